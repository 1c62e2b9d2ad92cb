// Host-side checks of the runtime's validation and parsing paths, built with
// the address and undefined-behaviour sanitizers on host code only and run
// without a GPU: every creating call with invalid arguments (enumerations
// out of range included, as a C caller may pass them), the workspace cap, the
// plan rule over a sweep of inputs, the tuning-file parser on malformed
// files, and the VTK writer.  Exits non-zero on the first failed check; a
// sanitizer report aborts the run.

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>
#include <vector>

#include "expint.h"
#include "plan.hpp"
// the tuning-file parser and its caches have internal linkage
#include "autotune.cpp"

extern "C" {
// tests/sanitize/c_caller.c: enumeration arguments passed as a C caller does
int c_create_raw_bc(const expint_grid* g, const expint_dfield* d, double rho, int bc, const expint_opts* o,
                    expint_ctx** out);
int c_write_vtk_raw_dtype(const char* path, int nx, int ny, int nz, double h, const void* f, int dtype,
                          const char* name, const uint8_t* labels);
}

namespace {

int g_fail = 0;

void check(bool ok, const char* what) {
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s (last error: %s)\n", what, expint_last_error());
    ++g_fail;
  }
}

template <typename E>
void set_raw(E* e, int v) {
  static_assert(sizeof(E) == sizeof(int), "C enumerations are int-sized here");
  std::memcpy(e, &v, sizeof v);
}

int create(expint_grid g, expint_dfield d, double rho, int bc, const expint_opts& o) {
  expint_ctx* c = reinterpret_cast<expint_ctx*>(0x1);
  const int rc = c_create_raw_bc(&g, &d, rho, bc, &o, &c);
  check(c == nullptr, "context is NULL after an error");
  return rc;
}

void create_paths() {
  const double cd[3] = {0.0, 0.13, 0.013};
  expint_grid g{8, 8, 8, 1.0};
  expint_dfield d{reinterpret_cast<const uint8_t*>(0x1234), 3, cd, nullptr};
  expint_opts o;
  check(expint_opts_default(&o) == EXPINT_OK, "opts default");
  check(expint_opts_default(nullptr) == EXPINT_EINVAL, "opts default NULL");
  check(expint_create(nullptr, &d, 0.0, EXPINT_NOFLUX, &o, nullptr) == EXPINT_EINVAL, "NULL out");
  const double nan = std::numeric_limits<double>::quiet_NaN(), inf = std::numeric_limits<double>::infinity();
  struct Case {
    const char* name;
    void (*mut)(expint_grid&, expint_dfield&, expint_opts&, double&, int&);
    int want;
  };
  static const Case cases[] = {
      {"nx 0", [](expint_grid& g, expint_dfield&, expint_opts&, double&, int&) { g.nx = 0; }, EXPINT_EINVAL},
      {"nz negative", [](expint_grid& g, expint_dfield&, expint_opts&, double&, int&) { g.nz = -5; }, EXPINT_EINVAL},
      {"huge grid",
       [](expint_grid& g, expint_dfield&, expint_opts&, double&, int&) { g.nx = g.ny = g.nz = 2000000000; },
       EXPINT_EINVAL},
      {"h 0", [](expint_grid& g, expint_dfield&, expint_opts&, double&, int&) { g.h = 0.0; }, EXPINT_EINVAL},
      {"h inf",
       [](expint_grid& g, expint_dfield&, expint_opts&, double&, int&) {
         g.h = std::numeric_limits<double>::infinity();
       },
       EXPINT_EINVAL},
      {"rho nan",
       [](expint_grid&, expint_dfield&, expint_opts&, double& r, int&) { r = std::numeric_limits<double>::quiet_NaN(); },
       EXPINT_EINVAL},
      {"rho negative", [](expint_grid&, expint_dfield&, expint_opts&, double& r, int&) { r = -1.0; }, EXPINT_EINVAL},
      {"bc 7", [](expint_grid&, expint_dfield&, expint_opts&, double&, int& b) { b = 7; }, EXPINT_EINVAL},
      {"bc -1", [](expint_grid&, expint_dfield&, expint_opts&, double&, int& b) { b = -1; }, EXPINT_EINVAL},
      {"dtype 9", [](expint_grid&, expint_dfield&, expint_opts& o, double&, int&) { set_raw(&o.dtype, 9); },
       EXPINT_EINVAL},
      {"algo 5", [](expint_grid&, expint_dfield&, expint_opts& o, double&, int&) { set_raw(&o.algo, 5); },
       EXPINT_EINVAL},
      {"mp -3", [](expint_grid&, expint_dfield&, expint_opts& o, double&, int&) { set_raw(&o.mp, -3); },
       EXPINT_EINVAL},
      {"sweeps 4", [](expint_grid&, expint_dfield&, expint_opts& o, double&, int&) { set_raw(&o.sweeps, 4); },
       EXPINT_EINVAL},
      {"scheme 3", [](expint_grid&, expint_dfield&, expint_opts& o, double&, int&) { set_raw(&o.scheme, 3); },
       EXPINT_EINVAL},
      {"tau nan",
       [](expint_grid&, expint_dfield&, expint_opts& o, double&, int&) {
         o.tau = std::numeric_limits<double>::quiet_NaN();
       },
       EXPINT_EINVAL},
      {"tol inf",
       [](expint_grid&, expint_dfield&, expint_opts& o, double&, int&) {
         o.tol = std::numeric_limits<double>::infinity();
       },
       EXPINT_EINVAL},
      {"s only", [](expint_grid&, expint_dfield&, expint_opts& o, double&, int&) { o.s = 3; }, EXPINT_EINVAL},
      {"m 61", [](expint_grid&, expint_dfield&, expint_opts& o, double&, int&) { o.s = 1, o.m = 61; },
       EXPINT_EINVAL},
      {"m huge", [](expint_grid&, expint_dfield&, expint_opts& o, double&, int&) { o.s = 1, o.m = 2147483647; },
       EXPINT_EINVAL},
      {"n_classes 0", [](expint_grid&, expint_dfield& d, expint_opts&, double&, int&) { d.n_classes = 0; },
       EXPINT_EINVAL},
      {"n_classes 9", [](expint_grid&, expint_dfield& d, expint_opts&, double&, int&) { d.n_classes = 9; },
       EXPINT_EINVAL},
      {"class_D NULL", [](expint_grid&, expint_dfield& d, expint_opts&, double&, int&) { d.class_D = nullptr; },
       EXPINT_EINVAL},
      {"both forms", [](expint_grid&, expint_dfield& d, expint_opts&, double&, int&) { d.D = &d; }, EXPINT_EINVAL},
      {"no form", [](expint_grid&, expint_dfield& d, expint_opts&, double&, int&) { d.labels = nullptr; },
       EXPINT_EINVAL},
      {"mp without modal",
       [](expint_grid&, expint_dfield&, expint_opts& o, double&, int&) { o.mp = EXPINT_MP_BF16_SPLIT; },
       EXPINT_EUNSUPPORTED},
      {"modal 40^3",
       [](expint_grid& g, expint_dfield&, expint_opts& o, double&, int&) {
         g.nx = g.ny = g.nz = 40;
         o.algo = EXPINT_ALGO_MODAL;
       },
       EXPINT_EUNSUPPORTED},
      {"linearised modal",
       [](expint_grid& g, expint_dfield&, expint_opts& o, double&, int&) {
         g.nx = g.ny = g.nz = 32;
         o.algo = EXPINT_ALGO_MODAL;
         o.scheme = EXPINT_SCHEME_LINEARISED;
       },
       EXPINT_EUNSUPPORTED},
  };
  for (const Case& cs : cases) {
    expint_grid gg = g;
    expint_dfield dd = d;
    expint_opts oo = o;
    double rho = 0.025;
    int bc = EXPINT_NOFLUX;
    cs.mut(gg, dd, oo, rho, bc);
    const int rc = create(gg, dd, rho, bc, oo);
    if (rc != cs.want) std::fprintf(stderr, "case %s: rc %d, want %d\n", cs.name, rc, cs.want);
    check(rc == cs.want, cs.name);
    check(std::strlen(expint_last_error()) > 0, "an error message is set");
  }
  {
    double bad[3] = {0.0, nan, 0.013};
    expint_dfield dd = d;
    dd.class_D = bad;
    check(create(g, dd, 0.025, EXPINT_NOFLUX, o) == EXPINT_EINVAL, "class_D nan");
    bad[1] = -inf;
    check(create(g, dd, 0.025, EXPINT_NOFLUX, o) == EXPINT_EINVAL, "class_D -inf");
  }
  // the workspace cap, decided before the device is touched
  setenv("EXPINT_MAX_BYTES", "1000", 1);
  check(create(g, d, 0.025, EXPINT_NOFLUX, o) == EXPINT_ENOMEM, "workspace cap");
  setenv("EXPINT_MAX_BYTES", "not a number", 1);
  unsetenv("EXPINT_MAX_BYTES");
  expint_destroy(nullptr);
}

void batch_paths() {
  const double cd[3] = {0.0, 0.13, 0.013};
  expint_grid g[2] = {{8, 8, 8, 1.0}, {4, 6, 8, 1.0}};
  expint_dfield d[2] = {{reinterpret_cast<const uint8_t*>(0x1234), 3, cd, nullptr},
                        {reinterpret_cast<const uint8_t*>(0x1234), 3, cd, nullptr}};
  double rho[2] = {0.02, 0.03};
  expint_opts o;
  expint_opts_default(&o);
  expint_batch* b = reinterpret_cast<expint_batch*>(0x1);
  check(expint_batch_create(0, g, d, rho, EXPINT_NOFLUX, &o, &b) == EXPINT_EINVAL && b == nullptr, "batch count 0");
  check(expint_batch_create(2, g, d, nullptr, EXPINT_NOFLUX, &o, &b) == EXPINT_EINVAL, "batch rho NULL");
  rho[1] = -0.5;
  check(expint_batch_create(2, g, d, rho, EXPINT_NOFLUX, &o, &b) == EXPINT_EINVAL, "batch rho negative");
  rho[1] = 0.03;
  g[1].ny = 0;
  check(expint_batch_create(2, g, d, rho, EXPINT_NOFLUX, &o, &b) == EXPINT_EINVAL, "batch bad grid");
  g[1].ny = 6;
  d[1].n_classes = 12;
  check(expint_batch_create(2, g, d, rho, EXPINT_NOFLUX, &o, &b) == EXPINT_EINVAL, "batch n_classes");
  d[1].n_classes = 3;
  set_raw(&o.scheme, 11);
  check(expint_batch_create(2, g, d, rho, EXPINT_NOFLUX, &o, &b) != EXPINT_OK, "batch scheme");
  expint_batch_destroy(nullptr);
}

void plan_paths() {
  using expint::choose_plan;
  int s = 0, m = 0;
  check(choose_plan(0.0, 1e-6, std::log(64.0), &s, &m) && s == 1 && m == 1, "plan nu = 0");
  check(!choose_plan(-1.0, 1e-6, 1.0, &s, &m), "plan nu < 0");
  check(!choose_plan(std::numeric_limits<double>::quiet_NaN(), 1e-6, 1.0, &s, &m), "plan nu nan");
  check(!choose_plan(std::numeric_limits<double>::infinity(), 1e-6, 1.0, &s, &m), "plan nu inf");
  check(!choose_plan(1.0, 0.0, 1.0, &s, &m), "plan tol 0");
  check(!choose_plan(1.0, 1e-6, 1.0, &s, &m, 0), "plan m_min 0");
  for (double nu : {1e-300, 1e-12, 1e-3, 0.5, 1.0, 11.39, 21.1, 100.0, 1e4, 3e5}) {
    for (double tol : {1e-16, 1e-13, 1e-6, 1e-2}) {
      for (double th : {0.1, std::log(16.0), std::log(64.0), std::log(1024.0), 50.0}) {
        const bool ok = choose_plan(nu, tol, th, &s, &m);
        if (ok) {
          check(s >= 1 && m >= 1 && m <= expint::kPlanMaxDegree, "plan range");
          check(nu / s <= th * (1 + 1e-12), "plan theta cap");
        }
      }
    }
  }
}

void tune_file_paths() {
  const char* path = "sanitize_tune.txt";
  const std::vector<std::string> bodies = {
      "",
      "sweep",
      "sweep 1 2 3",
      "sweep 128 128 128 1 0 7 64 4 2 1 32 1\n",
      "sweep 128 128 128 1 0 7 64 4 3 1 32 1\n",  // lp 3: invalid, dropped
      "sweep 99999999999 2 3 4 5 6 7 8 9 10 11 12\n",
      "pair 8 8 8 1 0 0 8 8\npair 8 8 8 1 0 1 5 -3\n",
      "sweep -1 -1 -1 -1 -1 -1 -1 -1 -1 -1 -1 -1\nbogus 1 2 3\nsweep 4 4 4 1 0 7 64 4 1 0 64 0\n",
      std::string(4000, 'x') + " 1 2 3\n",
      "sweep 4 4 4 1 0 7 64 4 1 0 64 0 sweep 4 4 4 1 0 7 64 4 1 0 64",
  };
  for (size_t i = 0; i < bodies.size(); ++i) {
    FILE* f = std::fopen(path, "w");
    check(f != nullptr, "tune file written");
    if (!f) return;
    std::fputs(bodies[i].c_str(), f);
    std::fclose(f);
    // a different name each time, so the parser reads it again
    const std::string named = std::string(path) + "." + std::to_string(i);
    std::rename(path, named.c_str());
    setenv("EXPINT_TUNE_FILE", named.c_str(), 1);
    {
      std::lock_guard<std::mutex> lk(expint::g_mu);
      expint::load_tune_file();
      for (const auto& kv : expint::g_cache) check(expint::tiling_valid(kv.second), "cached tilings are valid");
    }
    std::remove(named.c_str());
  }
  setenv("EXPINT_TUNE_FILE", "/nonexistent/dir/tune.txt", 1);
  {
    std::lock_guard<std::mutex> lk(expint::g_mu);
    expint::load_tune_file();
    expint::append_tune_file("sweep 1 1 1 1 1 1 64 4 1 0 64 0\n");
  }
  unsetenv("EXPINT_TUNE_FILE");
}

void vtk_paths() {
  const int nx = 3, ny = 4, nz = 5;
  std::vector<float> f32(nx * ny * nz);
  std::vector<double> f64(nx * ny * nz);
  std::vector<uint8_t> lab(nx * ny * nz);
  for (int p = 0; p < nx * ny * nz; ++p) {
    f32[p] = 0.01f * p;
    f64[p] = 0.02 * p;
    lab[p] = static_cast<uint8_t>(p % 3);
  }
  check(expint_write_vtk("sanitize_a.vtk", nx, ny, nz, 1.0, f32.data(), EXPINT_F32, "u", lab.data()) == EXPINT_OK,
        "vtk f32");
  check(expint_write_vtk("sanitize_b.vtk", nx, ny, nz, 0.5, f64.data(), EXPINT_F64, "tumour_density", nullptr) ==
            EXPINT_OK,
        "vtk f64");
  check(expint_write_vtk("sanitize_c.vtk", nx, ny, nz, 1.0, f32.data(), EXPINT_F32, "bad name!", nullptr) ==
            EXPINT_EINVAL,
        "vtk name");
  check(expint_write_vtk("sanitize_c.vtk", nx, ny, nz, 1.0, f32.data(), EXPINT_F32, std::string(65, 'a').c_str(),
                         nullptr) == EXPINT_EINVAL,
        "vtk long name");
  check(c_write_vtk_raw_dtype("sanitize_c.vtk", nx, ny, nz, 1.0, f32.data(), 4, "u", nullptr) == EXPINT_EINVAL,
        "vtk dtype");
  check(expint_write_vtk("sanitize_c.vtk", 2000000000, 2000000000, 2000000000, 1.0, f32.data(), EXPINT_F32, "u",
                         nullptr) == EXPINT_EINVAL,
        "vtk huge grid");
  check(expint_write_vtk("/nonexistent/dir/x.vtk", nx, ny, nz, 1.0, f32.data(), EXPINT_F32, "u", nullptr) ==
            EXPINT_EIO,
        "vtk unwritable");
  std::remove("sanitize_a.vtk");
  std::remove("sanitize_b.vtk");
}

void diagnostics_paths() {
  int64_t d2 = 0;
  check(expint_tumour_size_static(nullptr, EXPINT_F32, 4, 4, 4, 0.5, &d2, nullptr, nullptr) == EXPINT_EINVAL,
        "static size NULL");
  check(expint_tumour_size_static(reinterpret_cast<void*>(0x1), 7, 4, 4, 4, 0.5, &d2, nullptr, nullptr) ==
            EXPINT_EINVAL,
        "static size dtype");
  check(expint_tumour_size_static(reinterpret_cast<void*>(0x1), EXPINT_F32, 400, 400, 400, 0.5, &d2, nullptr,
                                  nullptr) == EXPINT_EINVAL,
        "static size too large");
  check(expint_tumour_size_static(reinterpret_cast<void*>(0x1), EXPINT_F32, 1, 1 << 20, 1 << 20, 0.5, &d2, nullptr,
                                  nullptr) == EXPINT_EUNSUPPORTED,
        "static size cross-section");
  const int32_t th[3] = {10, 20, 15};
  check(expint_labels_from_intensity(reinterpret_cast<const uint8_t*>(0x10), 4, 4, 4, th, 3, 4, 4, 4,
                                     reinterpret_cast<uint8_t*>(0x1000), nullptr) == EXPINT_EINVAL,
        "labels thresholds not increasing");
  check(expint_labels_from_intensity(reinterpret_cast<const uint8_t*>(0x10), 4, 4, 4, th, 9, 4, 4, 4,
                                     reinterpret_cast<uint8_t*>(0x1000), nullptr) == EXPINT_EINVAL,
        "labels threshold count");
  check(expint_labels_from_intensity(reinterpret_cast<const uint8_t*>(0x1000), 8, 8, 8, th, 2, 8, 8, 8,
                                     reinterpret_cast<uint8_t*>(0x1100), nullptr) == EXPINT_EINVAL,
        "labels overlap");
}

}  // namespace

// FastDiv (the kernels' tile decomposition) against the division operator:
// every divisor the launches can see up to 4096 on dividends at the edges of
// each quotient, and large divisors and dividends up to 2^31 - 1.
void fastdiv_paths() {
  unsigned long long bad = 0;
  auto one = [&](uint32_t d, uint32_t x) {
    if (expint::FastDiv(d).div(x) != x / d) ++bad;
  };
  for (uint32_t d = 1; d <= 4096; ++d) {
    for (uint32_t x = 0; x < 3 * d + 3; ++x) one(d, x);
    for (uint32_t q : {1000u, 65535u, 1000000u, (0x7fffffffu / d) - 1, 0x7fffffffu / d}) {
      for (uint32_t r : {0u, 1u, d - 1}) {
        const unsigned long long x = static_cast<unsigned long long>(q) * d + r;
        if (x <= 0x7fffffffull) one(d, static_cast<uint32_t>(x));
      }
    }
    one(d, 0x7fffffffu);
  }
  for (uint32_t d : {65535u, 65536u, 65537u, 1000003u, 0x3fffffffu, 0x40000000u, 0x40000001u, 0x7fffffffu})
    for (uint32_t x : {0u, 1u, d - 1, d, d + 1, 2 * (d - 1) + 1, 0x7ffffffeu, 0x7fffffffu})
      if (x <= 0x7fffffffu) one(d, x);
  check(bad == 0, "FastDiv equals integer division");
}

int main() {
  fastdiv_paths();
  create_paths();
  batch_paths();
  plan_paths();
  tune_file_paths();
  vtk_paths();
  diagnostics_paths();
  std::printf("host checks: %d failed\n", g_fail);
  return g_fail ? 1 : 0;
}
