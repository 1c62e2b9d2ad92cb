// Host side of the modal path: closed-form 1D eigenbases, operator upload in
// the precision of the mode products, and the six-product phi1 chain.
//
// Zero flux (grad u . n = 0, the PDE of section 2): orthonormal cosine modes
//   Q[i][k] = c_k cos(pi k (i + 1/2) / n),  c_0 = sqrt(1/n), c_k = sqrt(2/n),
//   lambda_k = -(4/h^2) sin^2(pi k / (2n));
// zero ghost values (Dirichlet): orthonormal sine modes
//   Q[i][k] = sqrt(2/(n+1)) sin(pi (k+1)(i+1) / (n+1)),
//   lambda_k = -(4/h^2) sin^2(pi (k+1) / (2(n+1))).
// The forward transform applies Q^T (Qop[k][i] = Q[i][k]), the inverse Q.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "context.hpp"
#include "modal.hpp"

using namespace expint;

namespace {

uint16_t to_bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return static_cast<uint16_t>(u >> 16);
}
float bf16_bits_to_float(uint16_t h) {
  const uint32_t u = static_cast<uint32_t>(h) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

void eigen_1d(int n, double h, expint_bc bc, std::vector<double>& Q, std::vector<double>& lam) {
  Q.assign(static_cast<size_t>(n) * n, 0.0);
  lam.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < n; ++k) {
    if (bc == EXPINT_NOFLUX) {
      const double sn = std::sin(pi * k / (2.0 * n));
      lam[k] = -(4.0 / (h * h)) * sn * sn;
      const double ck = k == 0 ? std::sqrt(1.0 / n) : std::sqrt(2.0 / n);
      for (int i = 0; i < n; ++i) Q[static_cast<size_t>(i) * n + k] = ck * std::cos(pi * k * (i + 0.5) / n);
    } else {
      const double sn = std::sin(pi * (k + 1) / (2.0 * (n + 1)));
      lam[k] = -(4.0 / (h * h)) * sn * sn;
      const double ck = std::sqrt(2.0 / (n + 1));
      for (int i = 0; i < n; ++i) Q[static_cast<size_t>(i) * n + k] = ck * std::sin(pi * (k + 1) * (i + 1) / (n + 1.0));
    }
  }
}

// Upload one n x n operator (row i', column i) in the element type of prec.
int upload_op(expint_ctx* c, const std::vector<double>& op, int n, void** dst) {
  const size_t nn = static_cast<size_t>(n) * n;
  int rc;
  const int prec = c->modal.prec;
  if (prec == kPrecF64) {
    if ((rc = c->arena.alloc(dst, nn * sizeof(double)))) return rc;
    HIP_TRY(c, hipMemcpy(*dst, op.data(), nn * sizeof(double), hipMemcpyHostToDevice));
  } else if (prec == kPrecF32) {
    std::vector<float> f(nn);
    for (size_t i = 0; i < nn; ++i) f[i] = static_cast<float>(op[i]);
    if ((rc = c->arena.alloc(dst, nn * sizeof(float)))) return rc;
    HIP_TRY(c, hipMemcpy(*dst, f.data(), nn * sizeof(float), hipMemcpyHostToDevice));
  } else {
    std::vector<uint16_t> bits(2 * nn);
    for (size_t i = 0; i < nn; ++i) {
      if (prec == kPrecBF16) {
        const uint16_t hi = to_bf16_bits(static_cast<float>(op[i]));
        const double r = op[i] - static_cast<double>(bf16_bits_to_float(hi));
        bits[i] = hi;
        bits[nn + i] = to_bf16_bits(static_cast<float>(r));
      } else {
        const _Float16 hi = static_cast<_Float16>(op[i]);
        const double r = (op[i] - static_cast<double>(hi)) * 2048.0;  // lo scaled by 2^11, as in the kernel
        const _Float16 lo = static_cast<_Float16>(r);
        std::memcpy(&bits[i], &hi, 2);
        std::memcpy(&bits[nn + i], &lo, 2);
      }
    }
    if ((rc = c->arena.alloc(dst, 2 * nn * sizeof(uint16_t)))) return rc;
    HIP_TRY(c, hipMemcpy(*dst, bits.data(), 2 * nn * sizeof(uint16_t), hipMemcpyHostToDevice));
  }
  return EXPINT_OK;
}

}  // namespace

namespace expint {

int modal_setup(expint_ctx* c) {
  if (!c->labels_form) return set_error(EXPINT_EUNSUPPORTED, "the modal path needs the label form of D");
  if (c->g.nx % 32 || c->g.ny % 32 || c->g.nz % 32)
    return set_error(EXPINT_EUNSUPPORTED, "the modal path needs every grid dimension to be a multiple of 32");
  if (c->dtype == EXPINT_F64 && c->mp != EXPINT_MP_NONE)
    return set_error(EXPINT_EUNSUPPORTED, "split matrix-core products are for FP32 contexts");
  // uniform D over the classes present
  unsigned* mask = nullptr;
  int rc = c->arena.alloc(reinterpret_cast<void**>(&mask), sizeof(unsigned));
  if (rc) return rc;
  HIP_TRY(c, hipMemsetAsync(mask, 0, sizeof(unsigned), c->stream));
  HIP_TRY(c, launch_label_mask(c->labels, c->g.n, mask, c->stream));
  unsigned hmask = 0;
  HIP_TRY(c, hipMemcpyAsync(&hmask, mask, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->arena.release(mask);
  c->modal.present = hmask;
  if ((rc = modal_diffusivity(c, c->class_D, true))) return rc;
  c->modal.prec = c->dtype == EXPINT_F64 ? kPrecF64
                  : c->mp == EXPINT_MP_BF16_SPLIT ? kPrecBF16
                  : c->mp == EXPINT_MP_FP16_SPLIT ? kPrecF16
                                                  : kPrecF32;
  const int dims[3] = {c->g.nx, c->g.ny, c->g.nz};
  for (int ax = 0; ax < 3; ++ax) {
    const int n = dims[ax];
    std::vector<double> Q, lam;
    eigen_1d(n, c->h, c->bc, Q, lam);
    std::vector<double> fwd(static_cast<size_t>(n) * n), inv(static_cast<size_t>(n) * n);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < n; ++k) {
        fwd[static_cast<size_t>(k) * n + i] = Q[static_cast<size_t>(i) * n + k];  // Q^T
        inv[static_cast<size_t>(i) * n + k] = Q[static_cast<size_t>(i) * n + k];
      }
    if ((rc = upload_op(c, fwd, n, &c->modal.q[ax][0]))) return rc;
    if ((rc = upload_op(c, inv, n, &c->modal.q[ax][1]))) return rc;
    if ((rc = c->arena.alloc(reinterpret_cast<void**>(&c->modal.lam[ax]), n * sizeof(double)))) return rc;
    HIP_TRY(c, hipMemcpy(c->modal.lam[ax], lam.data(), n * sizeof(double), hipMemcpyHostToDevice));
    // zero flux, FP64 or FP32, a power-of-two length, tile rows within a
    // 32-bit offset: the products along this axis run as fast cosine
    // transforms (EXPINT_MODAL_DCT=0: dense products)
    const char* de = std::getenv("EXPINT_MODAL_DCT");
    const long post = ax == 0 ? static_cast<long>(c->g.ny) * c->g.nz : ax == 1 ? c->g.nz : 1;
    if (c->bc == EXPINT_NOFLUX && (c->modal.prec == kPrecF64 || c->modal.prec == kPrecF32) && dct_axis_ok(n) &&
        dct_rows_ok(c->modal.prec, n, ax == 2 ? 1 : 0, post) && !(de && de[0] == '0')) {
      std::vector<double> tw, mk;
      dct_tables(n, tw, mk);
      if ((rc = c->arena.alloc(reinterpret_cast<void**>(&c->modal.dct_tw[ax]), tw.size() * sizeof(double)))) return rc;
      if ((rc = c->arena.alloc(reinterpret_cast<void**>(&c->modal.dct_mk[ax]), mk.size() * sizeof(double)))) return rc;
      HIP_TRY(c, hipMemcpy(c->modal.dct_tw[ax], tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice));
      HIP_TRY(c, hipMemcpy(c->modal.dct_mk[ax], mk.data(), mk.size() * sizeof(double), hipMemcpyHostToDevice));
    }
  }
  const size_t fb = c->field_bytes();
  if ((rc = c->arena.alloc(&c->modal.t[0], fb))) return rc;
  if ((rc = c->arena.alloc(&c->modal.t[1], fb))) return rc;
  return EXPINT_OK;
}

bool modal_fuses_rhs(const expint_ctx* c) { return c->modal.dct_tw[2] != nullptr; }

int modal_diffusivity(expint_ctx* c, const double* class_D, bool set) {
  bool first = true;
  double Dc = 0.0;
  for (int a = 0; a < c->nclass; ++a) {
    if (!(c->modal.present & (1u << a))) continue;
    if (first) {
      Dc = class_D[a];
      first = false;
    } else if (class_D[a] != Dc) {
      return set_error(EXPINT_EUNSUPPORTED, "the modal path needs a uniform diffusivity (classes %d differ)", a);
    }
  }
  if (set) c->modal.Dc = Dc;
  return EXPINT_OK;
}

// out = tau phi1(tau A) b (add_into_out: out += ...), by six mode products;
// with u_rhs the first pass forms b = A u_rhs + f(u_rhs) itself.
int modal_phi1(expint_ctx* c, const void* b, void* out, bool add_into_out, const void* u_rhs) {
  const auto& md = c->modal;
  const int nx = c->g.nx, ny = c->g.ny, nz = c->g.nz;
  ModalArgs a;
  a.lam_x = md.lam[0];
  a.lam_y = md.lam[1];
  a.lam_z = md.lam[2];
  a.tauD = c->tau * md.Dc;
  a.tau = c->tau;
  a.nz = nz;
  auto run = [&](int side, int epi, int axis, int dir, const void* in, void* o, int pre, int n, long post) -> int {
    a.in = in;
    a.out = o;
    a.q = md.q[axis][dir];
    a.pre = pre;
    a.n = n;
    a.post = post;
    HIP_TRY(c, launch_mode_product(md.prec, side, epi, a, c->stream));
    return EXPINT_OK;
  };
  // an axis with fast-transform tables runs its products as DCTs (mode
  // kDctFwd / kDctInv; along x the forward transform, the multiplier and the
  // inverse transform in one pass), the others as dense products
  DctArgs d;
  d.lam_x = a.lam_x;
  d.lam_y = a.lam_y;
  d.lam_z = a.lam_z;
  d.tauD = a.tauD;
  d.tau = a.tau;
  d.nz = nz;
  auto run_dct = [&](int side, int mode, int epi, int axis, const void* in, void* o, int pre, int n, long post) -> int {
    d.in = in;
    d.out = o;
    d.tw = md.dct_tw[axis];
    d.mk = md.dct_mk[axis];
    d.pre = pre;
    d.n = n;
    d.post = post;
    HIP_TRY(c, launch_mode_dct(md.prec, side, mode, epi, d, c->stream));
    return EXPINT_OK;
  };
  const long nyz = static_cast<long>(ny) * nz;
  int rc;
  // forward: z (right), y (left), x (left, with the multiplier)
  if (u_rhs && !md.dct_tw[2]) return set_error(EXPINT_EINVAL, "the right-hand side is fused only where z runs as fast transforms");
  if (md.dct_tw[2] && u_rhs) {
    d.dh2 = md.Dc / (c->h * c->h);
    d.rho = c->rho;
    d.nx = nx;
    d.ny = ny;
    rc = run_dct(1, kDctRhsFwd, kEpiStore, 2, u_rhs, md.t[0], nx * ny, nz, 1);
  } else if (md.dct_tw[2]) {
    rc = run_dct(1, kDctFwd, kEpiStore, 2, b, md.t[0], nx * ny, nz, 1);
  } else {
    rc = run(1, kEpiStore, 2, 0, b, md.t[0], nx * ny, nz, 1);
  }
  if (rc) return rc;
  if (md.dct_tw[1]) rc = run_dct(0, kDctFwd, kEpiStore, 1, md.t[0], md.t[1], nx, ny, nz);
  else rc = run(0, kEpiStore, 1, 0, md.t[0], md.t[1], nx, ny, nz);
  if (rc) return rc;
  // x: the field ends in `cur`, `spare` is free
  void* cur = md.t[0];
  void* spare = md.t[1];
  if (md.dct_tw[0]) {
    if ((rc = run_dct(0, kDctFwdMulInv, kEpiStore, 0, md.t[1], md.t[0], 1, nx, nyz))) return rc;
  } else {
    if ((rc = run(0, kEpiMul, 0, 0, md.t[1], md.t[0], 1, nx, nyz))) return rc;
    if ((rc = run(0, kEpiStore, 0, 1, md.t[0], md.t[1], 1, nx, nyz))) return rc;
    cur = md.t[1];
    spare = md.t[0];
  }
  // inverse: y (left), z (right, into out)
  if (md.dct_tw[1]) rc = run_dct(0, kDctInv, kEpiStore, 1, cur, spare, nx, ny, nz);
  else rc = run(0, kEpiStore, 1, 1, cur, spare, nx, ny, nz);
  if (rc) return rc;
  const int zepi = add_into_out ? kEpiAddU : kEpiStore;
  if (md.dct_tw[2]) rc = run_dct(1, kDctInv, zepi, 2, spare, out, nx * ny, nz, 1);
  else rc = run(1, zepi, 2, 1, spare, out, nx * ny, nz, 1);
  return rc;
}

}  // namespace expint
