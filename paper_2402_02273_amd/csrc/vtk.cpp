// Legacy VTK output of a field on the grid (section 3.3 shows its 3-D
// results through ParaView, which reads this format).  Host code only: the
// field and labels are host arrays in the library's layout, z fastest,
// (i * ny + j) * nz + k; the file puts library axis i on VTK's x axis, so the
// values are written x fastest (i innermost), big-endian, as the format asks.

#include <cctype>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "context.hpp"
#include "internal.hpp"

using namespace expint;

namespace {

template <typename T>
void put_be(std::vector<unsigned char>& out, T v) {
  unsigned char b[sizeof(T)];
  std::memcpy(b, &v, sizeof(T));
  for (size_t q = 0; q < sizeof(T); ++q) out.push_back(b[sizeof(T) - 1 - q]);  // the host is little-endian
}

bool valid_name(const char* s) {
  if (!s || !*s || std::strlen(s) > 64) return false;
  for (const char* p = s; *p; ++p)
    if (!(std::isalnum(static_cast<unsigned char>(*p)) || *p == '_')) return false;
  return true;
}

}  // namespace

extern "C" {

int expint_write_vtk(const char* path, int32_t nx, int32_t ny, int32_t nz, double h, const void* field,
                     expint_dtype dtype, const char* name, const uint8_t* labels) {
  if (!path || !field) return set_error(EXPINT_EINVAL, "NULL argument");
  if (nx < 1 || ny < 1 || nz < 1) return set_error(EXPINT_EINVAL, "grid dims must be >= 1");
  if (!(h > 0.0) || !std::isfinite(h)) return set_error(EXPINT_EINVAL, "h must be finite and > 0");
  if (enum_value(dtype) != EXPINT_F32 && enum_value(dtype) != EXPINT_F64)
    return set_error(EXPINT_EINVAL, "unknown dtype");
  if (!valid_name(name)) return set_error(EXPINT_EINVAL, "name must be 1..64 letters, digits or '_'");
  const int64_t n = product_within(nx, ny, nz, INT64_MAX / 8);
  if (n < 0) return set_error(EXPINT_EINVAL, "grid too large");
  const int w = dtype == EXPINT_F64 ? 8 : 4;
  std::FILE* f = std::fopen(path, "wb");
  if (!f) return set_error(EXPINT_EIO, "cannot open %s for writing", path);
  char head[512];
  const int hn = std::snprintf(head, sizeof(head),
                               "# vtk DataFile Version 3.0\n"
                               "tumour density\n"
                               "BINARY\n"
                               "DATASET STRUCTURED_POINTS\n"
                               "DIMENSIONS %d %d %d\n"
                               "ORIGIN 0 0 0\n"
                               "SPACING %.17g %.17g %.17g\n"
                               "POINT_DATA %lld\n"
                               "SCALARS %s %s 1\n"
                               "LOOKUP_TABLE default\n",
                               nx, ny, nz, h, h, h, static_cast<long long>(n), name, w == 8 ? "double" : "float");
  bool ok = std::fwrite(head, 1, static_cast<size_t>(hn), f) == static_cast<size_t>(hn);
  // one z-plane (k) of VTK points at a time: x = i fastest, then y = j
  std::vector<unsigned char> buf;
  buf.reserve(static_cast<size_t>(nx) * ny * w);
  for (int k = 0; k < nz && ok; ++k) {
    buf.clear();
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const int64_t p = (static_cast<int64_t>(i) * ny + j) * nz + k;
        if (w == 8) put_be(buf, static_cast<const double*>(field)[p]);
        else put_be(buf, static_cast<const float*>(field)[p]);
      }
    ok = std::fwrite(buf.data(), 1, buf.size(), f) == buf.size();
  }
  if (ok && labels) {
    const char* lh = "\nSCALARS labels unsigned_char 1\nLOOKUP_TABLE default\n";
    ok = std::fwrite(lh, 1, std::strlen(lh), f) == std::strlen(lh);
    for (int k = 0; k < nz && ok; ++k) {
      buf.clear();
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) buf.push_back(labels[(static_cast<int64_t>(i) * ny + j) * nz + k]);
      ok = std::fwrite(buf.data(), 1, buf.size(), f) == buf.size();
    }
  }
  if (ok) ok = std::fputc('\n', f) != EOF;
  if (std::fclose(f) != 0) ok = false;
  if (!ok) return set_error(EXPINT_EIO, "writing %s failed", path);
  return EXPINT_OK;
}

}  // extern "C"
