/* Calls made the way a C caller makes them: an enumeration argument is a
 * plain int converted to the enumeration type, which C defines for any int
 * value; the library must validate it before using it. */
#include "expint.h"

int c_create_raw_bc(const expint_grid* g, const expint_dfield* d, double rho, int bc, const expint_opts* o,
                    expint_ctx** out) {
  return expint_create(g, d, rho, (expint_bc)bc, o, out);
}

int c_write_vtk_raw_dtype(const char* path, int nx, int ny, int nz, double h, const void* f, int dtype,
                          const char* name, const uint8_t* labels) {
  return expint_write_vtk(path, nx, ny, nz, h, f, (expint_dtype)dtype, name, labels);
}
