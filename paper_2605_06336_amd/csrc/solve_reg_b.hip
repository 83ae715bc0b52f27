// Instantiations of the register-resident projected-problem kernels for padded size 40.
#include "solve_reg.h"

namespace nlrmm {
namespace reg {

template int launch_gks_solve_reg<40>(const double *, const double *, int, const double *,
                                          const double *, int, double, double *, double *,
                                          int *, hipStream_t, double *, int);
template int launch_compress_reg<40>(const double *, const double *, int, const double *,
                                         int, int, const double *, double *, int, double *,
                                         int *, int *, hipStream_t);

}  // namespace reg
}  // namespace nlrmm
