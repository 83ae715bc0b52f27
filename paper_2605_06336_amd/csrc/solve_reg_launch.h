// Launchers of the register-resident projected-problem kernels, one instantiation per padded
// size NB in {8, 16, ..., 56} (defined in solve_reg.h, instantiated in solve_reg_*.hip).
#pragma once
#include "internal.h"

namespace nlrmm {
namespace reg {

// Lst (optional, ldg * ldg + ldg doubles): receives the Cholesky factor of GA (rows) and its
// reciprocal diagonal; linc: it already holds them for the leading ell - 1 rows and columns
// of this GA, so only the appended row is formed.
template <int NB>
int launch_gks_solve_reg(const double *GA, const double *GP, int ldg, const double *rb,
                         const double *scal, int ell, double lam_fix, double *z, double *out,
                         int *status, hipStream_t s, double *Lst, int linc);
template <int NB>
int launch_compress_reg(const double *GA, const double *GP, int ldg, const double *lam, int ell,
                        int kmin, const double *z, double *T, int ldt, double *zout, int *kout,
                        int *status, hipStream_t s);

}  // namespace reg
}  // namespace nlrmm
