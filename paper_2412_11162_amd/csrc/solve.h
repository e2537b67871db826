// Right-hand sides, coupled-system data flow and field synthesis.
#pragma once
#include <hip/hip_runtime.h>
#include "lu.h"
#include "modal_math.h"

namespace pmlbie {

void launch_rhs_gather_point(const zd* raw, const int* rmap, int npt, int N, int M, int m0, int nrhs,
                             zd* b1, zd* b2, hipStream_t st);
// Interleaved system (equation 2i / 2i + 1 = upper / lower medium at node i,
// unknown 2l / 2l + 1 = u1 / phi1 at node l).  Right-hand sides from the
// lower-medium equations: row i of mode n at Alow + n * lstride + i * rstride.
void launch_lower_rhs(const zd* Alow, long lstride, long rstride, int N, int modes, int nrhs, const zd* b1,
                      const zd* b2, zd* rhs, hipStream_t st);
// One mode's interleaved matrix copied out in the block order [[K1 + I, -S1], [K2 - I, -S2]].
void launch_deinterleave(const zd* A, long n2, zd* out, hipStream_t st);
void launch_outputs(const zd* x, const zd* b1, const zd* b2, int N, int M, int nrhs, zd* u1, zd* p1,
                    zd* u2, zd* p2, hipStream_t st);
void launch_zero_column(zd* A, long n, int col, hipStream_t st);
void launch_fill_u32(unsigned* p, int n, unsigned v, hipStream_t st);
void launch_residual(const zd* A, long ms, int n, int modes, int nrhs, const zd* x, const zd* rhs,
                     zd* r, double* rs2, hipStream_t st);
void launch_sumsq(const double* sq, int n, int nvec, double* out, hipStream_t st);
void launch_sq(const zd* v, long count, double* sq, hipStream_t st);
void launch_axpy(zd* x, const zd* d, long count, hipStream_t st);
constexpr int FIELD_MAX_MODES = 1024;  // modes a field evaluation may sum
// Field at npts points for every right-hand side into out[r * ldo + p] (raw:
// the points' modal kernels against every node, [(p * N + l)][4][M + 1]).
void launch_field(const zd* raw, const double* W, int N, int M, int m0, int nrhs, int npts,
                  const int* medium, const double* theta, const zd* u1, const zd* p1, const zd* u2,
                  const zd* p2, zd* out, long ldo, hipStream_t st);

}  // namespace pmlbie
