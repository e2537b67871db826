// Right-hand sides, coupled-system data flow and field synthesis (Sec. 4.2).
#include "solve.h"
#include "rows16.h"

namespace pmlbie {

// b1 = -[u_tot0]_n, b2 = -[du_tot0/dnu_c]_n (modes n = m0..M, stored from
// index 0) from the raw modal values (modes 0..M) of the point-source pairs:
// raw[(inc * 2N + i)][s][n] with s = S1 for the pairs
// (node i, source) and s = K1 for the swapped pairs (source, node i) whose
// source-side conormal is the node's (the conormal derivative at the target
// of G~(r, r*) by the symmetry of G~).
__global__ void k_rhs_gather_point(const zd* __restrict__ raw, const int* __restrict__ rmap,
                                   int npt, int N, int M, int m0, int nrhs, zd* __restrict__ b1,
                                   zd* __restrict__ b2) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long tot = (long)(M + 1 - m0) * npt * N;
  if (e >= tot) return;
  const int i = (int)(e % N);
  const int pidx = (int)((e / N) % npt);
  const int nk = (int)(e / ((long)N * npt));  // kept mode index, mode m0 + nk
  const int n = m0 + nk;
  const long q1 = (long)pidx * 2 * N + i, q2 = q1 + N;
  const long o = ((long)nk * nrhs + rmap[pidx]) * N + i;
  b1[o] = -raw[q1 * 4 * (M + 1) + n];
  b2[o] = -raw[q2 * 4 * (M + 1) + (M + 1) + n];
}

// Right-hand sides of the interleaved system (equation 2i upper medium,
// 2i + 1 lower medium; unknown 2l = u1, 2l + 1 = phi1 at node l):
// rhs[2i] = 0, rhs[2i + 1] = sum_l Alow_i(2l) b1_l + Alow_i(2l + 1) b2_l, where
// Alow_i is the lower-medium equation [K2 - D2, -S2] of node i (row i of
// Alow at Alow + n * lstride + i * rstride).  64 rows per workgroup, every
// right-hand side at once (rows16.h); grid (row blocks, modes).
template <bool MM>
__global__ __launch_bounds__(256) void k_lower_rhs(const zd* __restrict__ Alow, long lstride, long rstride,
                                                   int N, int nrhs, const zd* __restrict__ b1,
                                                   const zd* __restrict__ b2, zd* __restrict__ rhs) {
  const int n = blockIdx.y;
  const zd* a = Alow + (long)n * lstride;
  const zd* x1 = b1 + (long)n * nrhs * N;
  const zd* x2 = b2 + (long)n * nrhs * N;
  zd* out = rhs + (long)n * nrhs * 2 * N;
  const int rbase = blockIdx.x * R16_ROWS;
  zd acc[4];
  bool ow;
  int og;
  rows16_acc<double, MM>(a, rstride, rbase, N, 0, 2 * N, nrhs,
                     [&](int s, int c) { return (c & 1) ? x2[(long)s * N + (c >> 1)] : x1[(long)s * N + (c >> 1)]; },
                     acc, ow, og);
  const int lane = threadIdx.x & 63;
  const int i = rbase + lane;
  if (i >= N || !ow) return;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int s = 4 * og + q;
    if (s < nrhs) {
      out[(long)s * 2 * N + 2 * i] = zd{0.0, 0.0};
      out[(long)s * 2 * N + 2 * i + 1] = acc[q];
    }
  }
}

// u1 = x[2i], phi1 = x[2i + 1] (interleaved unknowns), u2 = u1 - b1,
// phi2 = phi1 - b2 (transmission conditions), layout [mode][rhs][node].
__global__ void k_outputs(const zd* __restrict__ x, const zd* __restrict__ b1,
                          const zd* __restrict__ b2, int N, int M, int nrhs, zd* __restrict__ u1,
                          zd* __restrict__ p1, zd* __restrict__ u2, zd* __restrict__ p2) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long tot = (long)(M + 1) * nrhs * N;
  if (e >= tot) return;
  const int i = (int)(e % N);
  const long nr = e / N;  // mode * nrhs + r
  const zd xu = x[nr * 2 * N + 2 * i], xp = x[nr * 2 * N + 2 * i + 1];
  if (u1) u1[e] = xu;
  if (p1) p1[e] = xp;
  if (u2) u2[e] = xu - b1[e];
  if (p2) p2[e] = xp - b2[e];
}

// The interleaved system of one mode in the block order of the C ABI:
// out[R][C] with R, C < N the upper-medium equation / u1 unknown of node R, C
// and R, C >= N the lower-medium equation / phi1 unknown of node R - N, C - N.
__global__ void k_deinterleave(const zd* __restrict__ A, long n2, zd* __restrict__ out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n2 * n2) return;
  const long N = n2 >> 1;
  const long R = e / n2, C = e % n2;
  const long r = R < N ? 2 * R : 2 * (R - N) + 1;
  const long c = C < N ? 2 * C : 2 * (C - N) + 1;
  out[e] = A[r * n2 + c];
}

// Field modes by the Green representation (Sec. 4.2, eq. eqfujs) and the
// synthesis u = (1/2pi) sum_n u_n e^{i n theta} with u_{-n} = u_n over the
// built modes n = m0..M (boundary data stored from index 0):
//   u_n(x) = sgn sum_l W_l [S_n(x, r_l) phi_n(r_l) - K_n(x, r_l) u_n(r_l)],
// sgn = +1 in the upper medium, -1 in the lower one.  raw[(p * N + l)][s][n].
// One workgroup per point: threads take nodes l (the solution values of one
// mode are read coalesced), each node's kernels serve every right-hand side,
// a block reduction sums them; the result goes to out[r * ldo + p].
template <int RB>
__global__ __launch_bounds__(256) void k_field(const zd* __restrict__ raw, const double* __restrict__ W,
                                               int N, int M, int m0, int nrhs, const int* __restrict__ medium,
                                               const double* __restrict__ theta, const zd* __restrict__ u1,
                                               const zd* __restrict__ p1, const zd* __restrict__ u2,
                                               const zd* __restrict__ p2, zd* __restrict__ out, long ldo) {
  __shared__ double fn[FIELD_MAX_MODES];
  __shared__ zd part[4][RB];
  const int p = blockIdx.x, tid = threadIdx.x;
  const int md = medium[p];
  const double sgn = md == 1 ? 1.0 : -1.0;
  const int sS = md == 1 ? 0 : 2, sK = md == 1 ? 1 : 3;
  const zd* U = md == 1 ? u1 : u2;
  const zd* P = md == 1 ? p1 : p2;
  for (int n = m0 + tid; n <= M; n += 256)
    fn[n - m0] = (n == 0 ? 1.0 : 2.0) * cos(n * theta[p]) * sgn * (0.5 / PMLBIE_PI);
  __syncthreads();
  // every node's kernels are read once and weighted by the densities of all
  // right-hand sides (loops over the compile-time bound RB >= nrhs keep the
  // accumulators in registers)
  zd acc[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) acc[r] = zd{0.0, 0.0};
  for (int l = tid; l < N; l += 256) {
    const zd* rw = raw + ((long)p * N + l) * 4 * (M + 1);
    zd ul[RB];
#pragma unroll
    for (int r = 0; r < RB; ++r) ul[r] = zd{0.0, 0.0};
    for (int n = m0; n <= M; ++n) {
      const zd sv = fn[n - m0] * rw[sS * (M + 1) + n];
      const zd kv = fn[n - m0] * rw[sK * (M + 1) + n];
      const long base = (long)(n - m0) * nrhs * N + l;
#pragma unroll
      for (int r = 0; r < RB; ++r)
        if (r < nrhs) ul[r] = ul[r] + (sv * P[base + (long)r * N] - kv * U[base + (long)r * N]);
    }
#pragma unroll
    for (int r = 0; r < RB; ++r) acc[r] = acc[r] + W[l] * ul[r];
  }
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    if (r >= nrhs) break;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      acc[r].re += __shfl_xor(acc[r].re, off);
      acc[r].im += __shfl_xor(acc[r].im, off);
    }
    if ((tid & 63) == 0) part[tid >> 6][r] = acc[r];
  }
  __syncthreads();
  if (tid < nrhs) out[(long)tid * ldo + p] = part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
}

// Residual of the FP64 systems: r = rhs - A x for all modes and right-hand
// sides (A row-major n x n per mode), 64 rows per workgroup with every
// right-hand side at once (rows16.h: A read once, lane per row); rs2 receives
// |r_i|^2 for the convergence test.  Grid (row blocks, modes).
template <bool MM>
__global__ __launch_bounds__(256) void k_residual(const zd* __restrict__ A, long ms, int n,
                                                  int nrhs, const zd* __restrict__ x,
                                                  const zd* __restrict__ rhs, zd* __restrict__ r,
                                                  double* __restrict__ rs2) {
  const int md = blockIdx.y;
  const zd* a = A + (long)md * ms;
  const zd* xm = x + (long)md * nrhs * n;
  const int rbase = blockIdx.x * R16_ROWS;
  zd acc[4];
  bool ow;
  int og;
  rows16_acc<double, MM>(a, n, rbase, n, 0, n, nrhs, [&](int s, int c) { return xm[(long)s * n + c]; }, acc, ow, og);
  const int lane = threadIdx.x & 63;
  const int i = rbase + lane;
  if (i >= n || !ow) return;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int s = 4 * og + q;
    if (s < nrhs) {
      const long e = ((long)md * nrhs + s) * n + i;
      const zd d = rhs[e] - acc[q];
      r[e] = d;
      rs2[e] = abs2(d);
    }
  }
}

// Per (mode, rhs) sums of squares of vectors of length n: out[v] = sum |.|^2.
__global__ __launch_bounds__(256) void k_sumsq(const double* __restrict__ sq, int n, double* __restrict__ out) {
  const double* p = sq + (long)blockIdx.x * n;
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += p[i];
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

__global__ void k_sq(const zd* __restrict__ v, long count, double* __restrict__ sq) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) sq[e] = abs2(v[e]);
}

__global__ void k_axpy(zd* __restrict__ x, const zd* __restrict__ d, long count) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < count) x[e] = x[e] + d[e];
}

// Column `col` of a row-major n x n matrix set to zero (test hook of the
// zero-pivot path).
__global__ void k_zero_column(zd* __restrict__ A, long n, int col) {
  const long r = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) A[r * n + col] = zd{0.0, 0.0};
}

// n unsigned counters set to v (a kernel, not a memset: callers may capture
// the work that uses it in a graph).
__global__ void k_fill_u32(unsigned* __restrict__ p, int n, unsigned v) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}

void launch_fill_u32(unsigned* p, int n, unsigned v, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
}
void launch_zero_column(zd* A, long n, int col, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_column, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, A, n, col);
}
void launch_residual(const zd* A, long ms, int n, int modes, int nrhs, const zd* x, const zd* rhs,
                     zd* r, double* rs2, hipStream_t st) {
  hipLaunchKernelGGL(nrhs > 8 ? k_residual<true> : k_residual<false>, dim3((n + R16_ROWS - 1) / R16_ROWS, modes),
                     dim3(256), 0, st, A, ms, n, nrhs, x, rhs, r, rs2);
}
void launch_sumsq(const double* sq, int n, int nvec, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sumsq, dim3(nvec), dim3(256), 0, st, sq, n, out);
}
void launch_sq(const zd* v, long count, double* sq, hipStream_t st) {
  hipLaunchKernelGGL(k_sq, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, v, count, sq);
}
void launch_axpy(zd* x, const zd* d, long count, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, x, d, count);
}

void launch_rhs_gather_point(const zd* raw, const int* rmap, int npt, int N, int M, int m0, int nrhs,
                             zd* b1, zd* b2, hipStream_t st) {
  const long tot = (long)(M + 1 - m0) * npt * N;
  hipLaunchKernelGGL(k_rhs_gather_point, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, raw,
                     rmap, npt, N, M, m0, nrhs, b1, b2);
}
void launch_lower_rhs(const zd* Alow, long lstride, long rstride, int N, int modes, int nrhs, const zd* b1,
                      const zd* b2, zd* rhs, hipStream_t st) {
  hipLaunchKernelGGL(nrhs > 8 ? k_lower_rhs<true> : k_lower_rhs<false>, dim3((N + R16_ROWS - 1) / R16_ROWS, modes), dim3(256), 0, st, Alow, lstride,
                     rstride, N, nrhs, b1, b2, rhs);
}
void launch_deinterleave(const zd* A, long n2, zd* out, hipStream_t st) {
  const long tot = n2 * n2;
  hipLaunchKernelGGL(k_deinterleave, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, A, n2, out);
}
void launch_outputs(const zd* x, const zd* b1, const zd* b2, int N, int M, int nrhs, zd* u1, zd* p1,
                    zd* u2, zd* p2, hipStream_t st) {
  const long tot = (long)(M + 1) * nrhs * N;
  hipLaunchKernelGGL(k_outputs, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, x, b1, b2, N,
                     M, nrhs, u1, p1, u2, p2);
}
void launch_field(const zd* raw, const double* W, int N, int M, int m0, int nrhs, int npts,
                  const int* medium, const double* theta, const zd* u1, const zd* p1, const zd* u2,
                  const zd* p2, zd* out, long ldo, hipStream_t st) {
  if (npts <= 0 || nrhs <= 0) return;
  if (nrhs == 1)
    hipLaunchKernelGGL(k_field<1>, dim3(npts), dim3(256), 0, st, raw, W, N, M, m0, nrhs, medium, theta, u1,
                       p1, u2, p2, out, ldo);
  else if (nrhs <= 4)
    hipLaunchKernelGGL(k_field<4>, dim3(npts), dim3(256), 0, st, raw, W, N, M, m0, nrhs, medium, theta, u1,
                       p1, u2, p2, out, ldo);
  else
    hipLaunchKernelGGL(k_field<LU_MAX_RHS>, dim3(npts), dim3(256), 0, st, raw, W, N, M, m0, nrhs, medium,
                       theta, u1, p1, u2, p2, out, ldo);
}

}  // namespace pmlbie
