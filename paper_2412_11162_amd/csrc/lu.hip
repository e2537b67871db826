// Batched per-mode complex LU with partial pivoting and the matching solves
// (the per-mode dense solve of Sec. 4.2, eqs. eqntdpsi1/2, done as one
// 2N x 2N system per mode).  Matrices are stored row-major.
//
// Right-looking blocked algorithm with panel width LU_NB:
//   1. panel factorisation, one workgroup per matrix: the panel is walked in
//      sub-panels of 4 (8) columns held in registers (pivot search, row exchange
//      and rank-1 updates never leave the chip), each followed by the update
//      of the panel columns to its right;
//   2. the panel's row interchanges applied to the trailing columns, then the
//      triangular solve U12 = L11^{-1} A12;
//   3. trailing update A22 -= L21 U12 on the matrix cores (MFMA), a complex
//      product as three real MFMA products.
// Look-ahead: the update of step k is split into the next panel's columns
// and the rest; the next panel is factored on a second stream while the rest
// of the update runs (the panel touches only its own columns).
// Row interchanges are not applied to the columns left of the current panel:
// the forward solve applies each panel's interchanges to the right-hand side
// just before using that panel's columns of L, which are stored in the row
// order that was current when the panel was factored.
#include "lu.h"
#include "rows16.h"

namespace pmlbie {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int PNL_T = 1024;  // threads of the panel kernel

template <typename T>
__device__ __forceinline__ void wave_argmax(T& v, int& idx) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    T ov = __shfl_xor(v, off);
    int oi = __shfl_xor(idx, off);
    if (ov > v || (ov == v && (unsigned)oi < (unsigned)idx)) {
      v = ov;
      idx = oi;
    }
  }
}

// ---------------------------------------------------------------------------
// Panel factorisation: columns [k0, k0 + nb), rows [k0, n).  Thread t owns the
// local rows t, t + PNL_T, ... (local row = row - k0); RPT rows per thread.
template <typename T, int RPT>
__global__ __launch_bounds__(PNL_T) void k_panel(cx<T>* __restrict__ A, long ms, int n, int k0,
                                                 int nb, int cs0, int ce, int* __restrict__ ipiv,
                                                 int* __restrict__ info) {
  // register sub-panel width: 8 columns where the registers allow it (FP32 up
  // to two rows per thread), which halves the passes of the in-leaf update
  constexpr int SUB = (sizeof(T) == 4 && RPT <= 2) ? 8 : 4;
  cx<T>* a = A + (long)blockIdx.x * ms;
  int* piv = ipiv + (long)blockIdx.x * n;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int m = n - k0;
  __shared__ T sv[PNL_T / 64];
  __shared__ int si[PNL_T / 64];
  __shared__ cx<T> prow[SUB];
  __shared__ cx<T> sx[2][SUB];
  __shared__ cx<T> sinv;
  __shared__ int sp;
  __shared__ cx<T> L8[SUB][SUB];
  __shared__ cx<T> Ur[SUB][LU_NB];
  __shared__ cx<T> Ls[PNL_T][SUB];
  const cx<T> zero{T(0), T(0)};
  cx<T> x[RPT][SUB];
  for (int s0 = 0; s0 < nb; s0 += SUB) {
    // unconditional loads (rows past the end re-read the last row) so that
    // they are all in flight together; those rows are then zeroed
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int rl = tid + PNL_T * q;
      const cx<T>* src = a + (long)(k0 + min(rl, m - 1)) * n + k0 + s0;
#pragma unroll
      for (int jj = 0; jj < SUB; ++jj) x[q][jj] = src[jj];
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q)
#pragma unroll
      for (int jj = 0; jj < SUB; ++jj)
        if (tid + PNL_T * q >= m) x[q][jj] = zero;
#pragma unroll
    for (int jj = 0; jj < SUB; ++jj) {
      const int cl = s0 + jj;
      T best = T(-1);
      int bi = -1;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int rl = tid + PNL_T * q;
        if (rl >= cl && rl < m) {
          const T v = cabs1(x[q][jj]);
          if (v > best) {
            best = v;
            bi = rl;
          }
        }
      }
      wave_argmax(best, bi);
      if (lane == 0) {
        sv[wid] = best;
        si[wid] = bi;
      }
      __syncthreads();
      if (tid == 0) {
        T b = sv[0];
        int p = si[0];
        for (int w = 1; w < PNL_T / 64; ++w)
          if (sv[w] > b || (sv[w] == b && (unsigned)si[w] < (unsigned)p)) {
            b = sv[w];
            p = si[w];
          }
        if (p < 0) p = cl;
        sp = p;
        piv[k0 + cl] = k0 + p;
        if (!(b > T(0)) && info[blockIdx.x] == 0) info[blockIdx.x] = k0 + cl + 1;
      }
      __syncthreads();
      const int p = sp;
      // the diagonal row cl < LU_NB <= PNL_T lives in slot 0 of thread cl
      const int op = p % PNL_T, qp = p / PNL_T;
      if (p != cl) {
        if (tid == cl)
#pragma unroll
          for (int j2 = 0; j2 < SUB; ++j2) sx[0][j2] = x[0][j2];
        if (tid == op)
#pragma unroll
          for (int q = 0; q < RPT; ++q)
            if (q == qp)
#pragma unroll
              for (int j2 = 0; j2 < SUB; ++j2) sx[1][j2] = x[q][j2];
        // the rest of the two rows in memory over the enclosing LU_NB panel,
        // columns [cs0, ce); the trailing columns get the panel's interchanges
        // afterwards (k_laswp), so that the panel may run beside an update of
        // them
        for (int c = cs0 - k0 + tid; c < ce - k0; c += PNL_T)
          if (c < s0 || c >= s0 + SUB) {
            cx<T>* r1 = a + (long)(k0 + cl) * n + k0 + c;
            cx<T>* r2 = a + (long)(k0 + p) * n + k0 + c;
            const cx<T> t1 = *r1;
            *r1 = *r2;
            *r2 = t1;
          }
        __syncthreads();
        if (tid == cl)
#pragma unroll
          for (int j2 = 0; j2 < SUB; ++j2) x[0][j2] = sx[1][j2];
        if (tid == op)
#pragma unroll
          for (int q = 0; q < RPT; ++q)
            if (q == qp)
#pragma unroll
              for (int j2 = 0; j2 < SUB; ++j2) x[q][j2] = sx[0][j2];
      }
      if (tid == cl) {
#pragma unroll
        for (int j2 = 0; j2 < SUB; ++j2) prow[j2] = x[0][j2];
        const cx<T> pv = x[0][jj];
        sinv = (pv.re != T(0) || pv.im != T(0)) ? inv(pv) : zero;
      }
      __syncthreads();
      const cx<T> ip = sinv;
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        const int rl = tid + PNL_T * q;
        if (rl > cl && rl < m) {
          const cx<T> l = x[q][jj] * ip;
          x[q][jj] = l;
#pragma unroll
          for (int j2 = jj + 1; j2 < SUB; ++j2) x[q][j2] = x[q][j2] - l * prow[j2];
        }
      }
      __syncthreads();
    }
    // write the sub-panel back
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int rl = tid + PNL_T * q;
      if (rl < m) {
        cx<T>* dst = a + (long)(k0 + rl) * n + k0 + s0;
#pragma unroll
        for (int jj = 0; jj < SUB; ++jj) dst[jj] = x[q][jj];
      }
    }
    const int wr = nb - s0 - SUB;  // panel columns right of the sub-panel
    if (wr <= 0) continue;
    // U rows of the sub-panel: Ur = L8^{-1} A[s0 .. s0+SUB-1][right part]
    if (tid >= s0 && tid < s0 + SUB)
#pragma unroll
      for (int jj = 0; jj < SUB; ++jj) L8[tid - s0][jj] = x[0][jj];
    __syncthreads();  // row exchanges in memory and L8 visible
    for (int e = tid; e < SUB * wr; e += PNL_T) {
      const int r = e / wr, c = e % wr;
      Ur[r][c] = a[(long)(k0 + s0 + r) * n + k0 + s0 + SUB + c];
    }
    __syncthreads();
    for (int c = tid; c < wr; c += PNL_T) {
#pragma unroll
      for (int r = 1; r < SUB; ++r) {
        cx<T> acc = Ur[r][c];
#pragma unroll
        for (int j = 0; j < r; ++j) acc = acc - L8[r][j] * Ur[j][c];
        Ur[r][c] = acc;
      }
    }
    __syncthreads();
    for (int e = tid; e < SUB * wr; e += PNL_T) {
      const int r = e / wr, c = e % wr;
      a[(long)(k0 + s0 + r) * n + k0 + s0 + SUB + c] = Ur[r][c];
    }
    // rows below: A[r][right] -= L[r][0..SUB-1] Ur, one block of PNL_T rows at
    // a time with L staged in LDS so that the row segments are read coalesced;
    // UNR independent row segments in flight per step
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int base = PNL_T * q;
      if (base >= m) break;
#pragma unroll
      for (int jj = 0; jj < SUB; ++jj) Ls[tid][jj] = x[q][jj];
      __syncthreads();
      const int rlo = max(base, s0 + SUB), rhi = min(base + PNL_T, m);
      // thread -> (column c, first row rs), rows strided by PNL_T / wr
      const int c = tid % wr, rs = tid / wr, stride = PNL_T / wr;
      if (rs < stride) {
        cx<T> u[SUB];
#pragma unroll
        for (int j = 0; j < SUB; ++j) u[j] = Ur[j][c];
        cx<T>* col = a + (long)k0 * n + k0 + s0 + SUB + c;
        constexpr int UNR = 4;
        for (int r1 = rlo + rs; r1 < rhi; r1 += UNR * stride) {
          cx<T> v[UNR];
          // unconditional loads (rows past the end re-read the last row), so
          // that all UNR of them are in flight together
#pragma unroll
          for (int h = 0; h < UNR; ++h) v[h] = col[(long)min(r1 + h * stride, rhi - 1) * n];
#pragma unroll
          for (int h = 0; h < UNR; ++h) {
            const int rl = r1 + h * stride;
            if (rl < rhi) {
              cx<T> acc = v[h];
#pragma unroll
              for (int j = 0; j < SUB; ++j) acc = acc - Ls[rl - base][j] * u[j];
              col[(long)rl * n] = acc;
            }
          }
        }
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// X = L11^{-1} B for a tile of trsm_cols<T>() columns, held in LDS.  The
// rows are taken in blocks of JB = trsm_jb<T>(): the triangle of a block is
// solved by wavefronts without barriers (lane = row of the block x one of
// 64 / JB columns; the solved value of row q comes by a shuffle from lane q
// of the same group), then the rows below get the block's rank-JB update.
// With W == nullptr, B = A12 (columns k0 + nb .. cend - 1 of the panel rows)
// is overwritten by U12; otherwise B is the identity and X = L11^{-1} is
// written to W + b * LU_NB^2 (row-major, leading dimension LU_NB).  Blocks
// and tiles are 16 wide so that several workgroups fit in one CU's LDS.
template <typename T>
constexpr int trsm_jb() {
  return 16;
}
template <typename T>
constexpr int trsm_cols() {
  return 16;
}  // measured faster than 32 for both precisions (more workgroups per CU)
template <typename T>
__global__ __launch_bounds__(256) void k_trsm(cx<T>* __restrict__ A, long ms, int n, int k0,
                                              int nb, int cend, cx<T>* __restrict__ W) {
  constexpr int JB = trsm_jb<T>(), TC = trsm_cols<T>(), G = 64 / JB;
  cx<T>* a = A + (long)blockIdx.y * ms;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int cbase = (W ? 0 : k0 + nb) + blockIdx.x * TC;
  const int cmax = W ? nb : cend;
  __shared__ cx<T> Xs[LU_NB][TC + 1];
  __shared__ cx<T> Lb[LU_NB][JB + 1];
  const cx<T> zero{T(0), T(0)};
  for (int e = tid; e < nb * TC; e += 256) {
    const int r = e / TC, cc = e % TC, c = cbase + cc;
    if (W)
      Xs[r][cc] = cx<T>{(c < cmax && r == c) ? T(1) : T(0), T(0)};
    else
      Xs[r][cc] = c < cmax ? a[(long)(k0 + r) * n + c] : zero;
  }
  for (int j0 = 0; j0 < nb; j0 += JB) {
    const int jn = min(JB, nb - j0);
    for (int e = j0 * JB + tid; e < nb * JB; e += 256) {
      const int r = e / JB, jj = e % JB;
      Lb[r][jj] = jj < jn ? a[(long)(k0 + r) * n + k0 + j0 + jj] : zero;
    }
    __syncthreads();
    {
      const int rr = lane % JB, gs = lane / JB, base = lane - rr;
      for (int cg = wid; cg < TC / G; cg += 4) {
        const int cc = G * cg + gs;
        cx<T> y = rr < jn ? Xs[j0 + rr][cc] : zero;
        for (int q = 0; q < jn; ++q) {
          const int src = base + q;
          const cx<T> yq{__shfl(y.re, src), __shfl(y.im, src)};
          if (rr > q && rr < jn) y = y - Lb[j0 + rr][q] * yq;
        }
        if (rr < jn) Xs[j0 + rr][cc] = y;
      }
    }
    __syncthreads();
    // rows below the block: a rank-jn update
    const int r0 = j0 + jn;
    for (int e = tid; e < (nb - r0) * TC; e += 256) {
      const int r = r0 + e / TC, cc = e % TC;
      cx<T> acc = Xs[r][cc];
      for (int q = 0; q < jn; ++q) acc = acc - Lb[r][q] * Xs[j0 + q][cc];
      Xs[r][cc] = acc;
    }
    __syncthreads();
  }
  for (int e = tid; e < nb * TC; e += 256) {
    const int r = e / TC, cc = e % TC, c = cbase + cc;
    if (c >= cmax) continue;
    if (W)
      W[(long)blockIdx.y * LU_NB * LU_NB + (long)r * LU_NB + c] = Xs[r][cc];
    else
      a[(long)(k0 + r) * n + c] = Xs[r][cc];
  }
}

// ---------------------------------------------------------------------------
// Trailing update C -= L21 U12 on MFMA (rows below k0 + nb, columns
// k0 + nb .. cend - 1).  Workgroup tile 64 x 64 (complex), four waves of
// 32 x 32, K staged through LDS in chunks (16 complex64 / 8 complex128
// columns, two 4-wide MFMA steps unrolled together); registers held to four waves
// per SIMD (three for FP64), whose interleaving hides the global and LDS
// latencies.  The complex product takes three real products (the 3M form): with
// T1 = Lr Ur, T2 = Li Ui, T3 = (Lr + Li)(Ur + Ui), Re C -= T1 - T2 and
// Im C -= T3 - T1 - T2.  Three accumulators start from C,
// V1 = 0, V2 = Cr, V3 = Ci - Cr, and collect V1 += T1, V2 += T2, V3 -= T3;
// then Cr' = V2 - V1 and Ci' = V3 + V1 + V2.  A quarter fewer MFMAs than
// four real products; the error bound stays normwise that of the complex
// product (the imaginary part loses its componentwise bound), which the
// factorisation's backward error and the refinement absorb.
template <typename T> struct mfma_t;
template <> struct mfma_t<double> {
  typedef v4d acc;
  __device__ __forceinline__ static acc op(double x, double y, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
  }
  // lane l, register j -> row of the 16 x 16 output tile (column = l % 16)
  __device__ __forceinline__ static int rowof(int lane, int j) { return (lane >> 4) + 4 * j; }
};
template <> struct mfma_t<float> {
  typedef v4f acc;
  __device__ __forceinline__ static acc op(float x, float y, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int rowof(int lane, int j) { return 4 * (lane >> 4) + j; }
};

// U12 = L11^{-1} A12 on MFMA, in place: one workgroup per strip of 64
// trailing columns of the panel rows (it reads the whole strip before writing
// it), W = L11^{-1} from k_trsm.  Eight waves, each with two 16-row tiles
// (t and 7 - t) x 32 columns; the K chunks above a tile's rows are skipped (W
// is lower triangular), which leaves every wave the same work.
template <typename T>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_trsm_mfma(
    cx<T>* __restrict__ A, long ms, int n, int k0, int nb, int cbeg, int cend, const cx<T>* __restrict__ W) {
  typedef typename mfma_t<T>::acc acc_t;
  cx<T>* a = A + (long)blockIdx.y * ms;
  const cx<T>* w = W + (long)blockIdx.y * LU_NB * LU_NB;
  const int c0 = cbeg + blockIdx.x * 64;
  constexpr int KC = 16;
  __shared__ T Lre[KC][LU_NB + 4], Lim[KC][LU_NB + 4];  // W chunk: [k][row]
  __shared__ T Bre[KC][64 + 4], Bim[KC][64 + 4];        // A12 chunk: [k][col]
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  // wave: 16-row tiles t and 7 - t of the strip (W is lower triangular, so
  // tile t needs the first t + 1 K chunks: every wave has the same work)
  const int rt0 = 16 * (wid & 3), rt1 = 16 * (7 - (wid & 3)), wc = (wid >> 2) * 32;
  acc_t cr[2][2], ci[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      cr[x][y] = acc_t{0, 0, 0, 0};
      ci[x][y] = acc_t{0, 0, 0, 0};
    }
  // global -> register prefetch of the next K chunk overlaps the MFMA work
  // on the current one
  cx<T> pw[4], pa[2];
  auto gload = [&](int kk) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + 512 * t;
      const int k = e % KC, r = e / KC;
      pw[t] = (r < nb && kk + k < nb) ? w[(long)r * LU_NB + kk + k] : cx<T>{T(0), T(0)};
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int e = tid + 512 * t;
      const int cc = e & 63, k = e >> 6;
      const int gc = c0 + cc, gk = kk + k;
      pa[t] = (gc < cend && gk < nb) ? a[(long)(k0 + gk) * n + gc] : cx<T>{T(0), T(0)};
    }
  };
  gload(0);
  for (int kk = 0; kk < nb; kk += KC) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = tid + 512 * t;
      const int k = e % KC, r = e / KC;
      Lre[k][r] = pw[t].re;
      Lim[k][r] = pw[t].im;
    }
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int e = tid + 512 * t;
      const int cc = e & 63, k = e >> 6;
      Bre[k][cc] = pa[t].re;
      Bim[k][cc] = pa[t].im;
    }
    __syncthreads();
    if (kk + KC < nb) gload(kk + KC);
    if (kk < rt1 + 16) {
      const bool both = kk < rt0 + 16;  // tile rt0 still below the diagonal
#pragma unroll 1
      for (int k4 = 0; k4 < KC; k4 += 4) {
        const int kx = k4 + (lane >> 4), lx = lane & 15;
        T lr[2], li[2], br[2], bi[2];
        lr[0] = Lre[kx][rt0 + lx];
        li[0] = Lim[kx][rt0 + lx];
        lr[1] = Lre[kx][rt1 + lx];
        li[1] = Lim[kx][rt1 + lx];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          br[t] = Bre[kx][wc + 16 * t + lx];
          bi[t] = Bim[kx][wc + 16 * t + lx];
        }
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y) {
            if (x == 0 && !both) continue;
            cr[x][y] = mfma_t<T>::op(lr[x], br[y], cr[x][y]);
            cr[x][y] = mfma_t<T>::op(-li[x], bi[y], cr[x][y]);
            ci[x][y] = mfma_t<T>::op(lr[x], bi[y], ci[x][y]);
            ci[x][y] = mfma_t<T>::op(li[x], br[y], ci[x][y]);
          }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = (x == 0 ? rt0 : rt1) + mfma_t<T>::rowof(lane, j);
        const int gc = c0 + wc + 16 * y + (lane & 15);
        if (r < nb && gc < cend) a[(long)(k0 + r) * n + gc] = cx<T>{cr[x][y][j], ci[x][y][j]};
      }
}

// Tile order: workgroups are dealt to the 8 XCDs round-robin, so XCD x
// receives the contiguous range x*ceil(T/8) .. of the logical tile sequence;
// inside a matrix the sequence walks groups of 8 tile rows column by column,
// so the tiles in flight on one XCD share L21 rows and U12 columns in its L2.
template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 3 : 4))) void k_gemm_update(cx<T>* __restrict__ A, long ms, int n,
                                                     int k0, int nb, int cbeg, int cend, int tx, int ty,
                                                     int batch, int rend, const int* __restrict__ rmap,
                                                     int mapk, const cx<double>* __restrict__ csrc,
                                                     const int* __restrict__ cmap) {
  typedef typename mfma_t<T>::acc acc_t;
  const long tiles = (long)tx * ty * batch;
  const long per_xcd = (tiles + 7) / 8;
  const long lt = (long)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (lt >= tiles) return;
  const long per_mat = (long)tx * ty;
  const int bz = (int)(lt / per_mat);
  const int t = (int)(lt % per_mat);
  constexpr int GM = 8;
  const int grp = t / (GM * tx), in = t % (GM * tx);
  const int rows_in_grp = min(GM, ty - grp * GM);
  const int by = grp * GM + in % rows_in_grp, bx = in / rows_in_grp;
  cx<T>* a = A + (long)bz * ms;
  const int m0 = k0 + nb;
  const int r0 = m0 + by * 64;    // tile rows of C
  const int c0 = cbeg + bx * 64;  // tile columns of C (cbeg >= k0 + nb)
  // K chunk: 16 for complex64 (half the barriers), 8 for complex128 (16
  // would spill the prefetch registers at three waves per SIMD)
  constexpr int KC = sizeof(T) == 4 ? 16 : 8;
  constexpr int NP = KC / 4;  // prefetched elements of L21 and of U12 per thread
  __shared__ T Lre[KC][64 + 4], Lim[KC][64 + 4], Lsm[KC][64 + 4];  // L21 chunk: [k][row]
  __shared__ T Ure[KC][64 + 4], Uim[KC][64 + 4], Usm[KC][64 + 4];  // U12 chunk: [k][col]
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wr = (wid & 1) * 32, wc = (wid >> 1) * 32;
  // the accumulators start from C (loaded before the K loop, so its latency
  // overlaps the first chunk) and the products are subtracted; with csrc, C
  // is read from the FP64 matrices, row r at row cmap[r], and rounded to T
  // (complex64 only: the complex128 kernel keeps its registers)
  acc_t v1[2][2], v2[2][2], v3[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int gr = r0 + wr + 16 * x + mfma_t<T>::rowof(lane, j);
        const int gc = c0 + wc + 16 * y + (lane & 15);
        cx<T> v{T(0), T(0)};
        if (gc < cend && gr < rend) {
          if constexpr (sizeof(T) == 4) {
            if (csrc) {
              const cx<double> w = csrc[(long)bz * ms + (long)cmap[(long)bz * n + gr] * n + gc];
              v = cx<T>{(T)w.re, (T)w.im};
            } else {
              v = a[(long)gr * n + gc];
            }
          } else {
            v = a[(long)gr * n + gc];
          }
        }
        v1[x][y][j] = T(0);
        v2[x][y][j] = v.re;
        v3[x][y][j] = v.im - v.re;
      }
  // global -> register prefetch of the next K chunk overlaps the MFMA work
  // on the current one; each thread moves NP elements of L21 and of U12
  cx<T> pl[NP], pu[NP];
  // a thread's rows of L21 are the same in every chunk: the storage rows of
  // the first mapk columns (through rmap) are read once
  int mrow[NP];
#pragma unroll
  for (int t = 0; t < NP; ++t) {
    const int gr = r0 + (tid + 256 * t) / KC;
    mrow[t] = (rmap && gr < rend) ? rmap[(long)bz * n + gr] : gr;
  }
  auto gload = [&](int kk) {
#pragma unroll
    for (int t = 0; t < NP; ++t) {
      const int e = tid + 256 * t;
      const int k = e % KC, rr = e / KC;  // row-major L21: k contiguous
      const int gr = r0 + rr, gk = kk + k;
      const int lr = gk < mapk ? mrow[t] : gr;
      pl[t] = (gr < rend && gk < nb) ? a[(long)lr * n + k0 + gk] : cx<T>{T(0), T(0)};
      const int cc = e & 63, ku = e >> 6;  // row-major U12: columns contiguous
      const int gc = c0 + cc, gku = kk + ku;
      pu[t] = (gc < cend && gku < nb) ? a[(long)(k0 + gku) * n + gc] : cx<T>{T(0), T(0)};
    }
  };
  gload(0);
  for (int kk = 0; kk < nb; kk += KC) {
#pragma unroll
    for (int t = 0; t < NP; ++t) {
      const int e = tid + 256 * t;
      const int k = e % KC, rr = e / KC;
      Lre[k][rr] = pl[t].re;
      Lim[k][rr] = pl[t].im;
      Lsm[k][rr] = pl[t].re + pl[t].im;
      const int cc = e & 63, ku = e >> 6;
      Ure[ku][cc] = pu[t].re;
      Uim[ku][cc] = pu[t].im;
      Usm[ku][cc] = pu[t].re + pu[t].im;
    }
    __syncthreads();
    if (kk + KC < nb) gload(kk + KC);
#pragma unroll 2
    for (int k4 = 0; k4 < KC; k4 += 4) {
      const int kx = k4 + (lane >> 4), lx = lane & 15;
      T lr[2], li[2], ls[2], ur[2], ui[2], us[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        lr[t] = Lre[kx][wr + 16 * t + lx];  // X[p][k] = L[row p][k]
        li[t] = Lim[kx][wr + 16 * t + lx];
        ls[t] = Lsm[kx][wr + 16 * t + lx];
        ur[t] = Ure[kx][wc + 16 * t + lx];  // Y[k][q] = U[k][col q]
        ui[t] = Uim[kx][wc + 16 * t + lx];
        us[t] = Usm[kx][wc + 16 * t + lx];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)      // row sub-tile
#pragma unroll
        for (int y = 0; y < 2; ++y) {  // column sub-tile
          v1[x][y] = mfma_t<T>::op(lr[x], ur[y], v1[x][y]);
          v2[x][y] = mfma_t<T>::op(li[x], ui[y], v2[x][y]);
          v3[x][y] = mfma_t<T>::op(-ls[x], us[y], v3[x][y]);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int gr = r0 + wr + 16 * x + mfma_t<T>::rowof(lane, j);
        const int gc = c0 + wc + 16 * y + (lane & 15);
        if (gc < cend && gr < rend)
          a[(long)gr * n + gc] = cx<T>{v2[x][y][j] - v1[x][y][j], v3[x][y][j] + v1[x][y][j] + v2[x][y][j]};
      }
}

// ---------------------------------------------------------------------------
// Solves with the factors, panel by panel; nrhs right-hand sides stored as
// b[mat][rhs][n] (overwritten by the solution).
//   forward, panel [k0, k0+nb): (1) one workgroup per matrix applies the
//   panel's row interchanges to b and solves the unit lower diagonal block;
//   (2) many workgroups update the rows below, one wavefront per row.
//   backward: (3) the upper diagonal block, (4) the rows above.
// Columns [j0, j0 + jn) of the diagonal block, rows [r_lo, r_hi), into Lb,
// by 256 threads: a thread issues all of its loads before its first LDS
// store, so their latencies overlap instead of adding up.
template <typename T>
__device__ __forceinline__ void stage_cols(const cx<T>* __restrict__ a, int n, int k0, int r_lo, int r_hi,
                                           int j0, int jn, cx<T> (*Lb)[33]) {
  constexpr int PER = LU_NB * 32 / 256;
  cx<T> v[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = r_lo * 32 + (int)threadIdx.x + 256 * i;
    const int r = e >> 5, jj = e & 31;
    v[i] = (e < r_hi * 32 && jj < jn) ? a[(long)(k0 + r) * n + k0 + j0 + jj] : cx<T>{T(0), T(0)};
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = r_lo * 32 + (int)threadIdx.x + 256 * i;
    if (e < r_hi * 32) Lb[e >> 5][e & 31] = v[i];
  }
}

// Triangle of a 32-column block of the diagonal block, solved by one
// wavefront without barriers: lane l holds the entries (row j0 + (l & 31),
// rhs 2 t + (l >> 5)) in slot t < NT (NT >= (nrhs + 1) / 2, slots beyond the
// right-hand sides hold zeros), so the entry (row j0 + jj, same rhs) of slot
// t sits in lane (l & 32) + jj, slot t.  Lower: unit diagonal, forward;
// upper: divided by the diagonal, backward.  A step's NT broadcasts are
// issued together, then the NT updates.
template <typename T, typename TB, bool UPPER, int NT>
__device__ __forceinline__ void tri_wave(cx<T> (*Lb)[33], cx<TB> (*yb)[LU_MAX_RHS], int j0, int jn,
                                         int nrhs) {
  const int lane = threadIdx.x & 63, rr = lane & 31, hs = lane >> 5;
  cx<TB> y[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int s2 = 2 * t + hs;
    y[t] = (rr < jn && s2 < nrhs) ? yb[j0 + rr][s2] : cx<TB>{TB(0), TB(0)};
  }
  // upper: each lane's own row's diagonal inverse, once (y / d is y * inv(d))
  cx<TB> dinv{TB(0), TB(0)};
  if (UPPER && rr < jn) {
    const cx<T> d = Lb[j0 + rr][rr];
    dinv = inv(cx<TB>{(TB)d.re, (TB)d.im});
  }
  for (int q = 0; q < jn; ++q) {
    const int jj = UPPER ? jn - 1 - q : q;
    const cx<T> lj = Lb[j0 + rr][jj];
    if (UPPER && rr == jj) {
#pragma unroll
      for (int t = 0; t < NT; ++t) y[t] = y[t] * dinv;
    }
    const int src = (lane & 32) + jj;
    const bool below = UPPER ? rr < jj : (rr > jj && rr < jn);
    cx<TB> yj[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) yj[t] = cx<TB>{__shfl(y[t].re, src), __shfl(y[t].im, src)};
    if (below) {
      const cx<TB> l{(TB)lj.re, (TB)lj.im};
#pragma unroll
      for (int t = 0; t < NT; ++t) y[t] = y[t] - l * yj[t];
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int s2 = 2 * t + hs;
    if (rr < jn && s2 < nrhs) yb[j0 + rr][s2] = y[t];
  }
}

template <typename T, typename TB, int NT>
__global__ __launch_bounds__(256) void k_solve_diag(const cx<T>* __restrict__ A, long ms, int n,
                                                    int k0, int nb, const int* __restrict__ ipiv,
                                                    cx<TB>* __restrict__ B, int nrhs, int upper) {
  const cx<T>* a = A + (long)blockIdx.x * ms;
  const int* piv = ipiv + (long)blockIdx.x * n;
  cx<TB>* b = B + (long)blockIdx.x * nrhs * n;
  const int tid = threadIdx.x;
  constexpr int JB = 32;
  __shared__ cx<TB> yb[LU_NB][LU_MAX_RHS];
  __shared__ cx<T> Lb[LU_NB][JB + 1];  // a block of JB columns of the diagonal block
  __shared__ cx<TB> ext[LU_NB][LU_MAX_RHS];  // pivot rows below the panel
  __shared__ int pv[LU_NB], slot[LU_NB];
  static_assert(JB == 32, "tri_wave holds 32 rows per half wavefront");
  constexpr int PERB = LU_NB * LU_MAX_RHS / 256;
  {
    cx<TB> v[PERB];
#pragma unroll
    for (int i = 0; i < PERB; ++i) {
      const int e = tid + 256 * i;
      v[i] = e < nb * nrhs ? b[(long)(e / nb) * n + k0 + e % nb] : cx<TB>{TB(0), TB(0)};
    }
#pragma unroll
    for (int i = 0; i < PERB; ++i) {
      const int e = tid + 256 * i;
      if (e < nb * nrhs) yb[e % nb][e / nb] = v[i];
    }
  }
  __syncthreads();
  if (!upper) {
    // the panel's row interchanges, in order.  A pivot row p below the panel
    // is read once into ext[slot] (slot: the first interchange naming p),
    // the interchanges then run in LDS, and the rows below are written back.
    if (tid < nb) pv[tid] = piv[k0 + tid] - k0;
    __syncthreads();
    if (tid < nb) {
      const int p = pv[tid];
      int sl = tid;
      if (p >= nb)
        for (int i = 0; i < tid; ++i)
          if (pv[i] == p) {
            sl = i;
            break;
          }
      slot[tid] = sl;
    }
    __syncthreads();
    {
      cx<TB> v[PERB];
#pragma unroll
      for (int i = 0; i < PERB; ++i) {
        const int e = tid + 256 * i, j = e % nb;
        v[i] = (e < nb * nrhs && pv[j] >= nb && slot[j] == j) ? b[(long)(e / nb) * n + k0 + pv[j]]
                                                               : cx<TB>{TB(0), TB(0)};
      }
#pragma unroll
      for (int i = 0; i < PERB; ++i) {
        const int e = tid + 256 * i;
        if (e < nb * nrhs) ext[e % nb][e / nb] = v[i];
      }
    }
    __syncthreads();
    if (tid < nrhs) {
      for (int j = 0; j < nb; ++j) {
        const int p = pv[j];
        if (p == j) continue;
        cx<TB>& o = p < nb ? yb[p][tid] : ext[slot[j]][tid];
        const cx<TB> t0 = yb[j][tid];
        yb[j][tid] = o;
        o = t0;
      }
    }
    __syncthreads();
    for (int e = tid; e < nb * nrhs; e += 256) {
      const int j = e % nb;
      if (pv[j] >= nb && slot[j] == j) b[(long)(e / nb) * n + k0 + pv[j]] = ext[j][e / nb];
    }
    for (int j0 = 0; j0 < nb; j0 += JB) {
      const int jn = min(JB, nb - j0);
      stage_cols(a, n, k0, j0, nb, j0, jn, Lb);
      __syncthreads();
      // the triangle of the block: one wavefront, register-held entries
      if (tid < 64) tri_wave<T, TB, false, NT>(Lb, yb, j0, jn, nrhs);
      __syncthreads();
      // rows below the block inside the panel: a rank-jn update
      for (int e = tid; e < (nb - j0 - jn) * nrhs; e += 256) {
        const int r = j0 + jn + e % (nb - j0 - jn), s2 = e / (nb - j0 - jn);
        cx<TB> acc = yb[r][s2];
        for (int jj = 0; jj < jn; ++jj) {
          const cx<T> l = Lb[r][jj];
          acc = acc - cx<TB>{(TB)l.re, (TB)l.im} * yb[j0 + jj][s2];
        }
        yb[r][s2] = acc;
      }
      __syncthreads();
    }
  } else {
    for (int j1 = nb; j1 > 0; j1 -= JB) {  // columns [j0, j1), last block first
      const int j0 = max(0, j1 - JB), jn = j1 - j0;
      stage_cols(a, n, k0, 0, j1, j0, jn, Lb);
      __syncthreads();
      if (tid < 64) tri_wave<T, TB, true, NT>(Lb, yb, j0, jn, nrhs);
      __syncthreads();
      // rows above the block: a rank-jn update
      for (int e = tid; e < j0 * nrhs; e += 256) {
        const int r = e % j0, s2 = e / j0;
        cx<TB> acc = yb[r][s2];
        for (int jj = 0; jj < jn; ++jj) {
          const cx<T> u = Lb[r][jj];
          acc = acc - cx<TB>{(TB)u.re, (TB)u.im} * yb[j0 + jj][s2];
        }
        yb[r][s2] = acc;
      }
      __syncthreads();
    }
  }
  for (int e = tid; e < nb * nrhs; e += 256) b[(long)(e / nb) * n + k0 + e % nb] = yb[e % nb][e / nb];
}

// rows [r0, r1) of b -= A[rows][k0 .. k0+nb) * b[k0 .. k0+nb) for every
// right-hand side: 64 rows per workgroup, LDS-staged tiles, lane per row
// (rows16.h); grid (row blocks of 64, matrices).
template <typename T, typename TB, bool MM>
__global__ __launch_bounds__(256) void k_solve_update(const cx<T>* __restrict__ A, long ms, int n,
                                                      int k0, int nb, cx<TB>* __restrict__ B,
                                                      int nrhs, int r0, int r1) {
  const cx<T>* a = A + (long)blockIdx.y * ms;
  cx<TB>* b = B + (long)blockIdx.y * nrhs * n;
  const int rbase = r0 + blockIdx.x * R16_ROWS;
  zd acc[4];
  bool ow;
  int og;
  rows16_acc<T, MM>(a, n, rbase, r1, k0, k0 + nb, nrhs,
                [&](int s2, int c) {
                  const cx<TB> v = b[(long)s2 * n + c];
                  return zd{(double)v.re, (double)v.im};
                },
                acc, ow, og);
  const int lane = threadIdx.x & 63;
  const int row = rbase + lane;
  if (row >= r1 || !ow) return;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int s2 = 4 * og + q;
    if (s2 < nrhs) {
      cx<TB>& o = b[(long)s2 * n + row];
      o = cx<TB>{o.re - (TB)acc[q].re, o.im - (TB)acc[q].im};
    }
  }
}

// ---------------------------------------------------------------------------
template <typename T, int RPT>
static void launch_panel(cx<T>* A, long ms, int n, int k0, int nb, int cs0, int ce, int batch, int* ipiv,
                         int* info, hipStream_t st) {
  hipLaunchKernelGGL((k_panel<T, RPT>), dim3(batch), dim3(PNL_T), 0, st, A, ms, n, k0, nb, cs0, ce, ipiv,
                     info);
}

template <typename T>
static void panel_any(cx<T>* A, long ms, int n, int k0, int nb, int cs0, int ce, int batch, int* ipiv,
                      int* info, hipStream_t st) {
  const int m = n - k0;
  if (m <= 1 * PNL_T) launch_panel<T, 1>(A, ms, n, k0, nb, cs0, ce, batch, ipiv, info, st);
  else if (m <= 2 * PNL_T) launch_panel<T, 2>(A, ms, n, k0, nb, cs0, ce, batch, ipiv, info, st);
  else if (m <= 4 * PNL_T) launch_panel<T, 4>(A, ms, n, k0, nb, cs0, ce, batch, ipiv, info, st);
  else launch_panel<T, 8>(A, ms, n, k0, nb, cs0, ce, batch, ipiv, info, st);
}

// Row interchanges of rows [k0, k0 + nb) applied, in order, to columns
// [c0, c1): one thread per column.
template <typename T>
__global__ __launch_bounds__(256) void k_laswp(cx<T>* __restrict__ A, long ms, int n, int k0, int nb, int c0,
                                               int c1, const int* __restrict__ ipiv) {
  cx<T>* a = A + (long)blockIdx.y * ms;
  const int* piv = ipiv + (long)blockIdx.y * n;
  const int c = c0 + blockIdx.x * 256 + threadIdx.x;
  if (c >= c1) return;
  for (int j = k0; j < k0 + nb; ++j) {
    const int p = piv[j];
    if (p != j) {
      cx<T>* r1 = a + (long)j * n + c;
      cx<T>* r2 = a + (long)p * n + c;
      const cx<T> t1 = *r1;
      *r1 = *r2;
      *r2 = t1;
    }
  }
}

// U12 = L11^{-1} A12 for columns [cbeg, cend) of the rows [k0, k0 + nb),
// cbeg >= k0 + nb: with W, W = L11^{-1} by the column solver and the product
// on MFMA; without, the column solver in place (cbeg = k0 + nb).
template <typename T>
static void trsm_part(cx<T>* A, long ms, int n, int k0, int nb, int cbeg, int cend, int batch, hipStream_t st,
                      cx<T>* W) {
  const int cols = cend - cbeg;
  if (cols <= 0) return;
  if (W) {
    hipLaunchKernelGGL(k_trsm<T>, dim3((nb + trsm_cols<T>() - 1) / trsm_cols<T>(), batch), dim3(256), 0, st, A, ms,
                       n, k0, nb, cend, W);
    hipLaunchKernelGGL(k_trsm_mfma<T>, dim3((cols + 63) / 64, batch), dim3(512), 0, st, A, ms, n, k0, nb, cbeg,
                       cend, (const cx<T>*)W);
  } else {
    hipLaunchKernelGGL(k_trsm<T>, dim3((cols + trsm_cols<T>() - 1) / trsm_cols<T>(), batch), dim3(256), 0, st, A, ms, n, k0, nb,
                       cend, (cx<T>*)nullptr);
  }
}

// A22 -= L21 U12 over the rows [k0 + nb, rend) (rend < 0: n) and columns
// [cbeg, cend); with rmap, the rows of the first mapk columns of L21 are
// read at rmap[row] (per matrix, n entries).
template <typename T>
static void gemm_part(cx<T>* A, long ms, int n, int k0, int nb, int cbeg, int cend, int batch, hipStream_t st,
                      int rend = -1, const int* rmap = nullptr, int mapk = 0, const cx<double>* csrc = nullptr,
                      const int* cmap = nullptr) {
  if (rend < 0) rend = n;
  const int cols = cend - cbeg, rows = rend - k0 - nb;
  if (cols <= 0 || rows <= 0) return;
  const int tx = (cols + 63) / 64, ty = (rows + 63) / 64;
  const long tiles = (long)tx * ty * batch;
  const long grid = ((tiles + 7) / 8) * 8;
  hipLaunchKernelGGL(k_gemm_update<T>, dim3((unsigned)grid), dim3(256), 0, st, A, ms, n, k0, nb, cbeg, cend,
                     tx, ty, batch, rend, rmap, mapk, csrc, cmap);
}

// D = S rounded to T over rows [r0, r1) x columns [c0, c1) of every matrix
// (grid y = matrix); with rmap, row r of D is read from row rmap[r] of S
// (per matrix, n entries).
template <typename T>
__global__ __launch_bounds__(256) void k_demote(const cx<double>* __restrict__ S, cx<T>* __restrict__ D, long ms,
                                                int n, int r0, int r1, int c0, int c1,
                                                const int* __restrict__ rmap) {
  const long cw = c1 - c0, cnt = (long)(r1 - r0) * cw;
  const cx<double>* s = S + (long)blockIdx.y * ms;
  cx<T>* d = D + (long)blockIdx.y * ms;
  const int* mp = rmap ? rmap + (long)blockIdx.y * n : nullptr;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < cnt; e += (long)gridDim.x * 256) {
    const int r = r0 + (int)(e / cw), c = c0 + (int)(e % cw);
    const cx<double> v = s[(long)(mp ? mp[r] : r) * n + c];
    d[(long)r * n + c] = cx<T>{(T)v.re, (T)v.im};
  }
}

// The row order that the interchanges of block [b1, b1 + nb1) leave, as
// storage rows of the columns left of it (which the interchanges do not
// touch): rmap[b n + r] for rows r in [b1, n).  One workgroup per matrix;
// the interchanges are applied in order to the identity in LDS.
__global__ __launch_bounds__(256) void k_row_map(const int* __restrict__ ipiv, int n, int b1, int nb1,
                                                 int* __restrict__ rmap) {
  __shared__ int sg[LU_MAX_N];
  const int* piv = ipiv + (long)blockIdx.x * n;
  int* out = rmap + (long)blockIdx.x * n;
  const int m = n - b1;
  for (int x = threadIdx.x; x < m; x += 256) sg[x] = b1 + x;
  __syncthreads();
  if (threadIdx.x == 0)
    for (int j = 0; j < nb1; ++j) {
      const int p = piv[b1 + j] - b1;
      if (p != j) {
        const int t = sg[j];
        sg[j] = sg[p];
        sg[p] = t;
      }
    }
  __syncthreads();
  for (int x = threadIdx.x; x < m; x += 256) out[b1 + x] = sg[x];
}

// One LU_NB block column [k0, k0 + nb), rows [k0, n): leaves of LU_LEAF
// columns by the register kernel, the block's columns right of a leaf
// updated by a column solve and an MFMA update of width LU_LEAF.  Row
// interchanges stay within the block's columns.
template <typename T>
static void factor_block(cx<T>* A, long ms, int n, int k0, int batch, int* ipiv, int* info, hipStream_t st) {
  const int nb = std::min(LU_NB, n - k0), ce = k0 + nb;
  for (int j0 = 0; j0 < nb; j0 += LU_LEAF) {
    const int lb = std::min(LU_LEAF, nb - j0);
    panel_any<T>(A, ms, n, k0 + j0, lb, k0, ce, batch, ipiv, info, st);
    trsm_part<T>(A, ms, n, k0 + j0, lb, k0 + j0 + lb, ce, batch, st, nullptr);
    gemm_part<T>(A, ms, n, k0 + j0, lb, k0 + j0 + lb, ce, batch, st);
  }
}

// Two blocks of LU_NB make a step (K = 2 LU_NB in the trailing update,
// whose rate is ~12% higher than at K = LU_NB).  A step's columns [s0, s0 +
// w) are factored within them: the first block, its interchanges and U rows
// on the second block's columns, the second block's update, the second
// block.  Then the step's interchanges and U rows on the trailing columns
// (the second block's U rows first take the first block's product), the
// update of the next step's columns, and the rest of the update, beside the
// next step's factorisation on a second stream.  The first block's L rows
// stay stored in the order of its own factorisation (the solves read them
// so); the update reads them through the row map of the second block's
// interchanges.
static int step_width(int n, int s0) { return std::min(2 * LU_NB, n - s0); }

int lu_update_steps(int n) {
  int k = 0;
  for (int s0 = 0; s0 + step_width(n, s0) < n; s0 += 2 * LU_NB) ++k;
  return k;
}

double lu_update_flops(int n, int batch) {
  double f = 0;
  for (int s0 = 0; s0 + step_width(n, s0) < n; s0 += 2 * LU_NB) {
    const double w = step_width(n, s0), m = n - s0 - w;
    f += 8.0 * m * m * w * batch;
  }
  return f;
}

template <typename T>
void lu_factor_batched(cx<T>* A, long ms, int n, int batch, int* ipiv, int* info, cx<T>* work,
                       hipStream_t st, LuTimers* tm, hipStream_t st2, hipEvent_t* la_ev, int* rmap,
                       const cx<double>* src, int* smap) {
  const bool la = st2 != nullptr && la_ev != nullptr;
  auto demote = [&](int r0, int r1, int c0, int c1, const int* map) {
    const long cnt = (long)(r1 - r0) * (c1 - c0);
    if (cnt <= 0) return;
    const unsigned gx = (unsigned)std::min<long>((cnt + 255) / 256, 64);
    hipLaunchKernelGGL(k_demote<T>, dim3(gx, batch), dim3(256), 0, st, src, A, ms, n, r0, r1, c0, c1, map);
  };
  auto laswp = [&](int k0, int nb, int c0, int c1, hipStream_t sx) {
    if (c1 > c0)
      hipLaunchKernelGGL(k_laswp<T>, dim3((c1 - c0 + 255) / 256, batch), dim3(256), 0, sx, A, ms, n, k0, nb, c0, c1,
                         (const int*)ipiv);
  };
  auto factor_step = [&](int s0, hipStream_t sx) {
    const int w = step_width(n, s0), wa = std::min(LU_NB, w), b1 = s0 + wa, e = s0 + w;
    factor_block<T>(A, ms, n, s0, batch, ipiv, info, sx);
    if (w > wa) {
      laswp(s0, wa, b1, e, sx);
      trsm_part<T>(A, ms, n, s0, wa, b1, e, batch, sx, nullptr);
      gemm_part<T>(A, ms, n, s0, wa, b1, e, batch, sx);
      factor_block<T>(A, ms, n, b1, batch, ipiv, info, sx);
    }
  };
  // with src, A is filled from it: complex64 starts with the first step's
  // columns and takes the rest inside the first step; complex128 (whose
  // update kernel does not read src) copies all of it first
  const bool fused = src != nullptr && sizeof(T) == 4;
  if (src) demote(0, n, 0, fused ? step_width(n, 0) : n, nullptr);
  factor_step(0, st);
  int step = 0;
  for (int s0 = 0; s0 < n; s0 += 2 * LU_NB, ++step) {
    const int w = step_width(n, s0), wa = std::min(LU_NB, w), b1 = s0 + wa, c1 = s0 + w;
    if (c1 >= n) break;
    // with src, the first step takes the rows [0, w) of the columns right of
    // it from src in the row order its interchanges leave (smap: the step's
    // w interchanges applied in order to the identity) instead of applying
    // the interchanges; its trailing update reads C from src in that order
    const bool from_src = fused && s0 == 0;
    if (from_src) {
      hipLaunchKernelGGL(k_row_map, dim3(batch), dim3(256), 0, st, (const int*)ipiv, n, 0, w, smap);
      demote(0, w, c1, n, smap);
    } else {
      laswp(s0, wa, c1, n, st);
    }
    trsm_part<T>(A, ms, n, s0, wa, c1, n, batch, st, work);
    const int* map = nullptr;
    if (w > wa) {
      if (!from_src) laswp(b1, w - wa, c1, n, st);
      hipLaunchKernelGGL(k_row_map, dim3(batch), dim3(256), 0, st, (const int*)ipiv, n, b1, w - wa, rmap);
      map = rmap;
      gemm_part<T>(A, ms, n, s0, wa, c1, n, batch, st, c1, map, wa);
      trsm_part<T>(A, ms, n, b1, w - wa, c1, n, batch, st, work);
    }
    const int c2 = std::min(n, c1 + 2 * LU_NB);
    const bool t = tm && tm->gemm_begin && tm->gemm_end;
    if (t) (void)hipEventRecord(tm->gemm_begin[step], st);
    const cx<double>* csrc = from_src ? src : nullptr;
    const int* cmap = from_src ? smap : nullptr;
    gemm_part<T>(A, ms, n, s0, w, c1, c2, batch, st, n, map, wa, csrc, cmap);
    if (la) {
      (void)hipEventRecord(la_ev[0], st);
      (void)hipStreamWaitEvent(st2, la_ev[0], 0);
      factor_step(c1, st2);
      (void)hipEventRecord(la_ev[1], st2);
    }
    {
      // the rest in 8 column pieces.  Between two pieces the stream drains,
      // and the next step's leaf panels waiting on the second stream get
      // whole compute units (a panel workgroup needs one): the LU is ~5%
      // (complex128) and ~4% (complex64) shorter, while the update's measured
      // interval includes the panels' share of the machine.
      const int pieces = 8;
      const int wp = ((n - c2 + pieces - 1) / pieces + 63) / 64 * 64;
      for (int cb = c2; cb < n; cb += wp)
        gemm_part<T>(A, ms, n, s0, w, cb, std::min(n, cb + wp), batch, st, n, map, wa, csrc, cmap);
    }
    if (t) (void)hipEventRecord(tm->gemm_end[step], st);
    if (la)
      (void)hipStreamWaitEvent(st, la_ev[1], 0);
    else
      factor_step(c1, st);
  }
}

template <typename T, typename TB>
void lu_solve_batched(const cx<T>* A, long ms, int n, int batch, const int* ipiv, cx<TB>* B,
                      int nrhs, hipStream_t st) {
  // off-diagonal block updates: the matrix-core form for 9 to 16 vectors
  auto upd = nrhs > 8 ? &k_solve_update<T, TB, true> : &k_solve_update<T, TB, false>;
  // diagonal blocks: (nrhs + 1) / 2 slots a lane, rounded up to 1, 2, 4 or 8
  auto diag = nrhs > 8   ? &k_solve_diag<T, TB, 8>
              : nrhs > 4 ? &k_solve_diag<T, TB, 4>
              : nrhs > 2 ? &k_solve_diag<T, TB, 2>
                         : &k_solve_diag<T, TB, 1>;
  for (int k0 = 0; k0 < n; k0 += LU_NB) {
    const int nb = std::min(LU_NB, n - k0);
    hipLaunchKernelGGL(diag, dim3(batch), dim3(256), 0, st, A, ms, n, k0, nb, ipiv, B, nrhs, 0);
    const int r0 = k0 + nb, r1 = n;
    if (r1 > r0)
      hipLaunchKernelGGL(upd, dim3((r1 - r0 + R16_ROWS - 1) / R16_ROWS, batch), dim3(256), 0,
                         st, A, ms, n, k0, nb, B, nrhs, r0, r1);
  }
  for (int k0 = ((n - 1) / LU_NB) * LU_NB; k0 >= 0; k0 -= LU_NB) {
    const int nb = std::min(LU_NB, n - k0);
    hipLaunchKernelGGL(diag, dim3(batch), dim3(256), 0, st, A, ms, n, k0, nb, ipiv, B, nrhs, 1);
    if (k0 > 0)
      hipLaunchKernelGGL(upd, dim3((k0 + R16_ROWS - 1) / R16_ROWS, batch), dim3(256), 0, st,
                         A, ms, n, k0, nb, B, nrhs, 0, k0);
  }
}

template void lu_factor_batched<double>(zd*, long, int, int, int*, int*, zd*, hipStream_t, LuTimers*, hipStream_t,
                                        hipEvent_t*, int*, const zd*, int*);
template void lu_factor_batched<float>(zf*, long, int, int, int*, int*, zf*, hipStream_t, LuTimers*, hipStream_t,
                                       hipEvent_t*, int*, const zd*, int*);
template void lu_solve_batched<double, double>(const zd*, long, int, int, const int*, zd*, int,
                                               hipStream_t);
template void lu_solve_batched<float, double>(const zf*, long, int, int, const int*, zd*, int,
                                              hipStream_t);

}  // namespace pmlbie
