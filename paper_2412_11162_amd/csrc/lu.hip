// Batched per-mode complex LU with partial pivoting and the matching solves
// (the per-mode dense solve of Sec. 4.2, eqs. eqntdpsi1/2, done as one
// 2N x 2N system per mode).  Right-looking blocked algorithm, panel width NB:
//   1. panel factorisation (one workgroup per matrix),
//   2. row interchanges of the trailing columns fused with the triangular
//      solve U12 = L11^{-1} A12,
//   3. trailing update A22 -= L21 U12 on the matrix cores (MFMA), complex
//      products as four real MFMA products.
// Row interchanges are not applied to the columns left of the current panel:
// the forward solve applies each panel's interchanges to the right-hand side
// just before using that panel's columns of L, which are stored in the row
// order that was current when the panel was factored.
#include "lu.h"

namespace pmlbie {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ void wave_argmax(T& v, int& idx) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    T ov = __shfl_xor(v, off);
    int oi = __shfl_xor(idx, off);
    if (ov > v || (ov == v && oi < idx)) {
      v = ov;
      idx = oi;
    }
  }
}

// ---------------------------------------------------------------------------
// Panel factorisation: columns [k0, k0 + nb), rows [k0, n).
template <typename T>
__global__ __launch_bounds__(256) void k_panel(cx<T>* __restrict__ A, long ms, int n, int k0,
                                               int nb, int* __restrict__ ipiv,
                                               int* __restrict__ info) {
  cx<T>* a = A + (long)blockIdx.x * ms;
  int* piv = ipiv + (long)blockIdx.x * n;
  __shared__ T sv[4];
  __shared__ int si[4];
  __shared__ cx<T> prow[LU_NB];
  __shared__ int sp;
  __shared__ cx<T> sinv;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int j = 0; j < nb; ++j) {
    const int c = k0 + j;
    const cx<T>* col = a + (long)c * n;
    T best = T(-1);
    int bi = c;
    for (int r = c + tid; r < n; r += 256) {
      T v = cabs1(col[r]);
      if (v > best) {
        best = v;
        bi = r;
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
      for (int w = 1; w < 4; ++w)
        if (sv[w] > b || (sv[w] == b && si[w] < p)) {
          b = sv[w];
          p = si[w];
        }
      sp = p;
      piv[c] = p;
      if (b == T(0)) {
        if (info[blockIdx.x] == 0) info[blockIdx.x] = c + 1;
        sinv = cx<T>{T(0), T(0)};
      }
    }
    __syncthreads();
    const int p = sp;
    if (p != c) {
      for (int cc = k0 + tid; cc < k0 + nb; cc += 256) {
        cx<T> t0 = a[(long)cc * n + c];
        a[(long)cc * n + c] = a[(long)cc * n + p];
        a[(long)cc * n + p] = t0;
      }
    }
    __syncthreads();
    for (int cc = c + 1 + tid; cc < k0 + nb; cc += 256) prow[cc - k0] = a[(long)cc * n + c];
    if (tid == 0) {
      cx<T> pv = a[(long)c * n + c];
      if (pv.re != T(0) || pv.im != T(0)) sinv = inv(pv);
    }
    __syncthreads();
    const cx<T> ip = sinv;
    cx<T>* colc = a + (long)c * n;
    for (int r = c + 1 + tid; r < n; r += 256) {
      cx<T> l = colc[r] * ip;
      colc[r] = l;
      for (int cc = c + 1; cc < k0 + nb; ++cc) {
        cx<T>* dst = a + (long)cc * n + r;
        *dst = *dst - l * prow[cc - k0];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Row interchanges + U12 = L11^{-1} A12 for a tile of 64 trailing columns.
// Thread (col = tid % 64, rg = tid / 64) holds rows rg, rg + 4, ... of the
// panel rows of its column.
template <typename T>
__global__ __launch_bounds__(256) void k_swap_trsm(cx<T>* __restrict__ A, long ms, int n, int k0,
                                                   int nb, const int* __restrict__ ipiv) {
  cx<T>* a = A + (long)blockIdx.y * ms;
  const int* piv = ipiv + (long)blockIdx.y * n;
  const int tid = threadIdx.x, cl = tid & 63, rg = tid >> 6;
  const int c = k0 + nb + blockIdx.x * 64 + cl;
  const bool act = c < n;
  __shared__ cx<T> xs[64];
  __shared__ int spv[LU_NB];
  for (int j = tid; j < nb; j += 256) spv[j] = piv[k0 + j];
  __syncthreads();
  cx<T>* colp = a + (long)(act ? c : 0) * n;
  if (act && rg == 0) {
    for (int j = 0; j < nb; ++j) {
      const int p = spv[j];
      if (p != k0 + j) {
        cx<T> t0 = colp[k0 + j];
        colp[k0 + j] = colp[p];
        colp[p] = t0;
      }
    }
  }
  __syncthreads();
  constexpr int R = LU_NB / 4;
  cx<T> x[R];
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int r = rg + 4 * t;
    x[t] = (act && r < nb) ? colp[k0 + r] : cx<T>{T(0), T(0)};
  }
  for (int j = 0; j < nb; ++j) {
    if ((j & 3) == rg) xs[cl] = x[j >> 2];
    __syncthreads();
    const cx<T> xj = xs[cl];
    const cx<T>* Lc = a + (long)(k0 + j) * n + k0;
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int r = rg + 4 * t;
      if (r > j && r < nb) x[t] = x[t] - Lc[r] * xj;
    }
    __syncthreads();
  }
  if (act) {
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int r = rg + 4 * t;
      if (r < nb) colp[k0 + r] = x[t];
    }
  }
}

// ---------------------------------------------------------------------------
// Trailing update C -= L21 U12 on MFMA.  Workgroup tile 64 x 64 (complex),
// four waves of 32 x 32, K staged through LDS in chunks of 16.
// The MFMA computes the transposed tile C^T = U12^T L21^T so that each lane's
// accumulators map to 16 consecutive rows of a column of C.
template <typename T> struct mfma_t;
template <> struct mfma_t<double> {
  typedef v4d acc;
  __device__ __forceinline__ static acc op(double x, double y, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
  }
  // lane l, register j -> (row of C^T tile, col) = (l/16 + 4j, l%16)
  __device__ __forceinline__ static int rowof(int lane, int j) { return (lane >> 4) + 4 * j; }
};
template <> struct mfma_t<float> {
  typedef v4f acc;
  __device__ __forceinline__ static acc op(float x, float y, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int rowof(int lane, int j) { return 4 * (lane >> 4) + j; }
};

template <typename T>
__global__ __launch_bounds__(256) void k_gemm_update(cx<T>* __restrict__ A, long ms, int n,
                                                     int k0, int nb) {
  typedef typename mfma_t<T>::acc acc_t;
  cx<T>* a = A + (long)blockIdx.z * ms;
  const int m0 = k0 + nb;  // first trailing row/column
  const int r0 = m0 + blockIdx.x * 64;  // tile rows of C
  const int c0 = m0 + blockIdx.y * 64;  // tile columns of C
  constexpr int KC = 16;
  __shared__ T Lre[KC][64 + 1], Lim[KC][64 + 1];  // L21 chunk: [k][row]
  __shared__ T Ure[KC][64 + 1], Uim[KC][64 + 1];  // U12 chunk: [k][col]
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wr = (wid & 1) * 32, wc = (wid >> 1) * 32;  // wave sub-tile offsets
  acc_t cr[2][2], ci[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      cr[x][y] = acc_t{0, 0, 0, 0};
      ci[x][y] = acc_t{0, 0, 0, 0};
    }
  for (int kk = 0; kk < nb; kk += KC) {
    // load L21[r0 .. r0+63][k0+kk .. +15] and U12[k0+kk .. +15][c0 .. c0+63]
    for (int e = tid; e < 64 * KC; e += 256) {
      const int rr = e & 63, k = e >> 6;
      const int gr = r0 + rr, gk = k0 + kk + k;
      cx<T> v = (gr < n && kk + k < nb) ? a[(long)gk * n + gr] : cx<T>{T(0), T(0)};
      Lre[k][rr] = v.re;
      Lim[k][rr] = v.im;
    }
    for (int e = tid; e < 64 * KC; e += 256) {
      const int k = e % KC, cc = e / KC;
      const int gc = c0 + cc, gk = k0 + kk + k;
      cx<T> v = (gc < n && kk + k < nb) ? a[(long)gc * n + gk] : cx<T>{T(0), T(0)};
      Ure[k][cc] = v.re;
      Uim[k][cc] = v.im;
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < KC; k4 += 4) {
      const int kx = k4 + (lane >> 4), lx = lane & 15;
      T ur[2], ui[2], lr[2], li[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        ur[t] = Ure[kx][wc + 16 * t + lx];   // X = U^T: X[p][k] = U[k][col p]
        ui[t] = Uim[kx][wc + 16 * t + lx];
        lr[t] = Lre[kx][wr + 16 * t + lx];   // Y = L^T: Y[k][q] = L[row q][k]
        li[t] = Lim[kx][wr + 16 * t + lx];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)      // column sub-tile (U)
#pragma unroll
        for (int y = 0; y < 2; ++y) {  // row sub-tile (L)
          cr[x][y] = mfma_t<T>::op(ur[x], lr[y], cr[x][y]);
          cr[x][y] = mfma_t<T>::op(-ui[x], li[y], cr[x][y]);
          ci[x][y] = mfma_t<T>::op(ur[x], li[y], ci[x][y]);
          ci[x][y] = mfma_t<T>::op(ui[x], lr[y], ci[x][y]);
        }
    }
    __syncthreads();
  }
  // C^T tile (p = column offset, q = row offset): lane -> q = lane % 16.
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int gc = c0 + wc + 16 * x + mfma_t<T>::rowof(lane, j);
        const int gr = r0 + wr + 16 * y + (lane & 15);
        if (gc < n && gr < n) {
          cx<T>* p = a + (long)gc * n + gr;
          cx<T> v = *p;
          v.re -= cr[x][y][j];
          v.im -= ci[x][y][j];
          *p = v;
        }
      }
}

// ---------------------------------------------------------------------------
// Solves with the factors, one workgroup per matrix, nrhs right-hand sides
// stored as b[mat][rhs][n] (overwritten by the solution).
template <typename T, typename TB>
__global__ __launch_bounds__(256) void k_solve(const cx<T>* __restrict__ A, long ms, int n,
                                               const int* __restrict__ ipiv, cx<TB>* __restrict__ B,
                                               int nrhs) {
  const cx<T>* a = A + (long)blockIdx.x * ms;
  const int* piv = ipiv + (long)blockIdx.x * n;
  cx<TB>* b = B + (long)blockIdx.x * nrhs * n;
  const int tid = threadIdx.x;
  __shared__ cx<TB> yb[LU_NB][LU_MAX_RHS];
  // forward: panel by panel
  for (int k0 = 0; k0 < n; k0 += LU_NB) {
    const int nb = min(LU_NB, n - k0);
    if (tid < nrhs) {
      cx<TB>* v = b + (long)tid * n;
      for (int j = 0; j < nb; ++j) {
        const int p = piv[k0 + j];
        if (p != k0 + j) {
          cx<TB> t0 = v[k0 + j];
          v[k0 + j] = v[p];
          v[p] = t0;
        }
      }
    }
    __syncthreads();
    // unit lower triangular block, sequential in j; threads over (row, rhs)
    for (int e = tid; e < nb * nrhs; e += 256) yb[e % nb][e / nb] = b[(long)(e / nb) * n + k0 + e % nb];
    __syncthreads();
    for (int j = 0; j < nb; ++j) {
      for (int e = tid; e < nb * nrhs; e += 256) {
        const int r = e % nb, s = e / nb;
        if (r > j) {
          cx<T> l = a[(long)(k0 + j) * n + k0 + r];
          cx<TB> lc{(TB)l.re, (TB)l.im};
          yb[r][s] = yb[r][s] - lc * yb[j][s];
        }
      }
      __syncthreads();
    }
    for (int e = tid; e < nb * nrhs; e += 256) b[(long)(e / nb) * n + k0 + e % nb] = yb[e % nb][e / nb];
    __syncthreads();
    // update rows below
    for (int r = k0 + nb + tid; r < n; r += 256) {
      for (int s = 0; s < nrhs; ++s) {
        cx<TB> acc = b[(long)s * n + r];
        for (int j = 0; j < nb; ++j) {
          cx<T> l = a[(long)(k0 + j) * n + r];
          cx<TB> lc{(TB)l.re, (TB)l.im};
          acc = acc - lc * yb[j][s];
        }
        b[(long)s * n + r] = acc;
      }
    }
    __syncthreads();
  }
  // backward
  for (int k0 = ((n - 1) / LU_NB) * LU_NB; k0 >= 0; k0 -= LU_NB) {
    const int nb = min(LU_NB, n - k0);
    for (int e = tid; e < nb * nrhs; e += 256) yb[e % nb][e / nb] = b[(long)(e / nb) * n + k0 + e % nb];
    __syncthreads();
    for (int j = nb - 1; j >= 0; --j) {
      if (tid < nrhs) {
        cx<T> u = a[(long)(k0 + j) * n + k0 + j];
        cx<TB> uc{(TB)u.re, (TB)u.im};
        yb[j][tid] = yb[j][tid] / uc;
      }
      __syncthreads();
      for (int e = tid; e < nb * nrhs; e += 256) {
        const int r = e % nb, s = e / nb;
        if (r < j) {
          cx<T> u = a[(long)(k0 + j) * n + k0 + r];
          cx<TB> uc{(TB)u.re, (TB)u.im};
          yb[r][s] = yb[r][s] - uc * yb[j][s];
        }
      }
      __syncthreads();
    }
    for (int e = tid; e < nb * nrhs; e += 256) b[(long)(e / nb) * n + k0 + e % nb] = yb[e % nb][e / nb];
    __syncthreads();
    for (int r = tid; r < k0; r += 256) {
      for (int s = 0; s < nrhs; ++s) {
        cx<TB> acc = b[(long)s * n + r];
        for (int j = 0; j < nb; ++j) {
          cx<T> u = a[(long)(k0 + j) * n + r];
          cx<TB> uc{(TB)u.re, (TB)u.im};
          acc = acc - uc * yb[j][s];
        }
        b[(long)s * n + r] = acc;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
template <typename T>
void lu_factor_batched(cx<T>* A, long ms, int n, int batch, int* ipiv, int* info, hipStream_t st,
                       LuTimers* tm) {
  for (int k0 = 0; k0 < n; k0 += LU_NB) {
    const int nb = std::min(LU_NB, n - k0);
    if (tm && tm->panel_begin) hipEventRecord(tm->panel_begin[k0 / LU_NB], st);
    hipLaunchKernelGGL(k_panel<T>, dim3(batch), dim3(256), 0, st, A, ms, n, k0, nb, ipiv, info);
    const int rest = n - k0 - nb;
    if (rest > 0) {
      dim3 g1((rest + 63) / 64, batch);
      hipLaunchKernelGGL(k_swap_trsm<T>, g1, dim3(256), 0, st, A, ms, n, k0, nb, ipiv);
      if (tm && tm->gemm_begin) hipEventRecord(tm->gemm_begin[k0 / LU_NB], st);
      dim3 g2((rest + 63) / 64, (rest + 63) / 64, batch);
      hipLaunchKernelGGL(k_gemm_update<T>, g2, dim3(256), 0, st, A, ms, n, k0, nb);
      if (tm && tm->gemm_end) hipEventRecord(tm->gemm_end[k0 / LU_NB], st);
    }
  }
}

template <typename T, typename TB>
void lu_solve_batched(const cx<T>* A, long ms, int n, int batch, const int* ipiv, cx<TB>* B,
                      int nrhs, hipStream_t st) {
  hipLaunchKernelGGL((k_solve<T, TB>), dim3(batch), dim3(256), 0, st, A, ms, n, ipiv, B, nrhs);
}

template void lu_factor_batched<double>(zd*, long, int, int, int*, int*, hipStream_t, LuTimers*);
template void lu_factor_batched<float>(zf*, long, int, int, int*, int*, hipStream_t, LuTimers*);
template void lu_solve_batched<double, double>(const zd*, long, int, int, const int*, zd*, int,
                                               hipStream_t);
template void lu_solve_batched<float, double>(const zf*, long, int, int, const int*, zd*, int,
                                              hipStream_t);

}  // namespace pmlbie
