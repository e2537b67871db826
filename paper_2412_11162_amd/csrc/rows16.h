// Row blocks of a row-major complex matrix applied to up to 16 vectors, the
// shape of every matrix-vector product around the per-mode solve (Sec. 4.2):
// the block updates of the triangular solves, the right-hand sides from the
// lower-medium equations and the FP64 residuals of the refinement.
//
//   acc[row][s] = sum_{c0 <= c < c1} A[row][c] y_s(c),  s < nrhs <= 16.
//
// A workgroup of four wavefronts takes 64 consecutive rows.  Column chunks of
// 32 are staged in LDS: the 64 x 32 tile of A (row segments loaded
// coalesced into registers one chunk ahead, so the next chunk's HBM reads
// overlap this chunk's arithmetic; rows padded to 33 entries so that the
// lane-per-row reads hit distinct banks) and the 32 values of every vector.
// Up to 8 vectors: lane l owns row r + l.  The vectors are dealt to G = 1 or
// 2 groups of four (G = ceil(nrhs / 4)); the 4 / G wavefronts of a group
// split the chunk's columns and add their partial sums through LDS at the
// end.  The vector values a wavefront reads are one address for all lanes
// (broadcast), and each A element is read from HBM once.
// 9 to 16 vectors: the product is a 64 x 32 by 32 x 16 matrix product per
// chunk and runs on the FP64 matrix cores (v_mfma_f64_16x16x4, wavefront w
// takes rows 16 w .. 16 w + 15 against all 16 vectors), the complex product
// as three real ones (T1 = Ar Yr, T2 = Ai Yi, T3 = (Ar + Ai)(Yr + Yi); re =
// T1 - T2, im = T3 - T1 - T2); the results go through LDS back to the
// lane-per-row layout (wavefront w returns vectors 4 w .. 4 w + 3).  At 16
// vectors the FP64 vector arithmetic of the lane-per-row form costs about as
// much as the HBM reads of A; on the matrix cores it costs half.
#pragma once
#include "cplx.h"

namespace pmlbie {

constexpr int R16_ROWS = 64;
constexpr int R16_CHUNK = 32;

// Accumulate rows [rbase, rbase + 64) (clamped to rend) over columns
// [c0, c1); vec(s, c) gives y_s(c).  On return, for the wavefronts with
// out_wave true, acc[q] holds this lane's row times vector 4 g + q, where g =
// out_group.  Every thread must call it (it synchronises the workgroup).
// MM selects the matrix-core form (callers instantiate it for 9 to 16
// vectors, so that the lane-per-row form keeps its own register budget).
template <typename TA, bool MM, typename F>
__device__ __forceinline__ void rows16_acc(const cx<TA>* __restrict__ a, long lda, int rbase, int rend,
                                           int c0, int c1, int nrhs, F vec, zd (&acc)[4], bool& out_wave,
                                           int& out_group) {
  constexpr int PER = (R16_ROWS * R16_CHUNK) / 256;  // A elements per thread per chunk
  // the tile of A and, after the last chunk, the partial sums of the column
  // partitions or the matrix-core results share one LDS area
  constexpr int AS_BYTES = sizeof(cx<TA>) * R16_ROWS * (R16_CHUNK + 1);
  constexpr int RED_BYTES = sizeof(zd) * 3 * 4 * R16_ROWS;
  constexpr int OUT_BYTES = sizeof(zd) * R16_ROWS * 17;  // matrix-core results, rows padded
  constexpr int AREA = AS_BYTES > RED_BYTES ? (AS_BYTES > OUT_BYTES ? AS_BYTES : OUT_BYTES)
                                            : (RED_BYTES > OUT_BYTES ? RED_BYTES : OUT_BYTES);
  __shared__ __align__(16) unsigned char area[AREA];
  __shared__ zd Ys[16][R16_CHUNK + 1];  // padded: the matrix-core reads take one column of all 16
  auto As = reinterpret_cast<cx<TA>(*)[R16_CHUNK + 1]>(area);
  auto Red = reinterpret_cast<zd(*)[4][R16_ROWS]>(area);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  constexpr bool mm = MM;
  const int G = nrhs <= 4 ? 1 : (nrhs <= 8 ? 2 : 4);  // vector groups
  const int P = 4 / G;                                 // column partitions per group
  const int g = w % G, p = w / G;
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = zd{0.0, 0.0};
  typedef double v4d_ __attribute__((ext_vector_type(4)));
  [[maybe_unused]] v4d_ t1 = {0.0, 0.0, 0.0, 0.0}, t2 = t1, t3 = t1;
  constexpr int YPER = (16 * R16_CHUNK) / 256;  // vector values per thread per chunk
  cx<TA> pre[PER];
  zd ypre[YPER];
  auto load = [&](int cb) {
    const int cn = min(R16_CHUNK, c1 - cb);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = tid + 256 * k, r = e / R16_CHUNK, c = e % R16_CHUNK;
      const int rr = min(rbase + r, rend - 1);
      pre[k] = c < cn ? a[(long)rr * lda + cb + c] : cx<TA>{TA(0), TA(0)};
    }
#pragma unroll
    for (int k = 0; k < YPER; ++k) {
      const int e = tid + 256 * k, s = e / R16_CHUNK, c = e % R16_CHUNK;
      ypre[k] = (s < nrhs && c < cn) ? vec(s, cb + c) : zd{0.0, 0.0};
    }
  };
  if (c0 < c1) load(c0);
  for (int cb = c0; cb < c1; cb += R16_CHUNK) {
    __syncthreads();  // the previous chunk's reads are done
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int e = tid + 256 * k;
      As[e / R16_CHUNK][e % R16_CHUNK] = pre[k];
    }
#pragma unroll
    for (int k = 0; k < YPER; ++k) {
      const int e = tid + 256 * k;
      Ys[e / R16_CHUNK][e % R16_CHUNK] = ypre[k];
    }
    __syncthreads();
    if (cb + R16_CHUNK < c1) load(cb + R16_CHUNK);  // in flight during the arithmetic below
    if constexpr (mm) {
      const int r = 16 * w + (lane & 15), kq = lane >> 4, s = lane & 15;
#pragma unroll
      for (int k4 = 0; k4 < R16_CHUNK; k4 += 4) {
        const cx<TA> av = As[r][k4 + kq];   // A[row r][k], row = lane % 16, k = lane / 16
        const zd yv = Ys[s][k4 + kq];        // Y[k][vector s]
        const double ar = (double)av.re, ai = (double)av.im;
        t1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, yv.re, t1, 0, 0, 0);
        t2 = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, yv.im, t2, 0, 0, 0);
        t3 = __builtin_amdgcn_mfma_f64_16x16x4f64(ar + ai, yv.re + yv.im, t3, 0, 0, 0);
      }
    } else if (4 * g < nrhs) {
#pragma unroll 8
      for (int c = p; c < R16_CHUNK; c += P) {
        const cx<TA> av = As[lane][c];
        const zd ad{(double)av.re, (double)av.im};
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = cfma(ad, Ys[4 * g + q][c], acc[q]);
      }
    }
  }
  out_group = g;
  out_wave = p == 0 && 4 * g < nrhs;
  if constexpr (mm) {
    // lane l, value j of the 16 x 16 tile: row 16 w + l / 16 + 4 j, vector
    // l % 16; back through LDS to lane = row, vectors 4 w .. 4 w + 3
    auto Out = reinterpret_cast<zd(*)[17]>(area);
    __syncthreads();  // the last chunk's tile reads are done
#pragma unroll
    for (int j = 0; j < 4; ++j)
      Out[16 * w + (lane >> 4) + 4 * j][lane & 15] = zd{t1[j] - t2[j], t3[j] - t1[j] - t2[j]};
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = Out[lane][4 * w + q];
    return;
  }
  if (P > 1) {
    __syncthreads();
    if (p > 0)
#pragma unroll
      for (int q = 0; q < 4; ++q) Red[w - G][q][lane] = acc[q];
    __syncthreads();
    if (p == 0)
      for (int pp = 1; pp < P; ++pp)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = acc[q] + Red[pp * G + g - G][q][lane];
  }
}

}  // namespace pmlbie
