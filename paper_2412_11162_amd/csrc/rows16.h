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
// Lane l owns row r + l.  The vectors are dealt to G = 1, 2 or 4 groups of
// four (G = ceil(nrhs / 4), 3 -> 4); the 4 / G wavefronts of a group split the
// chunk's columns and add their partial sums through LDS at the end.  The
// vector values a wavefront reads are one address for all lanes (broadcast),
// and each A element is read from HBM once.
#pragma once
#include "cplx.h"

namespace pmlbie {

constexpr int R16_ROWS = 64;
constexpr int R16_CHUNK = 32;

// Accumulate rows [rbase, rbase + 64) (clamped to rend) over columns
// [c0, c1); vec(s, c) gives y_s(c).  On return, for the wavefronts with
// out_wave true, acc[q] holds this lane's row times vector 4 g + q, where g =
// out_group.  Every thread must call it (it synchronises the workgroup).
template <typename TA, typename F>
__device__ __forceinline__ void rows16_acc(const cx<TA>* __restrict__ a, long lda, int rbase, int rend,
                                           int c0, int c1, int nrhs, F vec, zd (&acc)[4], bool& out_wave,
                                           int& out_group) {
  constexpr int PER = (R16_ROWS * R16_CHUNK) / 256;  // A elements per thread per chunk
  // the tile of A and, after the last chunk, the partial sums of the column
  // partitions share one LDS area
  constexpr int AS_BYTES = sizeof(cx<TA>) * R16_ROWS * (R16_CHUNK + 1);
  constexpr int RED_BYTES = sizeof(zd) * 3 * 4 * R16_ROWS;
  __shared__ __align__(16) unsigned char area[AS_BYTES > RED_BYTES ? AS_BYTES : RED_BYTES];
  __shared__ zd Ys[16][R16_CHUNK];
  auto As = reinterpret_cast<cx<TA>(*)[R16_CHUNK + 1]>(area);
  auto Red = reinterpret_cast<zd(*)[4][R16_ROWS]>(area);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int G = nrhs <= 4 ? 1 : (nrhs <= 8 ? 2 : 4);  // vector groups
  const int P = 4 / G;                                 // column partitions per group
  const int g = w % G, p = w / G;
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = zd{0.0, 0.0};
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
    if (4 * g < nrhs) {
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
