// Output of the modal-kernel paths: the per-mode system matrices or a raw
// modal buffer (Sec. 4.1-4.2).
#pragma once
#include "modal.h"

namespace pmlbie {

// Output: either the per-mode system matrices or a raw modal buffer.
//
// System matrix of mode n, row-major 2N x 2N at A + (n - m0) * mstride, with
// the unknowns and equations of each node interleaved: unknown 2l is u1 at
// node l and 2l + 1 is phi1 there; equation 2i is the upper medium's at node
// i and 2i + 1 the lower medium's.  The 2 x 2 block of a pair (i, l) is
//   [[K1_il - D1_il, -S1_il], [K2_il - D2_il, -S2_il]],
//   K_il = 2 W_l K_n(r_i, r_l), S_il = 2 W_l S_n(r_i, r_l),
// i.e. the system [[K1 - D1, -S1], [K2 - D2, -S2]] with rows and columns
// permuted symmetrically.  A pair's two entries of one equation are adjacent
// (32 bytes, one aligned sector), so the scattered per-pair mode writes of
// the far, split and direct paths fill whole sectors.
// Raw modal buffer: out[q][s][n], s in {S1, K1, S2, K2}.
struct OutSpec {
  zd* A;
  long n2;       // 2N
  long mstride;  // elements per mode matrix
  const double* W;
  zd* raw;
  int M;         // highest mode formed
  int m0;        // first mode kept in A (A + (n - m0) * mstride holds mode n)
};

// Element offset of sequence s (S1, K1, S2, K2) of pair (i, l) in a mode's
// interleaved matrix: equation 2i (+1 for the lower medium), unknown 2l for
// a K entry, 2l + 1 for an S entry.
__device__ __forceinline__ long sys_offset(long n2, long i, long l, int s) {
  return (2 * i + (s >> 1)) * n2 + 2 * l + ((s & 1) ? 0 : 1);
}

__device__ __forceinline__ void emit(const OutSpec& o, int2 dst, int n, zd S1, zd K1, zd S2,
                                     zd K2) {
  if (dst.y >= 0) {
    if (n < o.m0) return;
    const long i = dst.x, l = dst.y;
    const double w2 = 2.0 * o.W[l];
    zd* An = o.A + (long)(n - o.m0) * o.mstride;
    zd* up = An + 2 * i * o.n2 + 2 * l;
    up[0] = w2 * K1;
    up[1] = (-w2) * S1;
    up[o.n2] = w2 * K2;
    up[o.n2 + 1] = (-w2) * S2;
  } else {
    zd* r = o.raw + (long)dst.x * 4 * (o.M + 1);
    r[n] = S1;
    r[(o.M + 1) + n] = K1;
    r[2 * (o.M + 1) + n] = S2;
    r[3 * (o.M + 1) + n] = K2;
  }
}

__device__ __forceinline__ PairGeom node_pair(const NodesDev& nd, int i, int l) {
  PairGeom g;
  g.rt = zd{nd.rho[i], nd.I[i]};
  g.rs = zd{nd.rho[l], nd.I[l]};
  g.drho = zd{nd.rho[i] - nd.rho[l], nd.I[i] - nd.I[l]};
  g.dz = zd{nd.z[i] - nd.z[l], 0.0};
  g.nr = zd{nd.nr_re[l], nd.nr_im[l]};
  g.nz = zd{nd.nz_re[l], nd.nz_im[l]};
  return g;
}

// In-place radix-2 FFT (decimation in time, bit-reversed input) of NSEQ
// sequences of length NT held in LDS, one wavefront.  tw[k] = e^{-2 pi i k/NT}.
template <int NT, int NSEQ>
__device__ __forceinline__ void fft_lds(zd* buf, const zd* __restrict__ tw) {
#pragma unroll 1
  for (int len = 2; len <= NT; len <<= 1) {
    const int half = len >> 1, step = NT / len;
    for (int b = threadIdx.x; b < NSEQ * (NT / 2); b += 64) {
      const int s = b / (NT / 2), bb = b % (NT / 2);
      const int grp = bb / half, pos = bb % half;
      const int i0 = s * NT + grp * len + pos, i1 = i0 + half;
      const zd w = tw[pos * step];
      const zd u = buf[i0], v = buf[i1] * w;
      buf[i0] = u + v;
      buf[i1] = u - v;
    }
    __syncthreads();
  }
}

template <int NT>
__device__ __forceinline__ int bitrev(int j) {
  constexpr int LOG = __builtin_ctz(NT);
  return (int)(__brev((unsigned)j) >> (32 - LOG));
}

// ------------------------------------------------------------------------
// Classification of a pair (Sec. 4.1: well-separated pairs by FFT of the raw
// kernel; close pairs by the split; close pairs deep in the PML by graded
// direct quadrature, where cos(kR) grows like exp(max |Im kR|)).
// A far pair is also marked coarse when the same aliasing bound holds on the
// grid of half the length (its modes beyond L/2 - M are as negligible).  With
// cp.nt_small set, far pairs are judged on that shorter grid first (the main
// pass's grid) and the ones that need the full grid are CLASS_FAR_BIG.
__device__ __forceinline__ int classify(const PairGeom& g, const PairInv& v, const ClassParams& cp,
                                        bool* coarse = nullptr) {
  double delta, re0;
  singularity(v, delta, re0);
  const double sc = sqrt(cabs_(rho_product(g.rt, g.rs)));
  const double bw = cp.bw * cp.kmax * sc;
  if ((cp.nt_far - cp.M - bw) * delta >= cp.c_far) {
    int nt = cp.nt_far;
    if (cp.nt_small > 0 && cp.nt_small < cp.nt_far) {
      if ((cp.nt_small - cp.M - bw) * delta < cp.c_far) return CLASS_FAR_BIG;
      nt = cp.nt_small;
    }
    if (coarse) *coarse = (nt / 2 - cp.M - bw) * delta >= cp.c_far;
    return CLASS_FAR;
  }
  zd Rpi = csqrt_(v.d2 + v.c4);
  double grow = cp.kmax * fabs(Rpi.im) + cp.kmax_im * fabs(Rpi.re);
  if (grow > cp.g_split) return CLASS_DIRECT;
  if (cp.split_rho_small > 0.0 && fmax(cabs_(g.rt), cabs_(g.rs)) > cp.split_rho_small) return CLASS_SPLIT_BIG;
  return CLASS_SPLIT;
}

}  // namespace pmlbie
