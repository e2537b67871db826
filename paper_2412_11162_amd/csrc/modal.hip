// Modal-kernel generation on gfx950: pair x theta sampling of the
// complexified Green's function and its conormal derivative, batched
// azimuthal FFTs in LDS, the singular/smooth split with semi-analytic
// singular modes (Sec. 4.1, eqs. eq:s1, eq:k1, eqsnspml, eqknspml, and the
// convolution formula eqcon of Sec. 3.3), a graded direct azimuthal
// quadrature for near pairs deep in the PML where the split loses accuracy,
// and assembly of the per-mode Nystrom matrices (Sec. 4.1-4.2).
//
// Natural modes: F_n = int_{-pi}^{pi} e^{-i n D} F(D) dD.  Every kernel is
// even in D, so F_{-n} = F_n and only n = 0..M are formed.
#include "fft_wave.h"
#include "modal.h"
#include "modal_out.h"

namespace pmlbie {

// One mode value of sequence s in {S1, K1, S2, K2}, scaled.
__device__ __forceinline__ void emit_val(const OutSpec& o, int2 dst, int s, int n, double scale,
                                         zd val) {
  if (dst.y >= 0) {
    if (n < o.m0) return;
    const long i = dst.x, l = dst.y;
    const double w2 = 2.0 * o.W[l] * scale;
    // S entries carry the minus sign of [[K1 + I, -S1], [K2 - I, -S2]]
    const double f = (s & 1) ? w2 : -w2;
    o.A[(long)(n - o.m0) * o.mstride + sys_offset(o.n2, i, l, s)] = f * val;
  } else {
    o.raw[(long)dst.x * 4 * (o.M + 1) + (long)s * (o.M + 1) + n] = scale * val;
  }
}

// Modes 0..M of the two sequences (s0, s0 + 1) held in the output layout of
// fft_wave.
template <int R>
__device__ __forceinline__ void emit_pair(const OutSpec& o, int2 dst, int s0, double scale,
                                          const zd (&x)[2][R]) {
  const int b = threadIdx.x & 63;
#pragma unroll
  for (int sl = 0; sl < R; ++sl) {
    const int n = fft_wave_out_index<R>(b, sl);
    if (n <= o.M) {
      emit_val(o, dst, s0, n, scale, x[0][sl]);
      emit_val(o, dst, s0 + 1, n, scale, x[1][sl]);
    }
  }
}

// LDS of one pair (entries): two staging areas P1, P2 of two half-circle
// sequences each and the fft_wave exchange area E.  For R <= 16, E holds two
// sequences and P1 sits at its start (P1 is read into registers before the
// transform uses E); for R = 32 the sequences are transformed one at a time
// and P1, P2 and E are disjoint.
template <int R>
constexpr int pair_lds() {
  return R <= 16 ? (32 * R + 1) * 2 + 2 * fft_wave_lds<R>() : 4 * (32 * R + 1) + fft_wave_lds<R>();
}
// The far-pair path transforms one sequence at a time, so for R <= 16 its E
// needs only one exchange area (which also covers P1).
template <int R>
constexpr int far_lds() {
  return R <= 16 ? 2 * (32 * R + 1) + (fft_wave_lds<R>() > 2 * (32 * R + 1) ? fft_wave_lds<R>() : 2 * (32 * R + 1))
                 : pair_lds<R>();
}
template <int R>
__device__ __forceinline__ zd* pair_p1(zd* lds) {
  return lds + 2 * (32 * R + 1);
}
template <int R>
__device__ __forceinline__ zd* pair_e(zd* lds) {
  return R <= 16 ? lds + 2 * (32 * R + 1) : lds + 4 * (32 * R + 1);
}

// Load staged half-circle sequence(s) (j = 0..L/2 at st[j], st[H + j], ...)
// into the input layout of fft_wave, extended evenly: x[L - j] = x[j].
template <int R, int NS>
__device__ __forceinline__ void load_even(const zd* st, zd (&x)[NS][R]) {
  constexpr int L = 64 * R, H = L / 2 + 1;
  const int b = threadIdx.x & 63;
#pragma unroll
  for (int a = 0; a < R; ++a) {
    const int j = b + 64 * a;
    const int jj = j <= L / 2 ? j : L - j;
#pragma unroll
    for (int q = 0; q < NS; ++q) x[q][a] = st[q * H + jj];
  }
}

// Modes 0..M of one sequence s held in the output layout of fft_wave.
template <int R>
__device__ __forceinline__ void emit_seq(const OutSpec& o, int2 dst, int s, double scale,
                                         const zd (&x)[R]) {
  const int b = threadIdx.x & 63;
#pragma unroll
  for (int sl = 0; sl < R; ++sl) {
    const int n = fft_wave_out_index<R>(b, sl);
    if (n <= o.M) emit_val(o, dst, s, n, scale, x[sl]);
  }
}

// Transform the staged sequences (s0, s0 + 1) and emit their modes.
template <int R>
__device__ __forceinline__ void transform_emit(const zd* st, zd* E, const zd* __restrict__ tw,
                                               const OutSpec& o, int2 dst, int s0) {
  constexpr int H = 32 * R + 1;
  const double scale = 2.0 * PMLBIE_PI / (64 * R);
  if constexpr (R <= 16) {
    zd x[2][R];
    load_even<R, 2>(st, x);
    __syncthreads();
    fft_wave<R, 1>(*reinterpret_cast<zd(*)[1][R]>(&x[0]), E, tw);
    fft_wave<R, 1>(*reinterpret_cast<zd(*)[1][R]>(&x[1]), E, tw);
    emit_pair<R>(o, dst, s0, scale, x);
  } else {
#pragma unroll 1
    for (int q = 0; q < 2; ++q) {
      zd x[1][R];
      load_even<R, 1>(st + q * H, x);
      __syncthreads();
      fft_wave<R, 1>(x, E, tw);
      emit_seq<R>(o, dst, s0 + q, scale, x[0]);
    }
  }
}

// sin^2(D_j / 2) of the far grid of length L, stored after its L twiddles.
template <int R>
__device__ __forceinline__ double tw_s2(const zd* __restrict__ tw, int j) {
  return tw[64 * R + j].re;
}

// R = sqrt(R2) on the principal branch, 1 / R and 1 / R^2 at one sample of a
// far pair.  Far pairs keep |R2| well inside the double range (their R2 is
// bounded away from 0 on the real D axis), so the modulus needs no scaling,
// and since |R|^2 = |R2|, 1 / R = conj(R) / |R2|: two square roots and two
// divisions in all.
struct FarGeo {
  zd R, iR, iR2;
};
__device__ __forceinline__ FarGeo far_geo(zd R2) {
  const double x = R2.re, y = R2.im;
  const double r = sqrt(x * x + y * y);
  const double t = sqrt(0.5 * (r + fabs(x)));
  const double h = 0.5 / t;
  FarGeo f;
  f.R = x >= 0.0 ? zd{t, y * h} : zd{fabs(y) * h, copysign(t, y)};
  const double ir = 1.0 / r;
  f.iR = zd{f.R.re * ir, -f.R.im * ir};
  f.iR2 = f.iR * f.iR;
  return f;
}

// e^{i kR} from one exponential and one shared sine/cosine reduction.
__device__ __forceinline__ zd expi(zd kR) {
  double s, c;
  sincos(kR.re, &s, &c);
  const double m = exp(-kR.im);
  return zd{m * c, m * s};
}

// Raw-kernel FFT of one pair (one wavefront): the samples of S = G~ and
// K = dG~/dnu' for both wavenumbers on the half circle D_j = 2 pi j / L,
// j <= L/2 (R and the conormal factor are shared), staged in LDS, extended
// to the full circle (the kernels are even in D), transformed by fft_wave;
// modes 0..M are emitted.  A coarse pair is sampled at the odd j only (the
// L/2-point grid shifted by half a step) with doubled weights and zeros at
// the even j, so the same transform returns that grid's trapezoidal modes.
// sin^2(D_j / 2) is read from the table after the twiddles (tw_s2), R and
// its reciprocals come from far_geo.
template <int R>
__device__ __forceinline__ void far_pair(const PairInv& v, zd k1, zd k2, const zd* __restrict__ tw,
                                         zd* lds, const OutSpec& o, int2 dst, bool coarse) {
  constexpr int L = 64 * R, H = L / 2 + 1;
  zd* P2 = lds;
  zd* P1 = pair_p1<R>(lds);
  zd* E = pair_e<R>(lds);
  const int ns = coarse ? L / 4 : L / 2 + 1;
  const double w4pi = (coarse ? 2.0 : 1.0) * (0.25 / PMLBIE_PI);
#pragma unroll 1
  for (int q = threadIdx.x; q < ns; q += 64) {
    const int j = coarse ? 2 * q + 1 : q;
    const double s2 = tw_s2<R>(tw, j);
    const FarGeo f = far_geo(v.d2 + s2 * v.c4);
    const zd inv4piR = f.iR * w4pi;
    const zd iR2 = f.iR2;
    const zd N = v.N0 + s2 * v.N1;
    const zd kR1 = k1 * f.R, kR2 = k2 * f.R;
    const zd ikR1{-kR1.im, kR1.re}, ikR2{-kR2.im, kR2.re};
    const zd e1 = expi(kR1) * inv4piR, e2 = expi(kR2) * inv4piR;
    P1[j] = e1;
    P1[H + j] = N * e1 * (ikR1 - 1.0) * iR2;
    P2[j] = e2;
    P2[H + j] = N * e2 * (ikR2 - 1.0) * iR2;
    if (coarse) {
      const zd z0{0.0, 0.0};
      P1[j - 1] = z0;
      P1[H + j - 1] = z0;
      P2[j - 1] = z0;
      P2[H + j - 1] = z0;
    }
  }
  if (coarse && threadIdx.x == 0) {
    const zd z0{0.0, 0.0};
    P1[L / 2] = z0;
    P1[H + L / 2] = z0;
    P2[L / 2] = z0;
    P2[H + L / 2] = z0;
  }
  __syncthreads();
  transform_emit<R>(P1, E, tw, o, dst, 0);
  transform_emit<R>(P2, E, tw, o, dst, 2);
}

// Modes m0..M of one transformed sequence into a mode-strided column of A:
// base is the entry of mode m0, f the quadrature weight with the sign of the
// block.
template <int R>
__device__ __forceinline__ void emit_strided(zd* base, long mstride, int m0, int M, double f,
                                             const zd (&x)[R]) {
  const int b = threadIdx.x & 63;
#pragma unroll
  for (int sl = 0; sl < R; ++sl) {
    const int n = fft_wave_out_index<R>(b, sl);
    if (n >= m0 && n <= M) base[(long)(n - m0) * mstride] = f * x[sl];
  }
}

// Both orderings of a far pair at once: pair a = (i, l) (source l) and pair
// b = (l, i) (source i) share the distance R and e^{ikR}, hence the single
// layer S (reciprocity); only the double-layer numerators differ.  Per
// wavenumber: the samples of S, K_a, K_b on the half circle are staged in
// LDS, S and K_a are transformed together and emitted to a (S also to b),
// then K_b alone to b.  Two of the four complex exponentials and two of the
// eight transforms of two separate pairs are saved.  The coarse grid and the
// weights follow far_pair.  LDS for R <= 16: K_b at [0, H), S and K_a at
// [H, 3H), the exchange area of the transform from H on (S and K_a are in
// registers by then); for R = 32: S, K_a, K_b at [0, 3H) and the exchange area
// after them.  Within far_lds<R>() either way.
template <int R>
__device__ __forceinline__ void far_pair_sym(const PairInv& v, zd N0b, zd N1b, zd k1, zd k2,
                                             const zd* __restrict__ tw, zd* lds, const OutSpec& o, int2 da,
                                             int2 db, bool coarse) {
  if constexpr (R > 16) {
    // the 2048-point grid: S, K_a, K_b staged at [0, 3H), each transformed
    // alone with the exchange area E after them (a sequence of 32 slots per
    // lane is all the registers hold)
    constexpr int L = 64 * R, H = L / 2 + 1;
    zd* Sg = lds;
    zd* Ka = lds + H;
    zd* Kb = lds + 2 * H;
    zd* E = lds + 3 * H;
    const int ns = coarse ? L / 4 : L / 2 + 1;
    const double w4pi = (coarse ? 2.0 : 1.0) * (0.25 / PMLBIE_PI);
    const double scale = 2.0 * PMLBIE_PI / L;
    const double fa = 2.0 * o.W[da.y] * scale, fb = 2.0 * o.W[db.y] * scale;
    zd* const pa = o.A + (2L * da.x) * o.n2 + 2L * da.y;
    zd* const pb = o.A + (2L * db.x) * o.n2 + 2L * db.y;
    const int b = threadIdx.x & 63;
#pragma unroll 1
    for (int w = 0; w < 2; ++w) {
      const zd k = w == 0 ? k1 : k2;
#pragma unroll 1
      for (int q = b; q < ns; q += 64) {
        const int j = coarse ? 2 * q + 1 : q;
        const double s2 = tw_s2<R>(tw, j);
        const FarGeo f = far_geo(v.d2 + s2 * v.c4);
        const zd kR = k * f.R;
        const zd ikR{-kR.im, kR.re};
        const zd e = expi(kR) * (f.iR * w4pi);
        Sg[j] = e;
        Ka[j] = (v.N0 + s2 * v.N1) * e * (ikR - 1.0) * f.iR2;
        Kb[j] = (N0b + s2 * N1b) * e * (ikR - 1.0) * f.iR2;
        if (coarse) {
          const zd z0{0.0, 0.0};
          Sg[j - 1] = z0;
          Ka[j - 1] = z0;
          Kb[j - 1] = z0;
        }
      }
      if (coarse && b == 0) {
        const zd z0{0.0, 0.0};
        Sg[L / 2] = z0;
        Ka[L / 2] = z0;
        Kb[L / 2] = z0;
      }
      __syncthreads();
      const long row = w * o.n2;
#pragma unroll 1
      for (int sq = 0; sq < 3; ++sq) {
        zd x[1][R];
        load_even<R, 1>(lds + sq * H, x);
        fft_wave<R, 1>(x, E, tw);
        if (sq == 0) {
          emit_strided<R>(pa + row + 1, o.mstride, o.m0, o.M, -fa, x[0]);
          emit_strided<R>(pb + row + 1, o.mstride, o.m0, o.M, -fb, x[0]);
        } else if (sq == 1) {
          emit_strided<R>(pa + row, o.mstride, o.m0, o.M, fa, x[0]);
        } else {
          emit_strided<R>(pb + row, o.mstride, o.m0, o.M, fb, x[0]);
        }
      }
    }
    return;
  }
  constexpr int L = 64 * R, H = L / 2 + 1;
  zd* Kb = lds;
  zd* SK = lds + H;
  zd* E = lds + H;
  const int ns = coarse ? L / 4 : L / 2 + 1;
  const double w4pi = (coarse ? 2.0 : 1.0) * (0.25 / PMLBIE_PI);
  const double scale = 2.0 * PMLBIE_PI / L;
  // entries of mode m0 of both orderings (S entries at unknown 2l + 1 with
  // the block's minus sign, K entries at 2l)
  const double fa = 2.0 * o.W[da.y] * scale, fb = 2.0 * o.W[db.y] * scale;
  zd* const pa = o.A + (2L * da.x) * o.n2 + 2L * da.y;
  zd* const pb = o.A + (2L * db.x) * o.n2 + 2L * db.y;
  const int b = threadIdx.x & 63;
#pragma unroll 1
  for (int w = 0; w < 2; ++w) {
    const zd k = w == 0 ? k1 : k2;
#pragma unroll 1
    for (int q = b; q < ns; q += 64) {
      const int j = coarse ? 2 * q + 1 : q;
      const double s2 = tw_s2<R>(tw, j);
      const FarGeo f = far_geo(v.d2 + s2 * v.c4);
      const zd kR = k * f.R;
      const zd ikR{-kR.im, kR.re};
      const zd e = expi(kR) * (f.iR * w4pi);
      const zd iR2 = f.iR2;
      // the same products, in the same order, as far_pair
      SK[j] = e;
      SK[H + j] = (v.N0 + s2 * v.N1) * e * (ikR - 1.0) * iR2;
      Kb[j] = (N0b + s2 * N1b) * e * (ikR - 1.0) * iR2;
      if (coarse) {
        const zd z0{0.0, 0.0};
        SK[j - 1] = z0;
        SK[H + j - 1] = z0;
        Kb[j - 1] = z0;
      }
    }
    if (coarse && b == 0) {
      const zd z0{0.0, 0.0};
      SK[L / 2] = z0;
      SK[H + L / 2] = z0;
      Kb[L / 2] = z0;
    }
    __syncthreads();
    const long row = w * o.n2;  // lower-medium equation: one row down
    {
      zd x[2][R];
      load_even<R, 2>(SK, x);
      __syncthreads();
      fft_wave<R, 1>(*reinterpret_cast<zd(*)[1][R]>(&x[0]), E, tw);
      emit_strided<R>(pa + row + 1, o.mstride, o.m0, o.M, -fa, x[0]);
      emit_strided<R>(pb + row + 1, o.mstride, o.m0, o.M, -fb, x[0]);
      fft_wave<R, 1>(*reinterpret_cast<zd(*)[1][R]>(&x[1]), E, tw);
      emit_strided<R>(pa + row, o.mstride, o.m0, o.M, fa, x[1]);
    }
    {
      zd x[1][R];
      load_even<R, 1>(Kb, x);
      __syncthreads();
      fft_wave<R, 1>(x, E, tw);
      emit_strided<R>(pb + row, o.mstride, o.m0, o.M, fb, x[0]);
    }
  }
}

// Main grid over the unordered pairs {i, l} (i < l) off the near panels,
// both orderings at once (the class, the coarse flag and the far pass are
// symmetric in the two points).  Far pairs are finished here (raw-kernel FFT
// over theta on this pass's grid of 64 R angles); the others are appended to
// the split / direct work lists in both orderings, and far pairs that need a
// longer grid to the far_big list.  One wavefront per unordered pair.  The
// pairs are walked in 4 x 4 tiles of nodes (i = 4 I + r / 4, l = 4 J + r % 4):
// the 16 pairs of a tile fill whole 128-byte lines of both orderings' rows
// (4 nodes x (u, phi) columns), where a walk along one row of the triangle
// would write the transposed ordering one column at a time.  The tiles are
// taken in super-blocks of 16 x 16 (super-block rows BI <= BJ of their
// triangle, row-major inside), so that the tiles in flight on one XCD write
// the rows of 64 + 64 nodes, not of a whole row of tiles (3-4% faster).  No waves-per-SIMD bound: held
// to two waves the R = 8 pass spills its loop invariants to scratch and runs
// a third slower than at one wave without spills.
constexpr int FAR_TILE = 4;
constexpr int FAR_SB = 16;  // tiles per side of a super-block
__host__ __device__ inline long far_tile_slots(int N) {
  const long nt = (N + FAR_TILE - 1) / FAR_TILE;
  const long ns = (nt + FAR_SB - 1) / FAR_SB;
  return ns * (ns + 1) / 2 * (FAR_SB * FAR_SB) * (FAR_TILE * FAR_TILE);
}
template <int R>
__global__ __launch_bounds__(64) void k_grid_far(NodesDev nd, ClassParams cp, zd k1, zd k2,
                                                 const zd* __restrict__ tw, OutSpec o,
                                                 WorkList split, WorkList direct, WorkList far_big,
                                                 WorkList split_big) {
  __shared__ zd lds[far_lds<R>()];
  const int N = nd.N;
  const long NT = (N + FAR_TILE - 1) / FAR_TILE;
  const long NS = (NT + FAR_SB - 1) / FAR_SB;
  const long total = far_tile_slots(N);
  const double tn = 2.0 * NS + 1.0;
  // workgroups are dealt to the 8 XCDs round-robin; each XCD takes a
  // contiguous run of tiles so that the lines they write meet in one L2
  const long lb = (long)(blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  for (long p = lb; p < total; p += gridDim.x) {
    const long t = p >> 4;
    const int r = (int)(p & 15);
    const long sb = t / (FAR_SB * FAR_SB);
    const int ts = (int)(t % (FAR_SB * FAR_SB));
    // super-block row BI starts at s(BI) = BI (2 NS + 1 - BI) / 2
    long BI = (long)floor(0.5 * (tn - sqrt(tn * tn - 8.0 * (double)sb)));
    if (BI < 0) BI = 0;
    while (BI > 0 && BI * (2 * NS + 1 - BI) / 2 > sb) --BI;
    while ((BI + 1) * (2 * NS - BI) / 2 <= sb) ++BI;
    const long BJ = sb - BI * (2 * NS + 1 - BI) / 2 + BI;
    const long I = BI * FAR_SB + ts / FAR_SB, J = BJ * FAR_SB + ts % FAR_SB;
    if (I > J || J >= NT) continue;
    const int i = (int)(FAR_TILE * I) + (r >> 2), l = (int)(FAR_TILE * J) + (r & 3);
    if (l <= i || l >= N) continue;
    const int dp = nd.panel[i] - nd.panel[l];
    if (dp >= -1 && dp <= 1) continue;  // near panels: product integration
    const PairGeom g = node_pair(nd, i, l);
    const PairInv v = pair_invariants(g);
    bool coarse = false;
    const int cls = classify(g, v, cp, &coarse);
    if (cls != CLASS_FAR) {
      // far pairs on the long grid are listed once (i, l), i < l, and
      // transformed in both orderings from the list (k_list_far_sym); the
      // other classes list both orderings
      if (threadIdx.x < (cls == CLASS_FAR_BIG ? 1 : 2)) {
        WorkList& wl = cls == CLASS_SPLIT ? split
                       : (cls == CLASS_DIRECT ? direct : (cls == CLASS_FAR_BIG ? far_big : split_big));
        const unsigned slot = atomicAdd(wl.count, 1u);
        if (slot < wl.cap) {
          wl.geom[slot] = threadIdx.x == 0 ? g : node_pair(nd, l, i);
          wl.dest[slot] = threadIdx.x == 0 ? make_int2(i, l) : make_int2(l, i);
        }
      }
      continue;
    }
    // the conormal numerator of the ordering (l, i): source i, target l
    const zd nrb{nd.nr_re[i], nd.nr_im[i]}, nzb{nd.nz_re[i], nd.nz_im[i]};
    const zd N0b = nrb * g.drho + nzb * g.dz;  // -(n_i . (r~_l - r~_i))
    const zd N1b = 2.0 * (nrb * g.rs);
    far_pair_sym<R>(v, N0b, N1b, k1, k2, tw, lds, o, make_int2(i, l), make_int2(l, i), coarse);
  }
}

// Wave-aggregated append of this lane's pair to the work list of its class
// (one counter update per wavefront and class).
__device__ __forceinline__ void append_by_class(int cls, const PairGeom& g, int2 dst, WorkList far,
                                                WorkList split, WorkList direct, WorkList split_big) {
  const int lane = threadIdx.x & 63;
  // list slots: far (the far lists of this path are transformed on the full
  // grid, so CLASS_FAR_BIG joins them), split, direct, split on the full grid
  if (cls == CLASS_SPLIT_BIG) cls = 3;
  else if (cls == CLASS_FAR_BIG) cls = CLASS_FAR;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const unsigned long long mask = __ballot(cls == c);
    if (mask == 0) continue;
    const int leader = __ffsll((long long)mask) - 1;
    WorkList& wl = c == CLASS_FAR ? far : (c == CLASS_SPLIT ? split : (c == CLASS_DIRECT ? direct : split_big));
    unsigned base = 0;
    if (lane == leader) base = atomicAdd(wl.count, (unsigned)__popcll(mask));
    base = __shfl(base, leader);
    if (cls == c) {
      const unsigned slot = base + (unsigned)__popcll(mask & ((1ull << lane) - 1ull));
      if (slot < wl.cap) {
        wl.geom[slot] = g;
        wl.dest[slot] = dst;
      }
    }
  }
}

// Classification only (the surrogate path): every (target i, source l) pair
// off the near panels goes to the far / split / direct work list of its class
// with destination (i, l); one thread per pair.
__global__ __launch_bounds__(256) void k_grid_classify(NodesDev nd, ClassParams cp, WorkList far,
                                                       WorkList split, WorkList direct, WorkList split_big) {
  const long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int N = nd.N;
  int cls = -1, i = 0, l = 0;
  PairGeom g;
  if (p < (long)N * N) {
    l = (int)(p % N);
    i = (int)(p / N);
    const int dp = nd.panel[i] - nd.panel[l];
    if (dp < -1 || dp > 1) {  // near panels: product integration
      g = node_pair(nd, i, l);
      cls = classify(g, pair_invariants(g), cp);
    }
  }
  append_by_class(cls, g, make_int2(i, l), far, split, direct, split_big);
}

// Classification of an explicit pair list into far / split / direct work
// lists (destination = raw row q).
__global__ void k_classify_list(const PairGeom* __restrict__ geom, long count, ClassParams cp,
                                WorkList far, WorkList split, WorkList direct, WorkList split_big) {
  const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
  int cls = -1;
  PairGeom g;
  if (q < count) {
    g = geom[q];
    cls = classify(g, pair_invariants(g), cp);
  }
  append_by_class(cls, g, make_int2((int)q, -1), far, split, direct, split_big);
}

// Explicit list of far pairs (right-hand sides, field points).
template <int R>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_list_far(const PairGeom* __restrict__ geom,
                                                 const int2* __restrict__ dest, long first,
                                                 long count, zd k1, zd k2,
                                                 const zd* __restrict__ tw, OutSpec o,
                                                 ClassParams cp, int use_coarse) {
  __shared__ zd lds[far_lds<R>()];
  for (long t = blockIdx.x; t < count; t += gridDim.x) {
    const PairGeom g = geom[first + t];
    const PairInv v = pair_invariants(g);
    bool coarse = false;
    if (use_coarse) (void)classify(g, v, cp, &coarse);
    far_pair<R>(v, k1, k2, tw, lds, o, dest[first + t], coarse);
  }
}

// The long-grid far pairs of the main pass, one entry (i, l) per unordered
// pair: both orderings from one set of samples (far_pair_sym); the normal of
// node i gives the double-layer numerator of the ordering (l, i).
template <int R>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(R <= 16 ? 2 : 1))) void k_list_far_sym(
    const PairGeom* __restrict__ geom, const int2* __restrict__ dest, long count, NodesDev nd, zd k1, zd k2,
    const zd* __restrict__ tw, OutSpec o, ClassParams cp) {
  __shared__ zd lds[far_lds<R>()];
  for (long t = blockIdx.x; t < count; t += gridDim.x) {
    const PairGeom g = geom[t];
    const int2 d = dest[t];
    const PairInv v = pair_invariants(g);
    bool coarse = false;
    (void)classify(g, v, cp, &coarse);
    const zd nrb{nd.nr_re[d.x], nd.nr_im[d.x]}, nzb{nd.nz_re[d.x], nd.nz_im[d.x]};
    const zd N0b = nrb * g.drho + nzb * g.dz;  // -(n_i . (r~_l - r~_i))
    const zd N1b = 2.0 * (nrb * g.rs);
    far_pair_sym<R>(v, N0b, N1b, k1, k2, tw, lds, o, d, make_int2(d.y, d.x), coarse);
    __syncthreads();
  }
}

// Field points lie in one medium: the far pairs of a field chunk need the
// kernels of that medium's wavenumber only, i.e. sequences (0, 1) for the
// upper medium and (2, 3) for the lower one, half the samples, transforms and
// writes of far_pair.  The point of raw row q is q / N (rows p * N + l);
// medium[p] is 1 or 2.
template <int R>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_list_far_one(
    const PairGeom* __restrict__ geom, const int2* __restrict__ dest, long first, long count, zd k1, zd k2,
    const zd* __restrict__ tw, OutSpec o, const int* __restrict__ medium, int N) {
  constexpr int L = 64 * R, H = L / 2 + 1;
  __shared__ zd lds[far_lds<R>()];
  zd* P1 = pair_p1<R>(lds);
  zd* E = pair_e<R>(lds);
  const double w4pi = 0.25 / PMLBIE_PI;
  for (long t = blockIdx.x; t < count; t += gridDim.x) {
    const PairGeom g = geom[first + t];
    const int2 dst = dest[first + t];
    const PairInv v = pair_invariants(g);
    const int md = medium[dst.x / N];
    const zd k = md == 1 ? k1 : k2;
#pragma unroll 1
    for (int j = threadIdx.x; j < H; j += 64) {
      const double s2 = tw_s2<R>(tw, j);
      const FarGeo f = far_geo(v.d2 + s2 * v.c4);
      const zd kR = k * f.R;
      const zd ikR{-kR.im, kR.re};
      const zd e = expi(kR) * (f.iR * w4pi);
      P1[j] = e;
      P1[H + j] = (v.N0 + s2 * v.N1) * e * (ikR - 1.0) * f.iR2;
    }
    __syncthreads();
    transform_emit<R>(P1, E, tw, o, dst, md == 1 ? 0 : 2);
  }
}

// ------------------------------------------------------------------------
// Split pairs, phase 1 (one lane per pair): Q_{m-1/2}(chi), m = 0..MQ,
// chi = 1 + d2/(2 rho~ rho~'), and the factors that turn it into the
// semi-analytic modes of the singular factors, Zhat_m = modes of 1/(4 pi R)
// and Phat_m = modes of 1/R^3 (formed in phase 1b):
//   modes of (chi - cos D)^{-1/2} = 2 sqrt2 Q_{m-1/2}(chi)          (Heine)
//   modes of (chi - cos D)^{-3/2} = -4 sqrt2 Q'_{m-1/2}(chi)
// and R = sgn sqrt(c) sqrt(chi - cos D), c = 2 rho~ rho~', with the sign
// fixed by continuity against the principal R at D = pi.
__global__ __launch_bounds__(64) void k_split_singular(const PairGeom* __restrict__ geom,
                                                       long first, long count, int MQ,
                                                       zd* __restrict__ qtab,
                                                       zd* __restrict__ coef) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  const PairGeom g = geom[first + t];
  const PairInv v = pair_invariants(g);
  const zd c = 2.0 * (g.rt * g.rs);
  const zd chim1 = v.d2 / c;
  // Q is [m][pair], so that consecutive lanes write consecutive pairs
  legendre_q_half(chim1, MQ, qtab + t, count);
  const zd sc = csqrt_(c);
  const zd Rpi = csqrt_(v.d2 + v.c4);
  const zd Rsp = sc * csqrt_(chim1 + 2.0);
  const double sgn = cabs_(Rpi - Rsp) <= cabs_(Rpi + Rsp) ? 1.0 : -1.0;
  const double rt2 = 1.4142135623730950488;
  const zd isc = inv(sc);
  zd* cf = coef + 4 * t;
  cf[0] = (sgn * 2.0 * rt2 * (0.25 / PMLBIE_PI)) * isc;  // Zhat_m = cf0 Q_m
  cf[1] = (sgn * (-4.0) * rt2) * isc * isc * isc;        // Phat_m = cf1 Q'_m
  cf[2] = chim1;
  cf[3] = inv(chim1 * (chim1 + 2.0));                    // 1 / (chi^2 - 1)
}

// Split pairs, phase 1b: Zhat and Phat in pair-major tables (the layout the
// split kernel reads) from the mode-major Q table, through an LDS tile of 64
// pairs x 64 modes (plus the mode below the tile):
//   Q'_{m-1/2} = (m - 1/2)(chi Q_{m-1/2} - Q_{m-3/2}) / (chi^2 - 1),
// with Q_{-3/2} = Q_{1/2}.
__global__ __launch_bounds__(256) void k_split_tables(const zd* __restrict__ qtab,
                                                      const zd* __restrict__ coef, long count,
                                                      int MQ, zd* __restrict__ zhat,
                                                      zd* __restrict__ phat) {
  __shared__ zd Qs[65][65];  // [mode - m0 + 1][pair - p0]
  const long p0 = (long)blockIdx.x * 64;
  const int m0 = blockIdx.y * 64;
  for (int e = threadIdx.x; e < 65 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    const int m = (m0 == 0 && r == 0) ? (MQ >= 1 ? 1 : 0) : m0 - 1 + r;
    const long p = p0 + c;
    Qs[r][c] = (p < count && m <= MQ) ? qtab[(long)m * count + p] : zd{0.0, 0.0};
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int c = e >> 6, r = e & 63;  // a wavefront per pair, lanes over modes
    const long p = p0 + c;
    const int m = m0 + r;
    if (p >= count || m > MQ) continue;
    const zd* cf = coef + 4 * p;
    const zd qm = Qs[r + 1][c], qm1 = Qs[r][c];
    const zd num = cf[2] * qm + (qm - qm1);
    zhat[p * (MQ + 1) + m] = cf[0] * qm;
    phat[p * (MQ + 1) + m] = cf[1] * ((m - 0.5) * num * cf[3]);
  }
}

// Split pairs, phase 2 (one wavefront per pair).  With Zs and Ds the singular
// factors restricted to their modes |m| <= MQ (Dhat_m = -(e0 Phat_m +
// 4 pi e1 Zhat_m)/(4 pi)), the convolutions of the split become products on
// the angle grid D_j = 2 pi j / L:
//   S_n = modes of [Zs H1 + i ZH2],  K_n = modes of [Ds H3 + i DH4],
// which equal (1/2pi) sum_j Zhat_{n-j} H1hat_j + i ZH2hat_n (and the same for
// K) exactly for n <= M when L >= 2 MQ + 1 and the smooth parts carry no
// modes beyond MQ - M.  Zs, Ds come from one transform of the even mode
// sequences; the four products from one transform per wavenumber.
// CH (chL > 0): the substitution of Sec. 4.3 (eq. eqch1, split_smooth_ch) in
// place of H1, i H2, H3, i H4: S_n = modes of [Zs cH1 + Z (e^{iq} - cH1)],
// K_n = modes of [Ds cH3 + D (e^{iq} (1 - iq) - cH3)].
template <int R, bool CH>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_split(const PairGeom* __restrict__ geom,
                                              const int2* __restrict__ dest, long first,
                                              long count, int M, int MQ, zd k1, zd k2,
                                              const zd* __restrict__ tw,
                                              const zd* __restrict__ zhat,
                                              const zd* __restrict__ phat, OutSpec o, int chL) {
  constexpr int L = 64 * R, H = L / 2 + 1;
  __shared__ zd lds[pair_lds<R>()];
  zd* P2 = lds;
  zd* P1 = pair_p1<R>(lds);
  zd* E = pair_e<R>(lds);
  const double inv2pi = 0.5 / PMLBIE_PI;
  const int b = threadIdx.x & 63;
  for (long t = blockIdx.x; t < count; t += gridDim.x) {
    const PairGeom g = geom[first + t];
    const int2 dst = dest[first + t];
    const PairInv v = pair_invariants(g);
    const SplitCoef sc = split_coef(g, v);
    const zd* zz = zhat + t * (MQ + 1);
    const zd* pp = phat + t * (MQ + 1);
    const zd e0f = (-0.25 / PMLBIE_PI) * sc.e0;
    const zd e1f = -1.0 * sc.e1;
    {
      // Zs, Ds on the grid from their even mode sequences, staged in P2
      constexpr int NQ = R <= 16 ? 2 : 1;  // sequences per transform
#pragma unroll 1
      for (int q0 = 0; q0 < 2; q0 += NQ) {
        zd sg[NQ][R];
#pragma unroll
        for (int a = 0; a < R; ++a) {
          const int m = b + 64 * a;
          const int mm = m <= L / 2 ? m : L - m;
          zd zm{0.0, 0.0}, dm{0.0, 0.0};
          if (mm <= MQ) {
            zm = zz[mm];
            dm = e0f * pp[mm] + e1f * zm;
          }
#pragma unroll
          for (int q = 0; q < NQ; ++q) sg[q][a] = (q0 + q) == 0 ? zm : dm;
        }
        fft_wave<R, NQ>(sg, E, tw);
#pragma unroll
        for (int sl = 0; sl < R; ++sl) {
          const int j = fft_wave_out_index<R>(b, sl);
          if (j <= L / 2) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) P2[(q0 + q) * H + j] = inv2pi * sg[q][sl];
          }
        }
      }
    }
    __syncthreads();
    // products for both wavenumbers: medium 1 into P1, medium 2 over Zs, Ds
#pragma unroll 1
    for (int j = b; j <= L / 2; j += 64) {
      const double sh = sin(PMLBIE_PI * j / L);
      const zd Rd = csqrt_(v.d2 + (sh * sh) * v.c4);
      const zd zs = P2[j], ds = P2[H + j];
      if constexpr (CH) {
        zd H1c, Sr, H3c, Kr;
        split_smooth_ch(sc, Rd, k1, chL, H1c, Sr, H3c, Kr);
        P1[j] = zs * H1c + Sr;
        P1[H + j] = ds * H3c + Kr;
        split_smooth_ch(sc, Rd, k2, chL, H1c, Sr, H3c, Kr);
        P2[j] = zs * H1c + Sr;
        P2[H + j] = ds * H3c + Kr;
      } else {
        zd H1, ZH2, H3, DH4;
        split_smooth(sc, Rd, k1, H1, ZH2, H3, DH4);
        P1[j] = zs * H1 + zd{-ZH2.im, ZH2.re};
        P1[H + j] = ds * H3 + zd{-DH4.im, DH4.re};
        split_smooth(sc, Rd, k2, H1, ZH2, H3, DH4);
        P2[j] = zs * H1 + zd{-ZH2.im, ZH2.re};
        P2[H + j] = ds * H3 + zd{-DH4.im, DH4.re};
      }
    }
    __syncthreads();
    transform_emit<R>(P1, E, tw, o, dst, 0);
    transform_emit<R>(P2, E, tw, o, dst, 2);
  }
}

// ------------------------------------------------------------------------
// Direct pairs (close, deep in the PML): F_n = 2 sum_q w_q cos(n D_q) F(D_q)
// over a composite 16-point Gauss-Legendre rule on [0, pi] graded toward the
// nearest singularity Re D* with smallest piece ~ |Im D*|/4, and pieces short
// enough for the oscillation of cos(n D) exp(i k R).
// One wavefront per pair: 64 nodes are sampled at a time into LDS with the
// table cos(j D), j = 0..16; lane (a, g) = (lane / 16, lane % 16) then sums
// nodes a, a+4, ... of the batch into modes n = g + 16 r with the
// stride-16 Chebyshev recurrence cos((n+16)D) = 2 cos(16D) cos(nD) - cos((n-16)D).
#define DIRECT_MAX_PIECES 512
#define DIRECT_MPL 9  // modes per lane per pass (16 * 9 = 144 modes)

__global__ __launch_bounds__(64) void k_direct(const PairGeom* __restrict__ geom,
                                               const int2* __restrict__ dest, long first,
                                               long count, int M, zd k1, zd k2,
                                               const double* __restrict__ glx,
                                               const double* __restrict__ glw, OutSpec o,
                                               double omega_piece) {
  __shared__ double pa[DIRECT_MAX_PIECES], pb[DIRECT_MAX_PIECES];
  __shared__ int npieces;
  __shared__ zd fs[64][4];
  __shared__ double cw[64][18];  // cos(j D) j = 0..16, then weight
  const int lane = threadIdx.x;
  const int ga = lane >> 4, gm = lane & 15;
  const int mb = o.m0 & ~15;
  for (long t = blockIdx.x; t < count; t += gridDim.x) {
    const PairGeom g = geom[first + t];
    const int2 dst = dest[first + t];
    const PairInv v = pair_invariants(g);
    if (lane == 0) {
      double delta, re0;
      singularity(v, delta, re0);
      const double kabs = fmax(cabs_(k1), cabs_(k2));
      const double om = M + kabs * sqrt(cabs_(g.rt * g.rs)) + 1.0;
      const double hmax = omega_piece / om;      // longest piece for the oscillation
      const double hmin = fmax(0.25 * delta, 1e-15);
      int np = 0;
      // graded breakpoints around c = re0 (both sides), then uniform pieces
      double c = re0;
      // left side [0, c]: the walk from c toward 0 runs twice, first counting
      // its non-empty pieces, then storing each at its place in increasing
      // order (no private array: it would live in scratch memory)
      {
        int nl = 0;
        for (int pass = 0; pass < 2; ++pass) {
          int q = 0, nb = 0;
          double x = c, h = hmin;
          while (x > 0.0 && nb < 120) {
            const double step = fmin(h, hmax);
            const double nx = fmax(0.0, x - step);
            ++nb;
            if (x > nx) {
              if (pass) {
                pa[nl - 1 - q] = nx;
                pb[nl - 1 - q] = x;
              }
              ++q;
            }
            x = nx;
            h *= 2.0;
          }
          nl = q;
        }
        np = nl;
      }
      // right side [c, pi]
      {
        double x = c, h = hmin;
        while (x < PMLBIE_PI && np < DIRECT_MAX_PIECES) {
          double step = fmin(h, hmax);
          double nx = fmin(PMLBIE_PI, x + step);
          if (PMLBIE_PI - nx < 1e-3 * step) nx = PMLBIE_PI;
          pa[np] = x; pb[np] = nx; ++np;
          x = nx;
          h *= 2.0;
        }
      }
      npieces = np;
    }
    __syncthreads();
    const int nnodes = npieces * 16;
    // passes of 144 modes from the first mode the caller keeps (rounded down
    // to the recurrence stride), so a batch of at most 129 modes takes one
    for (int nbase = mb; nbase <= M; nbase += 16 * DIRECT_MPL) {
      zd acc[DIRECT_MPL][4];
#pragma unroll
      for (int r = 0; r < DIRECT_MPL; ++r)
#pragma unroll
        for (int s = 0; s < 4; ++s) acc[r][s] = zd{0.0, 0.0};
      for (int q0 = 0; q0 < nnodes; q0 += 64) {
        const int q = q0 + lane;
        if (q < nnodes) {
          const int pc = q >> 4, j = q & 15;
          const double a = pa[pc], b = pb[pc];
          const double D = 0.5 * (a + b) + 0.5 * (b - a) * glx[j];
          const double w = 0.5 * (b - a) * glw[j];
          const double sh = sin(0.5 * D);
          zd S1, K1, S2, K2;
          kernel_sample(v, sh * sh, k1, S1, K1);
          kernel_sample(v, sh * sh, k2, S2, K2);
          fs[lane][0] = S1;
          fs[lane][1] = K1;
          fs[lane][2] = S2;
          fs[lane][3] = K2;
          const double c1 = cos(D);
          double cm = 1.0, cc = c1;
          cw[lane][0] = 1.0;
          cw[lane][1] = c1;
          for (int jj = 2; jj <= 16; ++jj) {
            double cn = 2.0 * c1 * cc - cm;
            cm = cc;
            cc = cn;
            cw[lane][jj] = cn;
          }
          // base cosines for this pass: recurrence stride 16 starts at nbase
          cw[lane][17] = 2.0 * w;
        } else {
          fs[lane][0] = fs[lane][1] = fs[lane][2] = fs[lane][3] = zd{0.0, 0.0};
          cw[lane][17] = 0.0;
          for (int jj = 0; jj <= 16; ++jj) cw[lane][jj] = 1.0;
        }
        __syncthreads();
        for (int u = ga; u < 64; u += 4) {
          const double wq = cw[u][17];
          if (wq == 0.0) continue;
          const double c16 = cw[u][16];
          // cos(g D) and cos((g - 16) D) = cos((16 - g) D), then advance to nbase
          double cprev = cw[u][16 - gm], ccur = cw[u][gm];
          for (int r = 0; r < nbase / 16; ++r) {
            double cn = 2.0 * c16 * ccur - cprev;
            cprev = ccur;
            ccur = cn;
          }
          const zd f0 = fs[u][0], f1 = fs[u][1], f2 = fs[u][2], f3 = fs[u][3];
#pragma unroll
          for (int r = 0; r < DIRECT_MPL; ++r) {
            const double cwq = wq * ccur;
            acc[r][0] = acc[r][0] + cwq * f0;
            acc[r][1] = acc[r][1] + cwq * f1;
            acc[r][2] = acc[r][2] + cwq * f2;
            acc[r][3] = acc[r][3] + cwq * f3;
            double cn = 2.0 * c16 * ccur - cprev;
            cprev = ccur;
            ccur = cn;
          }
        }
        __syncthreads();
      }
      // reduce the 4 node groups (lanes gm, gm + 16, gm + 32, gm + 48)
#pragma unroll
      for (int r = 0; r < DIRECT_MPL; ++r)
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          zd a = acc[r][s];
          a.re += __shfl_xor(a.re, 16);
          a.im += __shfl_xor(a.im, 16);
          a.re += __shfl_xor(a.re, 32);
          a.im += __shfl_xor(a.im, 32);
          acc[r][s] = a;
        }
      if (ga == 0) {
#pragma unroll
        for (int r = 0; r < DIRECT_MPL; ++r) {
          const int n = nbase + gm + 16 * r;
          if (n <= M) emit(o, dst, n, acc[r][0], acc[r][1], acc[r][2], acc[r][3]);
        }
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------------------
// Near panels: product integration of the modal kernels at auxiliary source
// points against the Lagrange basis of the panel, plus the identity term of
// the smooth-point solid angle (K1 - D1 = K1 + I, K2 - D2 = K2 - I).
// One workgroup per (target, panel) job; raw modal values raw[q][s][n].
__global__ __launch_bounds__(256) void k_near(const NearJob* __restrict__ jobs, int njobs,
                                              const double* __restrict__ coef,
                                              const zd* __restrict__ raw, int M, OutSpec o) {
  const int jb = blockIdx.x;
  if (jb >= njobs) return;
  const NearJob J = jobs[jb];
  const int tot = 4 * (M + 1);
  // thread -> (sequence s, mode n): each raw value is read once per job and
  // weighted by the 16 Lagrange coefficients of its auxiliary point
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const int sq = e / (M + 1), n = e % (M + 1);
    if (n < o.m0) continue;  // raw values below the batch need not be there
    zd acc[16];
#pragma unroll
    for (int l = 0; l < 16; ++l) acc[l] = zd{0.0, 0.0};
    for (int q = J.q0; q < J.q1; ++q) {
      const zd r = raw[(long)q * 4 * (M + 1) + e];
      const double* c = coef + (long)q * 16;
#pragma unroll
      for (int l = 0; l < 16; ++l) acc[l] = acc[l] + c[l] * r;
    }
    const long i = J.target;
    zd* An = o.A + (long)(n - o.m0) * o.mstride;
    // K entries carry the identity term, S entries the minus sign
    const double diag = sq == 1 ? 1.0 : (sq == 3 ? -1.0 : 0.0);
#pragma unroll
    for (int l = 0; l < 16; ++l) {
      const long src = (long)J.panel * 16 + l;
      zd v = (sq & 1) ? acc[l] : -1.0 * acc[l];
      if (src == i) v.re += diag;
      An[sys_offset(o.n2, i, src, sq)] = v;
    }
  }
}

// Pair geometry of field points (rho, z; physical region, Im rho~ = 0) against
// every node: out[p * N + l], one thread per pair.
__global__ __launch_bounds__(256) void k_field_pairs(NodesDev nd, const double* __restrict__ pts, int np,
                                                     PairGeom* __restrict__ out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long N = nd.N;
  if (e >= (long)np * N) return;
  const int p = (int)(e / N), l = (int)(e % N);
  const double r = pts[2 * p], zz = pts[2 * p + 1];
  PairGeom q;
  q.rt = zd{r, 0.0};
  q.rs = zd{nd.rho[l], nd.I[l]};
  q.drho = zd{r - nd.rho[l], -nd.I[l]};
  q.dz = zd{zz - nd.z[l], 0.0};
  q.nr = zd{nd.nr_re[l], nd.nr_im[l]};
  q.nz = zd{nd.nz_re[l], nd.nz_im[l]};
  out[e] = q;
}

// Field points near the curve: the modal kernels of a point against the 16
// nodes of a nearby panel are replaced by product integrals over the panel
// (auxiliary points graded toward the closest curve point, Lagrange basis of
// the panel), already divided by the node weights that the field sum applies.
// One workgroup per (point, panel) job; raw_aux[q][s][n] at the auxiliary
// points, raw[(point * N + node)][s][n] the chunk's kernels.
__global__ __launch_bounds__(256) void k_field_near(const NearJob* __restrict__ jobs, int njobs,
                                                    const double* __restrict__ coef,
                                                    const zd* __restrict__ raw_aux, int N, int M,
                                                    zd* __restrict__ raw) {
  const int jb = blockIdx.x;
  if (jb >= njobs) return;
  const NearJob J = jobs[jb];
  const int tot = 4 * (M + 1);
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    zd acc[16];
#pragma unroll
    for (int l = 0; l < 16; ++l) acc[l] = zd{0.0, 0.0};
    for (int q = J.q0; q < J.q1; ++q) {
      const zd v = raw_aux[(long)q * tot + e];
      const double* c = coef + (long)q * 16;
#pragma unroll
      for (int l = 0; l < 16; ++l) acc[l] = acc[l] + c[l] * v;
    }
    zd* dst = raw + ((long)J.target * N + (long)J.panel * 16) * tot + e;
#pragma unroll
    for (int l = 0; l < 16; ++l) dst[(long)l * tot] = acc[l];
  }
}

// ------------------------------------------------------------------------
// Plane-wave right-hand sides (Sec. 2): the jump of the reference field
//   [u_tot0] = e^{-i k1 rho sin(phi) cos(theta)} g(z),
//   g(z) = e^{-i k1 z cos(phi)} + Rc e^{i k1 z cos(phi)} - (1 + Rc) e^{-i k* z},
// vanishes on the flat part z = 0 (where the PML acts), so it is evaluated at
// the physical node coordinates; its normal derivative is
// nu_rho d/drho + nu_z d/dz.  Modes by an azimuthal FFT of the samples (the
// data are even in theta).  One wavefront per (node, incidence);
// b1 = -[u_tot0]_n, b2 = -[du_tot0/dnu]_n at b[(n * nrhs + r) * N + i].
template <int NT>
__global__ __launch_bounds__(64) void k_rhs_plane(const double* __restrict__ rho,
                                                  const double* __restrict__ z,
                                                  const double* __restrict__ nur,
                                                  const double* __restrict__ nuz, int N,
                                                  const PlaneWave* __restrict__ pw, int npw,
                                                  const zd* __restrict__ tw, int M, int m0, int nrhs,
                                                  zd* __restrict__ b1, zd* __restrict__ b2) {
  __shared__ zd buf[2 * NT];
  const double scale = 2.0 * PMLBIE_PI / NT;
  for (long t = blockIdx.x; t < (long)N * npw; t += gridDim.x) {
    const int i = (int)(t % N), w = (int)(t / N);
    const PlaneWave P = pw[w];
    const double r = rho[i], zz = z[i];
    const zd I{0.0, 1.0};
    const zd e1 = cexp_(zd{0.0, -P.k1 * zz * P.c}), e2 = cexp_(zd{0.0, P.k1 * zz * P.c});
    const zd e3 = cexp_((-1.0 * zz) * (I * P.kst));
    const zd g = e1 + P.R * e2 - (P.R + 1.0) * e3;
    const zd gp = (-P.k1 * P.c) * (I * e1) + (P.k1 * P.c) * (I * (P.R * e2)) +
                  I * P.kst * (P.R + 1.0) * e3;
    const double a = P.k1 * r * P.s;
    for (int j = threadIdx.x; j <= NT / 2; j += 64) {
      const double ct = cos(2.0 * PMLBIE_PI * j / NT);
      const zd ph = cexp_(zd{0.0, -a * ct});
      const zd f = ph * g;
      // d/drho of the phase: -i k1 sin(phi) cos(theta)
      const zd df = nur[i] * ((-P.k1 * P.s * ct) * (I * f)) + nuz[i] * (ph * gp);
      const int ja = bitrev<NT>(j);
      buf[ja] = f;
      buf[NT + ja] = df;
      if (j > 0 && j < NT / 2) {
        const int jb = bitrev<NT>(NT - j);
        buf[jb] = f;
        buf[NT + jb] = df;
      }
    }
    __syncthreads();
    fft_lds<NT, 2>(buf, tw);
    for (int n = m0 + threadIdx.x; n <= M; n += 64) {
      const long e = ((long)(n - m0) * nrhs + P.rhs) * N + i;
      b1[e] = (-scale) * buf[n];
      b2[e] = (-scale) * buf[NT + n];
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------------
// Host launchers.
template <int R>
static void launch_far_t(const NodesDev& nd, const ClassParams& cp, zd k1, zd k2, const zd* tw,
                         const OutSpec& o, WorkList split, WorkList direct, WorkList far_big,
                         WorkList split_big, hipStream_t st) {
  const long total = far_tile_slots(nd.N);  // tile slots of the unordered pairs
  int grid = (int)std::min<long>((total + 7) / 8 * 8, 256L * 128);  // a multiple of 8
  if (grid < 8) grid = 8;
  hipLaunchKernelGGL(k_grid_far<R>, dim3(grid), dim3(64), 0, st, nd, cp, k1, k2, tw, o, split,
                     direct, far_big, split_big);
}

void launch_grid_far(const NodesDev& nd, const ClassParams& cp, zd k1, zd k2,
                     const zd* tw, zd* A, long mstride, int m0, const double* W, WorkList split,
                     WorkList direct, WorkList far_big, WorkList split_big, hipStream_t st) {
  OutSpec o{A, 2L * nd.N, mstride, W, nullptr, cp.M, m0};
  const int nt = (cp.nt_small > 0 && cp.nt_small < cp.nt_far) ? cp.nt_small : cp.nt_far;
  switch (nt) {
    case 512: launch_far_t<8>(nd, cp, k1, k2, tw, o, split, direct, far_big, split_big, st); break;
    case 1024: launch_far_t<16>(nd, cp, k1, k2, tw, o, split, direct, far_big, split_big, st); break;
    case 2048: launch_far_t<32>(nd, cp, k1, k2, tw, o, split, direct, far_big, split_big, st); break;
    default: break;
  }
}

void launch_grid_classify(const NodesDev& nd, const ClassParams& cp, WorkList far, WorkList split,
                          WorkList direct, WorkList split_big, hipStream_t st) {
  const long total = (long)nd.N * nd.N;
  hipLaunchKernelGGL(k_grid_classify, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, nd, cp, far,
                     split, direct, split_big);
}

template <int R>
static void launch_list_far_t(const PairGeom* geom, const int2* dest, long first, long count,
                              zd k1, zd k2, const zd* tw, const OutSpec& o, const ClassParams* cp,
                              hipStream_t st) {
  int grid = (int)std::min<long>(count, 256L * 128);
  hipLaunchKernelGGL(k_list_far<R>, dim3(grid), dim3(64), 0, st, geom, dest, first, count, k1, k2,
                     tw, o, cp ? *cp : ClassParams{}, cp ? 1 : 0);
}

template <int R>
static void launch_list_far_one_t(const PairGeom* geom, const int2* dest, long first, long count, zd k1,
                                  zd k2, const zd* tw, const OutSpec& o, const int* medium, int N,
                                  hipStream_t st) {
  int grid = (int)std::min<long>(count, 256L * 128);
  hipLaunchKernelGGL(k_list_far_one<R>, dim3(grid), dim3(64), 0, st, geom, dest, first, count, k1, k2, tw, o,
                     medium, N);
}

void launch_list_far_one(int nt, const PairGeom* geom, const int2* dest, long first, long count, int M,
                         zd k1, zd k2, const zd* tw, zd* raw, const int* medium, int N, hipStream_t st) {
  if (count <= 0) return;
  OutSpec o{nullptr, 0, 0, nullptr, raw, M, 0};
  switch (nt) {
    case 512: launch_list_far_one_t<8>(geom, dest, first, count, k1, k2, tw, o, medium, N, st); break;
    case 1024: launch_list_far_one_t<16>(geom, dest, first, count, k1, k2, tw, o, medium, N, st); break;
    case 2048: launch_list_far_one_t<32>(geom, dest, first, count, k1, k2, tw, o, medium, N, st); break;
    default: break;
  }
}

void launch_list_far(int nt, const PairGeom* geom, const int2* dest, long first, long count, int M,
                     int m0, zd k1, zd k2, const zd* tw, zd* A, long n2, long mstride,
                     const double* W, zd* raw, const ClassParams* cp, hipStream_t st) {
  if (count <= 0) return;
  OutSpec o{A, n2, mstride, W, raw, M, m0};
  switch (nt) {
    case 512: launch_list_far_t<8>(geom, dest, first, count, k1, k2, tw, o, cp, st); break;
    case 1024: launch_list_far_t<16>(geom, dest, first, count, k1, k2, tw, o, cp, st); break;
    case 2048: launch_list_far_t<32>(geom, dest, first, count, k1, k2, tw, o, cp, st); break;
    default: break;
  }
}

template <int R>
static void launch_list_far_sym_t(const PairGeom* geom, const int2* dest, long count, const NodesDev& nd, zd k1,
                                  zd k2, const zd* tw, const OutSpec& o, const ClassParams& cp, hipStream_t st) {
  int grid = (int)std::min<long>(count, 256L * 128);
  hipLaunchKernelGGL(k_list_far_sym<R>, dim3(grid), dim3(64), 0, st, geom, dest, count, nd, k1, k2, tw, o, cp);
}

void launch_list_far_sym(int nt, const PairGeom* geom, const int2* dest, long count, const NodesDev& nd, int M,
                         int m0, zd k1, zd k2, const zd* tw, zd* A, long n2, long mstride, const double* W,
                         const ClassParams& cp, hipStream_t st) {
  if (count <= 0) return;
  OutSpec o{A, n2, mstride, W, nullptr, M, m0};
  switch (nt) {
    case 512: launch_list_far_sym_t<8>(geom, dest, count, nd, k1, k2, tw, o, cp, st); break;
    case 1024: launch_list_far_sym_t<16>(geom, dest, count, nd, k1, k2, tw, o, cp, st); break;
    case 2048: launch_list_far_sym_t<32>(geom, dest, count, nd, k1, k2, tw, o, cp, st); break;
    default: break;
  }
}

void launch_classify_list(const PairGeom* geom, long count, const ClassParams& cp, WorkList far,
                          WorkList split, WorkList direct, WorkList split_big, hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_classify_list, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, geom,
                     count, cp, far, split, direct, split_big);
}

void launch_split_singular(const PairGeom* geom, long first, long count, int MQ, zd* qtab, zd* coef,
                           zd* zhat, zd* phat, hipStream_t st) {
  if (count <= 0) return;
  int blocks = (int)((count + 63) / 64);
  hipLaunchKernelGGL(k_split_singular, dim3(blocks), dim3(64), 0, st, geom, first, count, MQ, qtab,
                     coef);
  hipLaunchKernelGGL(k_split_tables, dim3((unsigned)((count + 63) / 64), (unsigned)((MQ + 64) / 64)),
                     dim3(256), 0, st, qtab, coef, count, MQ, zhat, phat);
}

template <int R>
static void launch_split_t(const PairGeom* geom, const int2* dest, long first, long count, int M,
                           int MQ, zd k1, zd k2, const zd* tw, const zd* zhat, const zd* phat,
                           const OutSpec& o, int chL, hipStream_t st) {
  int grid = (int)std::min<long>(count, 256L * 32);
  if (chL > 0)
    hipLaunchKernelGGL((k_split<R, true>), dim3(grid), dim3(64), 0, st, geom, dest, first, count, M, MQ, k1, k2, tw,
                       zhat, phat, o, chL);
  else
    hipLaunchKernelGGL((k_split<R, false>), dim3(grid), dim3(64), 0, st, geom, dest, first, count, M, MQ, k1, k2,
                       tw, zhat, phat, o, 0);
}

void launch_split(int nt, const PairGeom* geom, const int2* dest, long first, long count, int M,
                  int m0, int MQ, zd k1, zd k2, const zd* tw, const zd* zhat, const zd* phat,
                  zd* A, long n2, long mstride, const double* W, zd* raw, hipStream_t st, int chL) {
  if (count <= 0) return;
  OutSpec o{A, n2, mstride, W, raw, M, m0};
  switch (nt) {
    case 512: launch_split_t<8>(geom, dest, first, count, M, MQ, k1, k2, tw, zhat, phat, o, chL, st); break;
    case 1024: launch_split_t<16>(geom, dest, first, count, M, MQ, k1, k2, tw, zhat, phat, o, chL, st); break;
    case 2048: launch_split_t<32>(geom, dest, first, count, M, MQ, k1, k2, tw, zhat, phat, o, chL, st); break;
    default: break;
  }
}

void launch_direct(const PairGeom* geom, const int2* dest, long first, long count, int M, int m0,
                   zd k1, zd k2, const double* glx, const double* glw, zd* A, long n2,
                   long mstride, const double* W, zd* raw, double omega_piece, hipStream_t st) {
  if (count <= 0) return;
  OutSpec o{A, n2, mstride, W, raw, M, m0};
  int grid = (int)std::min<long>(count, 256L * 24);
  hipLaunchKernelGGL(k_direct, dim3(grid), dim3(64), 0, st, geom, dest, first, count, M, k1, k2,
                     glx, glw, o, omega_piece);
}

void launch_rhs_plane(int nt, const double* rho, const double* z, const double* nur,
                      const double* nuz, int N, const PlaneWave* pw, int npw, const zd* tw, int M,
                      int m0, int nrhs, zd* b1, zd* b2, hipStream_t st) {
  if (npw <= 0) return;
  const int grid = std::min(N * npw, 256 * 32);
  switch (nt) {
    case 256: hipLaunchKernelGGL(k_rhs_plane<256>, dim3(grid), dim3(64), 0, st, rho, z, nur, nuz, N, pw, npw, tw, M, m0, nrhs, b1, b2); break;
    case 512: hipLaunchKernelGGL(k_rhs_plane<512>, dim3(grid), dim3(64), 0, st, rho, z, nur, nuz, N, pw, npw, tw, M, m0, nrhs, b1, b2); break;
    case 1024: hipLaunchKernelGGL(k_rhs_plane<1024>, dim3(grid), dim3(64), 0, st, rho, z, nur, nuz, N, pw, npw, tw, M, m0, nrhs, b1, b2); break;
    case 2048: hipLaunchKernelGGL(k_rhs_plane<2048>, dim3(grid), dim3(64), 0, st, rho, z, nur, nuz, N, pw, npw, tw, M, m0, nrhs, b1, b2); break;
    default: break;
  }
}

void launch_near(const NearJob* jobs, int njobs, const double* coef, const zd* raw, int M, int m0,
                 zd* A, long n2, long mstride, hipStream_t st) {
  if (njobs <= 0) return;
  OutSpec o{A, n2, mstride, nullptr, nullptr, M, m0};
  hipLaunchKernelGGL(k_near, dim3(njobs), dim3(256), 0, st, jobs, njobs, coef, raw, M, o);
}

void launch_field_pairs(const NodesDev& nd, const double* pts, int np, PairGeom* out, hipStream_t st) {
  const long tot = (long)np * nd.N;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_field_pairs, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, nd, pts, np, out);
}

void launch_field_near(const NearJob* jobs, int njobs, const double* coef, const zd* raw_aux, int N,
                       int M, zd* raw, hipStream_t st) {
  if (njobs <= 0) return;
  hipLaunchKernelGGL(k_field_near, dim3(njobs), dim3(256), 0, st, jobs, njobs, coef, raw_aux, N, M, raw);
}

}  // namespace pmlbie
