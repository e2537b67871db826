// Learned surrogate of the far-pair modal kernels: BF16 MFMA multilayer
// perceptron (forward, backward, Adam), its training labels by the raw-kernel
// FFT, and the a-posteriori acceptance of its modes in the operator build.
#include <cmath>
#include "fft_wave.h"
#include "modal_out.h"
#include "surrogate.h"

namespace pmlbie {

typedef __bf16 b8v __attribute__((ext_vector_type(8)));
typedef short s8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));

SgLayout::SgLayout() {
  long o = 0;
  for (int l = 0; l < SG_NL; ++l) {
    w[l] = o;
    o += (long)SG_D[l + 1] * SG_D[l];
  }
  for (int l = 0; l < SG_NL; ++l) {
    b[l] = o;
    o += SG_D[l + 1];
  }
  total = o;
}

__device__ __forceinline__ bf16 f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16 b) { return __uint_as_float((uint32_t)b << 16); }

// GELU with the exact error function and its derivative.
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// ---------------------------------------------------------------------------
// C(m, n) = sum_k A(m, k) B(k, n), BF16 operands with arbitrary strides,
// FP32 accumulation on MFMA 16x16x32; workgroup tile 64 x 64, four waves of
// 32 x 32, K chunks of 32 staged in LDS as [m][k] and [n][k].
enum { EPI_HID = 0, EPI_OUT = 1, EPI_DH = 2, EPI_DW = 3 };

struct GemmArgs {
  const bf16* A;
  long sam, sak;
  const bf16* B;
  long sbk, sbn;
  int M, N, K;
  const float* bias;
  float* zout;
  long ldz;
  bf16* hout;
  long ldh;
  const float* zprev;
  long ldzp;
};

template <int EPI>
__global__ __launch_bounds__(256) void k_sg_gemm(GemmArgs g) {
  __shared__ bf16 As[64][40], Bs[64][40];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wr = (wid & 1) * 32, wc = (wid >> 1) * 32;
  f4v acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = f4v{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < g.K; k0 += 32) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int e = tid + 256 * t;
      const int r = e >> 5, k = e & 31;
      const int gm = m0 + r, gn = n0 + r, gk = k0 + k;
      As[r][k] = (gm < g.M && gk < g.K) ? g.A[(long)gm * g.sam + (long)gk * g.sak] : (bf16)0;
      Bs[r][k] = (gn < g.N && gk < g.K) ? g.B[(long)gk * g.sbk + (long)gn * g.sbn] : (bf16)0;
    }
    __syncthreads();
    b8v a[2], b[2];
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const s8v va = *reinterpret_cast<const s8v*>(&As[wr + 16 * x + (lane & 15)][8 * (lane >> 4)]);
      const s8v vb = *reinterpret_cast<const s8v*>(&Bs[wc + 16 * x + (lane & 15)][8 * (lane >> 4)]);
      a[x] = __builtin_bit_cast(b8v, va);
      b[x] = __builtin_bit_cast(b8v, vb);
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[x], b[y], acc[x][y], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int m = m0 + wr + 16 * x + 4 * (lane >> 4) + j;
        const int n = n0 + wc + 16 * y + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        const float c = acc[x][y][j];
        if (EPI == EPI_HID) {
          const float z = c + g.bias[n];
          if (g.zout) g.zout[(long)m * g.ldz + n] = z;
          g.hout[(long)m * g.ldh + n] = f2bf(gelu(z));
        } else if (EPI == EPI_OUT) {
          g.zout[(long)m * g.ldz + n] = c + g.bias[n];
        } else if (EPI == EPI_DH) {
          g.hout[(long)m * g.ldh + n] = f2bf(c * gelu_d(g.zprev[(long)m * g.ldzp + n]));
        } else {
          g.zout[(long)m * g.ldz + n] = c;
        }
      }
}

template <int EPI>
static void gemm(const GemmArgs& g, hipStream_t st) {
  dim3 grid((g.N + 63) / 64, (g.M + 63) / 64);
  hipLaunchKernelGGL(k_sg_gemm<EPI>, grid, dim3(256), 0, st, g);
}

// ---------------------------------------------------------------------------
__global__ void k_sg_refresh(const float* __restrict__ p, long wo, int dout, int din, bf16* w16,
                             bf16* wt16) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)dout * din) return;
  const int o = (int)(e / din), i = (int)(e % din);
  const bf16 v = f2bf(p[wo + e]);
  w16[e] = v;
  wt16[(long)i * dout + o] = v;
}

__global__ void k_sg_features(const double* __restrict__ x, int n, double rho_max, bf16* h0) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)n * SG_D[0]) return;
  const int r = (int)(e / SG_D[0]), c = (int)(e % SG_D[0]);
  const double* xr = x + (long)r * SG_IN;
  double f = 0.0;
  if (c == 0) f = 2.0 * xr[0] / rho_max - 1.0;
  else if (c == 1) f = 2.0 * xr[1] / rho_max - 1.0;
  else if (c == 2) f = xr[2];
  else if (c == 3) f = (xr[3] - 17.5) / 12.5;
  else if (c == 4) f = (xr[4] - 2.5) / 1.5;
  else if (c == 5) f = xr[5];
  else if (c == 6) f = xr[6];
  else if (c == 7 || c == 8) {
    const zd rt{xr[0], xr[5]}, rs{xr[1], xr[6]};
    const zd dr = rt - rs;
    const zd d2 = dr * dr + zd{xr[2] * xr[2], 0.0};
    const double r0 = cabs_(csqrt_(d2));
    if (c == 7) f = xr[3] * r0 / 50.0;
    else f = xr[3] * (cabs_(csqrt_(d2 + 4.0 * (rt * rs))) - r0) / 100.0;
  }
  h0[e] = f2bf((float)f);
}

// dY = 2 (Y - T) / (n * SG_OUT) on the 390 outputs (0 on the padding), and the
// sum of squares into *loss.
__global__ __launch_bounds__(256) void k_sg_mse(const float* __restrict__ Y, const float* __restrict__ T,
                                                int n, bf16* dY, double* loss) {
  constexpr int D = SG_D[SG_NL];
  const long tot = (long)n * D;
  double s = 0.0;
  const float sc = 2.0f / ((float)n * SG_OUT);
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    const int r = (int)(e / D), c = (int)(e % D);
    float d = 0.f;
    if (c < SG_OUT) d = Y[e] - T[(long)r * SG_OUT + c];
    s += (double)d * d;
    dY[e] = f2bf(sc * d);
  }
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(loss, red[0]);
}

// Bias gradients: db[c] = sum_r dz[r][c].
__global__ __launch_bounds__(256) void k_sg_colsum(const bf16* __restrict__ dz, int n, int d, float* db) {
  const int c = blockIdx.x;
  float s = 0.f;
  for (int r = threadIdx.x; r < n; r += 256) s += bf2f(dz[(long)r * d + c]);
  __shared__ float red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[c] = red[0];
}

__global__ void k_sg_adam(float* p, const float* g, float* m, float* v, long n, float lr, float b1,
                          float b2, float c1, float c2, float eps) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.f - b1) * gi;
  const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  p[e] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
// Labels: one wavefront per sample.  Samples of S, P, Q on the half circle
// D_j = 2 pi j / L are staged in LDS, extended evenly and transformed by
// fft_wave; modes 0..64 are normalised (sg_norm) into T[sample][h * 130 + 2n + c].
template <int R>
__global__ __launch_bounds__(64) void k_sg_label(const SgSample* __restrict__ s, long n,
                                                 const zd* __restrict__ tw, float* __restrict__ T) {
  constexpr int L = 64 * R, H = L / 2 + 1;
  __shared__ zd st[3 * H];
  __shared__ zd E[2 * fft_wave_lds<R>()];
  const int b = threadIdx.x & 63;
  const double scale = 2.0 * PMLBIE_PI / L;
  for (long q = blockIdx.x; q < n; q += gridDim.x) {
    const SgSample S = s[q];
    const zd rt{S.rt_re, S.rt_im}, rs{S.rs_re, S.rs_im};
    const zd dr = rt - rs;
    const zd d2 = dr * dr + zd{S.dz * S.dz, 0.0};
    const zd c4 = 4.0 * (rt * rs);
    const zd ik{0.0, S.k};
    for (int j = b; j <= L / 2; j += 64) {
      const double sh = sin(PMLBIE_PI * j / L);
      const double s2 = sh * sh;
      const zd R2 = d2 + s2 * c4;
      const zd Rd = csqrt_(R2);
      const zd ikR = ik * Rd;
      const zd e = cexp_(ikR) * (inv(Rd) * (0.25 / PMLBIE_PI));
      const zd f = e * (ikR - 1.0) * inv(R2);
      st[j] = e;
      st[H + j] = (-1.0 * dr + (2.0 * s2) * rt) * f;
      st[2 * H + j] = (-S.dz) * f;
    }
    __syncthreads();
    zd e0;
    double sS, sK;
    sg_norm(rt, rs, S.dz, S.k, e0, sS, sK);
    const zd ie0 = inv(e0);
#pragma unroll 1
    for (int h = 0; h < 3; ++h) {
      zd x[1][R];
#pragma unroll
      for (int a = 0; a < R; ++a) {
        const int j = b + 64 * a;
        x[0][a] = st[h * H + (j <= L / 2 ? j : L - j)];
      }
      fft_wave<R, 1>(x, E, tw);
      const double nrm = scale / (h == 0 ? sS : sK);
#pragma unroll
      for (int sl = 0; sl < R; ++sl) {
        const int m = fft_wave_out_index<R>(b, sl);
        if (m < SG_MODES) {
          const zd y = nrm * (x[0][sl] * ie0);
          T[q * SG_OUT + h * 2 * SG_MODES + 2 * m] = (float)y.re;
          T[q * SG_OUT + h * 2 * SG_MODES + 2 * m + 1] = (float)y.im;
        }
      }
    }
    __syncthreads();
  }
}

__global__ void k_sg_pair_features(const PairGeom* __restrict__ g, long n, double k1, double k2,
                                   double S, double* __restrict__ x) {
  const long r = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= 2 * n) return;
  const PairGeom p = g[r >> 1];
  double* o = x + r * SG_IN;
  o[0] = p.rt.re;
  o[1] = p.rs.re;
  o[2] = p.dz.re;
  o[3] = (r & 1) ? k2 : k1;
  o[4] = S;
  o[5] = p.rt.im;
  o[6] = p.rs.im;
}

// Uniform draw in [0, 1) from a 64-bit key: the splitmix64 output function
// (Steele, Lea and Flood 2014) applied to key + its increment.
__device__ __forceinline__ double sg_hash01(unsigned long long key) {
  unsigned long long z = key + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

// Acceptance: one wavefront per pair; lane n < 64 holds mode n, lane 0 also
// mode 64.  The modal synthesis (1/2pi)(F_0 + 2 sum_n F_n cos nD) of S and K
// at SG_CHECK angles with a per-pair offset is compared with direct samples
// of the kernels (see sg_accept).
__global__ __launch_bounds__(64) void k_sg_accept(const PairGeom* __restrict__ geom,
                                                  const int2* __restrict__ dest, long n,
                                                  const float* __restrict__ Y, int M, zd k1, zd k2,
                                                  double tol, OutSpec o, WorkList fb,
                                                  unsigned* accepted, ClassParams cp) {
  constexpr int DY = SG_D[SG_NL];
  const int lane = threadIdx.x & 63;
  unsigned acc_count = 0;
  for (long q = blockIdx.x; q < n; q += gridDim.x) {
    const PairGeom g = geom[q];
    const int2 dst = dest[q];
    const PairInv v = pair_invariants(g);
    bool ok = true;
    if (M >= SG_MODES) {
      // modes beyond 64 must be negligible: the decay bound of the far class
      double delta, re0;
      singularity(v, delta, re0);
      const double bw = cp.bw * cp.kmax * sqrt(cabs_(g.rt * g.rs));
      ok = ((double)SG_MODES - bw) * delta >= cp.c_far;
    }
    zd Fs[2][2], Fk[2][2];  // [wavenumber][mode lane, mode 64]
    const double u = sg_hash01(((unsigned long long)(unsigned)dst.x << 32) | (unsigned)dst.y);
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      const zd k = w == 0 ? k1 : k2;
      const float* y = Y + (2 * q + w) * DY;
      zd e0;
      double sS, sK;
      sg_norm(g.rt, g.rs, g.dz.re, k.re, e0, sS, sK);
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int m = b == 0 ? lane : 64;
        const zd ys{y[2 * m], y[2 * m + 1]};
        const zd yp{y[2 * SG_MODES + 2 * m], y[2 * SG_MODES + 2 * m + 1]};
        const zd yq{y[4 * SG_MODES + 2 * m], y[4 * SG_MODES + 2 * m + 1]};
        Fs[w][b] = (sS * e0) * ys;
        Fk[w][b] = (sK * e0) * (g.nr * yp + g.nz * yq);
      }
      if (!ok) continue;
      double err = 0.0;
#pragma unroll 1
      for (int a = 0; a < SG_CHECK; ++a) {
        const double D = (a + u) * (PMLBIE_PI / SG_CHECK);
        const double c0 = lane == 0 ? 1.0 : 2.0 * cos(lane * D);
        zd ps = c0 * Fs[w][0], pk = c0 * Fk[w][0];
        if (lane == 0) {
          const double c64 = 2.0 * cos(64.0 * D);
          ps = ps + c64 * Fs[w][1];
          pk = pk + c64 * Fk[w][1];
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
          ps.re += __shfl_xor(ps.re, off);
          ps.im += __shfl_xor(ps.im, off);
          pk.re += __shfl_xor(pk.re, off);
          pk.im += __shfl_xor(pk.im, off);
        }
        const double sh = sin(0.5 * D);
        zd Sd, Kd;
        kernel_sample(v, sh * sh, k, Sd, Kd);
        const double inv2pi = 0.5 / PMLBIE_PI;
        err = fmax(err, fmax(cabs_(inv2pi * ps - Sd), cabs_(inv2pi * pk - Kd)));
      }
      if (4.0 * PMLBIE_PI * o.W[dst.y] * err > tol) ok = false;
    }
    if (ok) {
      if (lane <= M) emit(o, dst, lane, Fs[0][0], Fk[0][0], Fs[1][0], Fk[1][0]);
      if (lane == 0 && M >= 64) emit(o, dst, 64, Fs[0][1], Fk[0][1], Fs[1][1], Fk[1][1]);
      const zd z0{0.0, 0.0};
      for (int m = SG_MODES + lane; m <= M; m += 64) emit(o, dst, m, z0, z0, z0, z0);
      ++acc_count;
    } else if (lane == 0) {
      const unsigned slot = atomicAdd(fb.count, 1u);
      if (slot < fb.cap) {
        fb.geom[slot] = g;
        fb.dest[slot] = dst;
      }
    }
  }
  if (lane == 0 && acc_count) atomicAdd(accepted, acc_count);
}

// Per-mode error sums of the network outputs Y (rows of SG_D[SG_NL]) against
// targets T (rows of SG_OUT): one thread per (row, mode), block sums in LDS.
__global__ __launch_bounds__(256) void k_sg_mode_err(const float* __restrict__ Y, const float* __restrict__ T,
                                                     int n, double* err2, double* ref2) {
  __shared__ double se[SG_MODES], sr[SG_MODES];
  for (int m = threadIdx.x; m < SG_MODES; m += blockDim.x) se[m] = sr[m] = 0.0;
  __syncthreads();
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (long)n * SG_MODES) {
    const long r = e / SG_MODES;
    const int m = (int)(e % SG_MODES);
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int h = 0; h < 3; ++h)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int j = h * 2 * SG_MODES + 2 * m + c;
        const double t = T[r * SG_OUT + j], d = (double)Y[r * SG_D[SG_NL] + j] - t;
        a += d * d;
        b += t * t;
      }
    atomicAdd(&se[m], a);
    atomicAdd(&sr[m], b);
  }
  __syncthreads();
  for (int m = threadIdx.x; m < SG_MODES; m += blockDim.x) {
    atomicAdd(err2 + m, se[m]);
    atomicAdd(ref2 + m, sr[m]);
  }
}

// ---------------------------------------------------------------------------
// Host side.
hipError_t sg_alloc(SgNet& net) {
  SgLayout L;
  hipError_t e = hipSuccess;
  for (float** p : {&net.p, &net.g, &net.m, &net.v}) {
    if (e == hipSuccess) e = hipMalloc(p, L.total * sizeof(float));
    if (e == hipSuccess) e = hipMemset(*p, 0, L.total * sizeof(float));
  }
  for (int l = 0; l < SG_NL && e == hipSuccess; ++l) {
    const size_t n = (size_t)SG_D[l + 1] * SG_D[l];
    e = hipMalloc(&net.w16[l], n * sizeof(bf16));
    if (e == hipSuccess) e = hipMalloc(&net.wt16[l], n * sizeof(bf16));
  }
  net.steps = 0;
  return e;
}

void sg_free(SgNet& net) {
  for (float* p : {net.p, net.g, net.m, net.v})
    if (p) hipFree(p);
  net.p = net.g = net.m = net.v = nullptr;
  for (int l = 0; l < SG_NL; ++l) {
    if (net.w16[l]) hipFree(net.w16[l]);
    if (net.wt16[l]) hipFree(net.wt16[l]);
    net.w16[l] = net.wt16[l] = nullptr;
  }
}

hipError_t sg_work_alloc(SgWork& w, int cap) {
  if (w.cap >= cap) return hipSuccess;
  sg_work_free(w);
  hipError_t e = hipSuccess;
  for (int l = 0; l < SG_NL && e == hipSuccess; ++l) {
    e = hipMalloc(&w.h[l], (size_t)cap * SG_D[l] * sizeof(bf16));
    if (e == hipSuccess) e = hipMalloc(&w.z[l], (size_t)cap * SG_D[l + 1] * sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&w.dz[l], (size_t)cap * SG_D[l + 1] * sizeof(bf16));
  }
  if (e == hipSuccess) e = hipMalloc(&w.loss, sizeof(double));
  if (e != hipSuccess) {
    sg_work_free(w);
    return e;
  }
  w.cap = cap;
  return e;
}

void sg_work_free(SgWork& w) {
  for (int l = 0; l < SG_NL; ++l) {
    if (w.h[l]) hipFree(w.h[l]);
    if (w.z[l]) hipFree(w.z[l]);
    if (w.dz[l]) hipFree(w.dz[l]);
    w.h[l] = nullptr;
    w.z[l] = nullptr;
    w.dz[l] = nullptr;
  }
  if (w.loss) hipFree(w.loss);
  w.loss = nullptr;
  w.cap = 0;
}

void sg_refresh_bf16(SgNet& net, hipStream_t st) {
  SgLayout L;
  for (int l = 0; l < SG_NL; ++l) {
    const long e = (long)SG_D[l + 1] * SG_D[l];
    hipLaunchKernelGGL(k_sg_refresh, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, st, net.p, L.w[l],
                       SG_D[l + 1], SG_D[l], net.w16[l], net.wt16[l]);
  }
}

void sg_features(const double* x, int n, const SgFeat& f, SgWork& w, hipStream_t st) {
  const long e = (long)n * SG_D[0];
  hipLaunchKernelGGL(k_sg_features, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, st, x, n, f.rho_max,
                     w.h[0]);
}

void sg_forward(const SgNet& net, SgWork& w, int n, hipStream_t st) {
  SgLayout L;
  for (int l = 0; l < SG_NL; ++l) {
    GemmArgs g{};
    g.A = w.h[l];
    g.sam = SG_D[l];
    g.sak = 1;
    g.B = net.w16[l];
    g.sbk = 1;
    g.sbn = SG_D[l];
    g.M = n;
    g.N = SG_D[l + 1];
    g.K = SG_D[l];
    g.bias = net.p + L.b[l];
    g.zout = w.z[l];
    g.ldz = SG_D[l + 1];
    if (l + 1 < SG_NL) {
      g.hout = w.h[l + 1];
      g.ldh = SG_D[l + 1];
      gemm<EPI_HID>(g, st);
    } else {
      gemm<EPI_OUT>(g, st);
    }
  }
}

void sg_backward(SgNet& net, SgWork& w, int n, const float* T, hipStream_t st) {
  SgLayout L;
  hipMemsetAsync(w.loss, 0, sizeof(double), st);
  const long tot = (long)n * SG_D[SG_NL];
  hipLaunchKernelGGL(k_sg_mse, dim3((unsigned)std::min<long>((tot + 255) / 256, 1024)), dim3(256), 0, st,
                     w.z[SG_NL - 1], T, n, w.dz[SG_NL - 1], w.loss);
  for (int l = SG_NL - 1; l >= 0; --l) {
    const int dout = SG_D[l + 1], din = SG_D[l];
    GemmArgs g{};  // dW_l = dz_l^T h_l
    g.A = w.dz[l];
    g.sam = 1;
    g.sak = dout;
    g.B = w.h[l];
    g.sbk = din;
    g.sbn = 1;
    g.M = dout;
    g.N = din;
    g.K = n;
    g.zout = net.g + L.w[l];
    g.ldz = din;
    gemm<EPI_DW>(g, st);
    hipLaunchKernelGGL(k_sg_colsum, dim3(dout), dim3(256), 0, st, w.dz[l], n, dout, net.g + L.b[l]);
    if (l > 0) {
      GemmArgs d{};  // dz_{l-1} = (dz_l W_l) * gelu'(z_{l-1})
      d.A = w.dz[l];
      d.sam = dout;
      d.sak = 1;
      d.B = net.wt16[l];
      d.sbk = 1;
      d.sbn = dout;
      d.M = n;
      d.N = din;
      d.K = dout;
      d.hout = w.dz[l - 1];
      d.ldh = din;
      d.zprev = w.z[l - 1];
      d.ldzp = din;
      gemm<EPI_DH>(d, st);
    }
  }
}

void sg_loss(SgWork& w, int n, const float* T, hipStream_t st) {
  hipMemsetAsync(w.loss, 0, sizeof(double), st);
  const long tot = (long)n * SG_D[SG_NL];
  hipLaunchKernelGGL(k_sg_mse, dim3((unsigned)std::min<long>((tot + 255) / 256, 1024)), dim3(256), 0, st,
                     w.z[SG_NL - 1], T, n, w.dz[SG_NL - 1], w.loss);
}

void sg_adam(SgNet& net, double lr, hipStream_t st) {
  SgLayout L;
  net.steps += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)net.steps), c2 = 1.f - powf(b2, (float)net.steps);
  hipLaunchKernelGGL(k_sg_adam, dim3((unsigned)((L.total + 255) / 256)), dim3(256), 0, st, net.p, net.g, net.m,
                     net.v, L.total, (float)lr, b1, b2, c1, c2, 1e-8f);
  sg_refresh_bf16(net, st);
}

void sg_label(const SgSample* s, long n, int L, const zd* tw, float* T, hipStream_t st) {
  if (n <= 0) return;
  const int grid = (int)std::min<long>(n, 256L * 64);
  if (L == 512)
    hipLaunchKernelGGL(k_sg_label<8>, dim3(grid), dim3(64), 0, st, s, n, tw, T);
  else
    hipLaunchKernelGGL(k_sg_label<16>, dim3(grid), dim3(64), 0, st, s, n, tw, T);
}

void sg_pair_features(const PairGeom* g, long n, double k1, double k2, double S, double* x,
                      hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_sg_pair_features, dim3((unsigned)((2 * n + 255) / 256)), dim3(256), 0, st, g, n, k1,
                     k2, S, x);
}

void sg_accept(const PairGeom* g, const int2* dest, long n, const float* Y, int M, int m0, zd k1, zd k2,
               double tol, zd* A, long n2, long mstride, const double* W, WorkList fallback,
               unsigned* accepted, const ClassParams& cp, hipStream_t st) {
  if (n <= 0) return;
  OutSpec o{A, n2, mstride, W, nullptr, M, m0};
  const int grid = (int)std::min<long>(n, 256L * 32);
  hipLaunchKernelGGL(k_sg_accept, dim3(grid), dim3(64), 0, st, g, dest, n, Y, M, k1, k2, tol, o, fallback,
                     accepted, cp);
}

void sg_mode_errors(const float* Y, const float* T, int n, double* err2, double* ref2, hipStream_t st) {
  const long tot = (long)n * SG_MODES;
  if (tot <= 0) return;
  hipLaunchKernelGGL(k_sg_mode_err, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Y, T, n, err2, ref2);
}

}  // namespace pmlbie
