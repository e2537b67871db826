// One-wavefront FFT of length L = 64 R (R = 8, 16 or 32) with the data held in
// registers: an R-point DFT per lane, then the 64-point DFTs across lanes as
// two radix-8 passes, with two transposes through LDS (rows padded to 65
// entries so that eight consecutive lanes touch distinct banks).
//
//   input:  lane b, slot a holds x[b + 64 a], a < R
//   output: lane b, slot 8 r + c2 holds X[b + 64 r + 8 R c2], r < R / 8, c2 < 8
//   X[k] = sum_n x[n] e^{-2 pi i n k / L}
//
// For R = 8 the output slot c holds X[b + 64 c], the same layout as the input.
// The azimuthal kernels are even in the angle, so the forward transform also
// serves as the inverse one on their mode sequences.
#pragma once
#include "cplx.h"

namespace pmlbie {

// a * (-i)
__device__ __forceinline__ zd mul_mi(zd a) { return zd{a.im, -a.re}; }

// In-place forward 8-point DFT, natural order in and out.
__device__ __forceinline__ void dft8(zd* u) {
  const double h = 0.70710678118654752440;
  const zd a0 = u[0] + u[4], a1 = u[0] - u[4], a2 = u[2] + u[6], a3 = u[2] - u[6];
  const zd a4 = u[1] + u[5], a5 = u[1] - u[5], a6 = u[3] + u[7], a7 = u[3] - u[7];
  const zd e0 = a0 + a2, e2 = a0 - a2, e1 = a1 + mul_mi(a3), e3 = a1 - mul_mi(a3);
  const zd o0 = a4 + a6, o2 = a4 - a6, o1 = a5 + mul_mi(a7), o3 = a5 - mul_mi(a7);
  const zd t1 = h * zd{o1.re + o1.im, o1.im - o1.re};   // e^{-i pi/4} o1
  const zd t2 = mul_mi(o2);                              // e^{-i pi/2} o2
  const zd t3 = h * zd{o3.im - o3.re, -o3.re - o3.im};  // e^{-3i pi/4} o3
  u[0] = e0 + o0;
  u[4] = e0 - o0;
  u[1] = e1 + t1;
  u[5] = e1 - t1;
  u[2] = e2 + t2;
  u[6] = e2 - t2;
  u[3] = e3 + t3;
  u[7] = e3 - t3;
}

// In-place forward R-point DFT (R = 8; R = 16 and 32 as two half-length DFTs
// of the even and odd samples joined by the twiddles e^{-2 pi i k / R}).
template <int R>
__device__ __forceinline__ void dft_r(zd* v) {
  if constexpr (R == 8) {
    dft8(v);
  } else {
    static_assert(R == 16 || R == 32, "fft_wave supports L = 512, 1024 and 2048");
    constexpr int H = R / 2;
    zd e[H], o[H];
#pragma unroll
    for (int a = 0; a < H; ++a) {
      e[a] = v[2 * a];
      o[a] = v[2 * a + 1];
    }
    dft_r<H>(e);
    dft_r<H>(o);
    // cos and sin of pi k / 16, k = 0..16 (W_R^k = e^{-2 pi i k / R})
    constexpr double c16[17] = {1.0, 0.98078528040323044913, 0.92387953251128675613,
                                0.83146961230254523708, 0.70710678118654752440, 0.55557023301960222474,
                                0.38268343236508977173, 0.19509032201612826785, 0.0,
                                -0.19509032201612826785, -0.38268343236508977173, -0.55557023301960222474,
                                -0.70710678118654752440, -0.83146961230254523708, -0.92387953251128675613,
                                -0.98078528040323044913, -1.0};
    constexpr double s16[17] = {0.0, 0.19509032201612826785, 0.38268343236508977173,
                                0.55557023301960222474, 0.70710678118654752440, 0.83146961230254523708,
                                0.92387953251128675613, 0.98078528040323044913, 1.0,
                                0.98078528040323044913, 0.92387953251128675613, 0.83146961230254523708,
                                0.70710678118654752440, 0.55557023301960222474, 0.38268343236508977173,
                                0.19509032201612826785, 0.0};
    constexpr int st = 32 / R;  // angle 2 pi k / R = pi (st k) / 16
#pragma unroll
    for (int k = 0; k < H; ++k) {
      const zd t = o[k] * zd{c16[st * k], -s16[st * k]};
      v[k] = e[k] + t;
      v[k + H] = e[k] - t;
    }
  }
}

// Number of LDS entries one sequence needs.
template <int R>
constexpr int fft_wave_lds() {
  return R * 65;
}

// NS sequences at once (sharing the barriers); lds holds NS * R * 65 entries;
// tw[k] = e^{-2 pi i k / L}, k < L.
template <int R, int NS>
__device__ __forceinline__ void fft_wave(zd (&v)[NS][R], zd* lds, const zd* __restrict__ tw) {
  constexpr int ST = R * 65;
  const int b = threadIdx.x & 63;
  // pass 1: R-point DFT over a, twiddle e^{-2 pi i b k1 / L}
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    dft_r<R>(v[q]);
#pragma unroll
    for (int k1 = 0; k1 < R; ++k1) {
      const zd w = k1 == 0 ? zd{1.0, 0.0} : tw[b * k1];
      lds[q * ST + k1 * 65 + b] = k1 == 0 ? v[q][k1] : v[q][k1] * w;
    }
  }
  __syncthreads();
  // pass 2: job j = b + 64 r -> (k1, b2) = (j / 8, j % 8); 8-point DFT over
  // b1 of entry [k1][8 b1 + b2], twiddle e^{-2 pi i b2 c1 / 64}
#pragma unroll
  for (int q = 0; q < NS; ++q) {
#pragma unroll
    for (int r = 0; r < R / 8; ++r) {
      const int j = b + 64 * r, k1 = j >> 3, b2 = j & 7;
#pragma unroll
      for (int b1 = 0; b1 < 8; ++b1) v[q][8 * r + b1] = lds[q * ST + k1 * 65 + 8 * b1 + b2];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NS; ++q) {
#pragma unroll
    for (int r = 0; r < R / 8; ++r) {
      const int j = b + 64 * r, k1 = j >> 3, b2 = j & 7;
      zd* u = v[q] + 8 * r;
      dft8(u);
#pragma unroll
      for (int c1 = 0; c1 < 8; ++c1) {
        const zd val = c1 == 0 ? u[0] : u[c1] * tw[R * b2 * c1];
        lds[q * ST + k1 * 65 + c1 * 8 + b2] = val;
      }
    }
  }
  __syncthreads();
  // pass 3: job j = b + 64 r -> (k1, c1) = (j % R, j / R); 8-point DFT over b2
  // gives X[j + 8 R c2]
#pragma unroll
  for (int q = 0; q < NS; ++q) {
#pragma unroll
    for (int r = 0; r < R / 8; ++r) {
      const int j = b + 64 * r, k1 = j % R, c1 = j / R;
      zd* u = v[q] + 8 * r;
#pragma unroll
      for (int b2 = 0; b2 < 8; ++b2) u[b2] = lds[q * ST + k1 * 65 + c1 * 8 + b2];
      dft8(u);
    }
  }
  __syncthreads();
}

// Angle index of output slot s (see the layout above), lane b.
template <int R>
__device__ __forceinline__ int fft_wave_out_index(int b, int s) {
  return b + 64 * (s >> 3) + 8 * R * (s & 7);
}

}  // namespace pmlbie
