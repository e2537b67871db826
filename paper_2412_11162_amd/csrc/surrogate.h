// Learned surrogate for the modal kernels of well-separated pairs: a
// multilayer perceptron (MI355X BF16 MFMA, FP32 accumulation, FP32 master
// weights, Adam) that maps (rho, rho', dz, k, S) to the modes 0..64 of
//   S = G~,  P = (-(rho~ - rho~') + 2 rho~ sin^2(D/2)) f,  Q = (-dz) f,
//   f = e^{ikR} (ikR - 1) / (4 pi R^3),
// so that the conormal kernel is K = n'_rho P + n'_z Q (Sec. 3.1: the
// conormal numerator is linear in n'_c).  Targets are normalised by the
// phase e^{ik Re R0} and an amplitude scale (R0 = R at D = 0; sg_norm),
// which removes the oscillation of the kernels with k R0 and their PML decay.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <vector>
#include "modal.h"

namespace pmlbie {

constexpr int SG_IN = 7;          // raw inputs (rho, rho', dz, k, S, Im rho~, Im rho~')
constexpr int SG_NF = 9;          // features the input layer sees (padded to SG_D[0])
constexpr int SG_MODES = 65;      // modes 0..64
constexpr int SG_OUT = 6 * SG_MODES;  // 3 heads x (Re, Im) x modes = 390
constexpr int SG_NL = 5;          // layers (4 hidden of 256 + output)
constexpr int SG_D[SG_NL + 1] = {32, 256, 256, 256, 256, 400};  // padded widths

typedef uint16_t bf16;  // raw BF16 bits (round to nearest even on conversion)

// Offsets of layer l's weights (out x in, row-major) and biases in the flat
// FP32 parameter vector.
struct SgLayout {
  long w[SG_NL], b[SG_NL], total;
  SgLayout();
};

// One labelled sample: stretched coordinates of the pair and the wavenumber.
struct SgSample {
  double rt_re, rt_im, rs_re, rs_im, dz, k;
};

// Feature map of the raw inputs (rho, rho', dz, k, S, Im rho~, Im rho~') ->
// network input, O(1) ranges: 2 rho / rho_max - 1, 2 rho' / rho_max - 1, dz,
// (k - 17.5) / 12.5, (S - 2.5) / 1.5, Im rho~, Im rho~' (the PML stretching of
// the two points), k |R0| / 50 and k (|R_pi| - |R0|) / 100 (the phase scale
// and the phase swing of e^{ikR} over the angle; R0, R_pi = R at D = 0, pi).
struct SgFeat {
  double rho_max;  // a1 + T of the PML the network is trained for
};

// Normalisation of one sample: F_n = scale_h e0 (y_re + i y_im) with the
// phase e0 = e^{ik Re R0} and the amplitude a = max |e^{ikR}| over
// sin^2(D/2) in {0, 1/2, 1} (in the PML |e^{ikR}| = e^{-k Im R} varies with
// the angle):  scale_S = a / (4 pi |R0|),
// scale_K = a (|k| |R0| + 1)(|R0| + |rho~|) / (4 pi |R0|^3).
HD inline void sg_norm(zd rt, zd rs, double dz, double k, zd& e0, double& sS, double& sK) {
  const zd dr = rt - rs;
  const zd d2 = dr * dr + zd{dz * dz, 0.0};
  const zd c4 = 4.0 * (rt * rs);
  const zd R0 = csqrt_(d2);
  const double imin = fmin(R0.im, fmin(csqrt_(d2 + 0.5 * c4).im, csqrt_(d2 + c4).im));
  const double a = exp(-k * imin);
  const double r = cabs_(R0);
  e0 = zd{cos(k * R0.re), sin(k * R0.re)};
  sS = a / (4.0 * PMLBIE_PI * r);
  sK = a * (fabs(k) * r + 1.0) * (r + cabs_(rt)) / (4.0 * PMLBIE_PI * r * r * r);
}

// Device state of the network and its optimiser.
struct SgNet {
  float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // FP32 params, grads, Adam moments
  bf16* w16[SG_NL] = {};   // BF16 weights (out x in)
  bf16* wt16[SG_NL] = {};  // BF16 transposed weights (in x out)
  int steps = 0;           // Adam step counter
};

// Work buffers of a batch of up to cap rows.
struct SgWork {
  int cap = 0;
  bf16* h[SG_NL] = {};    // layer inputs (cap x SG_D[l]); h[0] = features
  float* z[SG_NL] = {};   // pre-activations (cap x SG_D[l+1])
  bf16* dz[SG_NL] = {};   // gradients w.r.t. pre-activations
  double* loss = nullptr; // loss accumulator
};

hipError_t sg_alloc(SgNet& net);
void sg_free(SgNet& net);
hipError_t sg_work_alloc(SgWork& w, int cap);
void sg_work_free(SgWork& w);
void sg_refresh_bf16(SgNet& net, hipStream_t st);
// Features of rows [0, n): x[row][0..4] FP64 on the device -> h[0] (BF16, padded).
void sg_features(const double* x, int n, const SgFeat& f, SgWork& w, hipStream_t st);
// Forward pass of n rows; keep pre-activations when training; Y = z[SG_NL-1].
void sg_forward(const SgNet& net, SgWork& w, int n, hipStream_t st);
// Loss (mean square over the 390 outputs) against targets T (n x SG_OUT,
// FP32) and gradients into net.g; returns nothing, loss in w.loss.
void sg_backward(SgNet& net, SgWork& w, int n, const float* T, hipStream_t st);
// Sum of squared errors of the n rows of the last forward pass into w.loss.
void sg_loss(SgWork& w, int n, const float* T, hipStream_t st);
void sg_adam(SgNet& net, double lr, hipStream_t st);
// Labels of n samples by the raw-kernel FFT of length L (512 or 1024).
void sg_label(const SgSample* s, long n, int L, const zd* tw, float* T, hipStream_t st);
// Raw inputs of the far pairs of a list, two rows per pair (k1, k2):
// x[row] = (rho, rho', dz, k, S, Im rho~, Im rho~').
void sg_pair_features(const PairGeom* g, long n, double k1, double k2, double S, double* x,
                      hipStream_t st);
// Acceptance of the network's modes for the far pairs [first, first + n) of a
// list, Y rows 2q (k1) and 2q + 1 (k2): the network's modal synthesis
// (modes 0..64) is compared with direct samples of S and K at SG_CHECK
// angles pi (a + u) / SG_CHECK, a < SG_CHECK, with an offset u in [0, 1) drawn
// per pair (splitmix64 of its destination), so that no fixed pattern of mode
// errors can pass unseen for all pairs; the samples hold every mode, so the
// check also bounds the modes beyond 64 the synthesis leaves out.  When
// M > 64 a pair is only offered if its modes beyond 64 are below e^{-c_far}
// by the decay bound of the classification ((65 - bw) delta >= c_far); its
// modes 65..M are then zero.  Accepted pairs (4 pi W_l |error| <= tol over
// the angles and both media) get modes 0..M in A; the others go to the
// fallback list.
constexpr int SG_CHECK = 8;
void sg_accept(const PairGeom* g, const int2* dest, long n, const float* Y, int M, int m0, zd k1, zd k2,
               double tol, zd* A, long n2, long mstride, const double* W, WorkList fallback,
               unsigned* accepted, const ClassParams& cp, hipStream_t st);
// Relative RMS error per mode of the network over n samples (features x,
// targets T): err2[m] += sum over the 3 heads of |Y - T|^2 at mode m,
// ref2[m] += |T|^2 (device accumulators of 65 doubles each).
void sg_mode_errors(const float* Y, const float* T, int n, double* err2, double* ref2, hipStream_t st);

}  // namespace pmlbie
