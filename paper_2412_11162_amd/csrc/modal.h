// Modal-kernel generation: data structures shared by the host orchestration
// and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <algorithm>
#include "modal_math.h"

namespace pmlbie {

// CLASS_FAR_BIG: a far pair whose aliasing bound holds on the full angle grid
// but not on the shorter grid the main pass runs on (see ClassParams.nt_small).
// CLASS_SPLIT_BIG: a split pair whose smooth parts need the full grid (its
// |rho~| exceeds ClassParams.split_rho_small).
enum { CLASS_FAR = 0, CLASS_SPLIT = 1, CLASS_DIRECT = 2, CLASS_FAR_BIG = 3, CLASS_SPLIT_BIG = 4 };

// Node tables of the Nystrom discretisation, structure of arrays on the device.
struct NodesDev {
  int N;
  const double *rho, *I, *z, *W;
  const double *nr_re, *nr_im, *nz_re, *nz_im;
  const int* panel;
};

// Thresholds of the pair classification.
struct ClassParams {
  int M;          // highest mode kept
  int nt_far;     // FFT length of the raw-kernel path
  double bw;      // oscillation bandwidth factor: B = bw |k| sqrt|rho~ rho~'|
  double kmax;    // max |Re k| over the media
  double kmax_im; // max |Im k|
  double c_far;   // far if (nt_far - M - B) * delta >= c_far
  double g_split; // split if max |Im kR| <= g_split, else direct quadrature
  // > 0 and < nt_far: the main pass transforms far pairs on this shorter grid
  // when their aliasing bound holds there, and classes the other far pairs
  // CLASS_FAR_BIG (transformed on the full grid from a list)
  int nt_small = 0;
  // > 0: split pairs with max(|rho~_t|, |rho~_s|) above this are
  // CLASS_SPLIT_BIG; the others are resolved on the shorter grid nt_small
  // (their smooth parts' bandwidth 1.15 |k| |rho~| + 16 fits below it)
  double split_rho_small = 0.0;
};

// Device work list of pairs handed from the classifier to the split and
// direct kernels.
struct WorkList {
  PairGeom* geom;
  int2* dest;
  unsigned* count;
  unsigned cap;
};

// One plane-wave incidence (theta_inc = 0): k1, cos and sin of the polar
// angle, the transmitted wavenumber k* and the flat-interface reflection
// coefficient Rc, and the right-hand-side slot.
struct PlaneWave {
  double k1, c, s;
  zd kst, R;
  int rhs;
};

// One near-panel product-integration job: target node, source panel, and its
// auxiliary points q0..q1-1.
struct NearJob {
  int target, panel, q0, q1;
};

// The main grid over the unordered node pairs off the near panels: far pairs
// are transformed in place in both orderings, split and direct pairs appended
// to their lists in both orderings.  The pass runs on the grid of
// cp.nt_small when it is set (tw its twiddles), on cp.nt_far otherwise; far
// pairs that need the full grid go to far_big once per unordered pair (i, l),
// i < l (launch_list_far_sym).
void launch_grid_far(const NodesDev& nd, const ClassParams& cp, zd k1, zd k2,
                     const zd* tw, zd* A, long mstride, int m0, const double* W, WorkList split,
                     WorkList direct, WorkList far_big, WorkList split_big, hipStream_t st);
// Classification only (surrogate path): far / split / direct lists with
// destinations (i, l).
void launch_grid_classify(const NodesDev& nd, const ClassParams& cp, WorkList far, WorkList split,
                          WorkList direct, WorkList split_big, hipStream_t st);
// Far pairs of an explicit list; with cp, the pairs the classification marks
// coarse are sampled on the half-length grid, as in the main grid.
// The long-grid far pairs the main pass lists once per unordered pair (i, l):
// both orderings into A (modes m0..M).
void launch_list_far_sym(int nt, const PairGeom* geom, const int2* dest, long count, const NodesDev& nd, int M,
                         int m0, zd k1, zd k2, const zd* tw, zd* A, long n2, long mstride, const double* W,
                         const ClassParams& cp, hipStream_t st);
void launch_list_far(int nt, const PairGeom* geom, const int2* dest, long first, long count, int M,
                     int m0, zd k1, zd k2, const zd* tw, zd* A, long n2, long mstride,
                     const double* W, zd* raw, const ClassParams* cp, hipStream_t st);
void launch_classify_list(const PairGeom* geom, long count, const ClassParams& cp, WorkList far,
                          WorkList split, WorkList direct, WorkList split_big, hipStream_t st);
// Singular-part modes of split pairs: qtab ([MQ + 1][count], mode-major)
// and coef (4 per pair) are work space; zhat, phat receive [count][MQ + 1]
// (pair-major), read by launch_split.
void launch_split_singular(const PairGeom* geom, long first, long count, int MQ, zd* qtab, zd* coef,
                           zd* zhat, zd* phat, hipStream_t st);
// chL > 0: the smooth parts with the substitution of Sec. 4.3 of order chL.
void launch_split(int nt, const PairGeom* geom, const int2* dest, long first, long count, int M,
                  int m0, int MQ, zd k1, zd k2, const zd* tw, const zd* zhat, const zd* phat,
                  zd* A, long n2, long mstride, const double* W, zd* raw, hipStream_t st, int chL = 0);
// Graded direct rule, modes m0..M; with raw output (A null) the modes from m0
// rounded down to 16 up to M are written, so a caller reading every mode
// passes m0 = 0.
void launch_direct(const PairGeom* geom, const int2* dest, long first, long count, int M, int m0,
                   zd k1, zd k2, const double* glx, const double* glw, zd* A, long n2,
                   long mstride, const double* W, zd* raw, double omega_piece, hipStream_t st);
// Plane-wave right-hand sides of modes m0..M (b[(n - m0) * nrhs + r][node]).
void launch_rhs_plane(int nt, const double* rho, const double* z, const double* nur,
                      const double* nuz, int N, const PlaneWave* pw, int npw, const zd* tw, int M,
                      int m0, int nrhs, zd* b1, zd* b2, hipStream_t st);
void launch_near(const NearJob* jobs, int njobs, const double* coef, const zd* raw, int M, int m0,
                 zd* A, long n2, long mstride, hipStream_t st);
// Far pairs of a field chunk (raw rows q = p * N + l) for the medium of each
// point only: raw sequences (0, 1) where medium[p] == 1, (2, 3) where it is 2.
void launch_list_far_one(int nt, const PairGeom* geom, const int2* dest, long first, long count, int M,
                         zd k1, zd k2, const zd* tw, zd* raw, const int* medium, int N, hipStream_t st);
// Pair geometry of np field points pts[2 * p] = (rho, z) (physical region)
// against every node, out[p * N + l].
void launch_field_pairs(const NodesDev& nd, const double* pts, int np, PairGeom* out, hipStream_t st);
// Near-curve field points: job targets are chunk-local point indices,
// raw[(point * N + node)][4][M + 1] receives the panel's 16 corrected entries.
void launch_field_near(const NearJob* jobs, int njobs, const double* coef, const zd* raw_aux, int N,
                       int M, zd* raw, hipStream_t st);

}  // namespace pmlbie
