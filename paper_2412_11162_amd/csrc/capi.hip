// C ABI of the solver: context, argument checks, orchestration of the HIP
// kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <future>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/pmlbie.h"
#include "host_geom.h"
#include "lu.h"
#include "modal.h"
#include "solve.h"
#include "surrogate.h"

using namespace pmlbie;

namespace {

struct DevErr : std::runtime_error {
  int code;
  DevErr(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                       \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess)                                                               \
      throw DevErr(e_ == hipErrorOutOfMemory ? PMLBIE_ENOMEM : PMLBIE_EDEVICE,          \
                   std::string(#x) + ": " + hipGetErrorString(e_));                    \
  } while (0)

template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  void alloc(size_t count) {
    if (count <= n && p) return;
    release();
    if (count == 0) return;
    HIPCHK(hipMalloc((void**)&p, count * sizeof(T)));
    n = count;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  ~DBuf() { release(); }
};

}  // namespace

struct pmlbie_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t up_stream = nullptr;  // uploads of the near-panel tables
  hipEvent_t up_done = nullptr;
  hipStream_t lu_stream = nullptr;  // the LU's look-ahead panels
  hipEvent_t lu_ev[2] = {nullptr, nullptr};
  // host near-panel tables of the last build (auxiliary pair geometry,
  // Lagrange-weighted coefficients, jobs), reused as workspace
  std::vector<PairGeom> h_ageom;
  std::vector<double> h_acoef;
  std::vector<NearJob> h_ajobs;
  std::string err;
  int stage = 0;  // 0 created, 1 geometry, 2 media, 3 built, 4 solved
  Geometry geo;
  zd k1{0, 0}, k2{0, 0};
  double a2 = 0, T2 = 0, S2 = 0;
  // build parameters
  int n_theta = 0, M = 0, m0 = 0, nt_int = 0, nt_far = 0, B = 0, MQ = 0, precision = 0, flags = 0;
  int N = 0;
  ClassParams cp{};
  long long cnt_far = 0, cnt_split = 0, cnt_direct = 0, cnt_aux = 0, cnt_far_big = 0;
  // device data
  DBuf<double> nodes;  // 10 N doubles: rho, I, z, W, nr_re, nr_im, nz_re, nz_im, nu_rho, nu_z
  DBuf<PlaneWave> dpw;
  DBuf<zd> tw_pw;
  DBuf<int> rmap;
  DBuf<int> dpanel;
  DBuf<zd> tw_far, tw_int, tw_small;
  int nt_small = 0;  // grid of the main far pass (<= nt_far)
  double split_rho_small = 0.0;  // split pairs up to this |rho~| use the nt_small grid (0: none)
  DBuf<double> glx, glw;
  DBuf<zd> A, Alow, Akeep;
  DBuf<zf> A32;               // complex64 factors (mixed precision)
  DBuf<zd> rbuf, xs;          // refinement: residual / correction, iterate
  DBuf<double> rsq, rnorm;
  DBuf<int> ipiv, info;
  DBuf<zd> luw;  // inverses of the LU diagonal blocks
  DBuf<int> lumap;  // row maps of an LU step's second block, then (mixed) of the first step
  DBuf<PairGeom> lgeom;
  DBuf<int2> ldest;
  DBuf<unsigned> lcount;
  DBuf<zd> zhat, phat, qtab, qcoef;
  DBuf<zd> raw;
  DBuf<PairGeom> xgeom;
  DBuf<double> coef;
  DBuf<NearJob> jobs;
  // solution of the last solve
  int nrhs = 0;
  DBuf<zd> b1, b2, x, u1, p1, u2, p2;
  double stage_ms[16] = {0};
  double counters[16] = {0};
  // refinement stopping rule of the mixed-precision solve
  double ref_tol = 1e-10;
  int ref_maxit = 30;
  // > 0: the pairs of the direct class go through the split with the
  // substitution of Sec. 4.3 of this order (pmlbie_set_ch1_substitution)
  int ch1_L = 0;
  // one-shot test hook: zero this column of this mode's matrix before the LU
  int zc_mode = -1, zc_col = -1;
  // learned surrogate of the far-pair modes
  SgNet sg;
  SgWork sgw;
  bool sg_ready = false;
  double sg_a1 = 0, sg_T = 0, sg_tol = 1e-10;
  int sg_p = 0;
  DBuf<double> sgx[2];     // features (rho, rho', dz, k, S) of the sample sets
  DBuf<float> sgT[2];      // their normalised modal targets
  long sgn[2] = {0, 0};
  DBuf<zd> sgtw;           // twiddles of the labelling FFT
  DBuf<double> sgfx;       // features of the far pairs of one chunk
  DBuf<unsigned> sgcnt;    // accepted pairs, fallback count
  DBuf<PairGeom> sgfb_geom;  // far pairs the network's modes were not accepted for
  DBuf<int2> sgfb_dest;
  ~pmlbie_ctx() {
    sg_free(sg);
    sg_work_free(sgw);
  }
};

namespace {

// Longest piece of the direct azimuthal rule: h = kOmegaPiece / om with
// om = m_max + |k| sqrt|rho~ rho~'| + 1, the fastest oscillation of
// cos(n D) e^{ikR}.  The 16-point Gauss-Legendre error on a piece scales as
// (om h)^32 h (16!)^4 / (33 (32!)^3) relative to the integrand: ~1e-11 in the
// worst case (om h = 24 with k -> 0, m_max = 128), ~1e-16 for the direct pairs
// of the workloads, which sit deep in the PML where |k| sqrt|rho~ rho~'| is
// 45 - 80.
const double kOmegaPiece = 24.0;

int fail(pmlbie_ctx* c, int code, const std::string& m) {
  if (c) c->err = m;
  return code;
}

template <typename F>
int guarded(pmlbie_ctx* c, F&& f) {
  if (!c) return PMLBIE_EINVAL;
  try {
    HIPCHK(hipSetDevice(c->device));
    return f();
  } catch (const DevErr& e) {
    return fail(c, e.code, e.what());
  } catch (const std::invalid_argument& e) {
    return fail(c, PMLBIE_EINVAL, e.what());
  } catch (const std::bad_alloc&) {
    return fail(c, PMLBIE_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(c, PMLBIE_EDEVICE, e.what());
  }
}

struct Timer {
  hipStream_t st;
  hipEvent_t a, b;
  explicit Timer(hipStream_t s) : st(s) {
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    HIPCHK(hipEventRecord(a, st));
  }
  double stop() {
    HIPCHK(hipEventRecord(b, st));
    HIPCHK(hipEventSynchronize(b));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, a, b));
    return ms;
  }
  ~Timer() {
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
  }
};

// Split-path work on a device list [first, first+count): phase 1 (singular
// modes) in chunks, phase 2 (smooth FFTs + convolution).
void run_split(pmlbie_ctx* c, const PairGeom* geom, const int2* dest, long count, zd* A, long n2,
               long ms, const double* W, zd* raw, bool small_grid = false, int chL = 0) {
  // the full grid L (singular modes to MQ = L/2 - 1), or the shorter grid
  // of the pairs classed CLASS_SPLIT under ClassParams.split_rho_small
  const int nt = small_grid ? c->nt_small : c->nt_int;
  const int MQ = nt / 2 - 1;
  const zd* tw = small_grid ? c->tw_small.p : c->tw_int.p;
  // chunks of pairs sized to about 1 GiB per singular-part table: the
  // Legendre recurrences run one pair per lane and are latency bound, so the
  // chunk must hold several wavefronts per SIMD (tables sized for the full grid)
  const long CH = std::max(1L << 15, std::min(1L << 18, (1L << 30) / (16L * (c->MQ + 1))));
  for (long f = 0; f < count; f += CH) {
    const long cn = std::min(CH, count - f);
    c->zhat.alloc((size_t)CH * (c->MQ + 1));
    c->phat.alloc((size_t)CH * (c->MQ + 1));
    c->qtab.alloc((size_t)CH * (c->MQ + 1));
    c->qcoef.alloc((size_t)CH * 4);
    launch_split_singular(geom, f, cn, MQ, c->qtab.p, c->qcoef.p, c->zhat.p, c->phat.p, c->stream);
    HIPCHK(hipGetLastError());
    launch_split(nt, geom, dest, f, cn, c->M, c->m0, MQ, c->k1, c->k2, tw, c->zhat.p, c->phat.p, A, n2, ms, W,
                 raw, c->stream, chL);
    HIPCHK(hipGetLastError());
  }
}

// Far pairs of the grid through the surrogate: features, network forward,
// acceptance against direct kernel samples (accepted modes go into A), and
// the raw-kernel FFT for the rest.
void run_surrogate(pmlbie_ctx* c, const PairGeom* geom, const int2* dest, long count, long n2, long ms,
                   const double* W) {
  const long CH = 1L << 16;
  HIPCHK(sg_work_alloc(c->sgw, (int)(2 * CH)));
  c->sgfx.alloc((size_t)2 * CH * SG_IN);
  c->sgcnt.alloc(2);
  c->sgfb_geom.alloc(std::max<long>(count, 1));
  c->sgfb_dest.alloc(std::max<long>(count, 1));
  HIPCHK(hipMemsetAsync(c->sgcnt.p, 0, 2 * sizeof(unsigned), c->stream));
  WorkList fb{c->sgfb_geom.p, c->sgfb_dest.p, c->sgcnt.p + 1, (unsigned)std::max<long>(count, 1)};
  SgFeat f{c->sg_a1 + c->sg_T};
  for (long s = 0; s < count; s += CH) {
    const long cn = std::min(CH, count - s);
    sg_pair_features(geom + s, cn, c->k1.re, c->k2.re, c->geo.pml.S, c->sgfx.p, c->stream);
    sg_features(c->sgfx.p, (int)(2 * cn), f, c->sgw, c->stream);
    sg_forward(c->sg, c->sgw, (int)(2 * cn), c->stream);
    sg_accept(geom + s, dest + s, cn, c->sgw.z[SG_NL - 1], c->M, c->m0, c->k1, c->k2, c->sg_tol, c->A.p, n2, ms,
              W, fb, c->sgcnt.p, c->cp, c->stream);
    HIPCHK(hipGetLastError());
  }
  unsigned h[2];
  HIPCHK(hipMemcpy(h, c->sgcnt.p, sizeof(h), hipMemcpyDeviceToHost));
  c->counters[4] = (double)count;
  c->counters[5] = (double)h[0];
  launch_list_far(c->nt_far, c->sgfb_geom.p, c->sgfb_dest.p, 0, h[1], c->M, c->m0, c->k1, c->k2, c->tw_far.p,
                  c->A.p, n2, ms, W, nullptr, &c->cp, c->stream);
  HIPCHK(hipGetLastError());
}

// Explicit pair list (host) -> raw modal values raw[q][s][n]: upload, classify
// on the device into far / split / direct lists, run the three paths.
void run_pair_list_dev(pmlbie_ctx* c, size_t tot, zd* raw, long long* counts,
                       const int* medium = nullptr, int Nm = 0, bool two_grids = false, int m_lo = 0);

void run_pair_list(pmlbie_ctx* c, const std::vector<PairGeom>& g, zd* raw, long long* counts) {
  const size_t tot = g.size();
  if (tot == 0) return;
  c->xgeom.alloc(tot);
  HIPCHK(hipMemcpyAsync(c->xgeom.p, g.data(), tot * sizeof(PairGeom), hipMemcpyHostToDevice, c->stream));
  run_pair_list_dev(c, tot, raw, counts);
}

// The same with the pair geometry already in c->xgeom.  With medium (field
// points, rows q = p * Nm + l), the far pairs get the kernels of their point's
// medium only.  m_lo: the lowest mode the caller reads (the direct rule may
// leave the modes below it unwritten).
void run_pair_list_dev(pmlbie_ctx* c, size_t tot, zd* raw, long long* counts, const int* medium, int Nm,
                       bool two_grids, int m_lo) {
  if (tot == 0) return;
  c->lgeom.alloc(4 * tot > c->lgeom.n ? 4 * tot : c->lgeom.n);
  c->ldest.alloc(4 * tot > c->ldest.n ? 4 * tot : c->ldest.n);
  c->lcount.alloc(4);
  HIPCHK(hipMemsetAsync(c->lcount.p, 0, 4 * sizeof(unsigned), c->stream));
  WorkList wf{c->lgeom.p, c->ldest.p, c->lcount.p, (unsigned)tot};
  WorkList ws{c->lgeom.p + tot, c->ldest.p + tot, c->lcount.p + 1, (unsigned)tot};
  WorkList wd{c->lgeom.p + 2 * tot, c->ldest.p + 2 * tot, c->lcount.p + 2, (unsigned)tot};
  WorkList wsb{c->lgeom.p + 3 * tot, c->ldest.p + 3 * tot, c->lcount.p + 3, (unsigned)tot};
  ClassParams cpl = c->cp;
  if (two_grids) cpl.split_rho_small = c->split_rho_small;
  launch_classify_list(c->xgeom.p, (long)tot, cpl, wf, ws, wd, wsb, c->stream);
  HIPCHK(hipGetLastError());
  unsigned cnt[4];
  HIPCHK(hipMemcpy(cnt, c->lcount.p, sizeof(cnt), hipMemcpyDeviceToHost));
  if (counts) {
    counts[0] += cnt[0];
    counts[1] += cnt[1] + cnt[3];
    counts[2] += cnt[2];
  }
  if (medium)
    launch_list_far_one(c->nt_far, wf.geom, wf.dest, 0, cnt[0], c->M, c->k1, c->k2, c->tw_far.p, raw, medium,
                        Nm, c->stream);
  else
    launch_list_far(c->nt_far, wf.geom, wf.dest, 0, cnt[0], c->M, 0, c->k1, c->k2, c->tw_far.p, nullptr, 0,
                    0, nullptr, raw, nullptr, c->stream);
  HIPCHK(hipGetLastError());
  run_split(c, ws.geom, ws.dest, cnt[1], nullptr, 0, 0, nullptr, raw, cpl.split_rho_small > 0.0);
  run_split(c, wsb.geom, wsb.dest, cnt[3], nullptr, 0, 0, nullptr, raw);
  if (c->ch1_L > 0)
    run_split(c, wd.geom, wd.dest, cnt[2], nullptr, 0, 0, nullptr, raw, false, c->ch1_L);
  else
    launch_direct(wd.geom, wd.dest, 0, cnt[2], c->M, m_lo, c->k1, c->k2, c->glx.p, c->glw.p, nullptr, 0, 0,
                  nullptr, raw, kOmegaPiece, c->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
}

// ---------------------------------------------------------------------------
// Device scratch of the allocation-free modal-kernel call
// (pmlbie_modal_kernels_noalloc): a fixed array in the code object, one copy
// per device, held until the process ends.  Layout (bytes, 256-aligned):
// pair geometry, the far / split / direct work lists, their counters and the
// split path's singular-mode tables for chunks of kNaSplitChunk pairs.
constexpr long kNaMaxPairs = PMLBIE_NOALLOC_MAX_PAIRS;
constexpr long kNaSplitChunk = 256;
constexpr long kNaMaxModesQ = 1024;  // MQ + 1 = L / 2 <= 1024 (L <= 2048)
constexpr size_t na_round(size_t b) { return (b + 255) & ~size_t(255); }
constexpr size_t kNaGeom = 0;
constexpr size_t kNaLGeom = kNaGeom + na_round(sizeof(PairGeom) * kNaMaxPairs);
constexpr size_t kNaLDest = kNaLGeom + na_round(3 * sizeof(PairGeom) * kNaMaxPairs);
constexpr size_t kNaCount = kNaLDest + na_round(3 * sizeof(int2) * kNaMaxPairs);
constexpr size_t kNaQtab = kNaCount + 256;
constexpr size_t kNaTable = sizeof(zd) * kNaSplitChunk * kNaMaxModesQ;
constexpr size_t kNaZhat = kNaQtab + na_round(kNaTable);
constexpr size_t kNaPhat = kNaZhat + na_round(kNaTable);
constexpr size_t kNaCoef = kNaPhat + na_round(kNaTable);
constexpr size_t kNaBytes = kNaCoef + na_round(sizeof(zd) * 4 * kNaSplitChunk);
static_assert(sizeof(PairGeom) == 12 * sizeof(double), "the host pair layout is copied as is");

static __device__ __align__(256) unsigned char scratch[kNaBytes];

// Device address of `scratch` per device (the array's name is a host-side
// stand-in), resolved once per device by pmlbie_create with that device current.
constexpr int kNaMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[kNaMaxDevices] = {};

hipError_t resolve_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= kNaMaxDevices) return hipErrorInvalidDevice;
  if (g_scratch[device]) return hipSuccess;
  unsigned char* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess) g_scratch[device] = ptr;
  return e;
}

// Twiddles e^{-2 pi i k / nt}, k < nt / 2 (k < nt for a full table).  A full
// table is followed by sin^2(pi j / nt), j = 0..nt/2, in the real parts: the
// far pass's sin^2(D_j / 2) (tw_s2).
std::vector<zd> twiddles(int nt, bool full = false) {
  const int n = full ? nt : nt / 2;
  std::vector<zd> t(full ? nt + nt / 2 + 1 : n);
  for (int k = 0; k < n; ++k) {
    double a = -2.0 * PMLBIE_PI * k / nt;
    t[k] = zd{cos(a), sin(a)};
  }
  if (full)
    for (int j = 0; j <= nt / 2; ++j) {
      const double s = sin(PMLBIE_PI * j / nt);
      t[nt + j] = zd{s * s, 0.0};
    }
  return t;
}

int pow2_at_least(double x) {
  int p = 16;
  while (p < x) p <<= 1;
  return p;
}

}  // namespace

extern "C" {

int pmlbie_create(pmlbie_ctx** out, int device, void* stream) {
  if (!out) return PMLBIE_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return PMLBIE_EDEVICE;
  if (device < 0 || device >= ndev) return PMLBIE_EINVAL;
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) return PMLBIE_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return PMLBIE_EDEVICE;
  const hipError_t se = resolve_scratch(device);
  (void)hipSetDevice(prev);
  if (se != hipSuccess) return PMLBIE_EDEVICE;
  pmlbie_ctx* c = new (std::nothrow) pmlbie_ctx();
  if (!c) return PMLBIE_ENOMEM;
  c->device = device;
  c->stream = (hipStream_t)stream;
  *out = c;
  return PMLBIE_OK;
}

void pmlbie_destroy(pmlbie_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->up_stream) {
    (void)hipStreamSynchronize(c->up_stream);
    (void)hipStreamDestroy(c->up_stream);
  }
  if (c->up_done) (void)hipEventDestroy(c->up_done);
  if (c->lu_stream) {
    (void)hipStreamSynchronize(c->lu_stream);
    (void)hipStreamDestroy(c->lu_stream);
  }
  for (hipEvent_t& e : c->lu_ev)
    if (e) (void)hipEventDestroy(e);
  delete c;
}

const char* pmlbie_last_error(const pmlbie_ctx* c) { return c ? c->err.c_str() : "null context"; }

int pmlbie_set_geometry(pmlbie_ctx* c, int n_bumps, const double* bumps, double cos_freq,
                        double rho_c, const double* seg_breaks, int nodes_per_segment) {
  return guarded(c, [&]() -> int {
    if (n_bumps < 0 || n_bumps > 8 || (n_bumps > 0 && !bumps) || !seg_breaks)
      return fail(c, PMLBIE_EINVAL, "set_geometry: bad bump list");
    if (nodes_per_segment <= 0 || nodes_per_segment % 16)
      return fail(c, PMLBIE_EINVAL, "set_geometry: nodes_per_segment must be a positive multiple of 16");
    if (seg_breaks[0] != 0.0) return fail(c, PMLBIE_EINVAL, "set_geometry: curve must start on the axis");
    for (int s = 0; s < 4; ++s)
      if (!(seg_breaks[s + 1] > seg_breaks[s]))
        return fail(c, PMLBIE_EINVAL, "set_geometry: segment breaks must increase");
    Geometry g;
    for (int i = 0; i < n_bumps; ++i) {
      if (!(bumps[3 * i + 2] > 0)) return fail(c, PMLBIE_EINVAL, "set_geometry: bump width must be > 0");
      g.itf.amp.push_back(bumps[3 * i]);
      g.itf.cen.push_back(bumps[3 * i + 1]);
      g.itf.wid.push_back(bumps[3 * i + 2]);
    }
    g.itf.cos_freq = cos_freq;
    g.itf.rho_c = rho_c;
    g.breaks.assign(seg_breaks, seg_breaks + 5);
    g.nodes_per_segment = nodes_per_segment;
    c->geo = g;
    c->stage = 1;
    return PMLBIE_OK;
  });
}

int pmlbie_set_polyline(pmlbie_ctx* c, int n_vert, const double* verts, const int* panels,
                        int grade) {
  return guarded(c, [&]() -> int {
    if (n_vert < 2 || n_vert > PMLBIE_POLY_MAX_VERTS || !verts || !panels)
      return fail(c, PMLBIE_EINVAL, "set_polyline: need 2 <= n_vert <= 64 vertices and a panel count per segment");
    if (grade < 0 || grade > 24) return fail(c, PMLBIE_EINVAL, "set_polyline: grade must lie in [0, 24]");
    if (verts[0] != 0.0) return fail(c, PMLBIE_EINVAL, "set_polyline: the curve must start on the axis");
    for (int j = 1; j < n_vert; ++j) {
      if (!(verts[2 * j] > 0.0) || !std::isfinite(verts[2 * j]) || !std::isfinite(verts[2 * j + 1]))
        return fail(c, PMLBIE_EINVAL, "set_polyline: vertices after the first must have rho > 0");
      if (verts[2 * j] == verts[2 * j - 2] && verts[2 * j + 1] == verts[2 * j - 1])
        return fail(c, PMLBIE_EINVAL, "set_polyline: repeated vertex");
      if (panels[j - 1] < 2 || panels[j - 1] > 4096)
        return fail(c, PMLBIE_EINVAL, "set_polyline: 2 <= panels per segment <= 4096");
    }
    Geometry g;
    g.poly = true;
    g.verts.assign(verts, verts + 2 * n_vert);
    g.seg_panels.assign(panels, panels + n_vert - 1);
    g.grade = grade;
    // graded panels: the layout is fixed here, so the node count is known
    Geometry probe = g;
    probe.pml.a1 = verts[2 * n_vert - 2];
    probe.pml.T = 1.0;
    probe.build();
    if (probe.npanels() % 4)
      return fail(c, PMLBIE_EINVAL, "set_polyline: the total number of panels (after grading) must be a multiple of 4");
    c->geo = g;
    c->stage = 1;
    return PMLBIE_OK;
  });
}

int pmlbie_set_panels(pmlbie_ctx* c, int n_panels, const double* nodes) {
  return guarded(c, [&]() -> int {
    if (n_panels < 4 || n_panels > PMLBIE_MAX_PANELS || n_panels % 4 || !nodes)
      return fail(c, PMLBIE_EINVAL, "set_panels: need a multiple of 4 panels in [4, 65536] and their nodes");
    for (long i = 0; i < 32L * n_panels; ++i)
      if (!std::isfinite(nodes[i])) return fail(c, PMLBIE_EINVAL, "set_panels: non-finite node coordinate");
    for (long i = 0; i < 16L * n_panels; ++i)
      if (!(nodes[2 * i] > 0.0)) return fail(c, PMLBIE_EINVAL, "set_panels: every node needs rho > 0");
    Geometry g;
    g.curved = true;
    g.cnodes.assign(nodes, nodes + 32L * n_panels);
    if (const char* e = g.prepare_curved()) return fail(c, PMLBIE_EINVAL, e);
    c->geo = g;
    c->stage = 1;
    return PMLBIE_OK;
  });
}

int pmlbie_set_media_pml(pmlbie_ctx* c, double k1_re, double k1_im, double k2_re, double k2_im,
                         double a1, double T, double S, double a2, double T2, double S2, int p) {
  return guarded(c, [&]() -> int {
    if (c->stage < 1) return fail(c, PMLBIE_ESTATE, "set_media_pml: set the geometry first");
    if (!(a1 > 0) || !(T > 0) || !(S >= 0) || p < 2)
      return fail(c, PMLBIE_EINVAL, "set_media_pml: need a1 > 0, T > 0, S >= 0, p >= 2");
    if (fabs(c->geo.rho_end() - (a1 + T)) > 1e-12 * (a1 + T))
      return fail(c, PMLBIE_EINVAL, "set_media_pml: the curve must end at the outer PML edge a1 + T");
    if (const char* e = c->geo.poly_pml_error(a1)) return fail(c, PMLBIE_EINVAL, e);
    c->k1 = zd{k1_re, k1_im};
    c->k2 = zd{k2_re, k2_im};
    c->geo.pml.a1 = a1;
    c->geo.pml.T = T;
    c->geo.pml.S = S;
    c->geo.pml.p = p;
    c->a2 = a2;
    c->T2 = T2;
    c->S2 = S2;
    c->geo.build();
    c->N = c->geo.n();
    c->stage = 2;
    return PMLBIE_OK;
  });
}

int pmlbie_build_modal_operators(pmlbie_ctx* c, int n_theta, int m_max, int precision, int flags) {
  return pmlbie_build_modal_operators_range(c, n_theta, 0, m_max, precision, flags);
}

int pmlbie_build_modal_operators_range(pmlbie_ctx* c, int n_theta, int m_min, int m_max, int precision,
                                       int flags) {
  return guarded(c, [&]() -> int {
    if (c->stage < 2) return fail(c, PMLBIE_ESTATE, "build: set geometry and media first");
    if (n_theta < 16 || (n_theta & (n_theta - 1)))
      return fail(c, PMLBIE_EINVAL, "build: n_theta must be a power of two >= 16");
    if (m_max < 0 || m_max > n_theta / 2)
      return fail(c, PMLBIE_EINVAL, "build: need 0 <= m_max <= n_theta / 2");
    if (m_min < 0 || m_min > m_max) return fail(c, PMLBIE_EINVAL, "build: need 0 <= m_min <= m_max");
    if (precision != PMLBIE_FP64 && precision != PMLBIE_MIXED)
      return fail(c, PMLBIE_EINVAL, "build: precision must be PMLBIE_FP64 or PMLBIE_MIXED");
    if (2L * c->N > LU_MAX_N)
      return fail(c, PMLBIE_EINVAL, "build: at most " + std::to_string(LU_MAX_N / 2) +
                                        " curve nodes (the per-mode LU takes at most " + std::to_string(LU_MAX_N) +
                                        " unknowns)");
    const bool use_sg = (flags & PMLBIE_USE_SURROGATE) != 0;
    if (use_sg) {
      if (!c->sg_ready) return fail(c, PMLBIE_ESTATE, "build: no surrogate network (init, train or load one)");
      if (c->k1.im != 0.0 || c->k2.im != 0.0)
        return fail(c, PMLBIE_EINVAL, "build: the surrogate takes real wavenumbers");
      if (fabs(c->geo.pml.a1 - c->sg_a1) > 1e-12 || fabs(c->geo.pml.T - c->sg_T) > 1e-12 ||
          c->geo.pml.p != c->sg_p)
        return fail(c, PMLBIE_EINVAL, "build: the surrogate was trained for another PML geometry");
    }
    auto t_all = std::chrono::steady_clock::now();
    c->stage = 2;
    c->n_theta = n_theta;
    c->M = m_max;
    c->m0 = m_min;
    c->precision = precision;
    c->flags = flags;
    const int N = c->N, M = c->M, m0 = c->m0, nm = M - m0 + 1;
    const long n2 = 2L * N;
    const long ms = n2 * n2;
    // Angle grid L (one length for every FFT path): the smooth parts of the
    // split carry modes up to B ~ 1.15 |k| |rho~|max + 16 (the bandwidth of
    // cos kR in theta), the singular factors are kept to MQ = L/2 - 1, and
    // the products are exact for the kept modes 0..M when MQ - M >= B.
    const double kmax = std::max(cabs_(c->k1), cabs_(c->k2));
    const double rmax = cabs_(zd{c->geo.rho_end(), c->geo.Iint(c->geo.rho_end())});
    const double bneed = ceil(1.15 * kmax * rmax + 16.0);
    const int L = std::max(512, pow2_at_least(std::max<double>(n_theta, 2.0 * (M + bneed) + 2.0)));
    if (L > 2048) return fail(c, PMLBIE_EINVAL, "build: wavenumber or m_max too large for the azimuthal FFT");
    c->nt_int = L;
    c->MQ = L / 2 - 1;
    c->B = c->MQ - M;
    c->nt_far = L;
    c->cp.M = M;
    c->cp.nt_far = c->nt_far;
    c->cp.bw = 1.1;
    c->cp.kmax = std::max(fabs(c->k1.re), fabs(c->k2.re));
    c->cp.kmax_im = std::max(fabs(c->k1.im), fabs(c->k2.im));
    c->cp.c_far = 34.0;
    c->cp.g_split = 9.0;
    c->cp.nt_small = 0;
    // the main far pass runs on the shortest grid that holds modes 0..M
    // (512 at least); far pairs whose aliasing bound needs the full grid L
    // are listed and transformed on it afterwards
    c->nt_small = std::min(L, std::max(512, pow2_at_least(2.0 * (M + 1))));
    // split pairs whose smooth parts' bandwidth 1.15 |k| max(|rho~_t|, |rho~_s|) + 16
    // fits below the shorter grid (MQ_small - M of it) are split on that grid
    c->split_rho_small = 0.0;
    if (c->nt_small < L && kmax > 0.0) {
      const double r = ((double)(c->nt_small / 2 - 1 - M) - 16.0) / (1.15 * kmax);
      if (r > 0.0) c->split_rho_small = r;
    }

    Timer t_setup(c->stream);
    // node tables
    std::vector<double> nt(10L * N);
    for (int i = 0; i < N; ++i) {
      nt[i] = c->geo.rho[i];
      nt[N + i] = c->geo.I[i];
      nt[2L * N + i] = c->geo.z[i];
      nt[3L * N + i] = c->geo.W[i];
      nt[4L * N + i] = c->geo.nr_re[i];
      nt[5L * N + i] = c->geo.nr_im[i];
      nt[6L * N + i] = c->geo.nz_re[i];
      nt[7L * N + i] = c->geo.nz_im[i];
      nt[8L * N + i] = c->geo.nur[i];
      nt[9L * N + i] = c->geo.nuz[i];
    }
    c->nodes.alloc(nt.size());
    HIPCHK(hipMemcpyAsync(c->nodes.p, nt.data(), nt.size() * 8, hipMemcpyHostToDevice, c->stream));
    c->dpanel.alloc(N);
    HIPCHK(hipMemcpyAsync(c->dpanel.p, c->geo.panel.data(), N * sizeof(int), hipMemcpyHostToDevice,
                          c->stream));
    auto twf = twiddles(c->nt_far, true), twi = twiddles(c->nt_int, true), tws = twiddles(c->nt_small, true);
    c->tw_far.alloc(twf.size());
    c->tw_int.alloc(twi.size());
    c->tw_small.alloc(tws.size());
    HIPCHK(hipMemcpyAsync(c->tw_far.p, twf.data(), twf.size() * sizeof(zd), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->tw_int.p, twi.data(), twi.size() * sizeof(zd), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->tw_small.p, tws.data(), tws.size() * sizeof(zd), hipMemcpyHostToDevice, c->stream));
    c->glx.alloc(16);
    c->glw.alloc(16);
    HIPCHK(hipMemcpyAsync(c->glx.p, c->geo.glx, 16 * 8, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->glw.p, c->geo.glw, 16 * 8, hipMemcpyHostToDevice, c->stream));
    // operators
    c->A.alloc((size_t)nm * ms);
    c->ipiv.alloc((size_t)nm * n2);
    c->luw.alloc((size_t)nm * LU_NB * LU_NB);
    c->lumap.alloc(2 * (size_t)nm * n2);
    c->info.alloc(nm);
    HIPCHK(hipMemsetAsync(c->info.p, 0, nm * sizeof(int), c->stream));
    // work lists of the grid (split, direct, far and split on the full grid
    // share one allocation)
    const size_t cap = (size_t)N * N;
    c->lgeom.alloc(4 * cap);
    c->ldest.alloc(4 * cap);
    c->lcount.alloc(4);
    HIPCHK(hipMemsetAsync(c->lcount.p, 0, 4 * sizeof(unsigned), c->stream));
    // auxiliary near-panel points: built on the host while the device runs
    // the far, split and direct stages, into host tables that the context
    // keeps between builds (refilled every time; keeping the memory spares
    // the zero fill and page faults of ~150 MB at paper scale per build)
    std::vector<PairGeom>& ageom = c->h_ageom;
    std::vector<double>& acoef = c->h_acoef;
    std::vector<NearJob>& ajobs = c->h_ajobs;
    // longest auxiliary interval: |k| |1 + i sigma| h <= 4 keeps the 16-point
    // rule times a degree-15 Lagrange factor at rounding level
    const double keff = std::max(cabs_(c->k1), cabs_(c->k2)) * sqrt(1.0 + c->geo.pml.S * c->geo.pml.S);
    const double near_hmax = keff > 0.0 ? 4.0 / keff : 1e300;
    if (!c->up_stream) HIPCHK(hipStreamCreateWithFlags(&c->up_stream, hipStreamNonBlocking));
    if (!c->up_done) HIPCHK(hipEventCreateWithFlags(&c->up_done, hipEventDisableTiming));
    std::future<void> near_tables = std::async(std::launch::async, [&]() {
      HIPCHK(hipSetDevice(c->device));
      c->geo.build_near(ageom, acoef, ajobs, 6, near_hmax);
      // uploaded on their own stream while the far/split/direct stages run
      c->coef.alloc(acoef.size());
      c->jobs.alloc(ajobs.size());
      c->xgeom.alloc(std::max<size_t>(ageom.size(), 1));
      HIPCHK(hipMemcpyAsync(c->coef.p, acoef.data(), acoef.size() * 8, hipMemcpyHostToDevice, c->up_stream));
      HIPCHK(hipMemcpyAsync(c->jobs.p, ajobs.data(), ajobs.size() * sizeof(NearJob), hipMemcpyHostToDevice,
                            c->up_stream));
      HIPCHK(hipMemcpyAsync(c->xgeom.p, ageom.data(), ageom.size() * sizeof(PairGeom),
                            hipMemcpyHostToDevice, c->up_stream));
      HIPCHK(hipEventRecord(c->up_done, c->up_stream));
    });
    c->stage_ms[0] = t_setup.stop();

    NodesDev nd;
    nd.N = N;
    nd.rho = c->nodes.p;
    nd.I = c->nodes.p + N;
    nd.z = c->nodes.p + 2L * N;
    nd.W = c->nodes.p + 3L * N;
    nd.nr_re = c->nodes.p + 4L * N;
    nd.nr_im = c->nodes.p + 5L * N;
    nd.nz_re = c->nodes.p + 6L * N;
    nd.nz_im = c->nodes.p + 7L * N;
    nd.panel = c->dpanel.p;
    WorkList ws{c->lgeom.p, c->ldest.p, c->lcount.p, (unsigned)cap};
    WorkList wd{c->lgeom.p + cap, c->ldest.p + cap, c->lcount.p + 1, (unsigned)cap};

    // far pairs: raw-kernel FFT in the grid (those that need the full grid
    // listed in wf and transformed from the list), or listed for the surrogate
    WorkList wf{c->lgeom.p + 2 * cap, c->ldest.p + 2 * cap, c->lcount.p + 2, (unsigned)cap};
    WorkList wsb{c->lgeom.p + 3 * cap, c->ldest.p + 3 * cap, c->lcount.p + 3, (unsigned)cap};
    Timer t_far(c->stream);
    ClassParams cpg = c->cp;
    cpg.split_rho_small = c->split_rho_small;
    if (use_sg) {
      launch_grid_classify(nd, cpg, wf, ws, wd, wsb, c->stream);
    } else {
      cpg.nt_small = c->nt_small;
      launch_grid_far(nd, cpg, c->k1, c->k2, c->nt_small < c->nt_far ? c->tw_small.p : c->tw_far.p, c->A.p, ms,
                      m0, nd.W, ws, wd, wf, wsb, c->stream);
    }
    HIPCHK(hipGetLastError());
    unsigned counts[4] = {0, 0, 0, 0};
    HIPCHK(hipMemcpy(counts, c->lcount.p, 4 * sizeof(unsigned), hipMemcpyDeviceToHost));
    if (counts[0] > cap || counts[1] > cap || counts[2] > cap || counts[3] > cap)
      return fail(c, PMLBIE_EDEVICE, "build: work list overflow");
    c->counters[4] = 0;
    c->counters[5] = 0;
    // the main pass lists its long-grid far pairs once per unordered pair
    c->cnt_far_big = use_sg ? 0 : 2LL * counts[2];
    c->counters[6] = (double)c->cnt_far_big;
    if (use_sg) {
      run_surrogate(c, wf.geom, wf.dest, counts[2], n2, ms, nd.W);
    } else if (counts[2] > 0) {
      launch_list_far_sym(c->nt_far, wf.geom, wf.dest, counts[2], nd, M, m0, c->k1, c->k2, c->tw_far.p, c->A.p, n2,
                          ms, nd.W, c->cp, c->stream);
      HIPCHK(hipGetLastError());
    }
    c->stage_ms[1] = t_far.stop();
    c->cnt_split = counts[0] + counts[3];
    c->cnt_direct = counts[1];
    c->cnt_far = (long long)N * N - counts[0] - counts[1] - counts[3];

    Timer t_split(c->stream);
    run_split(c, c->lgeom.p, c->ldest.p, counts[0], c->A.p, n2, ms, nd.W, nullptr, c->split_rho_small > 0.0);
    run_split(c, wsb.geom, wsb.dest, counts[3], c->A.p, n2, ms, nd.W, nullptr);
    c->stage_ms[2] = t_split.stop();
    Timer t_direct(c->stream);
    if (c->ch1_L > 0)
      run_split(c, c->lgeom.p + cap, c->ldest.p + cap, counts[1], c->A.p, n2, ms, nd.W, nullptr, false, c->ch1_L);
    else
      launch_direct(c->lgeom.p + cap, c->ldest.p + cap, 0, counts[1], M, m0, c->k1, c->k2, c->glx.p,
                    c->glw.p, c->A.p, n2, ms, nd.W, nullptr, kOmegaPiece, c->stream);
    HIPCHK(hipGetLastError());
    c->stage_ms[3] = t_direct.stop();

    // near panels: modal kernels at the auxiliary points, then product integration
    Timer t_near(c->stream);
    near_tables.get();
    HIPCHK(hipStreamWaitEvent(c->stream, c->up_done, 0));
    c->cnt_aux = (long long)ageom.size();
    c->raw.alloc(std::max<size_t>(ageom.size(), 1) * 4 * (M + 1));
    long long dummy[3] = {0, 0, 0};
    run_pair_list_dev(c, ageom.size(), c->raw.p, dummy, nullptr, 0, true, m0);
    launch_near(c->jobs.p, (int)ajobs.size(), c->coef.p, c->raw.p, M, m0, c->A.p, n2, ms, c->stream);
    HIPCHK(hipGetLastError());
    c->stage_ms[4] = t_near.stop();
    // the near-panel pairs of the grid were not counted as far
    c->cnt_far -= 16LL * (long long)ajobs.size();
    if (c->zc_mode >= m0 && c->zc_mode <= M) {
      // the hook's column is in block order: u1 of node c, or phi1 of node c - N
      const int col = c->zc_col < N ? 2 * c->zc_col : 2 * (c->zc_col - N) + 1;
      launch_zero_column(c->A.p + (size_t)(c->zc_mode - m0) * ms, n2, col, c->stream);
      HIPCHK(hipGetLastError());
    }
    c->zc_mode = c->zc_col = -1;

    // keep what the solve needs: the unfactored operator (FP64) -- the lower
    // block row [K2 - D2, -S2] for the right-hand sides, and in mixed
    // precision the whole matrix for the residuals of the refinement
    const bool mixed = precision == PMLBIE_MIXED;
    if (mixed) {
      c->Alow.release();
    } else {
      c->A32.release();
      // the lower-medium equations are the odd rows of the interleaved system
      c->Alow.alloc((size_t)nm * N * n2);
      HIPCHK(hipMemcpy2DAsync(c->Alow.p, (size_t)n2 * sizeof(zd), c->A.p + n2, 2 * (size_t)n2 * sizeof(zd),
                              (size_t)n2 * sizeof(zd), (size_t)nm * N, hipMemcpyDeviceToDevice, c->stream));
    }
    if ((flags & PMLBIE_KEEP_OPERATORS) && !mixed) {
      c->Akeep.alloc((size_t)nm * ms);
      HIPCHK(hipMemcpyAsync(c->Akeep.p, c->A.p, (size_t)nm * ms * sizeof(zd),
                            hipMemcpyDeviceToDevice, c->stream));
    } else {
      c->Akeep.release();
    }

    // per-mode LU (complex128, or complex64 on FP32 MFMA in mixed precision)
    Timer t_lu(c->stream);
    const int npan = std::max(1, lu_update_steps((int)n2));
    std::vector<hipEvent_t> gb(npan), ge(npan);
    for (int k = 0; k < npan; ++k) {
      HIPCHK(hipEventCreate(&gb[k]));
      HIPCHK(hipEventCreate(&ge[k]));
    }
    LuTimers tm;
    tm.gemm_begin = gb.data();
    tm.gemm_end = ge.data();
    if (!c->lu_stream) HIPCHK(hipStreamCreateWithFlags(&c->lu_stream, hipStreamNonBlocking));
    for (hipEvent_t& e : c->lu_ev)
      if (!e) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    if (mixed) {
      // the complex64 copy is filled from the FP64 operators inside the LU's
      // first step (its second row map in lumap's second half)
      c->A32.alloc((size_t)nm * ms);
      lu_factor_batched<float>(c->A32.p, ms, (int)n2, nm, c->ipiv.p, c->info.p,
                               reinterpret_cast<zf*>(c->luw.p), c->stream, &tm, c->lu_stream, c->lu_ev, c->lumap.p,
                               c->A.p, c->lumap.p + (size_t)nm * n2);
    } else {
      lu_factor_batched<double>(c->A.p, ms, (int)n2, nm, c->ipiv.p, c->info.p, c->luw.p,
                                c->stream, &tm, c->lu_stream, c->lu_ev, c->lumap.p);
    }
    HIPCHK(hipGetLastError());
    c->stage_ms[5] = t_lu.stop();
    // algorithmic flops of the trailing updates (8 real flops per complex
    // multiply-add) and the number of their launches
    c->counters[2] = lu_update_flops((int)n2, nm);
    c->counters[3] = (double)lu_update_steps((int)n2);
    // summed durations of the trailing-update launches
    double gsum = 0;
    for (int k = 0; k < lu_update_steps((int)n2); ++k) {
      float ms1 = 0;
      if (hipEventElapsedTime(&ms1, gb[k], ge[k]) == hipSuccess) gsum += ms1;
    }
    for (int k = 0; k < npan; ++k) {
      (void)hipEventDestroy(gb[k]);
      (void)hipEventDestroy(ge[k]);
    }
    c->stage_ms[6] = gsum;
    std::vector<int> info(nm);
    HIPCHK(hipMemcpy(info.data(), c->info.p, nm * sizeof(int), hipMemcpyDeviceToHost));
    for (int n = 0; n < nm; ++n)
      if (info[n])
        return fail(c, PMLBIE_ESINGULAR,
                    "build: mode " + std::to_string(m0 + n) + " has a zero pivot at column " +
                        std::to_string((info[n] - 1) % 2 == 0 ? (info[n] - 1) / 2 : N + (info[n] - 1) / 2));
    c->stage_ms[10] = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_all).count();
    c->stage = 3;
    return PMLBIE_OK;
  });
}

int pmlbie_solve_modes(pmlbie_ctx* c, int n_rhs, const pmlbie_incidence* inc, void* d_u1,
                       void* d_phi1, void* d_u2, void* d_phi2) {
  return guarded(c, [&]() -> int {
    if (c->stage < 3) return fail(c, PMLBIE_ESTATE, "solve: build the operators first");
    if (n_rhs < 1 || n_rhs > LU_MAX_RHS || !inc) return fail(c, PMLBIE_EINVAL, "solve: 1 <= n_rhs <= 16");
    for (int r = 0; r < n_rhs; ++r) {
      if (inc[r].kind == 0) {
        if (!(inc[r].p[0] >= 0)) return fail(c, PMLBIE_EINVAL, "solve: source radius must be >= 0");
        if (!(inc[r].p[0] < c->geo.pml.a1)) return fail(c, PMLBIE_EINVAL, "solve: the point source must lie in the physical region rho < a1");
        if (!c->geo.above(inc[r].p[0], inc[r].p[1]))
          return fail(c, PMLBIE_EINVAL, "solve: the point source must lie in the upper medium");
      } else if (inc[r].kind == 1) {
        if (!(inc[r].p[0] >= 0 && inc[r].p[0] < 0.5 * PMLBIE_PI))
          return fail(c, PMLBIE_EINVAL, "solve: plane-wave polar angle must lie in [0, pi/2)");
        if (c->k1.im != 0.0 || c->k2.im != 0.0)
          return fail(c, PMLBIE_EINVAL, "solve: plane waves need real wavenumbers");
      } else {
        return fail(c, PMLBIE_EINVAL, "solve: incidence kind must be 0 (point source) or 1 (plane wave)");
      }
    }
    auto t0 = std::chrono::steady_clock::now();
    c->stage = 3;  // the solution of an earlier solve is being replaced
    const int N = c->N, M = c->M, m0 = c->m0, nm = M - m0 + 1;
    const long n2 = 2L * N, ms = n2 * n2;
    c->nrhs = n_rhs;
    Timer t_rhs(c->stream);
    // point sources: pairs (node i, source) and (source, node i)
    std::vector<PairGeom> g;
    std::vector<int> rmap;
    std::vector<PlaneWave> pws;
    for (int r = 0; r < n_rhs; ++r) {
      if (inc[r].kind == 1) {
        const double phi = inc[r].p[0], k1 = c->k1.re, k2 = c->k2.re;
        PlaneWave P;
        P.k1 = k1;
        P.c = cos(phi);
        P.s = sin(phi);
        // transmitted wavenumber and reflection coefficient of the flat interface (Sec. 2)
        if (k2 > fabs(k1 * P.s)) P.kst = zd{sqrt(k2 * k2 - k1 * k1 * P.s * P.s), 0.0};
        else P.kst = zd{0.0, sqrt(k1 * k1 * P.s * P.s - k2 * k2)};
        P.R = 2.0 * inv(zd{1.0, 0.0} + P.kst * (1.0 / (k1 * P.c))) - 1.0;
        P.rhs = r;
        pws.push_back(P);
        continue;
      }
      rmap.push_back(r);
      const double rs = inc[r].p[0], zs = inc[r].p[1];
      for (int i = 0; i < N; ++i) {
        PairGeom p;
        p.rt = zd{c->geo.rho[i], c->geo.I[i]};
        p.rs = zd{rs, 0.0};
        p.drho = zd{c->geo.rho[i] - rs, c->geo.I[i]};
        p.dz = zd{c->geo.z[i] - zs, 0.0};
        p.nr = zd{0.0, 0.0};
        p.nz = zd{0.0, 0.0};
        g.push_back(p);
      }
      for (int i = 0; i < N; ++i) {
        PairGeom p;
        p.rt = zd{rs, 0.0};
        p.rs = zd{c->geo.rho[i], c->geo.I[i]};
        p.drho = zd{rs - c->geo.rho[i], -c->geo.I[i]};
        p.dz = zd{zs - c->geo.z[i], 0.0};
        p.nr = zd{c->geo.nr_re[i], c->geo.nr_im[i]};
        p.nz = zd{c->geo.nz_re[i], c->geo.nz_im[i]};
        g.push_back(p);
      }
    }
    const size_t vec = (size_t)nm * n_rhs * N;
    c->b1.alloc(vec);
    c->b2.alloc(vec);
    c->x.alloc(2 * vec);
    if (!g.empty()) {
      c->raw.alloc(g.size() * 4 * (M + 1));
      run_pair_list(c, g, c->raw.p, nullptr);
      c->rmap.alloc(rmap.size());
      HIPCHK(hipMemcpyAsync(c->rmap.p, rmap.data(), rmap.size() * sizeof(int), hipMemcpyHostToDevice, c->stream));
      launch_rhs_gather_point(c->raw.p, c->rmap.p, (int)rmap.size(), N, M, m0, n_rhs, c->b1.p, c->b2.p,
                              c->stream);
      HIPCHK(hipGetLastError());
    }
    if (!pws.empty()) {
      // FFT length: the modes of exp(-i a cos theta) die out beyond |n| ~ a
      double amax = 0.0;
      for (const PlaneWave& P : pws) amax = std::max(amax, P.k1 * P.s * c->geo.rho_end());
      const int ntp = std::max(256, pow2_at_least(2.0 * (std::max<double>(M, amax) + 40.0)));
      if (ntp > 2048) return fail(c, PMLBIE_EINVAL, "solve: plane-wave data need more than 2048 azimuthal samples");
      auto twp = twiddles(ntp);
      c->tw_pw.alloc(twp.size());
      HIPCHK(hipMemcpyAsync(c->tw_pw.p, twp.data(), twp.size() * sizeof(zd), hipMemcpyHostToDevice, c->stream));
      c->dpw.alloc(pws.size());
      HIPCHK(hipMemcpyAsync(c->dpw.p, pws.data(), pws.size() * sizeof(PlaneWave), hipMemcpyHostToDevice, c->stream));
      launch_rhs_plane(ntp, c->nodes.p, c->nodes.p + 2L * N, c->nodes.p + 8L * N, c->nodes.p + 9L * N, N,
                       c->dpw.p, (int)pws.size(), c->tw_pw.p, M, m0, n_rhs, c->b1.p, c->b2.p, c->stream);
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(c->stream));
    }
    const bool mixed = c->precision == PMLBIE_MIXED;
    if (mixed)
      launch_lower_rhs(c->A.p + n2, ms, 2 * n2, N, nm, n_rhs, c->b1.p, c->b2.p, c->x.p, c->stream);
    else
      launch_lower_rhs(c->Alow.p, (long)N * n2, n2, N, nm, n_rhs, c->b1.p, c->b2.p, c->x.p, c->stream);
    HIPCHK(hipGetLastError());
    c->stage_ms[8] = t_rhs.stop();
    Timer t_sol(c->stream);
    double t_ref = 0.0;
    std::string noconv;  // set when the refinement stops short of its rule
    c->counters[0] = 0;
    c->counters[1] = 0;
    if (!mixed) {
      lu_solve_batched<double, double>(c->A.p, ms, (int)n2, nm, c->ipiv.p, c->x.p, n_rhs, c->stream);
      HIPCHK(hipGetLastError());
    } else {
      // FP64 iterative refinement with the complex64 factors:
      //   d = LU32 \ r (FP64 arithmetic), x += d, r = rhs - A64 x,
      // until ||r|| <= tol ||rhs|| for every mode and right-hand side.
      const long nv = (long)nm * n_rhs;
      const long len = nv * n2;
      c->rbuf.alloc(len);
      c->xs.alloc(len);
      c->rsq.alloc(len);
      c->rnorm.alloc(2 * nv);
      const double tol = c->ref_tol;
      const int maxit = c->ref_maxit;
      HIPCHK(hipMemsetAsync(c->xs.p, 0, len * sizeof(zd), c->stream));
      HIPCHK(hipMemcpyAsync(c->rbuf.p, c->x.p, len * sizeof(zd), hipMemcpyDeviceToDevice, c->stream));
      launch_sq(c->x.p, len, c->rsq.p, c->stream);
      launch_sumsq(c->rsq.p, (int)n2, (int)nv, c->rnorm.p + nv, c->stream);  // ||rhs||^2
      std::vector<double> hn(2 * nv);
      Timer t_r(c->stream);
      int it = 0;
      double worst = 0.0;
      for (; it < maxit; ++it) {
        lu_solve_batched<float, double>(c->A32.p, ms, (int)n2, nm, c->ipiv.p, c->rbuf.p, n_rhs, c->stream);
        launch_axpy(c->xs.p, c->rbuf.p, len, c->stream);
        launch_residual(c->A.p, ms, (int)n2, nm, n_rhs, c->xs.p, c->x.p, c->rbuf.p, c->rsq.p, c->stream);
        launch_sumsq(c->rsq.p, (int)n2, (int)nv, c->rnorm.p, c->stream);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpy(hn.data(), c->rnorm.p, 2 * nv * sizeof(double), hipMemcpyDeviceToHost));
        worst = 0.0;
        for (long v = 0; v < nv; ++v) {
          const double rr = sqrt(hn[v]), bb = sqrt(hn[nv + v]);
          const double rel = bb > 0 ? rr / bb : (rr > 0 ? 1.0 : 0.0);
          worst = std::max(worst, rel);
        }
        if (worst <= tol) {
          ++it;
          break;
        }
      }
      t_ref = t_r.stop();
      c->counters[0] = it;
      c->counters[1] = worst;
      HIPCHK(hipMemcpyAsync(c->x.p, c->xs.p, len * sizeof(zd), hipMemcpyDeviceToDevice, c->stream));
      if (worst > tol)
        noconv = "solve: refinement stopped at relative residual " + std::to_string(worst) + " after " +
                 std::to_string(it) + " iterations";
    }
    c->u1.alloc(vec);
    c->p1.alloc(vec);
    c->u2.alloc(vec);
    c->p2.alloc(vec);
    launch_outputs(c->x.p, c->b1.p, c->b2.p, N, nm - 1, n_rhs, c->u1.p, c->p1.p, c->u2.p, c->p2.p, c->stream);
    HIPCHK(hipGetLastError());
    const size_t bytes = vec * sizeof(zd);
    if (d_u1) HIPCHK(hipMemcpyAsync(d_u1, c->u1.p, bytes, hipMemcpyDeviceToDevice, c->stream));
    if (d_phi1) HIPCHK(hipMemcpyAsync(d_phi1, c->p1.p, bytes, hipMemcpyDeviceToDevice, c->stream));
    if (d_u2) HIPCHK(hipMemcpyAsync(d_u2, c->u2.p, bytes, hipMemcpyDeviceToDevice, c->stream));
    if (d_phi2) HIPCHK(hipMemcpyAsync(d_phi2, c->p2.p, bytes, hipMemcpyDeviceToDevice, c->stream));
    c->stage_ms[9] = t_ref;
    c->stage_ms[7] = t_sol.stop() + c->stage_ms[8];
    (void)t0;
    // the outputs hold the last iterate either way; only a converged solve
    // opens the field evaluation
    if (!noconv.empty()) return fail(c, PMLBIE_ENOCONV, noconv);
    c->stage = 4;
    return PMLBIE_OK;
  });
}

int pmlbie_evaluate_field(pmlbie_ctx* c, int n_pts, const double* rtz, double* out) {
  return guarded(c, [&]() -> int {
    if (c->stage < 4) return fail(c, PMLBIE_ESTATE, "evaluate_field: solve first");
    if (n_pts < 0 || (n_pts > 0 && (!rtz || !out))) return fail(c, PMLBIE_EINVAL, "evaluate_field: bad arguments");
    if (n_pts == 0) return PMLBIE_OK;
    const int N = c->N, M = c->M;
    if (M - c->m0 + 1 > FIELD_MAX_MODES) return fail(c, PMLBIE_EINVAL, "evaluate_field: too many modes");
    std::vector<int> med(n_pts);
    std::vector<double> th(n_pts);
    for (int p = 0; p < n_pts; ++p) {
      const double r = rtz[3 * p], zz = rtz[3 * p + 2];
      th[p] = rtz[3 * p + 1];
      if (!(r >= 0) || r >= c->geo.pml.a1) return fail(c, PMLBIE_EINVAL, "evaluate_field: points must lie in the physical region rho < a1");
      med[p] = c->geo.above(r, zz) ? 1 : 2;
    }
    DBuf<int> dmed;
    DBuf<double> dth;
    DBuf<zd> dout;
    dmed.alloc(n_pts);
    dth.alloc(n_pts);
    dout.alloc((size_t)n_pts * c->nrhs);
    HIPCHK(hipMemcpyAsync(dmed.p, med.data(), n_pts * sizeof(int), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(dth.p, th.data(), n_pts * 8, hipMemcpyHostToDevice, c->stream));
    // points in chunks whose modal kernels against every node take about 2 GiB
    const long per_pt = (long)N * 4 * (M + 1) * (long)sizeof(zd);
    const int chunk = (int)std::max(1L, std::min((long)n_pts, (2L << 30) / per_pt));
    std::vector<double> hpts(2L * chunk);
    DBuf<double> dpts;
    dpts.alloc(2L * chunk);
    NodesDev nd;
    nd.N = N;
    nd.rho = c->nodes.p;
    nd.I = c->nodes.p + N;
    nd.z = c->nodes.p + 2L * N;
    nd.W = c->nodes.p + 3L * N;
    nd.nr_re = c->nodes.p + 4L * N;
    nd.nr_im = c->nodes.p + 5L * N;
    nd.nz_re = c->nodes.p + 6L * N;
    nd.nz_im = c->nodes.p + 7L * N;
    nd.panel = c->dpanel.p;
    // points closer to a panel than its arclength: that panel's entries by
    // product integration (same interval cap as the build's near panels)
    const double keff = std::max(cabs_(c->k1), cabs_(c->k2)) * sqrt(1.0 + c->geo.pml.S * c->geo.pml.S);
    const double near_hmax = keff > 0.0 ? 4.0 / keff : 1e300;
    std::vector<PairGeom> fg;
    std::vector<double> fc;
    std::vector<NearJob> fj;
    DBuf<zd> fraw;
    DBuf<double> fcoef;
    DBuf<NearJob> fjobs;
    for (int p0 = 0; p0 < n_pts; p0 += chunk) {
      const int np = std::min(chunk, n_pts - p0);
      fg.clear();
      fc.clear();
      fj.clear();
      for (int p = p0; p < p0 + np; ++p)
        c->geo.field_near(rtz[3 * p], rtz[3 * p + 2], p - p0, 1.0, near_hmax, fg, fc, fj);
      for (const NearJob& J : fj)
        if (J.target < 0 || J.target >= np || J.panel < 0 || 16L * J.panel + 15 >= N || J.q0 < 0 ||
            J.q1 > (int)fg.size() || J.q0 > J.q1)
          return fail(c, PMLBIE_EDEVICE, "evaluate_field: inconsistent near-curve tables");
      // the point x node pair geometry is formed on the device from the
      // node tables already there
      for (int p = 0; p < np; ++p) {
        hpts[2 * p] = rtz[3 * (p0 + p)];
        hpts[2 * p + 1] = rtz[3 * (p0 + p) + 2];
      }
      HIPCHK(hipMemcpyAsync(dpts.p, hpts.data(), 2L * np * sizeof(double), hipMemcpyHostToDevice, c->stream));
      const size_t tot = (size_t)np * N;
      c->xgeom.alloc(tot);
      launch_field_pairs(nd, dpts.p, np, c->xgeom.p, c->stream);
      HIPCHK(hipGetLastError());
      c->raw.alloc(tot * 4 * (M + 1));
      run_pair_list_dev(c, tot, c->raw.p, nullptr, dmed.p + p0, N);  // synchronous: hpts may be reused
      if (!fj.empty()) {
        fraw.alloc(fg.size() * 4 * (M + 1));
        run_pair_list(c, fg, fraw.p, nullptr);
        fcoef.alloc(fc.size());
        fjobs.alloc(fj.size());
        HIPCHK(hipMemcpyAsync(fcoef.p, fc.data(), fc.size() * 8, hipMemcpyHostToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(fjobs.p, fj.data(), fj.size() * sizeof(NearJob), hipMemcpyHostToDevice,
                              c->stream));
        launch_field_near(fjobs.p, (int)fj.size(), fcoef.p, fraw.p, N, M, c->raw.p, c->stream);
        HIPCHK(hipGetLastError());
        // the host tables are refilled for the next chunk
        HIPCHK(hipStreamSynchronize(c->stream));
      }
      launch_field(c->raw.p, c->nodes.p + 3L * N, N, M, c->m0, c->nrhs, np, dmed.p + p0, dth.p + p0,
                   c->u1.p, c->p1.p, c->u2.p, c->p2.p, dout.p + p0, n_pts, c->stream);
      HIPCHK(hipGetLastError());
    }
    HIPCHK(hipMemcpyAsync(out, dout.p, (size_t)n_pts * c->nrhs * sizeof(zd), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return PMLBIE_OK;
  });
}

int pmlbie_get_info(const pmlbie_ctx* c, long long* info) {
  if (!c || !info) return PMLBIE_EINVAL;
  info[0] = c->N;
  info[1] = c->M;
  info[2] = c->nt_int;
  info[3] = c->nt_far;
  info[4] = c->cnt_far;
  info[5] = c->cnt_split;
  info[6] = c->cnt_direct;
  info[7] = c->cnt_aux;
  info[8] = c->B;
  return PMLBIE_OK;
}

int pmlbie_get_nodes(const pmlbie_ctx* c, double* out) {
  if (!c || !out) return PMLBIE_EINVAL;
  if (c->stage < 2) return PMLBIE_ESTATE;
  const Geometry& g = c->geo;
  for (int i = 0; i < g.n(); ++i) {
    double* o = out + 13L * i;
    o[0] = g.rho[i]; o[1] = g.I[i]; o[2] = g.z[i];
    o[3] = g.nr_re[i]; o[4] = g.nr_im[i]; o[5] = g.nz_re[i]; o[6] = g.nz_im[i];
    o[7] = g.W[i]; o[8] = g.panel[i]; o[9] = g.t[i]; o[10] = g.nur[i]; o[11] = g.nuz[i]; o[12] = g.jac[i];
  }
  return PMLBIE_OK;
}

int pmlbie_modal_kernels(pmlbie_ctx* c, int n_pairs, const double* geom, void* d_out) {
  return guarded(c, [&]() -> int {
    if (c->stage < 3) return fail(c, PMLBIE_ESTATE, "modal_kernels: build the operators first");
    if (n_pairs < 0 || (n_pairs > 0 && (!geom || !d_out))) return fail(c, PMLBIE_EINVAL, "modal_kernels: bad arguments");
    if (n_pairs == 0) return PMLBIE_OK;
    std::vector<PairGeom> g(n_pairs);
    for (int q = 0; q < n_pairs; ++q) {
      const double* s = geom + 12L * q;
      g[q].rt = zd{s[0], s[1]};
      g[q].rs = zd{s[2], s[3]};
      g[q].drho = zd{s[4], s[5]};
      g[q].dz = zd{s[6], s[7]};
      g[q].nr = zd{s[8], s[9]};
      g[q].nz = zd{s[10], s[11]};
    }
    run_pair_list(c, g, (zd*)d_out, nullptr);
    return PMLBIE_OK;
  });
}

int pmlbie_modal_kernels_noalloc(pmlbie_ctx* c, int n_pairs, const double* geom, void* d_out) {
  return guarded(c, [&]() -> int {
    if (c->stage < 3) return fail(c, PMLBIE_ESTATE, "modal_kernels_noalloc: build the operators first");
    if (n_pairs < 0 || (n_pairs > 0 && (!geom || !d_out)))
      return fail(c, PMLBIE_EINVAL, "modal_kernels_noalloc: bad arguments");
    if (n_pairs > kNaMaxPairs)
      return fail(c, PMLBIE_EINVAL, "modal_kernels_noalloc: " + std::to_string(n_pairs) +
                                        " pairs exceed the scratch limit of " + std::to_string(kNaMaxPairs));
    if (c->MQ + 1 > kNaMaxModesQ) return fail(c, PMLBIE_EINVAL, "modal_kernels_noalloc: angle grid too long");
    if (n_pairs == 0) return PMLBIE_OK;
    unsigned char* sp = g_scratch[c->device];
    if (!sp) return fail(c, PMLBIE_EDEVICE, "modal_kernels_noalloc: no scratch on this device");
    const long np = n_pairs;
    PairGeom* geo = reinterpret_cast<PairGeom*>(sp + kNaGeom);
    PairGeom* lg = reinterpret_cast<PairGeom*>(sp + kNaLGeom);
    int2* ld = reinterpret_cast<int2*>(sp + kNaLDest);
    unsigned* cnt = reinterpret_cast<unsigned*>(sp + kNaCount);
    zd* qtab = reinterpret_cast<zd*>(sp + kNaQtab);
    zd* zhat = reinterpret_cast<zd*>(sp + kNaZhat);
    zd* phat = reinterpret_cast<zd*>(sp + kNaPhat);
    zd* qcoef = reinterpret_cast<zd*>(sp + kNaCoef);
    zd* raw = reinterpret_cast<zd*>(d_out);
    // the host records (rho~_t, rho~_s, drho~, dz~, n_rho, n_z) are PairGeom
    HIPCHK(hipMemcpyAsync(geo, geom, np * sizeof(PairGeom), hipMemcpyHostToDevice, c->stream));
    launch_fill_u32(cnt, 4, 0u, c->stream);
    WorkList wf{lg, ld, cnt, (unsigned)np};
    WorkList ws{lg + np, ld + np, cnt + 1, (unsigned)np};
    WorkList wd{lg + 2 * np, ld + 2 * np, cnt + 2, (unsigned)np};
    // c->cp has no split on a shorter grid, so the fourth list stays empty
    // (capacity 0: nothing is ever written to it)
    WorkList wnone{lg, ld, cnt + 3, 0u};
    launch_classify_list(geo, np, c->cp, wf, ws, wd, wnone, c->stream);
    HIPCHK(hipGetLastError());
    unsigned h[3];
    HIPCHK(hipMemcpy(h, cnt, sizeof(h), hipMemcpyDeviceToHost));
    launch_list_far(c->nt_far, wf.geom, wf.dest, 0, h[0], c->M, 0, c->k1, c->k2, c->tw_far.p, nullptr, 0, 0,
                    nullptr, raw, nullptr, c->stream);
    HIPCHK(hipGetLastError());
    for (long f = 0; f < (long)h[1]; f += kNaSplitChunk) {
      const long cn = std::min<long>(kNaSplitChunk, (long)h[1] - f);
      launch_split_singular(ws.geom, f, cn, c->MQ, qtab, qcoef, zhat, phat, c->stream);
      HIPCHK(hipGetLastError());
      launch_split(c->nt_int, ws.geom, ws.dest, f, cn, c->M, 0, c->MQ, c->k1, c->k2, c->tw_int.p, zhat, phat,
                   nullptr, 0, 0, nullptr, raw, c->stream);
      HIPCHK(hipGetLastError());
    }
    if (c->ch1_L > 0) {
      for (long f = 0; f < (long)h[2]; f += kNaSplitChunk) {
        const long cn = std::min<long>(kNaSplitChunk, (long)h[2] - f);
        launch_split_singular(wd.geom, f, cn, c->MQ, qtab, qcoef, zhat, phat, c->stream);
        HIPCHK(hipGetLastError());
        launch_split(c->nt_int, wd.geom, wd.dest, f, cn, c->M, 0, c->MQ, c->k1, c->k2, c->tw_int.p, zhat, phat,
                     nullptr, 0, 0, nullptr, raw, c->stream, c->ch1_L);
      }
    } else {
      launch_direct(wd.geom, wd.dest, 0, h[2], c->M, 0, c->k1, c->k2, c->glx.p, c->glw.p, nullptr, 0, 0, nullptr,
                    raw, kOmegaPiece, c->stream);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    return PMLBIE_OK;
  });
}

int pmlbie_get_operator(pmlbie_ctx* c, int mode, void* d_out) {
  return guarded(c, [&]() -> int {
    if (c->stage < 3) return fail(c, PMLBIE_ESTATE, "get_operator: build first");
    // in mixed precision the FP64 operator is kept unfactored anyway
    const zd* src = c->precision == PMLBIE_MIXED ? c->A.p : c->Akeep.p;
    if (!src) return fail(c, PMLBIE_ESTATE, "get_operator: build with PMLBIE_KEEP_OPERATORS");
    if (mode < c->m0 || mode > c->M || !d_out) return fail(c, PMLBIE_EINVAL, "get_operator: mode outside the build");
    const size_t ms = (size_t)4 * c->N * c->N;
    // stored interleaved (node by node); returned in the block order of the ABI
    launch_deinterleave(src + (size_t)(mode - c->m0) * ms, 2L * c->N, (zd*)d_out, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    return PMLBIE_OK;
  });
}

int pmlbie_set_refinement(pmlbie_ctx* c, double tol, int max_iter) {
  if (!c) return PMLBIE_EINVAL;
  if (!(tol > 0.0 && tol < 1.0) || max_iter < 1 || max_iter > 100)
    return fail(c, PMLBIE_EINVAL, "set_refinement: need 0 < tol < 1 and 1 <= max_iter <= 100");
  c->ref_tol = tol;
  c->ref_maxit = max_iter;
  return PMLBIE_OK;
}

int pmlbie_set_ch1_substitution(pmlbie_ctx* c, int order) {
  if (!c) return PMLBIE_EINVAL;
  if (order < 0 || order > 12) return fail(c, PMLBIE_EINVAL, "set_ch1_substitution: order must be 0..12");
  c->ch1_L = order;
  return PMLBIE_OK;
}

int pmlbie_test_zero_column(pmlbie_ctx* c, int mode, int col) {
  if (!c) return PMLBIE_EINVAL;
  if (c->stage < 2) return fail(c, PMLBIE_ESTATE, "test_zero_column: set geometry and media first");
  if (mode < 0 || col < 0 || col >= 2 * c->N)
    return fail(c, PMLBIE_EINVAL, "test_zero_column: need mode >= 0 and 0 <= col < 2N");
  c->zc_mode = mode;
  c->zc_col = col;
  return PMLBIE_OK;
}

int pmlbie_get_stats(const pmlbie_ctx* c, double* stage_ms, double* counters) {
  if (!c) return PMLBIE_EINVAL;
  if (stage_ms) memcpy(stage_ms, c->stage_ms, sizeof(c->stage_ms));
  if (counters) memcpy(counters, c->counters, sizeof(c->counters));
  return PMLBIE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Learned surrogate (training, persistence, test hooks).
namespace {

// splitmix64 (Steele, Lea and Flood 2014): seeded uniform draws for the
// surrogate's initial weights and training geometries.
struct Rng {
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed) {}
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double u() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

struct SgHeader {
  char magic[8];
  int version, p;
  double a1, T;
  long nparams;
};

}  // namespace

extern "C" {

long pmlbie_surrogate_nparams(void) { return SgLayout().total; }

int pmlbie_surrogate_init(pmlbie_ctx* c, unsigned long long seed) {
  return guarded(c, [&]() -> int {
    if (c->stage < 2) return fail(c, PMLBIE_ESTATE, "surrogate_init: set geometry and media first");
    sg_free(c->sg);
    c->sg_ready = false;
    HIPCHK(sg_alloc(c->sg));
    SgLayout L;
    std::vector<float> p(L.total, 0.0f);
    Rng r(seed);
    for (int l = 0; l < SG_NL; ++l) {
      const int fin = l == 0 ? SG_NF : SG_D[l], fout = l == SG_NL - 1 ? SG_OUT : SG_D[l + 1];
      const double a = sqrt(6.0 / (fin + fout));
      for (int o = 0; o < fout; ++o)
        for (int i = 0; i < fin; ++i) p[L.w[l] + (long)o * SG_D[l] + i] = (float)(a * (2.0 * r.u() - 1.0));
    }
    HIPCHK(hipMemcpy(c->sg.p, p.data(), p.size() * sizeof(float), hipMemcpyHostToDevice));
    sg_refresh_bf16(c->sg, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    c->sg_a1 = c->geo.pml.a1;
    c->sg_T = c->geo.pml.T;
    c->sg_p = c->geo.pml.p;
    c->sg_ready = true;
    return PMLBIE_OK;
  });
}

int pmlbie_surrogate_make_samples(pmlbie_ctx* c, int which, long n, unsigned long long seed) {
  return guarded(c, [&]() -> int {
    if (which != 0 && which != 1) return fail(c, PMLBIE_EINVAL, "surrogate_make_samples: which is 0 or 1");
    if (n <= 0 || n > (1L << 24)) return fail(c, PMLBIE_EINVAL, "surrogate_make_samples: 0 < n <= 2^24");
    if (!c->sg_ready) return fail(c, PMLBIE_ESTATE, "surrogate_make_samples: no network");
    Rng r(seed);
    std::vector<SgSample> smp(n);
    std::vector<double> x((size_t)SG_IN * n);
    const double a1 = c->sg_a1, T = c->sg_T;
    long q = 0;
    while (q < n) {
      // one interface z = a exp(-(rho / w)^2) at the paper-scale resolution
      Geometry g;
      g.itf.amp = {0.6 * r.u()};
      g.itf.cen = {0.0};
      g.itf.wid = {0.5 + 1.5 * r.u()};
      g.itf.cos_freq = 0.0;
      g.itf.rho_c = a1;
      g.pml.a1 = a1;
      g.pml.T = T;
      g.pml.S = 1.0;  // Im rho~ is linear in S
      g.pml.p = c->sg_p;
      g.breaks = {0.0, 0.5 * a1, a1, a1 + 0.5 * T, a1 + T};
      g.nodes_per_segment = 512;
      g.build();
      const int N = g.n();
      for (long t = 0; t < 16384 && q < n;) {
        const int i = std::min(N - 1, (int)(r.u() * N)), l = std::min(N - 1, (int)(r.u() * N));
        const double h = 1.2 * std::max(g.pl[g.panel[i]], g.pl[g.panel[l]]);
        const double dr = g.rho[i] - g.rho[l], dz = g.z[i] - g.z[l];
        if (dr * dr + dz * dz <= 4.0 * h * h) continue;  // separation > 2 h
        const double S = 1.0 + 3.0 * r.u();
        const double k1 = 5.0 + 10.0 * r.u();
        const double k = r.u() < 0.5 ? k1 : k1 * (1.2 + 0.8 * r.u());
        smp[q] = SgSample{g.rho[i], S * g.I[i], g.rho[l], S * g.I[l], dz, k};
        const double xs[SG_IN] = {g.rho[i], g.rho[l], dz, k, S, S * g.I[i], S * g.I[l]};
        for (int j = 0; j < SG_IN; ++j) x[SG_IN * q + j] = xs[j];
        ++q;
        ++t;
      }
    }
    for (long a = n - 1; a > 0; --a) {  // shuffle the geometries together
      const long b = std::min(a, (long)(r.u() * (a + 1)));
      std::swap(smp[a], smp[b]);
      for (int j = 0; j < SG_IN; ++j) std::swap(x[SG_IN * a + j], x[SG_IN * b + j]);
    }
    DBuf<SgSample> ds;
    ds.alloc(n);
    HIPCHK(hipMemcpy(ds.p, smp.data(), n * sizeof(SgSample), hipMemcpyHostToDevice));
    const int L = 512;
    auto tw = twiddles(L, true);
    c->sgtw.alloc(tw.size());
    HIPCHK(hipMemcpy(c->sgtw.p, tw.data(), tw.size() * sizeof(zd), hipMemcpyHostToDevice));
    c->sgT[which].alloc((size_t)n * SG_OUT);
    c->sgx[which].alloc((size_t)n * SG_IN);
    HIPCHK(hipMemcpy(c->sgx[which].p, x.data(), x.size() * sizeof(double), hipMemcpyHostToDevice));
    sg_label(ds.p, n, L, c->sgtw.p, c->sgT[which].p, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    c->sgn[which] = n;
    return PMLBIE_OK;
  });
}

int pmlbie_surrogate_train(pmlbie_ctx* c, int steps, int batch, double lr, double* loss_out) {
  return guarded(c, [&]() -> int {
    if (!c->sg_ready) return fail(c, PMLBIE_ESTATE, "surrogate_train: no network");
    if (steps < 0 || batch < 64 || batch > 65536 || !(lr > 0))
      return fail(c, PMLBIE_EINVAL, "surrogate_train: steps >= 0, 64 <= batch <= 65536, lr > 0");
    const long n = c->sgn[0];
    if (n < batch) return fail(c, PMLBIE_ESTATE, "surrogate_train: fewer training samples than a batch");
    HIPCHK(sg_work_alloc(c->sgw, batch));
    DBuf<double> lsum;
    lsum.alloc(std::max(steps, 1));
    SgFeat f{c->sg_a1 + c->sg_T};
    for (int s = 0; s < steps; ++s) {
      long off = ((long)s * batch) % n;
      if (off + batch > n) off = 0;
      // cosine decay of the step size from lr to lr / 20
      const double lr_s = lr * (0.05 + 0.475 * (1.0 + cos(PMLBIE_PI * s / std::max(steps, 1))));
      sg_features(c->sgx[0].p + (long)SG_IN * off, batch, f, c->sgw, c->stream);
      sg_forward(c->sg, c->sgw, batch, c->stream);
      sg_backward(c->sg, c->sgw, batch, c->sgT[0].p + (long)SG_OUT * off, c->stream);
      sg_adam(c->sg, lr_s, c->stream);
      HIPCHK(hipMemcpyAsync(lsum.p + s, c->sgw.loss, sizeof(double), hipMemcpyDeviceToDevice, c->stream));
      HIPCHK(hipGetLastError());
    }
    std::vector<double> h(std::max(steps, 1));
    HIPCHK(hipMemcpy(h.data(), lsum.p, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    if (loss_out)
      for (int s = 0; s < steps; ++s) loss_out[s] = h[s] / ((double)batch * SG_OUT);
    return PMLBIE_OK;
  });
}

int pmlbie_surrogate_eval(pmlbie_ctx* c, int which, double* mse) {
  return guarded(c, [&]() -> int {
    if (which != 0 && which != 1) return fail(c, PMLBIE_EINVAL, "surrogate_eval: which is 0 or 1");
    if (!c->sg_ready || c->sgn[which] <= 0) return fail(c, PMLBIE_ESTATE, "surrogate_eval: no network or samples");
    const long n = c->sgn[which], CH = 1L << 15;
    HIPCHK(sg_work_alloc(c->sgw, (int)CH));
    SgFeat f{c->sg_a1 + c->sg_T};
    double tot = 0.0;
    for (long off = 0; off < n; off += CH) {
      const int cn = (int)std::min(CH, n - off);
      sg_features(c->sgx[which].p + (long)SG_IN * off, cn, f, c->sgw, c->stream);
      sg_forward(c->sg, c->sgw, cn, c->stream);
      sg_loss(c->sgw, cn, c->sgT[which].p + (long)SG_OUT * off, c->stream);
      double l = 0;
      HIPCHK(hipMemcpy(&l, c->sgw.loss, sizeof(double), hipMemcpyDeviceToHost));
      tot += l;
    }
    if (mse) *mse = tot / ((double)n * SG_OUT);
    return PMLBIE_OK;
  });
}

int pmlbie_surrogate_eval_modes(pmlbie_ctx* c, int which, double* rel) {
  return guarded(c, [&]() -> int {
    if (which != 0 && which != 1) return fail(c, PMLBIE_EINVAL, "surrogate_eval_modes: which is 0 or 1");
    if (!rel) return fail(c, PMLBIE_EINVAL, "surrogate_eval_modes: null output");
    if (!c->sg_ready || c->sgn[which] <= 0)
      return fail(c, PMLBIE_ESTATE, "surrogate_eval_modes: no network or samples");
    const long n = c->sgn[which], CH = 1L << 15;
    HIPCHK(sg_work_alloc(c->sgw, (int)CH));
    DBuf<double> acc;
    acc.alloc(2 * SG_MODES);
    HIPCHK(hipMemsetAsync(acc.p, 0, 2 * SG_MODES * sizeof(double), c->stream));
    SgFeat f{c->sg_a1 + c->sg_T};
    for (long off = 0; off < n; off += CH) {
      const int cn = (int)std::min(CH, n - off);
      sg_features(c->sgx[which].p + (long)SG_IN * off, cn, f, c->sgw, c->stream);
      sg_forward(c->sg, c->sgw, cn, c->stream);
      sg_mode_errors(c->sgw.z[SG_NL - 1], c->sgT[which].p + (long)SG_OUT * off, cn, acc.p, acc.p + SG_MODES,
                     c->stream);
      HIPCHK(hipGetLastError());
    }
    double h[2 * SG_MODES];
    HIPCHK(hipMemcpy(h, acc.p, sizeof(h), hipMemcpyDeviceToHost));
    for (int m = 0; m < SG_MODES; ++m) rel[m] = h[SG_MODES + m] > 0 ? sqrt(h[m] / h[SG_MODES + m]) : 0.0;
    return PMLBIE_OK;
  });
}

int pmlbie_surrogate_set_tolerance(pmlbie_ctx* c, double tol) {
  if (!c) return PMLBIE_EINVAL;
  if (!(tol >= 0)) return fail(c, PMLBIE_EINVAL, "surrogate_set_tolerance: tol >= 0");
  c->sg_tol = tol;
  return PMLBIE_OK;
}

int pmlbie_surrogate_save(pmlbie_ctx* c, void* blob, size_t* bytes) {
  return guarded(c, [&]() -> int {
    if (!bytes) return fail(c, PMLBIE_EINVAL, "surrogate_save: bytes is null");
    if (!c->sg_ready) return fail(c, PMLBIE_ESTATE, "surrogate_save: no network");
    SgLayout L;
    const size_t need = sizeof(SgHeader) + (size_t)L.total * sizeof(float);
    if (!blob) {
      *bytes = need;
      return PMLBIE_OK;
    }
    if (*bytes < need) return fail(c, PMLBIE_EINVAL, "surrogate_save: buffer too small");
    SgHeader hd{};
    memcpy(hd.magic, "PMLBIESG", 8);
    hd.version = 1;
    hd.p = c->sg_p;
    hd.a1 = c->sg_a1;
    hd.T = c->sg_T;
    hd.nparams = L.total;
    memcpy(blob, &hd, sizeof(hd));
    HIPCHK(hipMemcpy((char*)blob + sizeof(hd), c->sg.p, (size_t)L.total * sizeof(float), hipMemcpyDeviceToHost));
    *bytes = need;
    return PMLBIE_OK;
  });
}

int pmlbie_surrogate_load(pmlbie_ctx* c, const void* blob, size_t bytes) {
  return guarded(c, [&]() -> int {
    SgLayout L;
    SgHeader hd{};
    if (!blob || bytes < sizeof(hd)) return fail(c, PMLBIE_EINVAL, "surrogate_load: short blob");
    memcpy(&hd, blob, sizeof(hd));
    if (memcmp(hd.magic, "PMLBIESG", 8) != 0 || hd.version != 1 || hd.nparams != L.total ||
        bytes < sizeof(hd) + (size_t)L.total * sizeof(float))
      return fail(c, PMLBIE_EINVAL, "surrogate_load: not a surrogate blob of this layout");
    sg_free(c->sg);
    c->sg_ready = false;
    HIPCHK(sg_alloc(c->sg));
    HIPCHK(hipMemcpy(c->sg.p, (const char*)blob + sizeof(hd), (size_t)L.total * sizeof(float),
                     hipMemcpyHostToDevice));
    sg_refresh_bf16(c->sg, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    c->sg_a1 = hd.a1;
    c->sg_T = hd.T;
    c->sg_p = hd.p;
    c->sg_ready = true;
    return PMLBIE_OK;
  });
}

int pmlbie_surrogate_params(pmlbie_ctx* c, double* p, int get) {
  return guarded(c, [&]() -> int {
    if (!p) return fail(c, PMLBIE_EINVAL, "surrogate_params: null buffer");
    if (!c->sg_ready) return fail(c, PMLBIE_ESTATE, "surrogate_params: no network");
    SgLayout L;
    std::vector<float> f(L.total);
    if (get) {
      HIPCHK(hipMemcpy(f.data(), c->sg.p, f.size() * sizeof(float), hipMemcpyDeviceToHost));
      for (long i = 0; i < L.total; ++i) p[i] = f[i];
    } else {
      for (long i = 0; i < L.total; ++i) f[i] = (float)p[i];
      HIPCHK(hipMemcpy(c->sg.p, f.data(), f.size() * sizeof(float), hipMemcpyHostToDevice));
      sg_refresh_bf16(c->sg, c->stream);
      HIPCHK(hipGetLastError());
      HIPCHK(hipStreamSynchronize(c->stream));
    }
    return PMLBIE_OK;
  });
}

int pmlbie_surrogate_forward(pmlbie_ctx* c, int n, const double* x, double* y) {
  return guarded(c, [&]() -> int {
    if (n <= 0 || n > 65536 || !x || !y) return fail(c, PMLBIE_EINVAL, "surrogate_forward: 0 < n <= 65536");
    if (!c->sg_ready) return fail(c, PMLBIE_ESTATE, "surrogate_forward: no network");
    HIPCHK(sg_work_alloc(c->sgw, n));
    DBuf<double> dx;
    dx.alloc((size_t)n * SG_IN);
    HIPCHK(hipMemcpy(dx.p, x, (size_t)n * SG_IN * sizeof(double), hipMemcpyHostToDevice));
    SgFeat f{c->sg_a1 + c->sg_T};
    sg_features(dx.p, n, f, c->sgw, c->stream);
    sg_forward(c->sg, c->sgw, n, c->stream);
    HIPCHK(hipGetLastError());
    std::vector<float> h((size_t)n * SG_D[SG_NL]);
    HIPCHK(hipStreamSynchronize(c->stream));
    HIPCHK(hipMemcpy(h.data(), c->sgw.z[SG_NL - 1], h.size() * sizeof(float), hipMemcpyDeviceToHost));
    for (long r = 0; r < n; ++r)
      for (int j = 0; j < SG_OUT; ++j) y[r * SG_OUT + j] = h[r * SG_D[SG_NL] + j];
    return PMLBIE_OK;
  });
}

int pmlbie_surrogate_grad(pmlbie_ctx* c, int n, const double* x, const double* t, double* loss,
                          double* grad) {
  return guarded(c, [&]() -> int {
    if (n <= 0 || n > 65536 || !x || !t || !grad) return fail(c, PMLBIE_EINVAL, "surrogate_grad: 0 < n <= 65536");
    if (!c->sg_ready) return fail(c, PMLBIE_ESTATE, "surrogate_grad: no network");
    SgLayout L;
    HIPCHK(sg_work_alloc(c->sgw, n));
    DBuf<double> dx;
    dx.alloc((size_t)n * SG_IN);
    DBuf<float> dt;
    dt.alloc((size_t)n * SG_OUT);
    std::vector<float> tf((size_t)n * SG_OUT);
    for (size_t i = 0; i < tf.size(); ++i) tf[i] = (float)t[i];
    HIPCHK(hipMemcpy(dx.p, x, (size_t)n * SG_IN * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(dt.p, tf.data(), tf.size() * sizeof(float), hipMemcpyHostToDevice));
    SgFeat f{c->sg_a1 + c->sg_T};
    sg_features(dx.p, n, f, c->sgw, c->stream);
    sg_forward(c->sg, c->sgw, n, c->stream);
    sg_backward(c->sg, c->sgw, n, dt.p, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    std::vector<float> g(L.total);
    HIPCHK(hipMemcpy(g.data(), c->sg.g, g.size() * sizeof(float), hipMemcpyDeviceToHost));
    for (long i = 0; i < L.total; ++i) grad[i] = g[i];
    double l = 0;
    HIPCHK(hipMemcpy(&l, c->sgw.loss, sizeof(double), hipMemcpyDeviceToHost));
    if (loss) *loss = l / ((double)n * SG_OUT);
    return PMLBIE_OK;
  });
}

int pmlbie_surrogate_label(pmlbie_ctx* c, int n, const double* s, double* y) {
  return guarded(c, [&]() -> int {
    if (n <= 0 || n > (1 << 20) || !s || !y) return fail(c, PMLBIE_EINVAL, "surrogate_label: 0 < n <= 2^20");
    std::vector<SgSample> smp(n);
    for (int q = 0; q < n; ++q) smp[q] = SgSample{s[6 * q], s[6 * q + 1], s[6 * q + 2], s[6 * q + 3], s[6 * q + 4], s[6 * q + 5]};
    DBuf<SgSample> ds;
    ds.alloc(n);
    HIPCHK(hipMemcpy(ds.p, smp.data(), n * sizeof(SgSample), hipMemcpyHostToDevice));
    auto tw = twiddles(512, true);
    c->sgtw.alloc(tw.size());
    HIPCHK(hipMemcpy(c->sgtw.p, tw.data(), tw.size() * sizeof(zd), hipMemcpyHostToDevice));
    DBuf<float> dt;
    dt.alloc((size_t)n * SG_OUT);
    sg_label(ds.p, n, 512, c->sgtw.p, dt.p, c->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(c->stream));
    std::vector<float> h((size_t)n * SG_OUT);
    HIPCHK(hipMemcpy(h.data(), dt.p, h.size() * sizeof(float), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < h.size(); ++i) y[i] = h[i];
    return PMLBIE_OK;
  });
}

}  // extern "C"
