/*
 * pmlbie: FFT-accelerated PML boundary-integral solver for axisymmetric
 * two-layer acoustic scattering on one MI355X (gfx950).  C ABI.
 *
 * The method is that of Wang & Lu, "An FFT-accelerated PML-BIE solver for
 * three-dimensional acoustic wave scattering in layered media"
 * (arXiv 2412.11162):
 *   - problem: two homogeneous media separated by the axisymmetric interface
 *     z = h~(rho), Helmholtz equation with wavenumbers k1 (upper) and k2
 *     (lower), continuity of u and du/dnu across the interface (Sec. 2);
 *   - cylindrical PML by complex stretching rho~ = rho + i int sigma_1
 *     (Sec. 3.1, eqs. eqrhot, eqsgm1), truncation of the interface at the
 *     outer PML edge rho = a1 + T (Sec. 3.2);
 *   - azimuthal Fourier decomposition into decoupled per-mode curve integral
 *     equations (Sec. 3.3); per-mode coupled system of the two media with the
 *     transmission conditions (Sec. 4.2).
 *
 * Conventions
 *   - Every call returns PMLBIE_OK (0) or a negative status; nothing throws
 *     or aborts across the ABI.  pmlbie_last_error() describes the last
 *     failure of a context.
 *   - Calls run in order: set_geometry (or set_polyline, set_panels) -> set_media_pml ->
 *     build_modal_operators -> solve_modes -> evaluate_field; a call out of
 *     order returns PMLBIE_ESTATE.  Changing geometry or media invalidates
 *     later stages.
 *   - Complex arrays are interleaved (re, im) doubles.  "device" pointers are
 *     HIP device memory on the context's device (for example the data of a
 *     PyTorch tensor); "host" pointers are ordinary memory.
 *   - All work is ordered on the stream given to pmlbie_create; every call is
 *     synchronous on return.  A context is used by one host thread at a time.
 *   - Modes are natural: F_n = int_{-pi}^{pi} e^{-i n theta} F dtheta, which
 *     is sqrt(2 pi) times the paper's normalised mode (Sec. 3.3, eq. fmode1);
 *     only n = 0..m_max are stored since every quantity here is even in n.
 *   - The context owns all internal device buffers (operators, factors,
 *     work lists).  Output buffers belong to the caller.
 */
#ifndef PMLBIE_H
#define PMLBIE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pmlbie_ctx pmlbie_ctx;

enum {
  PMLBIE_OK = 0,
  PMLBIE_EINVAL = -1,    /* bad argument */
  PMLBIE_ESTATE = -2,    /* call out of order */
  PMLBIE_ENOMEM = -3,    /* device allocation failed */
  PMLBIE_EDEVICE = -4,   /* HIP runtime error */
  PMLBIE_ESINGULAR = -5, /* exactly singular mode matrix (zero pivot) */
  PMLBIE_ENOCONV = -6    /* iterative refinement did not converge */
};

enum { PMLBIE_FP64 = 0, PMLBIE_MIXED = 1 };
enum { PMLBIE_KEEP_OPERATORS = 1, PMLBIE_USE_SURROGATE = 2 };

/* Create a context on HIP device `device`, ordering work on `stream`
 * (a hipStream_t; NULL = the default stream).  *out receives the context. */
int pmlbie_create(pmlbie_ctx** out, int device, void* stream);
void pmlbie_destroy(pmlbie_ctx* ctx);
const char* pmlbie_last_error(const pmlbie_ctx* ctx);

/* Generating curve (Sec. 2, Sec. 4): the graph z = h~(rho) of
 *   h(rho) = [sum_i a_i exp(-((rho - c_i)/w_i)^2)] * (cos(f rho) if f != 0),
 *   h~ = h - h(rho_c) for rho < rho_c and 0 beyond (flat where the PML acts),
 * from the axis to rho = seg_breaks[4].  bumps: host, 3*n_bumps doubles
 * (a_i, c_i, w_i); seg_breaks: host, 5 increasing rho values with
 * seg_breaks[0] = 0; each of the four segments carries nodes_per_segment
 * Gauss-Legendre nodes in equal sub-panels of 16 (a positive multiple of 16).
 * N = 4 * nodes_per_segment nodes; node i lies on panel i / 16.
 * Errors: PMLBIE_EINVAL for n_bumps outside [0, 8], non-positive widths,
 * non-increasing breaks, nodes_per_segment not a multiple of 16. */
int pmlbie_set_geometry(pmlbie_ctx* ctx, int n_bumps, const double* bumps, double cos_freq,
                        double rho_c, const double* seg_breaks, int nodes_per_segment);

/* Generating curve with corners (Sec. 4: piecewise smooth curves, corner
 * singularities resolved by a graded mesh, eq. eqsxi; Sec. 5, Examples 1 and
 * 3): the polyline through n_vert vertices (rho_j, z_j), host array
 * verts[2 * n_vert] = rho_0, z_0, rho_1, z_1, ..., run from the axis
 * (rho_0 = 0) outward; every later vertex has rho > 0.  Segment j (vertex j
 * to j + 1) is cut into panels[j] equal panels of 16 Gauss-Legendre nodes;
 * at every corner (an interior vertex where the direction changes) the panel
 * touching it is cut again at the fractions 2^-grade, ..., 1/4, 1/2 of its
 * length measured from the corner, which clusters the nodes geometrically
 * toward the corner.  Node i lies on panel i / 16, panels in curve order.
 * The unit normal (z', -rho') / |r'| points into the lower medium.  The
 * curve must be flat (z = 0) where rho > a1, with a vertex at rho = a1, and
 * end at rho = a1 + T (checked by pmlbie_set_media_pml).
 * Errors: PMLBIE_EINVAL for n_vert outside [2, PMLBIE_POLY_MAX_VERTS],
 * rho_0 != 0, a later rho <= 0, a repeated vertex, panels[j] outside
 * [2, 4096], grade outside [0, 24], or a total panel count (after grading)
 * that is not a multiple of 4. */
#define PMLBIE_POLY_MAX_VERTS 64
int pmlbie_set_polyline(pmlbie_ctx* ctx, int n_vert, const double* verts, const int* panels,
                        int grade);

/* Generating curve given by its panels (any piecewise smooth curve, e.g.
 * the smooth non-graph curve of Sec. 5, Example 2, with the panels graded
 * toward its corners by the caller): nodes[32 * p + 2 * j + {0, 1}] = (rho, z)
 * of panel p at the j-th of the 16 Gauss-Legendre points of [-1, 1] (host,
 * ascending points, panels in curve order from the axis outward).  The curve
 * on a panel is the degree-15 interpolant of its nodes; consecutive panels
 * must join (to 1e-9 of the coordinates), the first must start on the axis
 * and the curve must be flat (z = 0) where rho > a1, no panel straddling a1,
 * and end at a1 + T (checked by pmlbie_set_media_pml).  The unit normal is
 * (z', -rho') / |r'|, into the lower medium.  Node i lies on panel i / 16.
 * Errors: PMLBIE_EINVAL for n_panels outside [4, PMLBIE_MAX_PANELS] or not a
 * multiple of 4, a node with rho <= 0 or non-finite, panels that do not join,
 * a curve that does not start on the axis. */
#define PMLBIE_MAX_PANELS 65536
int pmlbie_set_panels(pmlbie_ctx* ctx, int n_panels, const double* nodes);

/* Media and PML (Sec. 2, Sec. 3.1 eq. eqsgm1): wavenumbers k1 (upper medium),
 * k2 (lower medium), real or complex; radial PML from a1 with thickness T and
 * strength S; axial PML (a2, T2, S2), which never meets the curve; profile
 * order p >= 2.  The curve must end at the outer PML edge a1 + T.
 * Errors: PMLBIE_EINVAL (T <= 0, a1 <= 0, S < 0, p < 2, curve end != a1 + T,
 * a polyline that is not flat beyond a1 or has no vertex at a1),
 * PMLBIE_ESTATE (no geometry). */
int pmlbie_set_media_pml(pmlbie_ctx* ctx, double k1_re, double k1_im, double k2_re,
                         double k2_im, double a1, double T, double S, double a2, double T2,
                         double S2, int p);

/* Build the modal operators of modes n = 0..m_max (n_theta azimuthal
 * samples, a power of two >= 16; 0 <= m_max <= n_theta / 2), assemble the per-mode
 * 2N x 2N systems [[K1 + I, -S1], [K2 - I, -S2]] (Sec. 4.1-4.2) and factor
 * them (partial-pivoting LU).  The kernels are sampled on every
 * (target, source, theta) triple, split into singular and smooth parts where
 * needed (Sec. 4.1) and turned into modes by batched FFTs.
 * precision: PMLBIE_FP64 (complex128 throughout) or PMLBIE_MIXED
 * (complex64 LU with FP64 iterative refinement in solve_modes).
 * flags: PMLBIE_KEEP_OPERATORS keeps a copy of the assembled matrices for
 * pmlbie_get_operator; PMLBIE_USE_SURROGATE offers the well-separated
 * ("far") pairs to the learned surrogate first (needs a network for this PML
 * geometry and real wavenumbers): its modes 0..64 are kept where its modal
 * synthesis matches direct kernel samples at eight angles with a per-pair
 * offset to the tolerance of pmlbie_surrogate_set_tolerance; with m_max > 64
 * only pairs whose modes beyond 64 are negligible by the decay bound of the
 * classification are offered (their modes 65..m_max are zero); the
 * raw-kernel FFT takes the rest.
 * Errors: PMLBIE_EINVAL, PMLBIE_ESTATE, PMLBIE_ENOMEM, PMLBIE_EDEVICE,
 * PMLBIE_ESINGULAR (a zero pivot; pmlbie_last_error names the mode). */
int pmlbie_build_modal_operators(pmlbie_ctx* ctx, int n_theta, int m_max, int precision,
                                 int flags);

/* The same for the modes m_min..m_max only (0 <= m_min <= m_max), for mode
 * batches when the operators of all modes do not fit in device memory
 * (Sec. 4.2: the modes are independent systems).  Every pair is sampled and
 * transformed as in the full build (the FFT yields all modes at once); only
 * the kept modes are assembled and factored.  solve_modes then returns the
 * boundary data of modes m_min..m_max ([mode - m_min][rhs][node]),
 * evaluate_field sums those modes only, get_operator takes modes in the
 * range.  The surrogate needs m_min = 0. */
int pmlbie_build_modal_operators_range(pmlbie_ctx* ctx, int n_theta, int m_min, int m_max,
                                       int precision, int flags);

/* One incidence: kind 0 = point source at (rho, 0, z) = (p[0], p[1]) in the
 * upper medium (p[0] >= 0); kind 1 = plane wave with polar angle p[0]
 * (theta_inc = 0) (Sec. 2). */
typedef struct {
  int kind;
  double p[3];
} pmlbie_incidence;

/* Solve the coupled systems of all modes for n_rhs incidences (host array,
 * 1 <= n_rhs <= 16).  Outputs are device buffers of (m_max+1)*n_rhs*N
 * complex128, layout [mode][rhs][node]: u1 = scattered field of the upper
 * medium on the curve, phi1 = its conormal derivative, u2, phi2 the same for
 * the lower medium (u2 = u1 - b1, phi2 = phi1 - b2 by the transmission
 * conditions).  Any output pointer may be NULL.
 * Mixed precision refines x += LU32^{-1} (b - A64 x) in FP64 until
 * ||b - A64 x|| <= tol ||b|| for every mode and right-hand side
 * (pmlbie_set_refinement; default tol 1e-10, at most 30 iterations); the
 * iterate of the last step is returned even when it stops short.
 * Errors: PMLBIE_EINVAL, PMLBIE_ESTATE, PMLBIE_ENOCONV (mixed precision: the
 * rule was not met within the iteration cap; the outputs hold the last
 * iterate and pmlbie_last_error the residual reached). */
int pmlbie_solve_modes(pmlbie_ctx* ctx, int n_rhs, const pmlbie_incidence* inc, void* d_u1,
                       void* d_phi1, void* d_u2, void* d_phi2);

/* Scattered field at n_pts points (host array rtz of (rho, theta, z)
 * triples, physical region, off the curve), by the Green representation of
 * each medium (Sec. 4.2, eq. eqfujs) and the modal synthesis.  A panel closer
 * to a point than the panel's arclength is integrated on auxiliary points
 * graded toward the closest curve point, against the Lagrange interpolant of
 * the densities on its nodes (the panel rule alone fails there); the other
 * panels use their nodes.  out: host array, n_rhs * n_pts
 * complex128, layout [rhs][point].  n_pts = 0 is allowed.  The points are
 * processed in chunks whose point x node modal kernels take about 2 GiB of
 * device memory, so any number of points fits; PMLBIE_EINVAL for a point
 * outside rho < a1 or for more than 1024 summed modes. */
int pmlbie_evaluate_field(pmlbie_ctx* ctx, int n_pts, const double* rtz, double* out);

/* Stopping rule of the mixed-precision refinement (Sec. 4.2 systems solved
 * with complex64 factors and FP64 residuals): relative residual tol
 * (0 < tol < 1) and at most max_iter iterations (1..100).  Takes effect at
 * the next solve_modes.  Errors: PMLBIE_EINVAL. */
int pmlbie_set_refinement(pmlbie_ctx* ctx, double tol, int max_iter);

/* The substitution of Sec. 4.3 (eq. eqch1) for the close pairs deep in the
 * PML, for studying it against the graded direct rule: with order L > 0,
 * the pairs the classification gives to the direct rule (the "direct" class)
 * go instead through the split of Sec. 4.1 with H1 replaced by cH1(q, L) =
 * e^{iq} (Taylor polynomial of order L of H1 e^{-iq}), i H2 by e^{iq} - cH1,
 * and H3, i H4 the same way (H3 + i H4 = e^{iq} (1 - iq)); q = k R.  The
 * paper takes L = 5.  Read literally, the substitution leaves odd powers of q
 * in the smooth parts, and on these pairs the kernels it gives miss the
 * parity bar of the direct rule by orders of magnitude; the default (0)
 * keeps the direct rule.  Takes effect at the next build or modal-kernel
 * call.  Errors: PMLBIE_EINVAL (L outside 0..12). */
int pmlbie_set_ch1_substitution(pmlbie_ctx* ctx, int order);

/* ---- inspection ---------------------------------------------------------- */

/* Test hook of the zero-pivot path (Sec. 4.2 per-mode LU): the next build
 * sets column col (0 <= col < 2N) of mode `mode`'s assembled matrix to zero
 * before factoring it, so that its LU meets an exactly zero pivot and the
 * build returns PMLBIE_ESINGULAR naming the mode and column.  One shot: the
 * hook is cleared by that build; a mode outside the build's range leaves the
 * matrices untouched.  Errors: PMLBIE_EINVAL, PMLBIE_ESTATE (no media). */
int pmlbie_test_zero_column(pmlbie_ctx* ctx, int mode, int col);

/* Sizes of the current build: info[0] = N, [1] = m_max, [2] = angle grid L
 * of the split, [3] = angle grid of the far path (the same L), [4] = far
 * pairs, [5] = split pairs, [6] = direct pairs, [7] = auxiliary near-panel
 * points, [8] = modes of the smooth parts the split resolves beyond m_max
 * (L/2 - 1 - m_max). */
int pmlbie_get_info(const pmlbie_ctx* ctx, long long* info /* host, 9 */);

/* Node table (host output, N x 13 doubles per node): rho, Im rho~, z,
 * Re n_rho, Im n_rho, Re n_z, Im n_z, W (quadrature weight times rho |dr/dt|),
 * panel, t, nu_rho, nu_z, |dr/dt|. */
int pmlbie_get_nodes(const pmlbie_ctx* ctx, double* out);

/* Modal kernels S_n, K_n (natural modes, n = 0..m_max, both media) of
 * n_pairs explicit point pairs with the machinery of the build (pair
 * classification, FFT, split, graded quadrature).  geom: host, 12 doubles
 * per pair: rho~_t, rho~_s, rho~_t - rho~_s, z~_t - z~_s, n_rho, n_z of the
 * source (each complex as re, im).  out: device, n_pairs * 4 * (m_max+1)
 * complex128, layout [pair][S1, K1, S2, K2][mode]. */
int pmlbie_modal_kernels(pmlbie_ctx* ctx, int n_pairs, const double* geom, void* d_out);

/* Allocation-free variant of pmlbie_modal_kernels, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same arguments, kernels and output,
 * but every work buffer (pair records, the far / split / direct work lists,
 * the split path's singular-mode tables) lives in a fixed scratch array of
 * the library (about 14.3 MB per device, held until the process ends) and no
 * device or library allocation is made.  At most PMLBIE_NOALLOC_MAX_PAIRS
 * pairs per call (PMLBIE_EINVAL beyond).  All calls on one device share that
 * device's scratch: calls that overlap in time on one device (several host
 * threads, or several streams) race and must be serialised by the caller.
 * Errors: PMLBIE_EINVAL, PMLBIE_ESTATE (no build), PMLBIE_EDEVICE. */
#define PMLBIE_NOALLOC_MAX_PAIRS 4096
int pmlbie_modal_kernels_noalloc(pmlbie_ctx* ctx, int n_pairs, const double* geom, void* d_out);

/* Copy the assembled (unfactored) matrix of mode n (row-major 2N x 2N
 * complex128) to d_out; needs PMLBIE_KEEP_OPERATORS at build. */
int pmlbie_get_operator(pmlbie_ctx* ctx, int mode, void* d_out);

/* Stage wall-clock times of the last build/solve in ms (host, 16 doubles):
 * [0] setup, [1] far kernels, [2] split, [3] direct, [4] near panels,
 * [5] LU total, [6] LU trailing updates, [7] solve total, [8] right-hand
 * sides, [9] refinement, [10] build total; and counters (host, 16 doubles):
 * [0] refinement iterations, [1] final relative residual, [2] real flops of
 * all LU trailing updates (algorithmic: 8 per complex multiply-add; the
 * matrix cores execute 6 of them, the complex product being formed from
 * three real ones), [3] number of LU steps with a trailing update (stage [6]
 * sums, per step, the interval of its launches: the next step's columns, then
 * the rest in column pieces, between which the next step's factorisation
 * runs),
 * [4] far pairs offered to the surrogate, [5] pairs whose surrogate modes
 * were accepted, [6] far pairs transformed on the full angle grid (the others
 * on the shortest grid that holds modes 0..m_max, when that is shorter). */
int pmlbie_get_stats(const pmlbie_ctx* ctx, double* stage_ms, double* counters);

/* ---- Learned surrogate of the far-pair modes ------------------------------
 * A multilayer perceptron (raw inputs rho, rho', dz, k, S, Im rho~, Im rho~';
 * features: those scaled to O(1) plus the phase scale k |R0| and the phase
 * swing k (|R(pi)| - |R0|) of e^{ikR} over the angle; four hidden layers of
 * 256 with the erf GELU; 390 outputs) trained on modal kernels that the
 * raw-kernel FFT of the build generates.  It predicts modes 0..64 of
 *   S = G~, P = (-(rho~ - rho~') + 2 rho~ sin^2(D/2)) f, Q = -(z - z') f,
 *   f = e^{ikR}(ikR - 1)/(4 pi R^3)  (K = n'_rho P + n'_z Q, Sec. 3.1),
 * each normalised by the phase e^{ik Re R0} and an amplitude scale that
 * includes the largest PML decay factor |e^{ikR}| over the angle
 * (R0 = R at D = 0).
 * Weights: FP32 master copy and Adam moments on the device, BF16 copies for
 * the MFMA products (FP32 accumulation).  One network serves one PML
 * geometry (a1, T, p, fixed at init or load); S enters as an input.
 * Every call returns a status; PMLBIE_ESTATE when no network exists. */

/* Number of FP32 parameters of the network (weights and biases, padded
 * layouts: layer l is (out x in) row-major, in padded to 32 / 256). */
long pmlbie_surrogate_nparams(void);

/* Fresh network (Glorot-uniform weights from a splitmix64 stream seeded
 * with `seed`, zero biases) for the PML geometry of the current media. */
int pmlbie_surrogate_init(pmlbie_ctx* ctx, unsigned long long seed);

/* Sample set `which` (0 training, 1 held out) of n pairs: random interfaces
 * a exp(-(rho / w)^2), a ~ U[0, 0.6], w ~ U[0.5, 2], at 512 nodes per
 * segment; node pairs farther apart than twice the longer sub-panel;
 * S ~ U[1, 4]; k = k1 ~ U[5, 15] or k1 * U[1.2, 2] with equal odds.  Labels
 * by the raw-kernel FFT on the device (512 angles).  n <= 2^24. */
int pmlbie_surrogate_make_samples(pmlbie_ctx* ctx, int which, long n, unsigned long long seed);

/* `steps` Adam steps on consecutive batches of the training set (step size
 * decaying from lr to lr / 20 along a cosine); loss_out (host, steps
 * doubles, may be NULL) receives the mean squared error of each batch. */
int pmlbie_surrogate_train(pmlbie_ctx* ctx, int steps, int batch, double lr, double* loss_out);

/* Mean squared error of the network over sample set `which`. */
int pmlbie_surrogate_eval(pmlbie_ctx* ctx, int which, double* mse);

/* Relative RMS error per mode over sample set `which`: rel[n] (host, 65
 * doubles) = sqrt(sum |y - t|^2 / sum |t|^2) over the samples, the three
 * heads and both parts at mode n (normalised targets). */
int pmlbie_surrogate_eval_modes(pmlbie_ctx* ctx, int which, double* rel);

/* Acceptance tolerance of the build: a pair's surrogate modes are kept when
 * 4 pi W_l max |synthesis - direct sample| <= tol over the eight check
 * angles and both media (W_l the quadrature weight of the source node); the
 * quantity bounds every mode's error in the pair's matrix entries.  0
 * rejects all. */
int pmlbie_surrogate_set_tolerance(pmlbie_ctx* ctx, double tol);

/* Serialise / restore the network (header + FP32 parameters).  save with
 * blob = NULL stores the size in *bytes. */
int pmlbie_surrogate_save(pmlbie_ctx* ctx, void* blob, size_t* bytes);
int pmlbie_surrogate_load(pmlbie_ctx* ctx, const void* blob, size_t bytes);

/* Test hooks (host arrays).  params: get (1) or set (0) the FP32 parameters
 * (nparams doubles).  forward: x n x 7 raw inputs -> y n x 390 outputs.
 * grad: loss and gradient of the mean squared error against targets t
 * (n x 390) for the current parameters (no update).  label: normalised
 * FFT targets (n x 390) of samples s (n x 6: Re, Im rho~, Re, Im rho~',
 * z - z', k). */
int pmlbie_surrogate_params(pmlbie_ctx* ctx, double* p, int get);
int pmlbie_surrogate_forward(pmlbie_ctx* ctx, int n, const double* x, double* y);
int pmlbie_surrogate_grad(pmlbie_ctx* ctx, int n, const double* x, const double* t, double* loss,
                          double* grad);
int pmlbie_surrogate_label(pmlbie_ctx* ctx, int n, const double* s, double* y);

#ifdef __cplusplus
}
#endif
#endif /* PMLBIE_H */
