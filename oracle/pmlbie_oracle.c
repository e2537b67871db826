/*
 * Plain FP64 CPU oracle for the axisymmetric two-layer PML-BIE method
 * (Wang & Lu, "An FFT-accelerated PML-BIE solver for three-dimensional
 * acoustic wave scattering in layered media", arXiv 2412.11162).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this code; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the HIP path.
 *
 * What it computes, each from its plain definition:
 *   - the PML absorption profile sigma_1 and its primitive (Sec. 3.1, eq.
 *     eqsgm1, eqs. eqrhot/eqzt), integrated by adaptive Gauss-Kronrod;
 *   - the complexified Green's function G~ = exp(i k R)/(4 pi R) and its
 *     conormal derivative at the source (Sec. 3.1, the fundamental solution
 *     and eq. eqg1t), with R the principal square root of
 *     |r~ - r~'|^2 + 4 rho~ rho~' sin^2(Delta/2) (Sec. 4.3, the stable
 *     distance);
 *   - the natural azimuthal modes F_n = int_{-pi}^{pi} e^{-i n Delta} F dDelta
 *     (Sec. 3.3, eq. fmode3 without the 1/sqrt(2 pi)), by globally adaptive
 *     Gauss-Kronrod quadrature in Delta: no FFT and no kernel split;
 *   - the near-panel product integrals int_P F_n(r_i, r(t)) rho |r'| l_l(t) dt
 *     of the Nystrom discretisation on Gauss-Legendre panels, by globally
 *     adaptive Gauss-Kronrod quadrature in t whose every integrand value is
 *     itself an adaptive Delta integral.
 *
 * Conormal derivative: d/dnu_c = nu_c . grad_r with nu_c = A^T nu (Sec. 3.1),
 * which in the stretched variables reads
 *   n_rho d/drho~ + n_z d/dz~,  n_rho = nu_rho rho~ alpha_z / rho,
 *                               n_z   = nu_z rho~ alpha_rho / rho.
 * On every curve used here this coincides with the paper's kernel D of
 * Sec. 4.1 (nu_rho = 0 wherever sigma_1 != 0, and sigma_2 = 0 on the curve).
 */
#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------- */
/* Gauss-Kronrod 7/15 rule on [-1, 1] (the QUADPACK qk15 constants).         */
static const double XGK[8] = {
    0.991455371120812639206854697526329, 0.949107912342758524526189684047851,
    0.864864423359769072789712788640926, 0.741531185599394439863864773280788,
    0.586087235467691130294144845693013, 0.405845151377397166906606412076961,
    0.207784955007898467600689403773245, 0.000000000000000000000000000000000};
static const double WGK[8] = {
    0.022935322010529224963732008058970, 0.063092092629978553290700663189204,
    0.104790010322250183839876322541518, 0.140653259715525918745189590510238,
    0.169004726639267902826583426598550, 0.190350578064785409913256402421014,
    0.204432940075298892414161999234649, 0.209482141084727828012999174891714};
/* Gauss 7-point weights for XGK[1], XGK[3], XGK[5], XGK[7]. */
static const double WG[4] = {
    0.129484966168869693270611432679082, 0.279705391489276667901467771423780,
    0.381830050505118944950369775488975, 0.417959183673469387755102040816327};

typedef void (*vfun)(double x, void *ctx, cplx *out);

/* One GK15 panel: kronrod result in res, max |K - G| returned, and in
   *absint the largest Kronrod estimate of int |f_j| (the rounding floor). */
static double gk15(vfun f, void *ctx, int nout, double a, double b, cplx *res,
                   cplx *tmp, cplx *gsum, double *absint) {
  double c = 0.5 * (a + b), h = 0.5 * (b - a);
  for (int j = 0; j < nout; ++j) { res[j] = 0; gsum[j] = 0; }
  double amax = 0.0;
  for (int q = 0; q < 15; ++q) {
    int idx = q < 8 ? q : 14 - q;
    double x = q < 8 ? c - h * XGK[q] : c + h * XGK[14 - q];
    if (q == 7) x = c;
    f(x, ctx, tmp);
    double wk = WGK[idx];
    double wg = (idx % 2 == 1) ? WG[idx / 2] : 0.0;
    for (int j = 0; j < nout; ++j) {
      res[j] += wk * tmp[j];
      if (wg != 0.0) gsum[j] += wg * tmp[j];
      double m = wk * cabs(tmp[j]);
      if (m > amax) amax = m;
    }
  }
  *absint = amax * h;
  double err = 0;
  for (int j = 0; j < nout; ++j) {
    res[j] *= h;
    gsum[j] *= h;
    double e = cabs(res[j] - gsum[j]);
    if (e > err) err = e;
  }
  return err;
}

typedef struct { double a, b, err, absint; int depth; } ivl;

/*
 * Globally adaptive vector quadrature: keep bisecting the interval with the
 * largest error estimate until the summed estimate is below
 * max(abstol, reltol * max_j |I_j|, 200 eps int |f|) -- the last term is the
 * rounding floor below which no quadrature of f can resolve the integral; an
 * interval whose estimate is within 50 eps of its own int |f| is not split
 * further -- or the interval budget is spent.
 *
 * Bookkeeping: the vector of partial results is kept as a running sum (the
 * bisected interval's contribution taken out, its two halves added), so a
 * bisection costs O(nout) plus a scan of the scalar estimates, not a re-sum of
 * every interval's vector.  The running sum only serves the stopping test's
 * scale max_j |I_j|; the returned result is summed afresh over the final
 * intervals.  The rule (which interval is split, when to stop) is unchanged.
 * Returns the number of intervals used (negative if the budget ran out).
 */
static int adapt(vfun f, void *ctx, int nout, const double *brk, int nbrk,
                 double reltol, double abstol, int maxivl, cplx *result) {
  ivl *iv = (ivl *)malloc(sizeof(ivl) * maxivl);
  cplx *store = (cplx *)malloc(sizeof(cplx) * (size_t)nout * maxivl);
  cplx *tmp = (cplx *)malloc(sizeof(cplx) * nout * 3);
  cplx *gs = tmp + nout;
  cplx *run = tmp + 2 * (size_t)nout;
  int n = 0;
  for (int j = 0; j < nout; ++j) run[j] = 0;
  for (int s = 0; s + 1 < nbrk; ++s) {
    if (!(brk[s + 1] > brk[s])) continue;
    iv[n].a = brk[s]; iv[n].b = brk[s + 1]; iv[n].depth = 0;
    cplx *r = store + (size_t)n * nout;
    iv[n].err = gk15(f, ctx, nout, brk[s], brk[s + 1], r, tmp, gs, &iv[n].absint);
    for (int j = 0; j < nout; ++j) run[j] += r[j];
    ++n;
  }
  int ok = 1;
  for (;;) {
    double tot = 0, scale = 0, absint = 0;
    int worst = -1;
    double werr = -1;
    for (int s = 0; s < n; ++s) {
      tot += iv[s].err;
      absint += iv[s].absint;
      /* an interval whose estimate is at its own rounding level is final */
      int at_floor = iv[s].err <= 50.0 * DBL_EPSILON * iv[s].absint;
      if (iv[s].err > werr && iv[s].depth < 200 && !at_floor) { werr = iv[s].err; worst = s; }
    }
    for (int j = 0; j < nout; ++j) { double m = cabs(run[j]); if (m > scale) scale = m; }
    double tol = fmax(abstol, fmax(reltol * scale, 200.0 * DBL_EPSILON * absint));
    if (tot <= tol || worst < 0) break;
    if (n + 1 >= maxivl) { ok = 0; break; }
    double a = iv[worst].a, b = iv[worst].b, m = 0.5 * (a + b);
    int d = iv[worst].depth + 1;
    cplx *rw = store + (size_t)worst * nout, *rn = store + (size_t)n * nout;
    for (int j = 0; j < nout; ++j) run[j] -= rw[j];
    iv[worst].b = m; iv[worst].depth = d;
    iv[worst].err = gk15(f, ctx, nout, a, m, rw, tmp, gs, &iv[worst].absint);
    iv[n].a = m; iv[n].b = b; iv[n].depth = d;
    iv[n].err = gk15(f, ctx, nout, m, b, rn, tmp, gs, &iv[n].absint);
    for (int j = 0; j < nout; ++j) run[j] += rw[j] + rn[j];
    ++n;
  }
  for (int j = 0; j < nout; ++j) result[j] = 0;
  for (int s = 0; s < n; ++s) {
    cplx *r = store + (size_t)s * nout;
    for (int j = 0; j < nout; ++j) result[j] += r[j];
  }
  free(iv); free(store); free(tmp);
  return ok ? n : -n;
}

/* ------------------------------------------------------------------------- */
/* Geometry: interface graph, PML profile (Sec. 2, Sec. 3.1 eq. eqsgm1).     */
typedef struct {
  int nb;
  double amp[8], cen[8], wid[8];
  double cosf;   /* 0: no cosine factor */
  double a1, T, S;
  int p;
  double gl[16]; /* Gauss-Legendre nodes on [-1, 1] for the Lagrange basis */
  int poly;      /* 1: polyline of straight panels (Sec. 4, graded mesh); 2: curved panels
                    given by Chebyshev series */
} geom_t;

static geom_t G_;

void or_set_geometry(int nb, const double *bumps, double cosf, double a1,
                     double T, double S, int p, const double *gl16) {
  G_.nb = nb;
  for (int i = 0; i < nb && i < 8; ++i) {
    G_.amp[i] = bumps[3 * i]; G_.cen[i] = bumps[3 * i + 1]; G_.wid[i] = bumps[3 * i + 2];
  }
  G_.cosf = cosf; G_.a1 = a1; G_.T = T; G_.S = S; G_.p = p;
  for (int i = 0; i < 16; ++i) G_.gl[i] = gl16[i];
  G_.poly = 0;
}

/* Switch the near-panel integrals to straight panels (1: a panel is given by
   its start (rho_a, z_a) and its extent (d rho, d z)) or curved panels (2:
   Chebyshev series of rho(t), z(t) and of their derivatives). */
void or_set_poly(int on) { G_.poly = on; }

/* Chebyshev series sum_k c_k T_k(t), k < 16, by Clenshaw's recurrence. */
static double cheb_sum(const double *c, double t) {
  double b1 = 0.0, b2 = 0.0;
  for (int k = 15; k >= 1; --k) {
    double b0 = 2.0 * t * b1 - b2 + c[k];
    b2 = b1;
    b1 = b0;
  }
  return t * b1 - b2 + c[0];
}

/* (f(a) - f(b)) for a Chebyshev series without cancellation: the divided
   differences D_k = (T_k(a) - T_k(b)) / (a - b) obey D_0 = 0, D_1 = 1,
   D_{k+1} = 2 T_k(a) + 2 b D_k - D_{k-1}. */
static double cheb_diff(const double *c, double a, double b) {
  double Tm = 1.0, Tk = a, Dm = 0.0, Dk = 1.0, s = c[1];
  for (int k = 1; k < 15; ++k) {
    double Dn = 2.0 * Tk + 2.0 * b * Dk - Dm;
    double Tn = 2.0 * a * Tk - Tm;
    s += c[k + 1] * Dn;
    Dm = Dk; Dk = Dn; Tm = Tk; Tk = Tn;
  }
  return (a - b) * s;
}

static double gsum(double r) {
  double s = 0;
  for (int i = 0; i < G_.nb; ++i) { double u = (r - G_.cen[i]) / G_.wid[i]; s += G_.amp[i] * exp(-u * u); }
  return s;
}
static double gsum_d(double r) {
  double s = 0;
  for (int i = 0; i < G_.nb; ++i) {
    double u = (r - G_.cen[i]) / G_.wid[i];
    s += G_.amp[i] * exp(-u * u) * (-2.0 * u / G_.wid[i]);
  }
  return s;
}
/* g(r) - g(s) without cancellation: a e^{-v^2} expm1(-(u - v)(u + v)). */
static double gsum_diff(double r, double s) {
  double d = 0;
  for (int i = 0; i < G_.nb; ++i) {
    double u = (r - G_.cen[i]) / G_.wid[i], v = (s - G_.cen[i]) / G_.wid[i];
    double du = (r - s) / G_.wid[i];
    d += G_.amp[i] * exp(-v * v) * expm1(-du * (u + v));
  }
  return d;
}
static double hraw_d(double r) {
  if (G_.cosf == 0) return gsum_d(r);
  return gsum_d(r) * cos(G_.cosf * r) - gsum(r) * G_.cosf * sin(G_.cosf * r);
}
/* h(r) - h(s) without cancellation. */
static double hraw_diff(double r, double s) {
  if (G_.cosf == 0) return gsum_diff(r, s);
  double cr = cos(G_.cosf * r);
  double dc = -2.0 * sin(0.5 * G_.cosf * (r + s)) * sin(0.5 * G_.cosf * (r - s));
  return gsum_diff(r, s) * cr + gsum(s) * dc;
}
/* The interface: h~ = h(rho) - h(a1) below a1, flat (0) beyond. */
double or_h(double r) { return r < G_.a1 ? hraw_diff(r, G_.a1) : 0.0; }
double or_hp(double r) { return r < G_.a1 ? hraw_d(r) : 0.0; }
double or_hdiff(double r, double s) {
  int ir = r < G_.a1, is = s < G_.a1;
  if (ir && is) return hraw_diff(r, s);
  if (ir) return hraw_diff(r, G_.a1);
  if (is) return -hraw_diff(s, G_.a1);
  return 0.0;
}

/* sigma_1 of eq. eqsgm1 (rho >= 0). */
double or_sigma(double r) {
  double a1 = G_.a1, T = G_.T, S = G_.S;
  int p = G_.p;
  if (r <= a1) return 0.0;
  if (r > a1 + T) return S;
  double rb = (r - (a1 + T)) / T;
  double f1 = (0.5 - 1.0 / p) * rb * rb * rb + rb / p + 0.5;
  double f2 = 1.0 - f1;
  double f1p = pow(f1, p), f2p = pow(f2, p);
  return 2.0 * S * f1p / (f1p + f2p);
}

static void sig_v(double x, void *ctx, cplx *out) { (void)ctx; out[0] = or_sigma(x); }

/* int_s^r sigma_1, adaptive, breakpoints at the profile's joints. */
double or_Idiff(double r, double s) {
  double lo = fmin(r, s), hi = fmax(r, s), sgn = r >= s ? 1.0 : -1.0;
  double a1 = G_.a1, b1 = G_.a1 + G_.T;
  if (hi <= a1) return 0.0;
  double brk[4]; int nb = 0;
  brk[nb++] = fmax(lo, a1);
  if (b1 > brk[0] && b1 < hi) brk[nb++] = b1;
  brk[nb++] = hi;
  cplx res;
  adapt(sig_v, NULL, 1, brk, nb, 1e-16, 1e-17, 400, &res);
  return sgn * creal(res);
}
double or_I(double r) { return or_Idiff(r, 0.0); }


/*
 * Geometry at rho on a panel of rho-length L (t in [-1, 1] maps linearly):
 * out = [rho, I(rho), z, h~', nu_rho, nu_z, |dr/dt|, Re n_rho, Im n_rho,
 *        Re n_z, Im n_z, sigma].  nu points into the lower medium (Sec. 2).
 */
void or_point(double rho, double L, double *out) {
  double hp = or_hp(rho);
  double sq = sqrt(1.0 + hp * hp);
  double nur = hp / sq, nuz = -1.0 / sq;
  double Iv = or_I(rho);
  double sg = or_sigma(rho);
  cplx rhot = rho + Iv * (cplx)_Complex_I;
  cplx alr = 1.0 + sg * (cplx)_Complex_I;
  cplx nr = nur * rhot / rho; /* alpha_z = 1 on the curve (sigma_2 = 0 there) */
  cplx nz = nuz * rhot * alr / rho;
  out[0] = rho; out[1] = Iv; out[2] = or_h(rho); out[3] = hp;
  out[4] = nur; out[5] = nuz; out[6] = 0.5 * L * sq;
  out[7] = creal(nr); out[8] = cimag(nr); out[9] = creal(nz); out[10] = cimag(nz);
  out[11] = sg;
}

/* ------------------------------------------------------------------------- */
/* Kernels and their azimuthal modes (Sec. 3.1, Sec. 3.3, Sec. 4.3).         */
typedef struct {
  cplx rt, rs;     /* rho~ of target and source */
  cplx drho, dz;   /* rho~_t - rho~_s and z~_t - z~_s, formed from differences */
  cplx nrs, nzs;   /* source conormal components (n_rho, n_z) */
  int nk;
  cplx k[2];
  int nmode;
  const int *modes;
} pairctx;

/*
 * Integrand over Delta in [0, pi]: for each wavenumber, 2 cos(n Delta) G~
 * and 2 cos(n Delta) dG~/dnu_c(r').  Layout out[(2*ik + {0,1})*nmode + j].
 */
static void pair_integrand(double D, void *vctx, cplx *out) {
  pairctx *p = (pairctx *)vctx;
  double s = sin(0.5 * D), s2 = s * s;
  cplx d2 = p->drho * p->drho + p->dz * p->dz;
  cplx R2 = d2 + 4.0 * p->rt * p->rs * s2;          /* stable distance, Sec. 4.3 */
  cplx R = csqrt(R2);                                /* principal branch, Sec. 3.1 */
  /* nu_c'.(r~' - r~ rotated) = n'_rho (rho~' - rho~ cos D) + n'_z (z~' - z~) */
  cplx N = -(p->nrs * p->drho + p->nzs * p->dz) + 2.0 * p->nrs * p->rt * s2;
  cplx Gv[2], Kv[2];
  for (int ik = 0; ik < p->nk; ++ik) {
    cplx ikR = p->k[ik] * R * (cplx)_Complex_I;
    cplx e = cexp(ikR);
    Gv[ik] = e / (4.0 * M_PI * R);
    Kv[ik] = N * e * (ikR - 1.0) / (4.0 * M_PI * R * R2);
  }
  for (int j = 0; j < p->nmode; ++j) {
    /* cos(n D) with the rounding of the product n D compensated: n D = a + b
       exactly (b by a fused multiply-add), cos(a + b) = cos a - b sin a to
       O(b^2); plain cos(n D) would carry an absolute error ~ n D eps, ~1e-13
       at n = 256, D ~ pi, above the quadrature's stopping floor */
    const double nn = (double)p->modes[j];
    const double a = nn * D, b = fma(nn, D, -a);
    double cn = 2.0 * (cos(a) - b * sin(a));
    for (int ik = 0; ik < p->nk; ++ik) {
      out[(2 * ik) * p->nmode + j] = cn * Gv[ik];
      out[(2 * ik + 1) * p->nmode + j] = cn * Kv[ik];
    }
  }
}

static double g_reltol_delta = 1e-14;

/* Modes of one pair by adaptive quadrature over Delta in [0, pi]. */
static int pair_modes(pairctx *p, cplx *out) {
  int nout = 2 * p->nk * p->nmode;
  double brk[96];
  int nb = 0;
  /* uniform pieces for oscillation, geometric pieces toward Delta = 0 */
  double sc = sqrt(cabs(p->rt * p->rs));
  double kmax = 0;
  int nmax = 0;
  for (int ik = 0; ik < p->nk; ++ik) kmax = fmax(kmax, cabs(p->k[ik]));
  for (int j = 0; j < p->nmode; ++j) nmax = p->modes[j] > nmax ? p->modes[j] : nmax;
  int nu = (int)ceil((nmax + 2.0 * kmax * sc) / 6.0);
  if (nu < 4) nu = 4;
  if (nu > 48) nu = 48;
  double d = cabs(csqrt(p->drho * p->drho + p->dz * p->dz));
  double delta = sc > 0 ? d / sc : M_PI;
  double first = M_PI / nu;
  double geo[40];
  int ng = 0;
  for (double x = first * 0.5; x > 0.25 * delta && ng < 40; x *= 0.5) geo[ng++] = x;
  brk[nb++] = 0.0;
  for (int g = ng - 1; g >= 0; --g) brk[nb++] = geo[g];
  for (int u = 1; u <= nu; ++u) brk[nb++] = M_PI * u / nu;
  int r = adapt(pair_integrand, p, nout, brk, nb, g_reltol_delta, 1e-300, 20000, out);
  return r;
}

static void fill_pair(pairctx *p, double rho_t, double I_t, double z_t,
                      double rho_s, double I_s, double z_s, cplx nrs, cplx nzs,
                      double drho, double dI, double dz) {
  p->rt = rho_t + I_t * (cplx)_Complex_I;
  p->rs = rho_s + I_s * (cplx)_Complex_I;
  p->drho = drho + dI * (cplx)_Complex_I;
  p->dz = dz;
  p->nrs = nrs;
  p->nzs = nzs;
  (void)z_t; (void)z_s;
}

void or_set_reltol(double r) { g_reltol_delta = r; }

/*
 * Modal kernels of npairs (target, source) pairs (oncurve = 1 when both
 * points of every pair lie on the interface).
 * tgt[3*p] = (rho, I, z); src[7*p] = (rho, I, z, Re n_rho, Im n_rho, Re n_z,
 * Im n_z).  The differences rho - rho', z - z' and I - I' are formed from the
 * interface and profile definitions directly (or_hdiff, or_Idiff), not by
 * subtracting rounded coordinates.
 * out[p][(2*ik + {S,K})][j] complex, natural normalisation.
 * Returns the number of pairs whose interval budget ran out.
 */
int or_modal_pairs(int npairs, const double *tgt, const double *src, int oncurve,
                   int nk, const double *kri, int nmode, const int *modes,
                   double *outd) {
  int bad = 0;
  cplx *out = (cplx *)outd;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : bad)
  for (int q = 0; q < npairs; ++q) {
    pairctx p;
    const double *T = tgt + 3 * q, *Sx = src + 7 * q;
    double drho = T[0] - Sx[0];
    /* both points on the interface: difference of the graph without
       cancellation; otherwise plain coordinates */
    double dz = oncurve ? or_hdiff(T[0], Sx[0]) : T[2] - Sx[2];
    double dI = or_Idiff(T[0], Sx[0]);
    fill_pair(&p, T[0], T[1], T[2], Sx[0], Sx[1], Sx[2],
              Sx[3] + Sx[4] * (cplx)_Complex_I, Sx[5] + Sx[6] * (cplx)_Complex_I,
              drho, dI, dz);
    p.nk = nk;
    for (int ik = 0; ik < nk; ++ik) p.k[ik] = kri[2 * ik] + kri[2 * ik + 1] * (cplx)_Complex_I;
    p.nmode = nmode;
    p.modes = modes;
    int r = pair_modes(&p, out + (size_t)q * 2 * nk * nmode);
    if (r < 0) bad++;
  }
  return bad;
}

/* ------------------------------------------------------------------------- */
/* Near-panel product integrals of the Nystrom discretisation.               */
typedef struct {
  double rho_t, I_t, z_t;    /* target node */
  double pa, L;              /* panel: rho = pa + (1 + t) L / 2 */
  double za, dzp;            /* straight panel: z = za + (1 + t) dzp / 2 */
  const double *cheb;        /* curved panel: 4 x 16 Chebyshev coefficients of rho, z, rho', z' */
  int self;                  /* 1: target lies on this panel at t_i */
  int offc;                  /* 1: target off the curve (a field point), closest to t_i */
  double ti;
  int nk;
  cplx k[2];
  int nmode;
  const int *modes;
  cplx *buf;                 /* 2*nk*nmode scratch */
} nearctx;

/* Lagrange basis polynomial l_l(t) on the 16 Gauss-Legendre nodes. */
static double lagr(int l, double t) {
  double v = 1.0;
  for (int m = 0; m < 16; ++m)
    if (m != l) v *= (t - G_.gl[m]) / (G_.gl[l] - G_.gl[m]);
  return v;
}

/*
 * Integrand at panel parameter t: F_n(r_i, r(t)) rho(t) |dr/dt| l_l(t) for the
 * 16 Lagrange functions.  Layout out[l][(2*ik+{S,K})][j].
 */
/* Straight panel at parameter t: the same 12 values as or_point. */
static void poly_point(const nearctx *c, double t, double *out) {
  double u = 0.5 * (1.0 + t);
  double rho = c->pa + u * c->L;
  double len = hypot(c->L, c->dzp);
  double nur = c->dzp / len, nuz = -c->L / len; /* (z', -rho') / |r'| */
  double Iv = or_I(rho), sg = or_sigma(rho);
  cplx rhot = rho + Iv * (cplx)_Complex_I;
  cplx nr = nur * rhot / rho;
  cplx nz = nuz * rhot * (1.0 + sg * (cplx)_Complex_I) / rho;
  out[0] = rho; out[1] = Iv; out[2] = c->za + u * c->dzp; out[3] = 0.0;
  out[4] = nur; out[5] = nuz; out[6] = 0.5 * len;
  out[7] = creal(nr); out[8] = cimag(nr); out[9] = creal(nz); out[10] = cimag(nz);
  out[11] = sg;
}

/* Curved panel at parameter t: the same 12 values as or_point. */
static void curved_point(const nearctx *c, double t, double *out) {
  double rho = cheb_sum(c->cheb, t), zz = cheb_sum(c->cheb + 16, t);
  double dr = cheb_sum(c->cheb + 32, t), dz = cheb_sum(c->cheb + 48, t);
  double len = hypot(dr, dz);
  double nur = dz / len, nuz = -dr / len;
  double Iv = or_I(rho), sg = or_sigma(rho);
  cplx rhot = rho + Iv * (cplx)_Complex_I;
  cplx nr = nur * rhot / rho;
  cplx nz = nuz * rhot * (1.0 + sg * (cplx)_Complex_I) / rho;
  out[0] = rho; out[1] = Iv; out[2] = zz; out[3] = 0.0;
  out[4] = nur; out[5] = nuz; out[6] = len;
  out[7] = creal(nr); out[8] = cimag(nr); out[9] = creal(nz); out[10] = cimag(nz);
  out[11] = sg;
}

static void near_integrand(double t, void *vctx, cplx *out) {
  nearctx *c = (nearctx *)vctx;
  double g[12];
  double rho, drho, dz;
  if (G_.poly == 2) {
    curved_point(c, t, g);
    rho = g[0];
    if (c->self) {
      drho = cheb_diff(c->cheb, c->ti, t);
      dz = cheb_diff(c->cheb + 16, c->ti, t);
    } else {
      drho = c->rho_t - rho;
      dz = c->z_t - g[2];
    }
  } else if (G_.poly) {
    poly_point(c, t, g);
    rho = g[0];
    if (c->self) {
      /* on the target's own straight panel the offset is (t_i - t)/2 times
         the panel extent, exactly */
      drho = 0.5 * (c->ti - t) * c->L;
      dz = 0.5 * (c->ti - t) * c->dzp;
    } else {
      drho = c->rho_t - rho;
      dz = c->z_t - g[2];
    }
  } else {
    rho = c->pa + 0.5 * (1.0 + t) * c->L;
    or_point(rho, c->L, g);
    /* rho_t - rho is exact in floating point for nearby points, and or_hdiff
       uses that same difference, so the pair geometry stays consistent down to
       the log singularity */
    drho = c->rho_t - rho;
    dz = c->offc ? c->z_t - g[2] : or_hdiff(c->rho_t, rho);
  }
  double dI = or_Idiff(c->rho_t, rho);
  pairctx p;
  fill_pair(&p, c->rho_t, c->I_t, c->z_t, rho, g[1], g[2],
            g[7] + g[8] * (cplx)_Complex_I, g[9] + g[10] * (cplx)_Complex_I, drho, dI, dz);
  p.nk = c->nk;
  p.k[0] = c->k[0]; p.k[1] = c->k[1];
  p.nmode = c->nmode;
  p.modes = c->modes;
  int nm = 2 * c->nk * c->nmode;
  if (drho == 0.0 && dz == 0.0 && dI == 0.0) {
    for (int j = 0; j < 16 * nm; ++j) out[j] = 0; /* the log singularity itself: measure zero */
    return;
  }
  pair_modes(&p, c->buf);
  double w = rho * g[6];
  for (int l = 0; l < 16; ++l) {
    double lw = w * lagr(l, t);
    for (int j = 0; j < nm; ++j) out[l * nm + j] = lw * c->buf[j];
  }
}

/*
 * Product integrals of nt targets against panels.  For target q:
 * tinfo[5*q] = (rho_t, I_t, z_t, t_i or 2 (not on panel), which: 0 self,
 * -1 left neighbour, +1 right neighbour, 2 a point off the curve whose
 * closest panel parameter is t_i), panel[68*q] = (pa, L, za, dz, 64
 * Chebyshev coefficients): the start rho and rho-extent, (straight panels)
 * the start z and z-extent, (curved panels) the series of rho, z, rho', z'.
 * out[q][l][(2*ik+{S,K})][j] = int_{-1}^{1} F_n(r_q, r(t)) rho |dr/dt| l_l(t) dt.
 */
int or_near_panels(int nt, const double *tinfo, const double *panel, int nk,
                   const double *kri, int nmode, const int *modes, double reltol,
                   double *outd) {
  int bad = 0;
  cplx *out = (cplx *)outd;
  int nm = 2 * nk * nmode;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad)
  for (int q = 0; q < nt; ++q) {
    nearctx c;
    const double *ti = tinfo + 5 * q;
    c.rho_t = ti[0]; c.I_t = ti[1]; c.z_t = ti[2];
    c.pa = panel[68 * q]; c.L = panel[68 * q + 1];
    c.za = panel[68 * q + 2]; c.dzp = panel[68 * q + 3];
    c.cheb = panel + 68 * q + 4;
    int which = (int)ti[4];
    c.self = which == 0;
    c.offc = which == 2;
    c.ti = ti[3];
    c.nk = nk;
    c.k[0] = kri[0] + kri[1] * (cplx)_Complex_I;
    c.k[1] = nk > 1 ? kri[2] + kri[3] * (cplx)_Complex_I : 0;
    c.nmode = nmode;
    c.modes = modes;
    c.buf = (cplx *)malloc(sizeof(cplx) * nm);
    double brk[64];
    int nb = 0;
    if (which == 0) {
      /* breakpoint at the log singularity, geometric refinement toward it */
      brk[nb++] = -1.0;
      double gl[30], gr[30];
      int ngl = 0, ngr = 0;
      for (double h = 0.5 * (c.ti + 1.0); h > 1e-6 && ngl < 30; h *= 0.25) gl[ngl++] = c.ti - h;
      for (double h = 0.5 * (1.0 - c.ti); h > 1e-6 && ngr < 30; h *= 0.25) gr[ngr++] = c.ti + h;
      for (int g = 0; g < ngl; ++g) brk[nb++] = gl[g];
      brk[nb++] = c.ti;
      for (int g = ngr - 1; g >= 0; --g) brk[nb++] = gr[g];
      brk[nb++] = 1.0;
    } else if (which == 2) {
      /* off-curve target: breakpoints graded toward its closest point t_i */
      brk[nb++] = -1.0;
      double gl[30], gr[30];
      int ngl = 0, ngr = 0;
      for (double h = 0.5 * (c.ti + 1.0); h > 1e-6 && ngl < 30; h *= 0.25) gl[ngl++] = c.ti - h;
      for (double h = 0.5 * (1.0 - c.ti); h > 1e-6 && ngr < 30; h *= 0.25) gr[ngr++] = c.ti + h;
      for (int g = 0; g < ngl; ++g) if (gl[g] > -1.0) brk[nb++] = gl[g];
      if (c.ti > -1.0 && c.ti < 1.0) brk[nb++] = c.ti;
      for (int g = ngr - 1; g >= 0; --g) if (gr[g] < 1.0) brk[nb++] = gr[g];
      brk[nb++] = 1.0;
    } else if (which == -1) {
      /* panel to the left: the shared endpoint is t = +1 */
      brk[nb++] = -1.0;
      for (double h = 1.0; h > 1e-4; h *= 0.25) brk[nb++] = 1.0 - h;
      brk[nb++] = 1.0;
    } else {
      brk[nb++] = -1.0;
      double tmp[16];
      int n = 0;
      for (double h = 1.0; h > 1e-4; h *= 0.25) tmp[n++] = -1.0 + h;
      for (int g = n - 1; g >= 0; --g) brk[nb++] = tmp[g];
      brk[nb++] = 1.0;
    }
    int r = adapt(near_integrand, &c, 16 * nm, brk, nb, reltol, 1e-300, 3000,
                  out + (size_t)q * 16 * nm);
    if (r < 0) bad++;
    free(c.buf);
  }
  return bad;
}

int or_num_threads(void) { return omp_get_max_threads(); }
