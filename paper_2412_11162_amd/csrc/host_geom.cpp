#include "host_geom.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace pmlbie {

// Gauss-Legendre nodes by Newton iteration on P_n (three-term recurrence).
void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = cos(PMLBIE_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

double Geometry::graw(double r) const {
  double s = 0;
  for (size_t i = 0; i < itf.amp.size(); ++i) {
    double u = (r - itf.cen[i]) / itf.wid[i];
    s += itf.amp[i] * exp(-u * u);
  }
  return s;
}
double Geometry::graw_d(double r) const {
  double s = 0;
  for (size_t i = 0; i < itf.amp.size(); ++i) {
    double u = (r - itf.cen[i]) / itf.wid[i];
    s += itf.amp[i] * exp(-u * u) * (-2.0 * u / itf.wid[i]);
  }
  return s;
}
// g(r) - g(r - dr) = sum a e^{-v^2} expm1(-(u - v)(u + v)), u - v = dr / w
double Geometry::graw_diff(double r, double dr) const {
  double s = 0;
  for (size_t i = 0; i < itf.amp.size(); ++i) {
    double u = (r - itf.cen[i]) / itf.wid[i];
    double du = dr / itf.wid[i];
    double v = u - du;
    s += itf.amp[i] * exp(-v * v) * expm1(-du * (u + v));
  }
  return s;
}
double Geometry::hraw_diff(double r, double dr) const {
  if (itf.cos_freq == 0.0) return graw_diff(r, dr);
  const double f = itf.cos_freq, rs = r - dr;
  double dc = -2.0 * sin(0.5 * f * (r + rs)) * sin(0.5 * f * dr);
  return graw_diff(r, dr) * cos(f * r) + graw(rs) * dc;
}
double Geometry::hraw_d(double r) const {
  if (itf.cos_freq == 0.0) return graw_d(r);
  const double f = itf.cos_freq;
  return graw_d(r) * cos(f * r) - graw(r) * f * sin(f * r);
}
double Geometry::h(double r) const { return r < itf.rho_c ? hraw_diff(r, r - itf.rho_c) : 0.0; }
double Geometry::hprime(double r) const { return r < itf.rho_c ? hraw_d(r) : 0.0; }
double Geometry::hdiff(double r, double dr) const {
  const double s = r - dr;
  const bool ir = r < itf.rho_c, is = s < itf.rho_c;
  if (ir && is) return hraw_diff(r, dr);
  if (ir) return h(r);
  if (is) return -h(s);
  return 0.0;
}

// x^p for an integer p >= 0 by repeated squaring
static inline double ipow(double x, int p) {
  double r = 1.0;
  while (p > 0) {
    if (p & 1) r *= x;
    x *= x;
    p >>= 1;
  }
  return r;
}

// sigma_1 of eq. eqsgm1
double Geometry::sigma(double r) const {
  const double a1 = pml.a1, T = pml.T, S = pml.S;
  const int p = pml.p;
  if (r <= a1) return 0.0;
  if (r > a1 + T) return S;
  double rb = (r - (a1 + T)) / T;
  double f1 = (0.5 - 1.0 / p) * rb * rb * rb + rb / p + 0.5;
  double f2 = 1.0 - f1;
  double f1p = ipow(f1, p), f2p = ipow(f2, p);
  return 2.0 * S * f1p / (f1p + f2p);
}

// int_lo^hi sigma by composite 16-point Gauss-Legendre on 8 pieces of the
// smooth stretch [a1, a1 + T] (and the constant part beyond).
static double sigma_int(const Geometry& g, double lo, double hi) {
  if (hi <= lo) return 0.0;
  const double a1 = g.pml.a1, b1 = g.pml.a1 + g.pml.T;
  double s = 0.0;
  double x0 = fmax(lo, a1), x1 = fmin(hi, b1);
  if (x1 > x0) {
    const int P = 8;
    for (int k = 0; k < P; ++k) {
      double a = x0 + (x1 - x0) * k / P, b = x0 + (x1 - x0) * (k + 1) / P;
      for (int j = 0; j < 16; ++j) s += 0.5 * (b - a) * g.glw[j] * g.sigma(0.5 * (a + b) + 0.5 * (b - a) * g.glx[j]);
    }
  }
  if (hi > b1) s += g.pml.S * (hi - fmax(lo, b1));
  return s;
}
double Geometry::Iint(double r) const { return sigma_int(*this, 0.0, r); }
// Panels never straddle a1 (a segment break), so sigma is smooth on each and
// one 16-point rule from the panel start is exact to rounding.
double Geometry::Ipanel(int p, double r) const {
  const double a = pa[p];
  if (r <= pml.a1) return 0.0;
  double s = 0.0;
  for (int j = 0; j < 16; ++j) s += 0.5 * (r - a) * glw[j] * sigma(a + 0.5 * (r - a) * (1.0 + glx[j]));
  return Ipa[p] + s;
}
double Geometry::Idiff(double r, double dr) const {
  if (fabs(dr) < 1e-2) {
    // short interval: 8-point rule on [r - dr, r] in the offset variable
    static const struct R8 {
      double x[8], w[8];
      R8() { gauss_legendre(8, x, w); }
    } r8;
    const double* x8 = r8.x;
    const double* w8 = r8.w;
    double s = 0.0;
    for (int j = 0; j < 8; ++j) s += 0.5 * w8[j] * sigma(r - dr * 0.5 * (1.0 + x8[j]));
    return s * dr;
  }
  return Iint(r) - Iint(r - dr);
}

void Geometry::point(int pn, double tpar, double& r, double& Ir, double& zz, zd& nr, zd& nz,
                     double& jacobian) const {
  double nu_r, nu_z, sq;
  if (curved) {
    double drt, dzt;
    curve_eval(pn, tpar, r, zz, drt, dzt);
    sq = hypot(drt, dzt);  // |dr/dt|
    nu_r = dzt / sq;
    nu_z = -drt / sq;
  } else if (poly) {
    // straight panel: r(t) = start + (1 + t)/2 (d rho, d z); the normal
    // (z', -rho') / |r'| points into the lower medium for a curve run from
    // the axis outward
    const double u = 0.5 * (1.0 + tpar);
    r = pa[pn] + u * pl[pn];
    zz = pz[pn] + u * pdz[pn];
    nu_r = pdz[pn] / plen[pn];
    nu_z = -pl[pn] / plen[pn];
    sq = 0.0;
  } else {
    r = pa[pn] + 0.5 * (1.0 + tpar) * pl[pn];
    zz = h(r);
    double hpv = hprime(r);
    sq = sqrt(1.0 + hpv * hpv);
    nu_r = hpv / sq;
    nu_z = -1.0 / sq;  // unit normal into the lower medium
  }
  Ir = Ipanel(pn, r);
  zd rt{r, Ir};
  zd ar{1.0, sigma(r)};
  // nu_c . grad_r in stretched variables: n_rho d/drho~ + n_z d/dz~,
  // n_rho = nu_rho rho~ alpha_z / rho, n_z = nu_z rho~ alpha_rho / rho (alpha_z = 1 on the curve)
  nr = (nu_r / r) * rt;
  nz = (nu_z / r) * (rt * ar);
  jacobian = curved ? sq : (poly ? 0.5 * plen[pn] : 0.5 * pl[pn] * sq);
}

// Legendre series on [-1, 1]: P_{k+1} = ((2k + 1) t P_k - k P_{k-1}) / (k + 1),
// P'_{k+1} = P'_{k-1} + (2k + 1) P_k.
void Geometry::curve_eval(int p, double t, double& r, double& zz, double& dr, double& dz) const {
  const double* cr = &cleg[32 * (size_t)p];
  const double* cz = cr + 16;
  double P0 = 1.0, P1 = t, D0 = 0.0, D1 = 1.0;
  r = cr[0] + cr[1] * t;
  zz = cz[0] + cz[1] * t;
  dr = cr[1];
  dz = cz[1];
  for (int k = 1; k < 15; ++k) {
    const double P2 = ((2 * k + 1) * t * P1 - k * P0) / (k + 1);
    const double D2 = D0 + (2 * k + 1) * P1;
    r += cr[k + 1] * P2;
    zz += cz[k + 1] * P2;
    dr += cr[k + 1] * D2;
    dz += cz[k + 1] * D2;
    P0 = P1; P1 = P2; D0 = D1; D1 = D2;
  }
}

// Divided differences Q_k = (P_k(a) - P_k(b)) / (a - b): Q_0 = 0, Q_1 = 1,
// Q_{k+1} = ((2k + 1)(P_k(a) + b Q_k) - k Q_{k-1}) / (k + 1).  h = ta - tb is
// passed exactly: the auxiliary offsets next to a target fall far below the
// spacing of doubles near ta, where ta - tb would round to zero.
void Geometry::curve_diff(int p, double ta, double tb, double h, double& dr, double& dz) const {
  const double* cr = &cleg[32 * (size_t)p];
  const double* cz = cr + 16;
  double P0 = 1.0, P1 = ta, Q0 = 0.0, Q1 = 1.0;
  double sr = cr[1], sz = cz[1];
  for (int k = 1; k < 15; ++k) {
    const double Q2 = ((2 * k + 1) * (P1 + tb * Q1) - k * Q0) / (k + 1);
    const double P2 = ((2 * k + 1) * ta * P1 - k * P0) / (k + 1);
    sr += cr[k + 1] * Q2;
    sz += cz[k + 1] * Q2;
    P0 = P1; P1 = P2; Q0 = Q1; Q1 = Q2;
  }
  dr = h * sr;
  dz = h * sz;
}

const char* Geometry::prepare_curved() {
  gauss_legendre(16, glx, glw);
  const size_t np = cnodes.size() / 32;
  cleg.assign(32 * np, 0.0);
  // c_k = (2k + 1)/2 sum_j w_j P_k(x_j) f_j, exact for the degree-15
  // interpolant; the panel's mean coordinate is taken out first, so that the
  // rounding of the coefficients scales with the panel's size and not with
  // its distance from the origin (the tangent of a short panel far out would
  // otherwise lose digits)
  for (size_t p = 0; p < np; ++p) {
    double mr = 0.0, mz = 0.0;
    for (int j = 0; j < 16; ++j) {
      mr += cnodes[32 * p + 2 * j] / 16.0;
      mz += cnodes[32 * p + 2 * j + 1] / 16.0;
    }
    for (int j = 0; j < 16; ++j) {
      double Pm = 0.0, Pk = 1.0;  // P_{k-1}, P_k at x_j
      for (int k = 0; k < 16; ++k) {
        const double f = 0.5 * (2 * k + 1) * glw[j] * Pk;
        cleg[32 * p + k] += f * (cnodes[32 * p + 2 * j] - mr);
        cleg[32 * p + 16 + k] += f * (cnodes[32 * p + 2 * j + 1] - mz);
        const double Pn = ((2 * k + 1) * glx[j] * Pk - k * Pm) / (k + 1);
        Pm = Pk;
        Pk = Pn;
      }
    }
    cleg[32 * p] += mr;
    cleg[32 * p + 16] += mz;
  }
  // outline: 33 points per panel for the medium test; joins and the axis
  outline.clear();
  for (size_t p = 0; p < np; ++p) {
    for (int k = (p == 0 ? 0 : 1); k <= 32; ++k) {
      double r, zz, a, b;
      curve_eval((int)p, -1.0 + k / 16.0, r, zz, a, b);
      outline.push_back(r);
      outline.push_back(zz);
    }
    if (p + 1 < np) {
      double r0, z0, r1, z1, a, b;
      curve_eval((int)p, 1.0, r0, z0, a, b);
      curve_eval((int)p + 1, -1.0, r1, z1, a, b);
      const double scale = std::max(1.0, fabs(r0) + fabs(z0));
      if (hypot(r1 - r0, z1 - z0) > 1e-9 * scale) return "set_panels: consecutive panels must join";
    }
  }
  if (fabs(outline[0]) > 1e-10) return "set_panels: the curve must start on the axis (rho = 0)";
  return nullptr;
}


// Panels of the polyline model.  Segment s runs from vertex s to vertex s+1
// and is cut at the fractions 0, 1/n, ..., 1 of its length (n = seg_panels[s]);
// where a segment end is a corner (an interior vertex at which the direction
// changes) the end panel is cut again at the fractions 2^-g, ..., 1/2 of its
// own length measured from the corner.
static void poly_layout(const Geometry& g, std::vector<double>& pa, std::vector<double>& pl,
                        std::vector<double>& pz, std::vector<double>& pdz) {
  const int nv = (int)g.verts.size() / 2, nseg = nv - 1;
  std::vector<char> corner(nv, 0);
  for (int j = 1; j < nv - 1; ++j) {
    const double ax = g.verts[2 * j] - g.verts[2 * j - 2], az = g.verts[2 * j + 1] - g.verts[2 * j - 1];
    const double bx = g.verts[2 * j + 2] - g.verts[2 * j], bz = g.verts[2 * j + 3] - g.verts[2 * j + 1];
    const double cr = ax * bz - az * bx, dt = ax * bx + az * bz;
    corner[j] = fabs(cr) > 1e-12 * hypot(ax, az) * hypot(bx, bz) || dt < 0.0;
  }
  pa.clear(); pl.clear(); pz.clear(); pdz.clear();
  for (int s = 0; s < nseg; ++s) {
    const double r0 = g.verts[2 * s], z0 = g.verts[2 * s + 1];
    const double dr = g.verts[2 * s + 2] - r0, dz = g.verts[2 * s + 3] - z0;
    const int n = g.seg_panels[s];
    std::vector<double> u;
    u.push_back(0.0);
    if (corner[s])
      for (int l = g.grade; l >= 1; --l) u.push_back(ldexp(1.0, -l) / n);
    for (int k = 1; k < n; ++k) u.push_back((double)k / n);
    if (corner[s + 1])
      for (int l = 1; l <= g.grade; ++l) u.push_back(1.0 - ldexp(1.0, -l) / n);
    u.push_back(1.0);
    for (size_t k = 0; k + 1 < u.size(); ++k) {
      pa.push_back(r0 + u[k] * dr);
      pz.push_back(z0 + u[k] * dz);
      pl.push_back((u[k + 1] - u[k]) * dr);
      pdz.push_back((u[k + 1] - u[k]) * dz);
    }
  }
}

bool Geometry::above(double r, double zz) const {
  if (!poly && !curved) return zz > h(r);
  if (r >= rho_end()) return zz > 0.0;
  // vertical ray from the point upward: an even number of crossings with the
  // curve (the polyline, or the outline of the curved panels) means the
  // point lies above it
  const std::vector<double>& V = curved ? outline : verts;
  const int nv = (int)V.size() / 2;
  int cross = 0;
  for (int j = 0; j + 1 < nv; ++j) {
    const double r0 = V[2 * j], z0 = V[2 * j + 1], r1 = V[2 * j + 2], z1 = V[2 * j + 3];
    if ((r0 < r) == (r1 < r)) continue;
    const double zc = z0 + (r - r0) / (r1 - r0) * (z1 - z0);
    if (zc > zz) ++cross;
  }
  return (cross & 1) == 0;
}

const char* Geometry::poly_pml_error(double a1) const {
  if (curved) {
    const size_t np = cnodes.size() / 32;
    for (size_t p = 0; p < np; ++p) {
      double lo = 1e300, hi = -1e300, zmax = 0.0;
      for (int k = 0; k <= 32; ++k) {
        double r, zz, a, b;
        curve_eval((int)p, -1.0 + k / 16.0, r, zz, a, b);
        lo = std::min(lo, r);
        hi = std::max(hi, r);
      }
      for (int j = 0; j < 16; ++j) zmax = std::max(zmax, fabs(cnodes[32 * p + 2 * j + 1]));
      if (hi > a1 * (1 + 1e-12) && lo < a1 * (1 - 1e-12))
        return "set_media_pml: a panel may not straddle the start of the PML (rho = a1)";
      if (hi > a1 * (1 + 1e-12) && zmax != 0.0) return "set_media_pml: the curve must be flat (z = 0) where rho > a1";
    }
    return nullptr;
  }
  if (!poly) return nullptr;
  const int nv = (int)verts.size() / 2;
  for (int j = 0; j + 1 < nv; ++j) {
    const double r0 = verts[2 * j], r1 = verts[2 * j + 2];
    const double lo = std::min(r0, r1), hi = std::max(r0, r1);
    if (hi > a1 && lo < a1)
      return "set_media_pml: a polyline vertex must lie at rho = a1 (no segment may straddle the start of the PML)";
    if (hi > a1 && (verts[2 * j + 1] != 0.0 || verts[2 * j + 3] != 0.0))
      return "set_media_pml: the polyline must be flat (z = 0) where rho > a1";
  }
  return nullptr;
}

void Geometry::build() {
  gauss_legendre(16, glx, glw);
  if (curved) {
    const int np = (int)(cnodes.size() / 32);
    pa.assign(np, 0.0); pl.assign(np, 0.0); pz.assign(np, 0.0); pdz.assign(np, 0.0);
    for (int p = 0; p < np; ++p) {
      double r0, z0, r1, z1, a, b;
      curve_eval(p, -1.0, r0, z0, a, b);
      curve_eval(p, 1.0, r1, z1, a, b);
      pa[p] = r0; pl[p] = r1 - r0; pz[p] = z0; pdz[p] = z1 - z0;
    }
    plen.assign(np, 1.0);  // replaced by the arclength below
  } else if (poly) {
    poly_layout(*this, pa, pl, pz, pdz);
    plen.resize(pa.size());
    for (size_t p = 0; p < pa.size(); ++p) plen[p] = hypot(pl[p], pdz[p]);
  } else {
    if (breaks.size() != 5) throw std::invalid_argument("geometry: need 5 segment breaks");
    if (nodes_per_segment <= 0 || nodes_per_segment % 16)
      throw std::invalid_argument("geometry: nodes per segment must be a positive multiple of 16");
    const int nsub = nodes_per_segment / 16;
    pa.clear();
    pl.clear();
    for (int s = 0; s < 4; ++s) {
      double a = breaks[s], b = breaks[s + 1];
      if (!(b > a)) throw std::invalid_argument("geometry: segment breaks must increase");
      for (int k = 0; k < nsub; ++k) {
        pa.push_back(a + (b - a) * k / nsub);
        pl.push_back((b - a) / nsub);
      }
    }
    // the parameter is linear in rho on a graph panel
    plen = pl;
  }
  const int np = npanels(), N = np * 16;
  Ipa.assign(np, 0.0);
  for (int p = 0; p < np; ++p) Ipa[p] = Iint(pa[p]);
  rho.assign(N, 0); I.assign(N, 0); z.assign(N, 0); hp.assign(N, 0); nur.assign(N, 0);
  nuz.assign(N, 0); jac.assign(N, 0); W.assign(N, 0); t.assign(N, 0);
  nr_re.assign(N, 0); nr_im.assign(N, 0); nz_re.assign(N, 0); nz_im.assign(N, 0);
  panel.assign(N, 0);
  for (int p = 0; p < np; ++p)
    for (int j = 0; j < 16; ++j) {
      const int i = 16 * p + j;
      zd nr, nz;
      point(p, glx[j], rho[i], I[i], z[i], nr, nz, jac[i]);
      if (curved) {
        // the nodes are the given coordinates (the interpolant passes
        // through them); the tangent is the interpolant's
        double r2, z2, drt, dzt;
        curve_eval(p, glx[j], r2, z2, drt, dzt);
        const double sp = hypot(drt, dzt);
        rho[i] = cnodes[32 * (size_t)p + 2 * j];
        z[i] = cnodes[32 * (size_t)p + 2 * j + 1];
        I[i] = Ipanel(p, rho[i]);
        hp[i] = 0.0;
        nur[i] = dzt / sp;
        nuz[i] = -drt / sp;
        const zd rt{rho[i], I[i]}, ar{1.0, sigma(rho[i])};
        nr = (nur[i] / rho[i]) * rt;
        nz = (nuz[i] / rho[i]) * (rt * ar);
      } else if (poly) {
        hp[i] = 0.0;  // not a graph
        nur[i] = pdz[p] / plen[p];
        nuz[i] = -pl[p] / plen[p];
      } else {
        hp[i] = hprime(rho[i]);
        double sq = sqrt(1.0 + hp[i] * hp[i]);
        nur[i] = hp[i] / sq;
        nuz[i] = -1.0 / sq;
      }
      nr_re[i] = nr.re; nr_im[i] = nr.im; nz_re[i] = nz.re; nz_im[i] = nz.im;
      W[i] = glw[j] * rho[i] * jac[i];
      t[i] = glx[j];
      panel[i] = p;
    }
  parc.assign(np, 0.0);
  for (int p = 0; p < np; ++p)
    for (int j = 0; j < 16; ++j) parc[p] += glw[j] * jac[16 * p + j];
  // on curved panels the parameter is not linear in a known length; the
  // arclength serves to size the auxiliary rules
  if (curved) plen = parc;
}

// Lagrange basis on the 16 Gauss-Legendre nodes, barycentric form; bw holds
// the barycentric weights 1 / prod_{m != l} (x_l - x_m).
static void lagrange_weights16(const double* xn, double* bw) {
  for (int l = 0; l < 16; ++l) {
    double p = 1.0;
    for (int m = 0; m < 16; ++m)
      if (m != l) p *= (xn[l] - xn[m]);
    bw[l] = 1.0 / p;
  }
}
static void lagrange16(const double* xn, const double* bw, double tq, double* out) {
  for (int l = 0; l < 16; ++l)
    if (tq == xn[l]) {
      for (int m = 0; m < 16; ++m) out[m] = m == l ? 1.0 : 0.0;
      return;
    }
  double den = 0.0;
  for (int l = 0; l < 16; ++l) den += bw[l] / (tq - xn[l]);
  for (int l = 0; l < 16; ++l) out[l] = (bw[l] / (tq - xn[l])) / den;
}

// Auxiliary rules.  Self panel: each side of the target is covered by
// `levels` intervals shrinking by 4 toward the target plus an innermost
// interval mapped by t = eps u^6 (smooths the log singularity), 16 points
// each.  Neighbour panels: intervals shrinking by 4 toward the shared
// endpoint until their length is below the target's distance to that end.
// Every interval longer than hmax (physical length) is cut into equal pieces
// of at most hmax, and the self-panel levels continue until the mapped
// interval is that short too: the kernel oscillates and grows at the rate
// |k| |1 + i sigma|, and the 16-point rule must resolve it times a degree-15
// Lagrange factor.
void Geometry::build_near(std::vector<PairGeom>& geom, std::vector<double>& coef,
                          std::vector<NearJob>& jobs, int self_levels, double hmax) const {
  const int N = n(), np = npanels();
  double bw[16];
  lagrange_weights16(glx, bw);
  struct Local {
    std::vector<PairGeom> g;
    std::vector<double> c;
    std::vector<NearJob> j;
  };
  std::vector<Local> loc(N);
#pragma omp parallel for schedule(dynamic, 8)
  for (int i = 0; i < N; ++i) {
    Local& L = loc[i];
    L.g.reserve(512);
    L.c.reserve(16 * 512);
    L.j.reserve(3);
    const int p0 = panel[i];
    for (int pn = p0 - 1; pn <= p0 + 1; ++pn) {
      if (pn < 0 || pn >= np) continue;
      NearJob J;
      J.target = i;
      J.panel = pn;
      J.q0 = (int)L.g.size();
      // points as (anchor, offset, side sign, weight): t = anchor + sgn * off
      struct AP { double anchor, off, sgn, w; };
      std::vector<AP> pts;
      // half the physical length per unit of panel parameter
      const double hs = 0.5 * plen[pn];
      // 16-point rule on offsets [lo, hi], in pieces of physical length <= hmax
      auto interval = [&](double anchor, double sgn, double lo, double hi) {
        const int np = std::max(1, (int)ceil((hi - lo) * hs / hmax - 1e-9));
        for (int k = 0; k < np; ++k) {
          const double a = lo + (hi - lo) * k / np, b = lo + (hi - lo) * (k + 1) / np;
          for (int j = 0; j < 16; ++j)
            pts.push_back({anchor, a + 0.5 * (b - a) * (1.0 + glx[j]), sgn, 0.5 * (b - a) * glw[j]});
        }
      };
      if (pn == p0) {
        const double ti = t[i];
        for (int side = -1; side <= 1; side += 2) {
          const double h = side > 0 ? 1.0 - ti : ti + 1.0;
          double hi = h;
          for (int lv = 0; lv < self_levels || hi * hs > hmax; ++lv) {
            double lo = hi * 0.25;
            interval(ti, (double)side, lo, hi);
            hi = lo;
          }
          const double eps = hi;
          for (int j = 0; j < 16; ++j) {
            double u = 0.5 * (1.0 + glx[j]);
            double u5 = u * u * u * u * u;
            pts.push_back({ti, eps * u5 * u, (double)side, eps * 0.5 * glw[j] * 6.0 * u5});
          }
        }
      } else {
        // shared endpoint of the neighbour panel: +1 if it lies left of p0
        const double anchor = pn < p0 ? 1.0 : -1.0;
        const double sgn = pn < p0 ? -1.0 : 1.0;
        // target distance to the shared end, in neighbour-panel units
        const double dist = (pn < p0 ? (1.0 + t[i]) : (1.0 - t[i])) * plen[p0] / plen[pn];
        double hi = 2.0;
        int nint = 0;
        while (true) {
          double lo = hi * 0.25;
          // at least three intervals, so that the rule also resolves the
          // Lagrange factor when the target is far from the shared end
          if (hi <= dist && nint >= 2) lo = 0.0;
          ++nint;
          interval(anchor, sgn, lo, hi);
          if (lo == 0.0) break;
          hi = lo;
        }
      }
      for (const AP& a : pts) {
        const double tp = a.anchor + a.sgn * a.off;
        double r, Ir, zz, jc;
        zd nr, nz;
        point(pn, tp, r, Ir, zz, nr, nz, jc);
        // target minus source, from the exact offset on the self panel
        double dr, dzv;
        if (pn == p0) {
          if (curved) {
            curve_diff(pn, t[i], tp, -a.sgn * a.off, dr, dzv);
          } else {
            dr = -a.sgn * a.off * 0.5 * pl[pn];
            dzv = poly ? -a.sgn * a.off * 0.5 * pdz[pn] : hdiff(rho[i], dr);
          }
        } else {
          dr = rho[i] - r;
          dzv = (poly || curved) ? z[i] - zz : hdiff(rho[i], dr);
        }
        PairGeom g;
        g.rt = zd{rho[i], I[i]};
        g.rs = zd{r, Ir};
        g.drho = zd{dr, fabs(dr) < 1e-2 ? Idiff(rho[i], dr) : I[i] - Ir};
        g.dz = zd{dzv, 0.0};
        g.nr = nr;
        g.nz = nz;
        L.g.push_back(g);
        double Lg[16];
        lagrange16(glx, bw, tp, Lg);
        const double base = 2.0 * a.w * r * jc;
        for (int l = 0; l < 16; ++l) L.c.push_back(base * Lg[l]);
      }
      J.q1 = (int)L.g.size();
      L.j.push_back(J);
    }
  }
  // concatenate in target order: offsets first, then every target copies its
  // own tables in parallel
  std::vector<size_t> og(N + 1, 0), oj(N + 1, 0);
  for (int i = 0; i < N; ++i) {
    og[i + 1] = og[i] + loc[i].g.size();
    oj[i + 1] = oj[i] + loc[i].j.size();
  }
  geom.resize(og[N]);
  coef.resize(16 * og[N]);
  jobs.resize(oj[N]);
#pragma omp parallel for schedule(dynamic, 16)
  for (int i = 0; i < N; ++i) {
    Local& L = loc[i];
    std::copy(L.g.begin(), L.g.end(), geom.begin() + og[i]);
    std::copy(L.c.begin(), L.c.end(), coef.begin() + 16 * og[i]);
    for (size_t k = 0; k < L.j.size(); ++k) {
      NearJob J = L.j[k];
      J.q0 += (int)og[i];
      J.q1 += (int)og[i];
      jobs[oj[i] + k] = J;
    }
    std::vector<PairGeom>().swap(L.g);
    std::vector<double>().swap(L.c);
  }
}

void Geometry::field_near(double r, double zz, int tag, double factor, double hmax,
                          std::vector<PairGeom>& geom, std::vector<double>& coef,
                          std::vector<NearJob>& jobs) const {
  double bw[16];
  lagrange_weights16(glx, bw);
  const double It = Iint(r);
  for (int pn = 0; pn < npanels(); ++pn) {
    // every point of the panel lies within its arclength of the middle node
    const double dmid = hypot(r - rho[16 * pn + 8], zz - z[16 * pn + 8]);
    if (dmid - parc[pn] >= factor * parc[pn]) continue;
    double dmin = 1e300;
    for (int j = 0; j < 16; ++j) dmin = std::min(dmin, hypot(r - rho[16 * pn + j], zz - z[16 * pn + j]));
    if (!(dmin < factor * parc[pn])) continue;
    // closest curve point: the best of 65 samples, refined by golden sections
    auto dist2 = [&](double tp) {
      double rr, Ir, z2, jc;
      zd nr, nz;
      point(pn, tp, rr, Ir, z2, nr, nz, jc);
      return (r - rr) * (r - rr) + (zz - z2) * (zz - z2);
    };
    int kb = 0;
    double db = 1e300;
    for (int k = 0; k <= 64; ++k) {
      const double d2 = dist2(-1.0 + k / 32.0);
      if (d2 < db) {
        db = d2;
        kb = k;
      }
    }
    double a = std::max(-1.0, -1.0 + (kb - 1) / 32.0), b = std::min(1.0, -1.0 + (kb + 1) / 32.0);
    const double gr = 0.5 * (sqrt(5.0) - 1.0);
    double x1 = b - gr * (b - a), x2 = a + gr * (b - a), f1 = dist2(x1), f2 = dist2(x2);
    for (int it = 0; it < 60; ++it) {
      if (f1 < f2) {
        b = x2; x2 = x1; f2 = f1; x1 = b - gr * (b - a); f1 = dist2(x1);
      } else {
        a = x1; x1 = x2; f1 = f2; x2 = a + gr * (b - a); f2 = dist2(x2);
      }
    }
    const double ts = 0.5 * (a + b);
    const double hs = 0.5 * parc[pn];  // physical length per unit of parameter (mean)
    // distance in units of the parameter; the rule on each side of ts shrinks
    // by 4 toward ts until the intervals are below it
    const double dpar = std::max(sqrt(dist2(ts)) / hs, 1e-12);
    NearJob J;
    J.target = tag;
    J.panel = pn;
    J.q0 = (int)geom.size();
    for (int side = -1; side <= 1; side += 2) {
      const double hside = side > 0 ? 1.0 - ts : ts + 1.0;
      if (!(hside > 0.0)) continue;
      double hi = hside;
      for (int nint = 0;; ++nint) {
        double lo = hi * 0.25;
        if ((hi <= dpar && nint >= 2) || nint >= 40) lo = 0.0;
        const int npc = std::max(1, (int)ceil((hi - lo) * hs / hmax - 1e-9));
        for (int k = 0; k < npc; ++k) {
          const double ia = lo + (hi - lo) * k / npc, ib = lo + (hi - lo) * (k + 1) / npc;
          for (int j = 0; j < 16; ++j) {
            const double off = ia + 0.5 * (ib - ia) * (1.0 + glx[j]);
            const double w = 0.5 * (ib - ia) * glw[j];
            const double tp = ts + side * off;
            double rr, Ir, z2, jc;
            zd nr, nz;
            point(pn, tp, rr, Ir, z2, nr, nz, jc);
            PairGeom g;
            g.rt = zd{r, It};
            g.rs = zd{rr, Ir};
            g.drho = zd{r - rr, It - Ir};
            g.dz = zd{zz - z2, 0.0};
            g.nr = nr;
            g.nz = nz;
            geom.push_back(g);
            double Lg[16];
            lagrange16(glx, bw, tp, Lg);
            for (int l = 0; l < 16; ++l) coef.push_back(w * rr * jc * Lg[l] / W[16 * pn + l]);
          }
        }
        if (lo == 0.0) break;
        hi = lo;
      }
    }
    J.q1 = (int)geom.size();
    jobs.push_back(J);
  }
}

}  // namespace pmlbie
