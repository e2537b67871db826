// Device numerics of the modal-kernel generator: the PML-complexified
// Green's function and its conormal derivative (Sec. 3.1), the stable
// complex distance (Sec. 4.3), the kernel split S = Z (H1 + i H2),
// K = D (H3 + i H4) of Sec. 4.1 with its smooth parts, and the semi-analytic
// modes Z_m, D_m of the singular factors through half-integer-degree
// Legendre functions Q_{m-1/2} (toroidal functions) evaluated from Carlson's
// symmetric elliptic integrals and three-term recurrences.
#pragma once
#include "cplx.h"

#ifndef PMLBIE_PI
#define PMLBIE_PI 3.141592653589793238462643383279502884
#endif

// Geometry of one (target, source) pair in the stretched coordinates.
struct PairGeom {
  zd rt, rs;    // rho~ of target and source
  zd drho, dz;  // rho~_t - rho~_s and z~_t - z~_s (formed from differences)
  zd nr, nz;    // conormal of the source: n_rho, n_z
};

// Invariants of a pair used by every sample: R^2 = d2 + c4 sin^2(D/2) and the
// conormal numerator N(D) = N0 + N1 sin^2(D/2).
struct PairInv {
  zd d2, c4, N0, N1;
};

// rho~_t rho~_s with both products rounded before the sum, so that the
// result does not depend on the order of the two points (a fused
// multiply-add of one ordering would round the other product only): the
// invariants of (i, l) and (l, i) are then the same to the bit.
HD zd rho_product(zd a, zd b) {
#pragma clang fp contract(off)
  const double p1 = a.re * b.re, p2 = a.im * b.im;
  const double p3 = a.re * b.im, p4 = a.im * b.re;
  return zd{p1 - p2, p3 + p4};
}

HD PairInv pair_invariants(const PairGeom& g) {
  PairInv v;
  v.d2 = g.drho * g.drho + g.dz * g.dz;
  v.c4 = 4.0 * rho_product(g.rt, g.rs);
  v.N0 = -(g.nr * g.drho + g.nz * g.dz);
  v.N1 = 2.0 * (g.nr * g.rt);
  return v;
}

// G~ and dG~/dnu_c(r') at one azimuth difference (s2 = sin^2(D/2)).
HD void kernel_sample(const PairInv& v, double s2, zd k, zd& S, zd& K) {
  zd R2 = v.d2 + s2 * v.c4;
  zd R = csqrt_(R2);
  zd ikR = zd{0.0, 1.0} * (k * R);
  zd e = cexp_(ikR);
  zd inv4piR = inv(R) * (0.25 / PMLBIE_PI);
  S = e * inv4piR;
  zd N = v.N0 + s2 * v.N1;
  K = N * e * (ikR - 1.0) * inv4piR * inv(R2);
}

// Split coefficients of the double-layer singular factor:
// D = -(e0/R^3 + e1/R)/(4 pi), with e0 = N0 - n_rho' d2/(2 rho~'), e1 = n_rho'/(2 rho~').
struct SplitCoef {
  zd e0, e1;
};
HD SplitCoef split_coef(const PairGeom& g, const PairInv& v) {
  zd h = inv(2.0 * g.rs);
  SplitCoef c;
  c.e1 = g.nr * h;
  c.e0 = v.N0 - c.e1 * v.d2;
  return c;
}

// cos q and sin q of a complex argument from one sine/cosine pair of Re q
// and one expm1 of Im q (cosh and sinh without cancellation).
HD void ccossin_(zd q, zd& c, zd& s) {
  const double sx = sin(q.re), cx = cos(q.re);
  const double em = expm1(q.im), ep = em + 1.0;
  const double h = 0.5 / ep;
  const double ch = 1.0 + em * em * h, sh = em * (em + 2.0) * h;
  c = zd{cx * ch, -sx * sh};
  s = zd{sx * ch, cx * sh};
}

// Smooth parts of the split at one sample (complex distance R) for
// wavenumber k, q = k R:
//   H1 = cos q, ZH2 = sin(q)/(4 pi R) = k sinc(q)/(4 pi), H3 = cos q + q sin q,
//   DH4 = D (sin q - q cos q) = -(1/4pi)(e0 k^3 + e1 k q^2) s3(q),
// with sinc(q) = sin(q)/q and s3(q) = (sin q - q cos q)/q^3, both entire in
// q^2 and summed from their Taylor series for |q| < 1.
HD void split_smooth(const SplitCoef& sc, zd R, zd k, zd& H1, zd& ZH2, zd& H3, zd& DH4) {
  const zd q = k * R;
  zd cq, sq;
  ccossin_(q, cq, sq);
  H1 = cq;
  H3 = cq + q * sq;
  const zd q2 = q * q;
  zd sn, s3;
  if (cabs1(q) < 1.0) {
    // sinc = sum_i (-1)^i q^{2i}/(2i+1)!, s3 = sum_i (-1)^i 2(i+1) q^{2i}/(2i+3)!
    zd pw{1.0, 0.0};
    sn = zd{0.0, 0.0};
    s3 = zd{0.0, 0.0};
    double f1 = 1.0;
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      const double sg = (i & 1) ? -1.0 : 1.0;
      const double f3 = f1 * (2.0 * i + 2.0) * (2.0 * i + 3.0);
      sn = sn + (sg / f1) * pw;
      s3 = s3 + (sg * (2.0 * i + 2.0) / f3) * pw;
      pw = pw * q2;
      f1 = f3;
    }
  } else {
    const zd iq = inv(q);
    sn = sq * iq;
    s3 = (sq - q * cq) * (iq * iq * iq);
  }
  ZH2 = (0.25 / PMLBIE_PI) * (k * sn);
  DH4 = (sc.e0 * (k * k * k) + sc.e1 * k * q2) * s3 * (-0.25 / PMLBIE_PI);
}

// The substitution of Sec. 4.3 (eq. eqch1) at one sample, q = k R: cH1 =
// e^{iq} P_L(q) with P_L the Taylor polynomial of order L of cos(q) e^{-iq},
// and cH3 = e^{iq} Q_L(q) with Q_L that of H3 e^{-iq}.  With Z = 1/(4 pi R)
// and the double-layer factor D, S = Z cH1 + Z (e^{iq} - cH1) and
// K = D cH3 + D (e^{iq} (1 - iq) - cH3) (H3 + i H4 = e^{iq} (1 - iq)).
// Returned: cH1, the S remainder, cH3 and the K remainder.  From
// cos(q) e^{-iq} = (1 + e^{-2iq}) / 2 and H3 e^{-iq} = ((1 - iq) + (1 + iq)
// e^{-2iq}) / 2: a_0 = 1, a_j = t_j / 2; b_0 = 1, b_1 = -i and
// b_j = (t_j + i t_{j-1}) / 2 for j >= 2, with t_j = (-2i)^j / j!; b_2 = 0
// exactly.  The remainders are summed from their series in q, so that no
// division by R occurs: Z (e^{iq} - cH1) = -e^{iq} k sum_{j>=1} a_j q^{j-1}
// / (4 pi) and D (e^{iq} (1 - iq) - cH3) = e^{iq} sum_{j>=3} b_j (e0 k^3
// q^{j-3} + e1 k q^{j-1}) / (4 pi).
HD void split_smooth_ch(const SplitCoef& sc, zd R, zd k, int L, zd& H1c, zd& Srem, zd& H3c, zd& Krem) {
  const zd q = k * R;
  zd cq, sq;
  ccossin_(q, cq, sq);
  const zd eq = cq + zd{-sq.im, sq.re};  // e^{iq}
  const zd k3 = k * k * k;
  zd P{1.0, 0.0}, Q{1.0, 0.0}, sr{0.0, 0.0}, kr{0.0, 0.0};
  zd t{1.0, 0.0};   // t_j
  zd qm{1.0, 0.0};  // q^{j-1}
  zd qm3{1.0, 0.0};  // q^{j-3} (from j = 3)
  for (int j = 1; j <= L; ++j) {
    const zd tp = t;
    t = zd{2.0 * t.im, -2.0 * t.re} * (1.0 / j);  // t_j = t_{j-1} (-2i) / j
    const zd a = 0.5 * t;
    const zd b = j == 1 ? zd{0.0, -1.0} : 0.5 * (t + zd{-tp.im, tp.re});
    sr = sr + a * qm;
    const zd qj = qm * q;
    P = P + a * qj;
    Q = Q + b * qj;
    if (j >= 3) {
      kr = kr + b * (sc.e0 * k3 * qm3 + sc.e1 * k * qm);
      qm3 = qm3 * q;
    }
    qm = qj;
  }
  const double f = 0.25 / PMLBIE_PI;
  H1c = eq * P;
  H3c = eq * Q;
  Srem = (-f) * (eq * (k * sr));
  Krem = f * (eq * kr);
}

// ---------------------------------------------------------------------------
// Carlson's symmetric elliptic integrals for complex arguments (duplication
// algorithm, Carlson 1995; valid for arguments off the negative real axis).
HD zd carlson_rf(zd x, zd y, zd z) {
  zd A0 = (x + y + z) * (1.0 / 3.0);
  double Qm = fmax(cabs_(A0 - x), fmax(cabs_(A0 - y), cabs_(A0 - z))) * 600.0;
  zd xm = x, ym = y, zm = z, Am = A0;
  double p4 = 1.0;
  for (int it = 0; it < 60 && p4 * Qm > cabs_(Am); ++it) {
    zd sx = csqrt_(xm), sy = csqrt_(ym), sz = csqrt_(zm);
    zd lam = sx * sy + sx * sz + sy * sz;
    xm = (xm + lam) * 0.25;
    ym = (ym + lam) * 0.25;
    zm = (zm + lam) * 0.25;
    Am = (Am + lam) * 0.25;
    p4 *= 0.25;
  }
  zd iA = inv(Am);
  zd X = (A0 - x) * iA * p4, Y = (A0 - y) * iA * p4;
  zd Z = -(X + Y);
  zd E2 = X * Y - Z * Z, E3 = X * Y * Z;
  zd ser = zd{1.0, 0.0} - E2 * (1.0 / 10.0) + E3 * (1.0 / 14.0) + E2 * E2 * (1.0 / 24.0) -
           E2 * E3 * (3.0 / 44.0);
  return ser * inv(csqrt_(Am));
}

HD zd carlson_rd(zd x, zd y, zd z) {
  zd A0 = (x + y + 3.0 * z) * (1.0 / 5.0);
  double Qm = fmax(cabs_(A0 - x), fmax(cabs_(A0 - y), cabs_(A0 - z))) * 1000.0;
  zd xm = x, ym = y, zm = z, Am = A0, sum = zd{0.0, 0.0};
  double p4 = 1.0;
  for (int it = 0; it < 60 && p4 * Qm > cabs_(Am); ++it) {
    zd sx = csqrt_(xm), sy = csqrt_(ym), sz = csqrt_(zm);
    zd lam = sx * sy + sx * sz + sy * sz;
    sum = sum + p4 * inv(sz * (zm + lam));
    xm = (xm + lam) * 0.25;
    ym = (ym + lam) * 0.25;
    zm = (zm + lam) * 0.25;
    Am = (Am + lam) * 0.25;
    p4 *= 0.25;
  }
  zd iA = inv(Am);
  zd X = (A0 - x) * iA * p4, Y = (A0 - y) * iA * p4;
  zd Z = -(X + Y) * (1.0 / 3.0);
  zd XY = X * Y, Z2 = Z * Z;
  zd E2 = XY - 6.0 * Z2;
  zd E3 = (3.0 * XY - 8.0 * Z2) * Z;
  zd E4 = 3.0 * (XY - Z2) * Z2;
  zd E5 = XY * Z2 * Z;
  zd ser = zd{1.0, 0.0} - E2 * (3.0 / 14.0) + E3 * (1.0 / 6.0) + E2 * E2 * (9.0 / 88.0) -
           E4 * (3.0 / 22.0) - E2 * E3 * (9.0 / 52.0) + E5 * (3.0 / 26.0);
  return p4 * ser * iA * inv(csqrt_(Am)) + 3.0 * sum;
}

// Q[m qs] = Q_{m-1/2}(chi) for m = 0..mq, chi = 1 + chim1 (chim1 passed exactly).
// Q_{-1/2} = sqrt2 RF(0, chi-1, chi+1); Q_{1/2} from RF and RD; higher
// degrees by forward recurrence when it is stable over the range, else by the
// backward (Miller) ratio recurrence normalised by Q_{-1/2}.
HD void legendre_q_half(zd chim1, int mq, zd* Q, long qs = 1) {
  const double rt2 = 1.4142135623730950488;
  zd chi = chim1 + 1.0;
  zd zero = zd{0.0, 0.0};
  zd rf = carlson_rf(zero, chim1, chim1 + 2.0);
  Q[0] = rt2 * rf;
  if (mq == 0) return;
  zd s = csqrt_(chim1) * csqrt_(chim1 + 2.0);
  double La = log(fmax(cabs_(chi + s), cabs_(chi - s)));  // -log of the decay ratio
  if (2.0 * mq * La <= 6.0) {
    zd rd = carlson_rd(zero, chim1, chim1 + 2.0);
    Q[qs] = rt2 * (-rf + (2.0 / 3.0) * (chim1 + 2.0) * rd);
    for (int m = 1; m < mq; ++m) {
      // (m + 1/2) Q_{m+1/2} = 2 m chi Q_{m-1/2} - (m - 1/2) Q_{m-3/2}
      Q[(m + 1) * qs] = ((2.0 * m) * chi * Q[m * qs] - (m - 0.5) * Q[(m - 1) * qs]) * (1.0 / (m + 0.5));
    }
  } else {
    int ns = mq + (int)ceil(19.0 / La) + 8;
    if (ns > mq + 6000) ns = mq + 6000;
    zd r = zero;  // r_{m} = Q_{m-1/2} / Q_{m-3/2}
    for (int m = ns; m > mq; --m) r = (m - 0.5) * inv((2.0 * m) * chi - (m + 0.5) * r);
    // keep the ratios for m = mq..1 in Q temporarily
    for (int m = mq; m >= 1; --m) {
      r = (m - 0.5) * inv((2.0 * m) * chi - (m + 0.5) * r);
      Q[m * qs] = r;
    }
    for (int m = 1; m <= mq; ++m) Q[m * qs] = Q[m * qs] * Q[(m - 1) * qs];
  }
}

// Singularity distance of the azimuthal integrand: the zeros of R^2 sit at
// sin^2(D*/2) = -d2/c4; returns |Im D*| and Re D* (folded into [0, pi]).
HD void singularity(const PairInv& v, double& delta, double& re0) {
  if (v.c4.re == 0.0 && v.c4.im == 0.0) {  // a point on the axis: no azimuthal dependence
    delta = 1e300;
    re0 = 0.0;
    return;
  }
  zd w = -(v.d2 / v.c4);
  zd sw = csqrt_(w);
  zd t = zd{0.0, 1.0} * sw + csqrt_(zd{1.0, 0.0} - w);
  // asin(sw) = -i log(t) = arg(t) - i log|t|
  double im = -log(cabs_(t));
  double re = atan2(t.im, t.re);
  delta = 2.0 * fabs(im);
  re0 = fmin(fabs(2.0 * re), PMLBIE_PI);
}
