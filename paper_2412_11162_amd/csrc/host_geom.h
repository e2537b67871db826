// Host-side geometry of the Nystrom discretisation: the interface graph, the
// PML stretching (Sec. 3.1, eqs. eqrhot, eqsgm1), Gauss-Legendre panels, the
// conormal (Sec. 3.1, nu_c = A^T nu), and the auxiliary quadrature points of
// the near-panel product integration.
#pragma once
#include <vector>
#include "modal.h"

namespace pmlbie {

struct Interface {
  std::vector<double> amp, cen, wid;  // Gaussian rings a exp(-((rho - c)/w)^2)
  double cos_freq = 0.0;              // optional factor cos(f rho)
  double rho_c = 0.0;                 // flat for rho >= rho_c: h~ = h - h(rho_c) below
};

struct Pml {
  double a1 = 0, T = 0, S = 0;
  int p = 6;
};

// Two curve models.  Graph: z = h~(rho) over four rho segments of equal
// panels.  Polyline: straight segments between vertices (rho_j, z_j) with
// corners allowed (Sec. 4, the graded mesh of eq. eqsxi); each segment holds
// a given number of equal panels, and the panel touching a corner is split
// geometrically toward it (`grade` halvings) so that the nodes cluster at the
// corner singularities.
class Geometry {
 public:
  Interface itf;
  Pml pml;
  std::vector<double> breaks;  // graph: segment breaks in rho, 5 values
  int nodes_per_segment = 0;
  // polyline model (used when poly is set)
  bool poly = false;
  std::vector<double> verts;   // 2 * n_vert: rho_0, z_0, rho_1, z_1, ...
  std::vector<int> seg_panels;  // equal panels per segment before grading
  int grade = 0;
  // curved-panel model (used when curved is set): the caller gives the
  // coordinates (rho, z) at the 16 Gauss-Legendre points of every panel, and
  // the curve on a panel is their degree-15 interpolant
  bool curved = false;
  std::vector<double> cnodes;   // [P][16][2] node coordinates
  std::vector<double> cleg;     // [P][2][16] Legendre coefficients of rho(t) and z(t)
  std::vector<double> outline;  // 2 * K points along the curve (medium test)
  // Legendre coefficients from cnodes; returns an error text or nullptr
  const char* prepare_curved();
  // r(t) and r'(t) on curved panel p
  void curve_eval(int p, double t, double& r, double& zz, double& dr, double& dz) const;
  // r(ta) - r(tb) on curved panel p without cancellation (divided
  // differences), h = ta - tb given exactly
  void curve_diff(int p, double ta, double tb, double h, double& dr, double& dz) const;

  // Gauss-Legendre rule of 16 nodes on [-1, 1].
  double glx[16], glw[16];

  // panels
  std::vector<double> pa, pl;  // start rho and rho-length (signed for polylines)
  std::vector<double> pz, pdz;  // polyline: start z and z-length
  std::vector<double> parc;     // panel arclength
  std::vector<double> plen;     // panel length in the variable its parameter is linear in
                                // (arclength for a polyline, rho for a graph)
  std::vector<double> Ipa;     // Im rho~ at each panel start
  // node tables
  std::vector<double> rho, I, z, hp, nur, nuz, jac, W, t;
  std::vector<double> nr_re, nr_im, nz_re, nz_im;
  std::vector<int> panel;

  void build();  // panels + node tables
  int n() const { return (int)rho.size(); }
  int npanels() const { return (int)pa.size(); }

  double rho_end() const {
    if (curved) return outline[outline.size() - 2];
    return poly ? verts[verts.size() - 2] : breaks[4];
  }
  // the point lies above the curve (in the upper medium); points on the
  // curve are not classified
  bool above(double r, double zz) const;
  // polyline checks against the PML: no panel straddles a1 and the curve is
  // flat (z = 0) wherever rho > a1; returns an error text or nullptr
  const char* poly_pml_error(double a1) const;

  double h(double r) const;            // h~(rho)
  double hprime(double r) const;       // h~'(rho)
  double hdiff(double r, double dr) const;  // h~(r) - h~(r - dr), no cancellation
  double sigma(double r) const;        // sigma_1
  double Iint(double r) const;         // int_0^r sigma_1
  double Ipanel(int p, double r) const;  // int_0^r sigma_1 for r on panel p
  double Idiff(double r, double dr) const;  // int_{r - dr}^{r} sigma_1
  // geometry of a curve point given by its panel and parameter
  void point(int panel, double tpar, double& r, double& Ir, double& zz, zd& nr, zd& nz,
             double& jacobian) const;

  // near-panel product integration: auxiliary points, their pair geometry
  // relative to the target, Lagrange-weighted quadrature coefficients, jobs
  void build_near(std::vector<PairGeom>& geom, std::vector<double>& coef,
                  std::vector<NearJob>& jobs, int self_levels, double hmax) const;

  // Field point (r, z) off the curve: for every panel closer than `factor`
  // times its arclength, auxiliary points graded toward the closest curve
  // point and coefficients w rho |r'| l_l(t) / W_l that turn their modal
  // kernels into the panel's 16 node entries (product integration of the
  // Lagrange-interpolated densities); appended as jobs with target = tag.
  void field_near(double r, double zz, int tag, double factor, double hmax,
                  std::vector<PairGeom>& geom, std::vector<double>& coef,
                  std::vector<NearJob>& jobs) const;

 private:
  double graw(double r) const;
  double graw_d(double r) const;
  double graw_diff(double r, double dr) const;
  double hraw_diff(double r, double dr) const;
  double hraw_d(double r) const;
};

void gauss_legendre(int n, double* x, double* w);

}  // namespace pmlbie
