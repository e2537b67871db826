// CPU driver for the library's host-side geometry (no device calls): builds a
// curve from the command line and prints its tables as plain numbers for the
// host-logic tests.  Not part of the library.
//
//   driver layout  <grade> <n_vert> rho0 z0 ... <panels per segment...>
//   driver tables  poly|graph|curved ...   (see parse_curve)
//   driver above   <curve...> -- r z r z ...
//   driver near    <curve...>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "host_geom.h"

using namespace pmlbie;

// curve spec: "poly grade nv (r z)*nv np*(nv-1)" | "graph npseg a w" |
// "curved file"; PML a1 T S follow as three numbers.
static int parse_curve(int argc, char** argv, int i, Geometry& g) {
  const std::string kind = argv[i++];
  if (kind == "poly") {
    g.poly = true;
    g.grade = atoi(argv[i++]);
    const int nv = atoi(argv[i++]);
    for (int k = 0; k < 2 * nv; ++k) g.verts.push_back(atof(argv[i++]));
    for (int k = 0; k < nv - 1; ++k) g.seg_panels.push_back(atoi(argv[i++]));
  } else if (kind == "graph") {
    g.nodes_per_segment = atoi(argv[i++]);
    g.itf.amp = {atof(argv[i++])};
    g.itf.cen = {0.0};
    g.itf.wid = {atof(argv[i++])};
  } else {
    FILE* f = fopen(argv[i++], "r");
    double v;
    while (f && fscanf(f, "%lf", &v) == 1) g.cnodes.push_back(v);
    if (f) fclose(f);
    g.curved = true;
    if (g.prepare_curved()) return -1;
  }
  g.pml.a1 = atof(argv[i++]);
  g.pml.T = atof(argv[i++]);
  g.pml.S = atof(argv[i++]);
  g.pml.p = 6;
  if (kind == "graph") {
    g.itf.rho_c = g.pml.a1;
    const double a1 = g.pml.a1, T = g.pml.T;
    g.breaks = {0.0, 0.5 * a1, a1, a1 + 0.5 * T, a1 + T};
  }
  g.build();
  (void)argc;
  return i;
}

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  const std::string cmd = argv[1];
  Geometry g;
  int i = parse_curve(argc, argv, 2, g);
  if (i < 0) {
    printf("error\n");
    return 1;
  }
  if (cmd == "layout") {
    for (int p = 0; p < g.npanels(); ++p) printf("%.17g %.17g %.17g %.17g\n", g.pa[p], g.pl[p], g.pz[p], g.pdz[p]);
  } else if (cmd == "tables") {
    for (int k = 0; k < g.n(); ++k)
      printf("%.17g %.17g %.17g %.17g %.17g %.17g %.17g\n", g.rho[k], g.I[k], g.z[k], g.W[k], g.nur[k], g.nuz[k],
             g.jac[k]);
  } else if (cmd == "above") {
    for (++i; i + 1 < argc; i += 2) printf("%d\n", g.above(atof(argv[i]), atof(argv[i + 1])) ? 1 : 2);
  } else if (cmd == "near") {
    std::vector<PairGeom> geom;
    std::vector<double> coef;
    std::vector<NearJob> jobs;
    g.build_near(geom, coef, jobs, 6, 1e300);
    // per job: target, panel, points, then sum over points of each of the 16
    // coefficients
    for (const NearJob& J : jobs) {
      printf("%d %d %d", J.target, J.panel, J.q1 - J.q0);
      for (int l = 0; l < 16; ++l) {
        double s = 0.0;
        for (int q = J.q0; q < J.q1; ++q) s += coef[16L * q + l];
        printf(" %.17g", s);
      }
      printf("\n");
    }
  }
  return 0;
}
