// Host build of the exact in-circle predicate (rd_predicates.h) for its
// CPU tests: the same source the GPU kernels compile, built with g++ and
// -ffp-contract=off.
#include <vector>

#include "rd_predicates.h"

extern "C" {

int rdp_incircle_filter(const double* a, const double* b, const double* c, const double* d) {
  return rd::pred::incircle_filter(a, b, c, d);
}

int rdp_incircle_exact(const double* a, const double* b, const double* c, const double* d) {
  std::vector<double> w(rd::pred::kIncircleScratch);
  return rd::pred::incircle_exact(a, b, c, d, w.data());
}

int rdp_orient(const double* a, const double* b, const double* c) { return rd::pred::orient(a, b, c); }

// Expansion product and sum of two doubles' products, for the arithmetic checks:
// out[0..n) = (a0 * a1) * (b0 * b1) as an expansion; returns n.
int rdp_product4(double a0, double a1, double b0, double b1, double* out) {
  double e[2], f[2], tmp[64];
  rd::pred::two_product(a0, a1, e[1], e[0]);
  rd::pred::two_product(b0, b1, f[1], f[0]);
  int ne = 0, nf = 0;
  double ez[2], fz[2];
  if (e[0] != 0.0) ez[ne++] = e[0];
  ez[ne++] = e[1];
  if (f[0] != 0.0) fz[nf++] = f[0];
  fz[nf++] = f[1];
  return rd::pred::mul(ne, ez, nf, fz, out, tmp);
}
}
