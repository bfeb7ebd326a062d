// B-spline evaluation shared by the host setup routines (collocation and Galerkin).
#pragma once

#include <cstdint>
#include <vector>

namespace fdg {

// Open uniform knot vector with E spans, kept as integer numerators over E:
// p+1 zeros, 1..E-1, p+1 copies of E.  Returns the numerators (E + 2p + 1 entries).
std::vector<int64_t> open_knots(int p, int E);

// Local evaluation of the p+1 B-splines that can be non-zero at x, with their first
// and second derivatives.  span is the index s with xi_s <= x < xi_{s+1} (the last
// non-empty span when x is the right end); on return f[r][t] holds the r-th
// derivative of B_{s-p+t}.  p <= 15.
struct LocalBasis {
  int span;
  double f[3][16];
};
void eval_local(const std::vector<double> &xi, int p, double x, LocalBasis &out);

}  // namespace fdg
