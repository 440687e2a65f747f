// Leja points on [-2, 2] (Sec. 2.2 maps the spectrum onto a pre-computed Leja
// sequence in [-2, 2]).  xi_0 = 2; xi_m maximises prod_{j<m} |x - xi_j| over the
// interval, ties going to the leftmost maximiser.
//
// Method: a running log-product on a uniform grid of 2^18 + 1 points locates
// the maximiser to within one grid step; a safeguarded Newton iteration on the
// derivative of the log-product, sum_j 1/(x - xi_j), then refines it inside
// that one-step bracket to full double precision.  End points are exact.
#include <cmath>
#include <vector>

namespace lj {

static double dlog(double x, const std::vector<double>& pts) {
  double g = 0.0;
  for (double p : pts) g += 1.0 / (x - p);
  return g;
}

static double d2log(double x, const std::vector<double>& pts) {
  double g = 0.0;
  for (double p : pts) g -= 1.0 / ((x - p) * (x - p));
  return g;
}

// zero of dlog inside (lo, hi) where dlog(lo) > 0 > dlog(hi): Newton steps,
// replaced by bisection whenever they leave the shrinking bracket
static double refine(double lo, double hi, const std::vector<double>& pts) {
  double x = 0.5 * (lo + hi);
  for (int it = 0; it < 400; ++it) {
    const double g = dlog(x, pts);
    if (g == 0.0) return x;
    if (g > 0.0) lo = x; else hi = x;
    double xn = x - g / d2log(x, pts);
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    if (xn == x) return x;
    x = xn;
  }
  return x;
}

int leja_points_host(double* out, int count) {
  const int G = (1 << 18) + 1;
  std::vector<double> grid(G), acc(G, 0.0);
  for (int i = 0; i < G; ++i) grid[i] = -2.0 + 4.0 * (double)i / (double)(G - 1);
  std::vector<double> pts;
  pts.push_back(2.0);
  for (int i = 0; i < G; ++i) acc[i] += std::log(std::fabs(grid[i] - 2.0));
  while ((int)pts.size() < count) {
    double best = -INFINITY;
    for (int i = 0; i < G; ++i) best = std::fmax(best, acc[i]);
    // leftmost grid point within rounding of the best value; a genuine
    // neighbour of the maximiser is lower by at least ~1e-10 on this grid
    const double tiny = 1e-12 * std::fmax(1.0, std::fabs(best));
    int ib = 0;
    while (!(acc[ib] >= best - tiny)) ++ib;
    double x;
    if (ib == 0) {
      x = -2.0;
    } else if (ib == G - 1) {
      x = 2.0;
    } else {
      // the log-product is concave between existing points, so its maximiser
      // lies within one grid step of the best grid point
      x = refine(grid[ib - 1], grid[ib + 1], pts);
    }
    pts.push_back(x);
    for (int i = 0; i < G; ++i) {
      const double d = std::fabs(grid[i] - x);
      acc[i] += (d == 0.0) ? -INFINITY : std::log(d);
    }
  }
  for (int i = 0; i < count; ++i) out[i] = pts[i];
  return 0;
}

}  // namespace lj
