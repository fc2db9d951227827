// Correlation-function estimators on top of the pair counts (Section 1: the
// natural estimator eqn:xi, the analytic random-pair counts of a periodic
// cube, and w_p as twice the line-of-sight integral of xi(r_p, pi)).  Host
// code on host arrays, O(bins); declared in include/countpairs.h.
#include "../../include/countpairs.h"

#include <cmath>
#include <limits>

namespace cp {
int report_error(int code, const char *msg);
}

namespace {

constexpr double kPi = 3.14159265358979323846;

int check_edges(const double *e, int nedges, double boxsize) {
  if (!e) return cp::report_error(CP_ERR_INVALID_ARG, "edges is NULL");
  if (nedges < 2) return cp::report_error(CP_ERR_INVALID_ARG, "nedges < 2");
  for (int k = 0; k < nedges; k++)
    if (!std::isfinite(e[k])) return cp::report_error(CP_ERR_INVALID_ARG, "edges not finite");
  if (e[0] < 0) return cp::report_error(CP_ERR_INVALID_ARG, "edges[0] < 0");
  for (int k = 1; k < nedges; k++)
    if (!(e[k] > e[k - 1]))
      return cp::report_error(CP_ERR_INVALID_ARG, "edges not strictly increasing");
  if (!(boxsize > 0) || !std::isfinite(boxsize))
    return cp::report_error(CP_ERR_INVALID_ARG, "boxsize must be positive and finite");
  // minimum-image shells beyond half the box are cut by the cube
  if (e[nedges - 1] > 0.5 * boxsize)
    return cp::report_error(CP_ERR_INVALID_ARG, "largest edge above boxsize / 2");
  return CP_OK;
}

// ordered pairs of n distinct points, or unordered ones
double pair_norm(int64_t n, int count_mode) {
  const double nn = (double)n * (double)(n > 0 ? n - 1 : 0);
  return count_mode == CP_UNIQUE ? 0.5 * nn : nn;
}

} // namespace

extern "C" {

int cp_rr_periodic_xi(int64_t n, double boxsize, const double *edges, int nedges,
                      int count_mode, double *rr) {
  int rc = check_edges(edges, nedges, boxsize);
  if (rc) return rc;
  if (n < 0) return cp::report_error(CP_ERR_INVALID_ARG, "n < 0");
  if (count_mode != CP_ORDERED && count_mode != CP_UNIQUE)
    return cp::report_error(CP_ERR_INVALID_ARG, "bad count_mode");
  if (!rr) return cp::report_error(CP_ERR_INVALID_ARG, "rr is NULL");
  // a pair's partner is uniform over the cube: the chance that it falls in
  // the shell [e_k, e_k+1) is the shell's volume over the box volume
  const double scale = pair_norm(n, count_mode) / (boxsize * boxsize * boxsize);
  for (int k = 0; k + 1 < nedges; k++) {
    const double a = edges[k], b = edges[k + 1];
    rr[k] = scale * (4.0 * kPi / 3.0) * (b * b * b - a * a * a);
  }
  return CP_OK;
}

int cp_rr_periodic_wp(int64_t n, double boxsize, const double *rp_edges, int nedges,
                      double pimax, int npibins, int count_mode, double *rr) {
  int rc = check_edges(rp_edges, nedges, boxsize);
  if (rc) return rc;
  if (n < 0) return cp::report_error(CP_ERR_INVALID_ARG, "n < 0");
  if (!(pimax > 0) || !std::isfinite(pimax) || pimax > 0.5 * boxsize)
    return cp::report_error(CP_ERR_INVALID_ARG, "pimax must be in (0, boxsize / 2]");
  if (npibins < 1) return cp::report_error(CP_ERR_INVALID_ARG, "npibins < 1");
  if (count_mode != CP_ORDERED && count_mode != CP_UNIQUE)
    return cp::report_error(CP_ERR_INVALID_ARG, "bad count_mode");
  if (!rr) return cp::report_error(CP_ERR_INVALID_ARG, "rr is NULL");
  // annulus area in r_p times the two slabs pi in [q_l, q_l+1) above and below
  const double scale = pair_norm(n, count_mode) / (boxsize * boxsize * boxsize);
  const double dpi = pimax / npibins;
  for (int k = 0; k + 1 < nedges; k++) {
    const double a = rp_edges[k], b = rp_edges[k + 1];
    const double area = kPi * (b * b - a * a);
    for (int l = 0; l < npibins; l++) rr[(size_t)k * npibins + l] = scale * area * 2.0 * dpi;
  }
  return CP_OK;
}

int cp_xi_natural(const uint64_t *dd, double dd_norm, const double *rr, double rr_norm,
                  int nbins, double *xi) {
  if (!dd || !rr || !xi) return cp::report_error(CP_ERR_INVALID_ARG, "NULL array");
  if (nbins < 1) return cp::report_error(CP_ERR_INVALID_ARG, "nbins < 1");
  if (!(dd_norm > 0) || !(rr_norm > 0) || !std::isfinite(dd_norm) || !std::isfinite(rr_norm))
    return cp::report_error(CP_ERR_INVALID_ARG, "normalisations must be positive and finite");
  for (int k = 0; k < nbins; k++) {
    const double r = rr[k] / rr_norm;
    xi[k] = r > 0 ? ((double)dd[k] / dd_norm) / r - 1.0
                  : std::numeric_limits<double>::quiet_NaN();
  }
  return CP_OK;
}

int cp_wp_integrate(const double *xi2d, int nrpbins, int npibins, double pimax, double *wp) {
  if (!xi2d || !wp) return cp::report_error(CP_ERR_INVALID_ARG, "NULL array");
  if (nrpbins < 1 || npibins < 1) return cp::report_error(CP_ERR_INVALID_ARG, "bins < 1");
  if (!(pimax > 0) || !std::isfinite(pimax))
    return cp::report_error(CP_ERR_INVALID_ARG, "pimax must be positive and finite");
  const double dpi = pimax / npibins;
  for (int k = 0; k < nrpbins; k++) {
    double s = 0.0;
    for (int l = 0; l < npibins; l++) s += xi2d[(size_t)k * npibins + l];
    wp[k] = 2.0 * dpi * s;
  }
  return CP_OK;
}

} // extern "C"
