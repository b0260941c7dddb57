// Reblocking analysis of a serially correlated series (host code): the
// blocking transformation of Flyvbjerg and Petersen (J. Chem. Phys. 91, 461,
// 1989) and the choice of level of Lee, Conduit, Nemec, Lopez Rios and
// Drummond (Phys. Rev. E 83, 066706, 2011).  The paper reblocks the per-block
// outputs of its driver as the run goes on (Sec. 3.1).
#include <math.h>
#include <string.h>

#include <vector>

#include "afqmc.h"

namespace afqmc {
// the thread-local message of afqmc_last_error (api.hip)
afqmc_status record_error(afqmc_status s, const char *msg);
}  // namespace afqmc

extern "C" afqmc_status afqmc_reblock(const double *x, int64_t n, afqmc_reblock_result *out) {
  if (!x || !out) return afqmc::record_error(AFQMC_ERR_ARG, "NULL series or result");
  if (n < 2) return afqmc::record_error(AFQMC_ERR_ARG, "need at least two samples");
  for (int64_t i = 0; i < n; ++i)
    if (!isfinite(x[i])) return afqmc::record_error(AFQMC_ERR_ARG, "the series holds a non-finite sample");
  memset(out, 0, sizeof(*out));
  std::vector<double> data(x, x + n);
  double total = 0.0;
  for (double v : data) total += v;
  out->n = n;
  out->mean = total / (double)n;
  out->optimal = -1;
  int lev = 0;
  while ((int64_t)data.size() >= 2 && lev < AFQMC_REBLOCK_LEVELS) {
    const int64_t m = (int64_t)data.size();
    double sum = 0.0;
    for (double v : data) sum += v;
    const double mean = sum / (double)m;
    double c0 = 0.0;
    for (double v : data) c0 += (v - mean) * (v - mean);
    c0 /= (double)m;
    const double se = sqrt(c0 / (double)(m - 1));
    out->count[lev] = m;
    out->level_mean[lev] = mean;
    out->std_err[lev] = se;
    out->std_err_err[lev] = se / sqrt(2.0 * (double)(m - 1));
    // pair averages for the next level; an odd last sample is dropped
    const int64_t half = m / 2;
    for (int64_t i = 0; i < half; ++i) data[i] = 0.5 * (data[2 * i] + data[2 * i + 1]);
    data.resize(half);
    ++lev;
  }
  out->nlevels = lev;
  const double e0 = out->std_err[0];
  for (int b = 0; b < lev; ++b) {
    const double r = e0 > 0.0 ? out->std_err[b] / e0 : 1.0;
    if (ldexp(1.0, 3 * b) > 2.0 * (double)n * (r * r) * (r * r)) {
      out->optimal = b;
      break;
    }
  }
  return AFQMC_OK;
}
