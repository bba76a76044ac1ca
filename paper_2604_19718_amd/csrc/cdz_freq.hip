// Frequency matching (Section S4e, algorithm "iterative"): codon bonuses f
// whose expected codon frequencies under the Boltzmann ensemble equal the
// frequencies b* of independent codon choice with target bonuses f*.
//
// Each evaluation is one forward + outside pass on the device (the codon
// marginals of eq. codon-marginal, through cdz_marginals); between
// evaluations the library updates the log bonuses x = log f with Anderson
// acceleration (Walker and Ni, SIAM J. Numer. Anal. 49 (2011), Algorithm AA,
// unit mixing).  The update is a least-squares problem of at most 61 rows
// (one per codon) and as many columns as evaluations so far, solved here by
// Householder QR; it costs microseconds against the tens of milliseconds of
// a pass, and the weights it produces go through the same host table set-up
// (build_tables) as every other call.
//
// Fixed-point map:  r(x) = log b* - log b(x),  g(x) = x + r(x), which
// multiplies the bonuses by desired over achieved frequencies as the prose
// of Section S4e states (the printed listing has the ratio inverted, which
// moves away from the target under the plain iteration).
#include <cmath>
#include <cstring>
#include <vector>

#include "cdz_freq.h"
#include "cdz_internal.h"

int codon_count(unsigned char letter);  // cdz_host.hip: slots of a residue letter

namespace {

// gamma = argmin || r - A gamma ||_2 for A with rows x cols (column-major,
// cols <= rows) by Householder QR; a column whose diagonal entry of R falls
// below 1e-14 of the largest one is dropped (gamma = 0 there).
void least_squares(std::vector<double> A, int rows, int cols, std::vector<double> r, std::vector<double> &gamma) {
  std::vector<double> diag(cols, 0.0);
  for (int j = 0; j < cols; j++) {
    double *a = &A[(size_t)j * rows];
    double nrm = 0;
    for (int i = j; i < rows; i++) nrm += a[i] * a[i];
    nrm = std::sqrt(nrm);
    if (nrm == 0) {
      diag[j] = 0;
      continue;
    }
    const double alpha = a[j] > 0 ? -nrm : nrm;  // R[j][j]
    // v = a[j..] - alpha e_j, H = I - 2 v v^T / (v^T v)
    a[j] -= alpha;
    double vv = 0;
    for (int i = j; i < rows; i++) vv += a[i] * a[i];
    for (int k = j + 1; k < cols; k++) {
      double *b = &A[(size_t)k * rows];
      double dot = 0;
      for (int i = j; i < rows; i++) dot += a[i] * b[i];
      const double s = 2 * dot / vv;
      for (int i = j; i < rows; i++) b[i] -= s * a[i];
    }
    double dot = 0;
    for (int i = j; i < rows; i++) dot += a[i] * r[i];
    const double s = 2 * dot / vv;
    for (int i = j; i < rows; i++) r[i] -= s * a[i];
    diag[j] = alpha;
  }
  double dmax = 0;
  for (int j = 0; j < cols; j++) dmax = std::fmax(dmax, std::fabs(diag[j]));
  gamma.assign(cols, 0.0);
  for (int j = cols - 1; j >= 0; j--) {
    if (!(std::fabs(diag[j]) > 1e-14 * dmax)) continue;
    double s = r[j];
    for (int k = j + 1; k < cols; k++) s -= A[(size_t)k * rows + j] * gamma[k];
    gamma[j] = s / diag[j];
  }
}

}  // namespace

extern "C" cdz_status cdz_match_frequencies(cdz_handle *h, const cdz_problem *prob, const double *f_target,
                                            double r_tol, int32_t max_eval, int32_t history, double *f_out,
                                            double *err, int32_t *n_eval, int32_t *converged) {
  if (!h || !prob || !prob->aa || !f_target || !f_out || !n_eval || prob->n_aa < 1)
    return cdz_fail(h, CDZ_ERR_ARG, "null argument");
  if (max_eval < 1 || !(r_tol > 0) || !std::isfinite(r_tol))
    return cdz_fail(h, CDZ_ERR_ARG, "max_eval < 1 or r_tol not positive");
  const int m = prob->n_aa;
  // the codons of the letters present, row-major over [26][6]
  int count[26] = {0};
  for (int a = 0; a < m; a++) {
    const unsigned char c = (unsigned char)prob->aa[a];
    if (c < 'A' || c > 'Z' || codon_count(c) == 0)
      return cdz_fail(h, CDZ_ERR_PROTEIN, "invalid residue letter at " + std::to_string(a));
    count[c - 'A']++;
  }
  std::vector<int> bin;       // active bin (letter * 6 + slot) per dimension
  int dim_of[26 * 6];         // dimension of a bin, -1 if inactive
  std::vector<double> lbs;    // log b*
  for (int L = 0; L < 26; L++) {
    for (int s = 0; s < 6; s++) dim_of[L * 6 + s] = -1;
    if (!count[L]) continue;
    const int d = codon_count((unsigned char)('A' + L));
    double tot = 0;
    for (int s = 0; s < d; s++) {
      const double f = f_target[L * 6 + s];
      if (!(f > 0) || !std::isfinite(f))
        return cdz_fail(h, CDZ_ERR_ARG, "target bonuses must be finite and positive on the protein's codons");
      tot += f;
    }
    for (int s = 0; s < d; s++) {
      dim_of[L * 6 + s] = (int)bin.size();
      bin.push_back(L * 6 + s);
      lbs.push_back(std::log(count[L] * f_target[L * 6 + s] / tot));
    }
  }
  const int D = (int)bin.size();
  std::vector<double> x(D), theta1((size_t)m * 6, 0.0), codon((size_t)m * 6), b(D), r(D), g(D);
  for (int k = 0; k < D; k++) x[k] = std::log(f_target[bin[k]]);
  std::vector<std::vector<double>> X, R, G;  // history of evaluated iterates, residuals, g
  cdz_problem p2 = *prob;
  p2.theta1 = theta1.data();
  *n_eval = 0;
  if (converged) *converged = 0;
  auto write_f = [&](const std::vector<double> &xv) {
    for (int k = 0; k < 26 * 6; k++) f_out[k] = 0.0;
    for (int k = 0; k < D; k++) f_out[bin[k]] = std::exp(xv[k]);
  };
  for (int it = 0; it < max_eval; it++) {
    for (int a = 0; a < m; a++) {
      const int L = prob->aa[a] - 'A', d = codon_count((unsigned char)prob->aa[a]);
      for (int s = 0; s < d; s++) theta1[(size_t)a * 6 + s] = x[dim_of[L * 6 + s]];
    }
    cdz_status st = cdz_marginals(h, &p2, nullptr, nullptr, nullptr, codon.data(), nullptr);
    if (st != CDZ_OK) return st;
    std::fill(b.begin(), b.end(), 0.0);
    for (int a = 0; a < m; a++) {
      const int L = prob->aa[a] - 'A', d = codon_count((unsigned char)prob->aa[a]);
      for (int s = 0; s < d; s++) b[dim_of[L * 6 + s]] += codon[(size_t)a * 6 + s];
    }
    double e = 0;
    for (int k = 0; k < D; k++) {
      if (!(b[k] > 0) || !std::isfinite(b[k]))
        return cdz_fail(h, CDZ_ERR_NUMERIC, "codon frequency not positive and finite");
      r[k] = lbs[k] - std::log(b[k]);
      g[k] = x[k] + r[k];
      e = std::fmax(e, std::fabs(r[k]));
    }
    if (err) err[it] = e;
    *n_eval = it + 1;
    if (e < r_tol) {
      write_f(x);
      if (converged) *converged = 1;
      return CDZ_OK;
    }
    X.push_back(x);
    R.push_back(r);
    G.push_back(g);
    int mk = history < 0 ? it : std::min<int>(history, it);
    mk = std::min(mk, D);
    if (mk == 0) {
      x = g;
      continue;
    }
    // columns i = it-mk .. it-1: R[i+1] - R[i] and G[i+1] - G[i]
    std::vector<double> DR((size_t)D * mk), gamma;
    for (int c = 0; c < mk; c++) {
      const int i = it - mk + c;
      for (int k = 0; k < D; k++) DR[(size_t)c * D + k] = R[i + 1][k] - R[i][k];
    }
    least_squares(DR, D, mk, r, gamma);
    for (int k = 0; k < D; k++) {
      double s = g[k];
      for (int c = 0; c < mk; c++) {
        const int i = it - mk + c;
        s -= (G[i + 1][k] - G[i][k]) * gamma[c];
      }
      x[k] = s;
    }
  }
  write_f(X.back());  // not converged: the last evaluated bonuses
  return CDZ_OK;
}
