/*
 * cdz_freq.h -- frequency matching on top of the marginals of libcdz.so.
 *
 * Section S4e (algorithm "iterative"): find codon bonuses f such that the
 * codon frequencies of the Boltzmann ensemble of (codon sequence, structure)
 * equal the frequencies b* that independent codon choice with target bonuses
 * f* would give, with Anderson acceleration of the fixed-point iteration
 * (the paper's runs used it with no history limit; Walker and Ni 2011).
 */
#ifndef CDZ_FREQ_H
#define CDZ_FREQ_H

#include "cdz.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Codons are indexed [26][6]: row = residue letter - 'A', column = slot in the
 * library's slot order (the codons of the letter sorted by spelling under
 * A < C < G < U).  Bonuses enter the model as theta1[a][s] = log f(aa[a], s);
 * prob->theta1 is ignored, prob->theta2 is kept.
 *
 *   f_target  [26][6] host doubles: target bonuses f*; every codon of a letter
 *             present in the protein must be finite and > 0 (CDZ_ERR_ARG),
 *             other entries are not read.  b*(L, s) = count(L) f*(L, s) /
 *             sum_t f*(L, t) over the residues of letter L.
 *   r_tol     stop when max |log(b / b*)| < r_tol over the present codons,
 *             b(L, s) = sum of the codon marginals Pr(codon of a = s) over the
 *             residues a of letter L (the paper used 0.002).
 *   max_eval  number of marginal evaluations (forward + outside passes) at most.
 *   history   Anderson history: 0 = the plain iteration f <- f b* / b; -1 =
 *             unlimited (capped at the number of present codons); k > 0 = the
 *             last k differences.
 *   f_out     [26][6] host doubles: the bonuses of the last evaluation (the one
 *             that met r_tol, if any); 0 on codons of absent letters.
 *   err       [max_eval] host doubles or NULL: max |log(b / b*)| per evaluation.
 *   n_eval    evaluations made.
 *   converged 1 if the tolerance was met, else 0 (may be NULL).
 * The first evaluation uses f = f*.  Runs on the handle's device, stream and
 * precision; each evaluation replaces the forward kept in the handle.
 * Errors: CDZ_ERR_ARG / CDZ_ERR_PROTEIN for bad arguments, any status of
 * cdz_marginals, CDZ_ERR_NUMERIC when a codon frequency is not positive and
 * finite.  A run that stops at max_eval without meeting r_tol returns CDZ_OK
 * with *converged = 0. */
cdz_status cdz_match_frequencies(cdz_handle *h, const cdz_problem *prob, const double *f_target,
                                 double r_tol, int32_t max_eval, int32_t history, double *f_out,
                                 double *err, int32_t *n_eval, int32_t *converged);

#ifdef __cplusplus
}
#endif
#endif /* CDZ_FREQ_H */
