/*
 * cdz_tensor.h -- the sequence-summed free energy under a tensor-based
 * secondary-structure model, on top of libcdz.so.
 *
 * Sections 3b-3c and SI S2b-S2c: per unpaired base b a matrix V_b, per side
 * of a base pair (x paired to y) and rank index rho a matrix B^rho_{x,y}, and a
 * matrix S for the weighted trace Tr_S[X] = Tr[S X].  A loop of a structure
 * contributes Tr_S of the product of the matrices along its backbone; the
 * partition function sums the product over loops over every structure, every
 * rho per pair and every codon sequence of the protein, each sequence weighed
 * by the single-codon tensor train of Section 3a (eq. single-tt) with the
 * codon bonus exp(theta1) on its middle core.  The dynamic program is the
 * single recursion of eq. dp-short on the flattened block matrix Q, whose
 * blocks Q_{i,j} are (gamma Sigma_i) x (gamma Sigma_j) (Section 3c), with the
 * folding function of eq. design-fold and Alg. fast-pf's propagation
 *     Q_{[0:j), j} = sum_k Q_{[0:j), k} E_{k,j}    (a triangular product).
 */
#ifndef CDZ_TENSOR_H
#define CDZ_TENSOR_H

#include "cdz.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Model parameters, host doubles, row-major, bases A=0 C=1 G=2 U=3.
 *   gamma  matrix dimension, 1..16
 *   xi     pair rank (number of rho), 1..4
 *   V      [4][gamma][gamma]            unpaired base
 *   B      [xi][4][4][gamma][gamma]     B[rho][x][y]: side at base x of a pair
 *                                       with base y (zero where x, y do not pair)
 *   S      [gamma][gamma]               weighted trace
 * Every entry must be finite and >= 0 (the scaling assumes non-negative
 * sums); CDZ_ERR_NUMERIC otherwise. */
typedef struct {
  int32_t gamma;
  int32_t xi;
  const double *V;
  const double *B;
  const double *S;
} cdz_tensor_model;

/* log Z of prob under the model, on the handle's device and stream, in the
 * handle's precision (CDZ_FP32_SCALED: FP32 with one power-of-two factor per
 * column of Q; CDZ_FP64: the same in FP64).
 *   prob->theta1  [n_aa][6] codon bonuses in slot order, or NULL;
 *   prob->theta2  must be NULL (the single-codon train carries no codon-pair
 *                 terms): CDZ_ERR_ARG otherwise.
 *   log_z         host double.
 *   prefix        [n_aa] host doubles or NULL: log Z of the first a+1 residues
 *                 (the codon boundaries of the same pass, where Sigma = 1).
 * The workspace (Q, (gamma Sigma)^2 entries with Sigma the summed train
 * dimensions, plus partial sums of the split propagation) is allocated for the
 * call and released before it returns.  Afterwards cdz_last_timings reports
 * [0] the device time of the whole pass and, with cdz_set_profiling on (else
 * 0), [3] the average propagation kernel and [4] the number of propagation
 * launches (one per position).  Errors: CDZ_ERR_ARG, CDZ_ERR_PROTEIN,
 * CDZ_ERR_NUMERIC, CDZ_ERR_NOMEM, CDZ_ERR_HIP. */
cdz_status cdz_tensor_logz(cdz_handle *h, const cdz_tensor_model *model, const cdz_problem *prob, double *log_z,
                           double *prefix);

/* Bond dimensions Sigma_p, p = 0..n (n = 3 n_aa), of prob's single-codon
 * train (Section 3a, eq. single-tt): 1 at codon boundaries, the number of
 * distinct first bases after one, the number of distinct third bases before
 * one.  Q has gamma * sum_p Sigma_p rows.  sig: [n + 1] host int32.  Host
 * only.  Errors: CDZ_ERR_ARG, CDZ_ERR_PROTEIN. */
cdz_status cdz_tensor_dims(const cdz_problem *prob, int32_t *sig);

#ifdef __cplusplus
}
#endif
#endif /* CDZ_TENSOR_H */
