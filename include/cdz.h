/*
 * cdz.h -- C ABI of the MI355X codon-constrained partition-function library.
 *
 * The library computes, for an amino-acid sequence psi (m residues, n = 3m
 * bases), the partition function summed jointly over every codon sequence
 * encoding psi and every non-crossing secondary structure of that sequence
 * (paper Section 2b, eqs. structure-q, sequence-q, amino-q), biased by
 * per-codon and codon-pair weights (the soft constraints of Section 3a).  From
 * it follow the pair matrix, base and codon marginals (Section 2c, eqs.
 * pair-probability, marginal-base, marginal-codon) and exact joint samples of
 * sequence and structure (Section 4a).  The secondary-structure model is a
 * nearest-neighbour loop model (see cdz_energy).  Every call runs its dynamic
 * program in HIP kernels on the device that is current when cdz_create is
 * called; the host only validates inputs and builds small per-position tables.
 *
 * Conventions
 *   - Bases A=0 C=1 G=2 U=3.  Pair types AU=0 CG=1 GC=2 UA=3 GU=4 UG=5.
 *   - Residues are the letters "ARNDCQEGHILKMFPSTWYV"; start and stop codons
 *     are not part of psi (SI S3c).  The codons of a residue are numbered in
 *     lexicographic order of their spelling under A<C<G<U ("slot" s, at most
 *     6 per residue); all per-codon inputs and outputs use this slot order
 *     and are padded with zeros to 6 slots.
 *   - Energies are in units of kT (the paper's unitless free energies); +inf
 *     marks a forbidden entry.
 *   - The caller owns every input and output buffer.  The handle owns all
 *     device workspace and keeps the last forward pass for cdz_marginals and
 *     cdz_sample on the same problem.
 *   - Every call returns a cdz_status; no exception crosses the ABI.  Inputs
 *     are validated before any device work.  cdz_last_error() describes the
 *     last failure of a handle.  Handles are not thread-safe; use one handle
 *     per host thread / stream.
 */
#ifndef CDZ_H
#define CDZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CDZ_OK = 0,
  CDZ_ERR_ARG = 1,      /* null pointer, n_aa < 1, n_samples < 0, bad option   */
  CDZ_ERR_PROTEIN = 2,  /* a letter outside the 20 standard amino acids        */
  CDZ_ERR_NUMERIC = 3,  /* non-finite weights/tables, or scaling out of range  */
  CDZ_ERR_NOMEM = 4,    /* device allocation failed                            */
  CDZ_ERR_BUDGET = 5,   /* workspace would exceed options.mem_budget_bytes     */
  CDZ_ERR_HIP = 6,      /* a HIP runtime call failed                           */
  CDZ_ERR_STATE = 7     /* sample/marginals without a usable forward pass      */
} cdz_status;

typedef enum {
  CDZ_FP32_SCALED = 0,  /* FP32 arrays, one power-of-two exponent per diagonal;
                           exponents, exterior loop and log Z in FP64          */
  CDZ_FP64 = 1          /* the same dynamic program entirely in FP64           */
} cdz_precision;

/* Nearest-neighbour loop model, energies in kT (+inf = forbidden).
 *   hairpin closed by (i,j), L = j-i-1 >= 3 unpaired bases:
 *       hairpin[L] (L <= 30) or hairpin[30] + extrap*ln(L/30),
 *       plus mismatch[b(i+1)][b(j-1)][type(i,j)]
 *   stacked pair (i,j) on (i+1,j-1): stack[type(i,j)][type(i+1,j-1)]
 *   bulge, one side empty, L in 1..30 unpaired: bulge[L]
 *   interior loop, l1,l2 >= 1, l1+l2 <= 30, inner pair (k,l):
 *       interior[l1+l2] + mismatch[b(i+1)][b(j-1)][type(i,j)]
 *                       + mismatch[b(l+1)][b(k-1)][type(l,k)]
 *   multiloop: ml_a + ml_b*(inner branches + 1) + ml_c*(unpaired bases)
 *   exterior loop: 0.  Hairpins need >= 3 unpaired bases; no pseudoknots.
 * The record is 229 doubles (36 + 3*31 + 96 + 4) in exactly this field order. */
typedef struct {
  double stack[6][6];
  double hairpin[31];
  double bulge[31];
  double interior[31];
  double mismatch[4][4][6];
  double ml_a, ml_b, ml_c;
  double extrap;
} cdz_energy;

/* One protein and its soft constraints (Section 3a).
 *   aa      : n_aa letters (not NUL-terminated necessarily).
 *   theta1  : [n_aa][6] log codon weights, slot order; NULL = all zero.
 *   theta2  : [n_aa][6][6] log codon-pair weights; theta2[a][x][y] weighs
 *             codon x at residue a-1 followed by codon y at residue a; row 0
 *             is ignored (open chain, no pair term before the first codon);
 *             NULL = no pair terms.
 * W(c) = exp(sum_a theta1[a][c_a] + sum_{a>=1} theta2[a][c_{a-1}][c_a]). */
typedef struct {
  int32_t n_aa;
  const char *aa;
  const double *theta1;
  const double *theta2;
} cdz_problem;

/* There is no autotuning option: every cell of every diagonal runs the same
 * work shape (one workgroup per cell, a fixed number of waves per SIMD), so
 * no tile or schedule choice is left to search. */
typedef struct {
  cdz_precision prec;
  size_t mem_budget_bytes; /* 0 = unlimited; else the device workspace stays
                              within it (memory-bounded form when needed, see
                              cdz_workspace_bytes), CDZ_ERR_BUDGET below the
                              minimum                                          */
  void *hip_stream;        /* hipStream_t to run on; NULL = the null stream     */
} cdz_options;

typedef struct cdz_handle cdz_handle;

/* Create a handle bound to the current HIP device.  `energy` is copied.
 * Returns CDZ_ERR_NUMERIC if an energy is NaN or -inf. */
cdz_status cdz_create(const cdz_energy *energy, const cdz_options *opts, cdz_handle **out);
void cdz_destroy(cdz_handle *h);

/* log Z (natural log of the partition function, = -q_psi of eq. amino-q).
 * Runs the forward pass and keeps it in the handle. */
cdz_status cdz_partition(cdz_handle *h, const cdz_problem *prob, double *log_z);

/* log Z plus marginals (Section 2c), all row-major host buffers of doubles:
 *   pair       [n][n]   P[i][j] = Pr(i pairs with j), P[i][i] = Pr(i unpaired)
 *   base       [n][4]   Pr(base of position p = b)
 *   codon      [n_aa][6] Pr(codon of residue a = slot s)  (= d log Z / d theta1)
 *   codon_pair [n_aa][6][6] Pr(codons of residues a-1, a = x, y), row 0 zero
 *                        (= d log Z / d theta2)
 * Any output pointer may be NULL.  Runs forward (unless the handle holds the
 * forward of the same problem) and the outside (adjoint) pass. */
cdz_status cdz_marginals(cdz_handle *h, const cdz_problem *prob, double *log_z,
                         double *pair, double *base, double *codon, double *codon_pair);

/* n_samples exact joint samples of (codon sequence, structure) from the
 * Boltzmann distribution, drawn by stochastic traceback of the forward pass
 * with Philox4x32-10 (key = seed, counter = (draw index, sample index, 0, 0)).
 *   codons [n_samples][n_aa]  slot of each residue
 *   pairs  [n_samples][n]     partner of each position, -1 = unpaired */
cdz_status cdz_sample(cdz_handle *h, const cdz_problem *prob, uint64_t seed,
                      int32_t n_samples, uint8_t *codons, int32_t *pairs);

/* cdz_sample for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same samples as cdz_sample with the same seed, drawn from the forward pass
 * the handle already holds for this problem (CDZ_ERR_STATE otherwise: call
 * cdz_partition or cdz_marginals on it first).  It allocates nothing: the
 * sampler's device workspace is one fixed array of 32 MiB per device, held
 * until the process ends, which needs per call
 *   n_samples * (20 (n + 16) + 8 (max(n, 498) + 64) + 5 n + n_aa + 4) + 1536
 * bytes (n = 3 n_aa; 1000 samples of 900 nt take 30.8 MB); a call needing
 * more returns CDZ_ERR_BUDGET before any device work.  All calls on one
 * device share that array and the next call overwrites it: calls that
 * overlap on one device (other streams, handles or threads) race, and the
 * caller must serialise them.  codons and pairs are host buffers laid out as
 * in cdz_sample. */
cdz_status cdz_sample_noalloc(cdz_handle *h, const cdz_problem *prob, uint64_t seed,
                              int32_t n_samples, uint8_t *codons, int32_t *pairs);

/* Batched forms (batching is this library's own; the paper treats one
 * protein at a time): `count` problems of uneven length on one handle.  The batch is split, in
 * order, into chunks whose device workspaces together fit the budget
 * (options.mem_budget_bytes, else 90% of the free device memory less 1 GiB);
 * inside a chunk one launch per diagonal index runs that diagonal of every
 * protein in the chunk.  Each protein's results equal those of the
 * single-problem call (bit for bit: same kernels, same order of operations).
 * Outputs are concatenated in batch order; with n_c = 3 * n_aa of problem c,
 * problem b's block starts at
 *   log_z      [count]                 b
 *   pair       n_c * n_c per problem    sum_{c<b} n_c^2
 *   base       n_c * 4                  4 * sum_{c<b} n_c
 *   codon      n_aa_c * 6               6 * sum_{c<b} n_aa_c
 *   codon_pair n_aa_c * 36              36 * sum_{c<b} n_aa_c
 *   codons     n_samples * n_aa_c       n_samples * sum_{c<b} n_aa_c
 *   pairs      n_samples * n_c          n_samples * sum_{c<b} n_c
 * with each block laid out as in the single-problem call.  Problem b's samples
 * are drawn with key seed + b (the samples cdz_sample gives with that seed).
 * The handle keeps no forward pass afterwards (cdz_sample / cdz_marginals on
 * a single problem recompute theirs).  Errors: CDZ_ERR_ARG for count < 0,
 * null lists or outputs, or n_samples < 0; a problem's validation error is
 * reported with its index in cdz_last_error; CDZ_ERR_BUDGET when one
 * protein's workspace alone exceeds mem_budget_bytes (CDZ_ERR_NOMEM without
 * a budget).  Outputs of problems before a failing chunk are written. */

/* Forward of every problem (log_z may be NULL), the outside pass when any
 * marginal output is non-NULL, and n_samples samples of each problem when
 * n_samples > 0 (codons and pairs then required), all in one call. */
cdz_status cdz_batch(cdz_handle *h, const cdz_problem *probs, int32_t count, int32_t n_samples,
                     uint64_t seed, double *log_z, double *pair, double *base, double *codon,
                     double *codon_pair, uint8_t *codons, int32_t *pairs);
cdz_status cdz_partition_batch(cdz_handle *h, const cdz_problem *probs, int32_t count, double *log_z);
cdz_status cdz_marginals_batch(cdz_handle *h, const cdz_problem *probs, int32_t count, double *log_z,
                               double *pair, double *base, double *codon, double *codon_pair);
cdz_status cdz_sample_batch(cdz_handle *h, const cdz_problem *probs, int32_t count, uint64_t seed,
                            int32_t n_samples, uint8_t *codons, int32_t *pairs);

/* Device workspace (bytes) that one problem needs in the handle's precision,
 * for `what`:
 *   CDZ_WS_FORWARD       forward arrays, all diagonals resident (cdz_partition,
 *                        cdz_sample without a budget)
 *   CDZ_WS_MARGINALS     forward + outside, all resident (cdz_marginals
 *                        without a budget; what each batch member takes)
 *   CDZ_WS_MARGINALS_MIN the least budget cdz_marginals accepts: forward +
 *                        outside with the interior-loop sums kept only as
 *                        checkpoints and one recomputed band of diagonals
 *                        (or the resident form where that is smaller, as for
 *                        sequences of about 120 nt and less)
 *   CDZ_WS_FORWARD_MIN   the least budget cdz_partition / cdz_sample accept:
 *                        forward with those sums in a ring of 3 diagonals
 * The single-problem calls use the resident form when it fits
 * options.mem_budget_bytes (or no budget is set), else the minimum form, whose
 * results are the same bit for bit; below the minimum they return
 * CDZ_ERR_BUDGET.  No device work. */
enum { CDZ_WS_FORWARD = 0, CDZ_WS_MARGINALS = 1, CDZ_WS_MARGINALS_MIN = 2, CDZ_WS_FORWARD_MIN = 3 };
cdz_status cdz_workspace_bytes(cdz_handle *h, const cdz_problem *prob, int32_t what, size_t *bytes);

/* Device-pointer form of the forward pass for callers that keep the weights
 * on the device (PyTorch), whose reverse mode (cdz_backward_dev) gives the
 * codon marginals as d log Z / d theta (Section 4c, eq. codon-marginal: the
 * codon probability is the derivative of log Z with respect to the log weight
 * on the codon's middle base).  theta1_dev [n_aa][6], theta2_dev [n_aa][6][6] or
 * NULL, doubles in device memory.  log_z is a host pointer.  The stream is the
 * handle's stream. */
cdz_status cdz_forward_dev(cdz_handle *h, int32_t n_aa, const char *aa,
                           const double *theta1_dev, const double *theta2_dev,
                           double *log_z);

/* Adjoint of cdz_forward_dev (Section 4c, eq. codon-marginal): writes
 * d(log Z)/d theta1 [n_aa][6] and d(log Z)/d theta2 [n_aa][6][6] (device
 * doubles; theta2 grad may be NULL), each scaled by grad_logz, for the
 * problem of the forward pass the handle holds now (a later call on another
 * problem replaces it: call cdz_forward_dev again first, which is free when
 * the handle already holds that problem).  CDZ_ERR_STATE without a forward
 * pass; CDZ_ERR_NUMERIC if the adjoint left the floating-point range. */
cdz_status cdz_backward_dev(cdz_handle *h, double grad_logz, double *dtheta1_dev,
                            double *dtheta2_dev);

/* Per-phase device times (ms) of the last call, measured with HIP events on
 * the handle's stream: [0] forward, [1] outside + marginals, [2] sampling,
 * [3] average forward diagonal kernel (profiling on, else 0), [4] launches. */
cdz_status cdz_last_timings(cdz_handle *h, double *ms5);

/* Drop the forward pass kept in the handle, so the next call recomputes it
 * (used to time complete passes). */
cdz_status cdz_reset(cdz_handle *h);

/* When on, every diagonal launch is bracketed by HIP events on the handle's
 * stream and cdz_kernel_timings reports summed kernel times:
 *   [0] forward diagonal kernels, ms   [1] their number of launches
 *   [2] outside diagonal kernels, ms   [3] their number of launches
 *   [4] edge-marginal kernel, ms       [5] sampling kernel, ms */
cdz_status cdz_set_profiling(cdz_handle *h, int on);
cdz_status cdz_kernel_timings(cdz_handle *h, double *ms6);

const char *cdz_status_string(cdz_status s);
const char *cdz_last_error(const cdz_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* CDZ_H */
