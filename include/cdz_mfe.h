/*
 * cdz_mfe.h -- minimum free energy over codon sequences and structures, with
 * an argmin traceback, on top of libcdz.so.
 *
 * Section 4d (minimization): the same dynamic program in the (min, +)
 * algebra (SI S2c), i.e. the zero-temperature limit of the partition
 * function: sums over decompositions become minima, products of Boltzmann
 * factors become sums of energies.  For a protein psi,
 *     MFE(psi) = min over codon assignments c and secondary structures s of
 *                E(phi(c), s) - log W(c)                     (kT),
 * with the loop model, slot order and weights W of cdz.h.
 */
#ifndef CDZ_MFE_H
#define CDZ_MFE_H

#include "cdz.h"

#ifdef __cplusplus
extern "C" {
#endif

/* MFE of prob under the handle's energy tables, computed in FP64 on the
 * handle's device and stream whatever the handle's precision, and one state
 * that attains it.
 *   mfe     host double: the minimum (kT); +inf if no codon sequence exists
 *           (never for valid proteins: the all-unpaired structure is finite).
 *   codons  [n_aa] host bytes or NULL: slot of each residue's codon.
 *   pairs   [n] host int32 or NULL (n = 3 n_aa): partner of each position, -1
 *           unpaired.
 * Among states of equal energy the one returned is fixed: every decision of
 * the traceback takes the first alternative of smallest value in a fixed order
 * (exterior: j unpaired by slot of j-1, then 0 pairs j, then k pairs j for k
 * ascending; a pair: hairpin, stack, bulge/interior windows by (l1, l2)
 * ascending, multiloop; multiloop parts: splits by u ascending, then the
 * one-branch forms).
 * The workspace (seven n x n x 36 FP64 arrays, 1.6 GB at 900 nt) is allocated
 * for the call and released before it returns.  Errors: CDZ_ERR_ARG,
 * CDZ_ERR_PROTEIN, CDZ_ERR_NUMERIC (non-finite weights), CDZ_ERR_NOMEM,
 * CDZ_ERR_HIP. */
cdz_status cdz_mfe(cdz_handle *h, const cdz_problem *prob, double *mfe, uint8_t *codons, int32_t *pairs);

/* Suboptimal states (SI S4d, Alg. subopt): every (codon assignment,
 * structure) whose energy is at most MFE + gap, in FP64 on the handle's
 * device and stream.
 *   gap         >= 0 (kT); the threshold is MFE + gap + 1e-9 max(1, |MFE|).
 *               The single argmin (the paper's gap < 0) is cdz_mfe.
 *   max_states  capacity of the outputs; with more states than that the first
 *               max_states are returned and *more is set.
 *   mfe         host double: the minimum.
 *   energies    [max_states] host doubles or NULL: each state's energy (kT).
 *   codons      [max_states][n_aa] host bytes or NULL: codon slots.
 *   pairs       [max_states][n] host int32 or NULL: partner per position, -1
 *               unpaired.
 *   count       host int32: states written.  more: host int32 or NULL.
 * States come in a fixed order (a depth-first search over the traceback's
 * decisions in the order documented for cdz_mfe), each exactly once.  The
 * workspace of cdz_mfe plus the search's (up to 2^20 pending alternatives of
 * 112 bytes, the outputs) is allocated for the call.  Errors: CDZ_ERR_ARG (a
 * negative or non-finite gap, max_states < 0), CDZ_ERR_PROTEIN,
 * CDZ_ERR_NUMERIC, CDZ_ERR_NOMEM, CDZ_ERR_BUDGET (more pending alternatives
 * than the search holds: lower the gap), CDZ_ERR_HIP. */
cdz_status cdz_subopt(cdz_handle *h, const cdz_problem *prob, double gap, int32_t max_states, double *mfe,
                      double *energies, uint8_t *codons, int32_t *pairs, int32_t *count, int32_t *more);

#ifdef __cplusplus
}
#endif
#endif /* CDZ_MFE_H */
