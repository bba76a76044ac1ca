/*
 * cdz_debug.h -- test and diagnostic hooks of libcdz.so.
 *
 * Not part of the product interface (include/cdz.h): these entry points exist
 * so that tests can reach states the normal calls do not produce on the
 * default inputs (the FP32 repeated pass, a forced storage form of the
 * interior-loop sums) and read intermediate results back.  Each takes a
 * handle created by cdz_create; none allocates device memory.  A hook that
 * changes how the next forward pass runs also drops the forward kept in the
 * handle, so the next call recomputes it.
 */
#ifndef CDZ_DEBUG_H
#define CDZ_DEBUG_H

#include <stddef.h>

#include "cdz.h"

#ifdef __cplusplus
extern "C" {
#endif

/* log Z of the last forward pass computed from the suffix exterior loop
 * (the prefix one is what cdz_partition returns); NaN for a null handle.  The
 * two are independent sums over the same arrays, a consistency check of the
 * exterior reduction (eq. complex-logq). */
double cdz_debug_logz_suffix(const cdz_handle *h);

/* Storage of the interior-loop sums in the last forward pass: -1 all
 * diagonals resident, 0 a ring of three diagonals, K > 0 checkpoints with
 * bands of K diagonals recomputed by the outside pass; -2 for a null handle. */
int cdz_debug_al_k(const cdz_handle *h);

/* Force that storage for the following passes regardless of the budget
 * (K = -2 restores the choice by budget).  Returns CDZ_ERR_ARG for K < -2. */
int cdz_debug_force_al_k(cdz_handle *h, int K);

/* FP32: span of the truncated pass that estimates the free-energy landscape
 * (0 = by length; else 4..512).  Returns CDZ_ERR_ARG outside that range. */
int cdz_debug_set_span(cdz_handle *h, int W);

/* FP32: number of exact passes the last forward repeated because a cell came
 * within the range-check threshold; -1 for a null handle. */
int cdz_debug_landscape_retries(const cdz_handle *h);

/* Binary exponent of the largest entry of the weakest cell in the first
 * and in the final range check of the last single-problem forward pass (the
 * two differ when the FP32 pass was repeated; -1100 stands for a cell that is
 * entirely zero).  CDZ_ERR_ARG for null arguments. */
int cdz_debug_weakest(const cdz_handle *h, int *first, int *final_);

/* Range-check threshold exponent e: a cell whose largest entry is below 2^-e
 * is too weak (0 = the default of the precision: 120 in FP32, 1020 in FP64).
 * Accepts 0..1074, else CDZ_ERR_ARG. */
int cdz_debug_set_low_exp(cdz_handle *h, int e);

/* Batched calls run each chunk's forward passes (up to the range check) and
 * its outside pass as hipGraphs, captured the first time a chunk's launch
 * sequence is seen and replayed when it recurs.  on = 0 launches every kernel
 * directly instead (for timing the two); CDZ_ERR_ARG for a null handle. */
int cdz_debug_set_graphs(cdz_handle *h, int on);

/* Captures and replays of those graphs in the last batched call. */
int cdz_debug_graph_counts(const cdz_handle *h, int *captures, int *replays);

/* Launch grouping of the diagonal kernels: a launch whose pieces of work (the
 * workgroup kinds of the forward and outside passes) would take at least wg
 * workgroups runs fused, one workgroup per cell index doing every kind in
 * turn; wg = 0 fuses every launch, wg = -1 returns the choice to the
 * library's tuner (which times candidate thresholds on the first passes of
 * each class of pass).  Results are the same either way.  CDZ_ERR_ARG for
 * wg < -1. */
int cdz_debug_set_fuse(cdz_handle *h, int wg);

/* Copy one workspace array of the last pass to host memory dst (bytes long):
 * which = 0..11 forward arrays (U Qb G F DI Qm1 Qm1Lr Qm1Lt Qm1p QmX Qm Qmt),
 * 12..24 adjoints (Qbb Qm1b Qm1pb QmXb QmXbt Qmb Qm1Lb DIb Gb Fb Ub UbL UbR),
 * 25 the diagonal exponents (int32, n + 1).  Elements are in the handle's
 * precision, ld x ld of them (*ld receives ld).  CDZ_ERR_STATE without a
 * forward pass, CDZ_ERR_ARG for a bad index or a short buffer. */
cdz_status cdz_debug_copy(cdz_handle *h, int which, void *dst, size_t bytes, long long *ld);

#ifdef __cplusplus
}
#endif
#endif /* CDZ_DEBUG_H */
