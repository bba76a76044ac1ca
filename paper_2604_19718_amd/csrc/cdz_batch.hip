// cdz_batch.hip -- batches of proteins of uneven length on one handle.
//
// The batch is split, in order, into chunks whose workspaces fit the memory
// budget.  Inside a chunk each diagonal index is ONE launch that covers that
// diagonal of every protein long enough to have it: the workgroups of the
// launch are dealt to the proteins by prefix offsets (cdz_batch_locate), so
// the cells of short proteins fill the device beside the long ones and the
// launch count is that of the longest protein, not the sum over proteins.
// The per-cell work is the single-protein kernels' (fwd_cell, out_cell,
// eta_edge, the sampler), so every protein's results equal those of the
// single-protein calls bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "cdz.h"
#include "cdz_dev.h"
#include "cdz_internal.h"

template <typename T>
__global__ void cdz_fwd_diag_batch(const DevProb<T> *probs, const int *off, int count, int dl);
template <typename T>
__global__ void cdz_exterior_trunc_batch(const DevProb<T> *probs, const int *W);
template <typename T>
__global__ void cdz_exterior_scan_batch(const DevProb<T> *probs, const int *W, const int *jend, int per);
template <typename T>
__global__ void cdz_landscape_batch(const DevProb<T> *probs);
template <typename T>
__global__ void cdz_spread_check_batch(const DevProb<T> *probs, const int *off, int count);
template <typename T>
__global__ void cdz_out_diag_batch(const DevProb<T> *probs, const DevAdj<T> *adjs, const int *off, int count,
                                   int dl);
template <typename T>
__global__ void cdz_eta_batch(const DevProb<T> *probs, const DevAdj<T> *adjs, const int *off, int count);
template <typename T>
__global__ void cdz_pairprob(DevProb<T> D, DevAdj<T> A, double r);

namespace {

const double kLn2 = 0.6931471805599453094;

// Host image of the small descriptor buffer of one phase (problem records and
// launch offset tables), uploaded to the handle's batch buffer in one copy.
struct Meta {
  std::vector<char> img;
  size_t put(const void *p, size_t bytes) {
    const size_t at = (img.size() + 255) / 256 * 256;
    img.resize(at + bytes);
    if (bytes) memcpy(img.data() + at, p, bytes);
    return at;
  }
};

// Offsets of a sequence of launches over `count` problems: launch l gives
// problem b wg(b, l) workgroups; its table is the count + 1 prefix sums.
struct Launches {
  int count = 0, nl = 0;
  std::vector<int> off;  // [nl][count + 1]
  template <typename F>
  Launches(int count_, int nl_, F wg) : count(count_), nl(nl_), off((size_t)nl_ * (count_ + 1)) {
    for (int l = 0; l < nl; l++) {
      int *o = &off[(size_t)l * (count + 1)];
      o[0] = 0;
      for (int b = 0; b < count; b++) o[b + 1] = o[b] + wg(b, l);
    }
  }
  int total(int l) const { return off[(size_t)l * (count + 1) + count]; }
  size_t at(int l) const { return (size_t)l * (count + 1); }
};

// the descriptor buffer of the handle, grown to `bytes`; the stream must be idle
cdz_status meta_upload(cdz_handle *h, const Meta &m, char **dev) {
  if (m.img.size() > h->bws_bytes) {
    if (h->bws) HIPCHK(h, hipFree(h->bws));
    h->bws = nullptr;
    h->bws_bytes = 0;
    if (hipMalloc(&h->bws, m.img.size()) != hipSuccess) {
      (void)hipGetLastError();
      return cdz_fail(h, CDZ_ERR_NOMEM, "batch descriptor allocation failed");
    }
    h->bws_bytes = m.img.size();
  }
  HIPCHK(h, hipMemcpyAsync(h->bws, m.img.data(), m.img.size(), hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));  // the host image may go away after this
  *dev = (char *)h->bws;
  return CDZ_OK;
}

template <typename T>
struct Chunk {
  std::vector<const HostTables *> t;
  std::vector<DevProb<T>> D;
  std::vector<DevAdj<T>> A;
  std::vector<double> res;  // [count][8] scalars of each forward
  int count() const { return (int)t.size(); }
  int nmax() const {
    int r = 0;
    for (auto *x : t) r = std::max(r, x->n);
    return r;
  }
};

// forward diagonals 0..dlmax[b] of the listed problems (dP: their records)
template <typename T>
cdz_status fwd_pass(cdz_handle *h, const DevProb<T> *dP, const int *dOff, const Launches &L, size_t shm) {
  for (int l = 0; l < L.nl; l++) {
    const int tot = L.total(l);
    if (tot == 0) continue;
    hipLaunchKernelGGL(cdz_fwd_diag_batch<T>, dim3(tot), dim3(CDZ_NT), shm, h->stream, dP, dOff + L.at(l),
                       L.count, l);
  }
  HIPCHK(h, hipGetLastError());
  return CDZ_OK;
}

Launches fwd_launches(const std::vector<int> &n, const std::vector<int> &dlmax) {
  int nl = 0;
  for (int x : dlmax) nl = std::max(nl, x + 1);
  return Launches((int)n.size(), nl, [&](int b, int t) { return t <= dlmax[b] ? fwd_nblocks(n[b], t) : 0; });
}

// Forward passes of every problem of the chunk (the sequence of the
// single-problem forward: FP32 landscape estimate, exact pass, spread check and
// the repeated pass where needed).
template <typename T>
cdz_status chunk_forward(cdz_handle *h, Chunk<T> &C) {
  const int cnt = C.count(), nmax = C.nmax();
  hipStream_t st = h->stream;
  const bool fp32 = std::is_same<T, float>::value;
  const size_t shm = fwd_lds_bytes<T>(nmax);
  if (shm > (size_t)h->lds_max)
    return cdz_fail(h, CDZ_ERR_ARG, "sequence of " + std::to_string(nmax) + " nt exceeds the LDS layout of the forward kernel");
  HIPCHK(h, hipFuncSetAttribute((const void *)cdz_fwd_diag_batch<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)shm));
  if (scan_lds_bytes(nmax) > (size_t)h->lds_max)
    return cdz_fail(h, CDZ_ERR_ARG, "sequence of " + std::to_string(nmax) + " nt exceeds the LDS layout of the exterior scan");
  HIPCHK(h, hipFuncSetAttribute((const void *)cdz_exterior_scan_batch<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)scan_lds_bytes(nmax)));
  std::vector<int> n(cnt), W(cnt), full(cnt), Wm1(cnt), nm1(cnt);
  for (int b = 0; b < cnt; b++) {
    n[b] = C.t[b]->n;
    W[b] = landscape_span(n[b], h->span);
    full[b] = n[b];
    Wm1[b] = W[b] - 1;  // truncated pass: prefix scan of the first W positions
    nm1[b] = n[b] - 1;  // exact pass: pairs of every span, every position
  }
  const Launches Ltr = fwd_launches(n, W), Lex = fwd_launches(n, full);
  const Launches Lsp(cnt, 1, [&](int b, int) { return n[b]; });
  Meta m;
  const size_t oP = m.put(C.D.data(), cnt * sizeof(DevProb<T>));
  const size_t oW = m.put(W.data(), cnt * sizeof(int));
  const size_t oWm1 = m.put(Wm1.data(), cnt * sizeof(int));
  const size_t oNm1 = m.put(nm1.data(), cnt * sizeof(int));
  const size_t oTr = m.put(Ltr.off.data(), Ltr.off.size() * sizeof(int));
  const size_t oEx = m.put(Lex.off.data(), Lex.off.size() * sizeof(int));
  const size_t oSp = m.put(Lsp.off.data(), Lsp.off.size() * sizeof(int));
  char *dev;
  cdz_status s = meta_upload(h, m, &dev);
  if (s != CDZ_OK) return s;
  const DevProb<T> *dP = (const DevProb<T> *)(dev + oP);
  HIPCHK(h, hipEventRecord(h->ev[0], st));
  for (int b = 0; b < cnt; b++) {
    HIPCHK(h, hipMemsetAsync(C.D[b].res, 0, 8 * sizeof(double), st));
    HIPCHK(h, hipMemsetAsync(C.D[b].maxb, 0, (n[b] + 1) * sizeof(unsigned), st));
    HIPCHK(h, hipMemsetAsync(C.D[b].E, 0, (n[b] + 1) * sizeof(int), st));
  }
  C.res.assign((size_t)cnt * 8, 0.0);
  if (fp32) {
    s = fwd_pass<T>(h, dP, (const int *)(dev + oTr), Ltr, shm);
    if (s != CDZ_OK) return s;
    hipLaunchKernelGGL(cdz_exterior_scan_batch<T>, dim3(cnt), dim3(CDZ_SCAN_NT), scan_lds_bytes(nmax), st, dP,
                       (const int *)(dev + oW), (const int *)(dev + oWm1), 1);
    hipLaunchKernelGGL(cdz_exterior_trunc_batch<T>, dim3(cnt), dim3(64), 0, st, dP, (const int *)(dev + oW));
    hipLaunchKernelGGL(cdz_landscape_batch<T>, dim3(cnt), dim3(1024), 0, st, dP);
    for (int b = 0; b < cnt; b++) {
      HIPCHK(h, hipMemsetAsync(C.D[b].maxb, 0, (n[b] + 1) * sizeof(unsigned), st));
      HIPCHK(h, hipMemsetAsync(C.D[b].E, 0, (n[b] + 1) * sizeof(int), st));
    }
    s = fwd_pass<T>(h, dP, (const int *)(dev + oEx), Lex, shm);
    if (s != CDZ_OK) return s;
    HIPCHK(h, hipGetLastError());
  } else {
    s = fwd_pass<T>(h, dP, (const int *)(dev + oEx), Lex, shm);
    if (s != CDZ_OK) return s;
  }
  hipLaunchKernelGGL(cdz_exterior_scan_batch<T>, dim3(2 * cnt), dim3(CDZ_SCAN_NT), scan_lds_bytes(nmax), st, dP,
                     (const int *)(dev + oNm1), (const int *)(dev + oNm1), 2);
  // range check of every exact pass: flags res[5] (weak cell), res[6]
  // (non-finite entry); FP32 problems with weak cells repeat the pass once
  // with the landscape of the exact pass and are checked again
  hipLaunchKernelGGL(cdz_spread_check_batch<T>, dim3(Lsp.total(0)), dim3(CDZ_NT), 0, st, dP,
                     (const int *)(dev + oSp), cnt);
  HIPCHK(h, hipGetLastError());
  for (int b = 0; b < cnt; b++)
    HIPCHK(h, hipMemcpyAsync(&C.res[(size_t)b * 8], C.D[b].res, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipStreamSynchronize(st));
  h->landscape_retries = 0;
  if (fp32) {
    std::vector<DevProb<T>> R;
    std::vector<int> rn;
    for (int b = 0; b < cnt; b++)
      if (C.res[(size_t)b * 8 + 5] != 0.0 && C.res[(size_t)b * 8 + 6] == 0.0) {
        R.push_back(C.D[b]);
        rn.push_back(n[b]);
      }
    h->landscape_retries = (int)R.size();
    if (!R.empty()) {
      const int rc = (int)R.size();
      const Launches Lr = fwd_launches(rn, rn);
      const Launches Lrs(rc, 1, [&](int k, int) { return rn[k]; });
      Meta mr;
      const size_t rP = mr.put(R.data(), rc * sizeof(DevProb<T>));
      const size_t rO = mr.put(Lr.off.data(), Lr.off.size() * sizeof(int));
      const size_t rS = mr.put(Lrs.off.data(), Lrs.off.size() * sizeof(int));
      std::vector<int> rm1(rc);
      for (int k = 0; k < rc; k++) rm1[k] = rn[k] - 1;
      const size_t rN = mr.put(rm1.data(), rc * sizeof(int));
      s = meta_upload(h, mr, &dev);
      if (s != CDZ_OK) return s;
      const DevProb<T> *dR = (const DevProb<T> *)(dev + rP);
      hipLaunchKernelGGL(cdz_landscape_batch<T>, dim3(rc), dim3(1024), 0, st, dR);
      for (int k = 0; k < rc; k++) {
        HIPCHK(h, hipMemsetAsync(R[k].maxb, 0, (rn[k] + 1) * sizeof(unsigned), st));
        HIPCHK(h, hipMemsetAsync(R[k].E, 0, (rn[k] + 1) * sizeof(int), st));
        HIPCHK(h, hipMemsetAsync(R[k].res + 5, 0, 3 * sizeof(double), st));
      }
      s = fwd_pass<T>(h, dR, (const int *)(dev + rO), Lr, shm);
      if (s != CDZ_OK) return s;
      hipLaunchKernelGGL(cdz_exterior_scan_batch<T>, dim3(2 * rc), dim3(CDZ_SCAN_NT), scan_lds_bytes(nmax), st, dR,
                         (const int *)(dev + rN), (const int *)(dev + rN), 2);
      hipLaunchKernelGGL(cdz_spread_check_batch<T>, dim3(Lrs.total(0)), dim3(CDZ_NT), 0, st, dR,
                         (const int *)(dev + rS), rc);
      HIPCHK(h, hipGetLastError());
    }
  }
  HIPCHK(h, hipEventRecord(h->ev[1], st));
  for (int b = 0; b < cnt; b++)
    HIPCHK(h, hipMemcpyAsync(&C.res[(size_t)b * 8], C.D[b].res, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipStreamSynchronize(st));
  float ms = 0;
  HIPCHK(h, hipEventElapsedTime(&ms, h->ev[0], h->ev[1]));
  h->times[0] += ms;
  for (int b = 0; b < cnt; b++) {
    const double *r = &C.res[(size_t)b * 8];
    if (r[6] != 0.0)
      return cdz_fail(h, CDZ_ERR_NUMERIC, "non-finite entries in the forward pass of a batch member (" +
                                              std::string(fp32 ? "FP32-scaled" : "FP64") + " range exceeded)");
    if (r[5] != 0.0)
      return cdz_fail(h, CDZ_ERR_NUMERIC, "cells of the forward pass of a batch member fell below 2^-" +
                                              std::to_string(C.D[b].lowExp) + " (" +
                                              std::string(fp32 ? "FP32-scaled" : "FP64") + " range exceeded)");
    if (!std::isfinite(r[0]) || !std::isfinite(r[1]))
      return cdz_fail(h, CDZ_ERR_NUMERIC, "log Z not finite (scaling out of range)");
  }
  return CDZ_OK;
}

// Outside passes and device marginals (edge marginals, pair probabilities)
template <typename T>
cdz_status chunk_outside(cdz_handle *h, Chunk<T> &C) {
  const int cnt = C.count(), nmax = C.nmax();
  hipStream_t st = h->stream;
  const size_t shm = out_lds_bytes<T>(nmax);
  if (shm > (size_t)h->lds_max)
    return cdz_fail(h, CDZ_ERR_ARG, "sequence of " + std::to_string(nmax) + " nt exceeds the LDS layout of the outside kernel");
  HIPCHK(h, hipFuncSetAttribute((const void *)cdz_out_diag_batch<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)shm));
  std::vector<int> n(cnt);
  for (int b = 0; b < cnt; b++) n[b] = C.t[b]->n;
  const Launches Lo(cnt, nmax, [&](int b, int dl) { return dl <= n[b] - 1 ? out_nblocks(n[b], dl) : 0; });
  const Launches Le(cnt, 1, [&](int b, int) { return n[b] >= 2 ? n[b] - 1 : 0; });
  Meta m;
  const size_t oP = m.put(C.D.data(), cnt * sizeof(DevProb<T>));
  const size_t oA = m.put(C.A.data(), cnt * sizeof(DevAdj<T>));
  const size_t oO = m.put(Lo.off.data(), Lo.off.size() * sizeof(int));
  const size_t oE = m.put(Le.off.data(), Le.off.size() * sizeof(int));
  char *dev;
  cdz_status s = meta_upload(h, m, &dev);
  if (s != CDZ_OK) return s;
  const DevProb<T> *dP = (const DevProb<T> *)(dev + oP);
  const DevAdj<T> *dA = (const DevAdj<T> *)(dev + oA);
  HIPCHK(h, hipEventRecord(h->ev[2], st));
  for (int b = 0; b < cnt; b++) {
    // accumulators of pushed adjoints start at zero
    const DevProb<T> &D = C.D[b];
    const DevAdj<T> &A = C.A[b];
    const size_t S2b = (size_t)D.ld * D.ld * sizeof(T);
    HIPCHK(h, hipMemsetAsync(A.UbL, 0, S2b, st));
    HIPCHK(h, hipMemsetAsync(A.UbR, 0, S2b, st));
    HIPCHK(h, hipMemsetAsync(A.UbL2, 0, S2b, st));
    HIPCHK(h, hipMemsetAsync(A.UbR2, 0, S2b, st));
    HIPCHK(h, hipMemsetAsync(A.DIbL, 0, S2b, st));
    HIPCHK(h, hipMemsetAsync(A.DIbR, 0, S2b, st));
    HIPCHK(h, hipMemsetAsync(A.etaV, 0, (size_t)n[b] * 36 * sizeof(double), st));
    HIPCHK(h, hipMemsetAsync(A.etaW, 0, (size_t)n[b] * 36 * sizeof(double), st));
  }
  for (int dl = nmax - 1; dl >= 0; dl--) {
    const int tot = Lo.total(dl);
    if (tot == 0) continue;
    hipLaunchKernelGGL(cdz_out_diag_batch<T>, dim3(tot), dim3(CDZ_NT), shm, st, dP, dA,
                       (const int *)(dev + oO) + Lo.at(dl), cnt, dl);
  }
  HIPCHK(h, hipGetLastError());
  if (eta_lds_bytes(nmax) > (size_t)h->lds_max)
    return cdz_fail(h, CDZ_ERR_ARG, "sequence of " + std::to_string(nmax) + " nt exceeds the LDS layout of the edge kernel");
  HIPCHK(h, hipFuncSetAttribute((const void *)cdz_eta_batch<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)eta_lds_bytes(nmax)));
  if (Le.total(0) > 0)
    hipLaunchKernelGGL(cdz_eta_batch<T>, dim3(Le.total(0)), dim3(CDZ_NT), eta_lds_bytes(nmax), st, dP, dA,
                       (const int *)(dev + oE), cnt);
  for (int b = 0; b < cnt; b++) {
    const double *r = &C.res[(size_t)b * 8];
    const double sc = std::exp(r[2] * kLn2 - r[0]);
    const long long nn = (long long)n[b] * n[b];
    hipLaunchKernelGGL(cdz_pairprob<T>, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, C.D[b], C.A[b], sc);
  }
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipEventRecord(h->ev[3], st));
  HIPCHK(h, hipStreamSynchronize(st));
  float ms = 0;
  HIPCHK(h, hipEventElapsedTime(&ms, h->ev[2], h->ev[3]));
  h->times[1] += ms;
  return CDZ_OK;
}

// output offsets of problem b in the concatenated outputs
struct OutOff {
  size_t pair = 0, base = 0, codon = 0, codon_pair = 0, samp_c = 0, samp_p = 0;
};

template <typename T>
cdz_status run_batch(cdz_handle *h, const std::vector<HostTables> &tabs, int32_t N, uint64_t seed, double *log_z,
                     double *pair, double *base, double *codon, double *codon_pair, uint8_t *codons,
                     int32_t *pairs) {
  const int count = (int)tabs.size();
  const bool adjoint = pair || base || codon || codon_pair;
  const bool sampling = N > 0;
  // workspace of each problem, laid out back to back inside a chunk
  std::vector<size_t> need(count);
  size_t biggest = 0;
  for (int b = 0; b < count; b++) {
    DevProb<T> D;
    DevAdj<T> A;
    memset(&D, 0, sizeof(D));
    memset(&A, 0, sizeof(A));
    need[b] = (carve<T>(nullptr, tabs[b], D, A, adjoint, CDZ_AL_RESIDENT) + 255) / 256 * 256;
    if ((unsigned long long)D.ld * (unsigned long long)D.ld > 0x7fffffffull)
      return cdz_fail(h, CDZ_ERR_ARG, "sequence of " + std::to_string(tabs[b].n) + " nt is too long for 32-bit block offsets");
    biggest = std::max(biggest, need[b]);
  }
  size_t budget = h->opt.mem_budget_bytes;
  if (budget == 0) {
    // what the device has left, with the handle's own workspace counted as free
    size_t fr = 0, tot = 0;
    HIPCHK(h, hipMemGetInfo(&fr, &tot));
    const size_t avail = fr + h->ws_bytes;
    const size_t reserve = (size_t)1 << 30;
    budget = avail > reserve ? (avail - reserve) / 10 * 9 : 0;
  }
  if (biggest > budget)
    return cdz_fail(h, h->opt.mem_budget_bytes ? CDZ_ERR_BUDGET : CDZ_ERR_NOMEM,
                    "workspace of " + std::to_string(biggest) + " bytes for one problem exceeds the budget");
  std::vector<OutOff> oo(count + 1);
  for (int b = 0; b < count; b++) {
    const size_t n = tabs[b].n, m = tabs[b].m;
    oo[b + 1].pair = oo[b].pair + n * n;
    oo[b + 1].base = oo[b].base + n * 4;
    oo[b + 1].codon = oo[b].codon + m * 6;
    oo[b + 1].codon_pair = oo[b].codon_pair + m * 36;
    oo[b + 1].samp_c = oo[b].samp_c + (size_t)N * m;
    oo[b + 1].samp_p = oo[b].samp_p + (size_t)N * n;
  }
  int start = 0;
  int retries = 0;
  while (start < count) {
    // greedy chunk [start, stop): as many problems as the budget holds
    int stop = start;
    size_t used = 0;
    while (stop < count && used + need[stop] <= budget) used += need[stop++];
    if (used > h->ws_bytes) {
      if (h->ws) HIPCHK(h, hipFree(h->ws));
      h->ws = nullptr;
      h->ws_bytes = 0;
      if (hipMalloc(&h->ws, used) != hipSuccess) {
        h->ws = nullptr;
        (void)hipGetLastError();
        return cdz_fail(h, CDZ_ERR_NOMEM, "hipMalloc of " + std::to_string(used) + " bytes failed");
      }
      h->ws_bytes = used;
    }
    Chunk<T> C;
    size_t at = 0;
    for (int b = start; b < stop; b++) {
      DevProb<T> D;
      DevAdj<T> A;
      memset(&D, 0, sizeof(D));
      memset(&A, 0, sizeof(A));
      carve<T>((char *)h->ws + at, tabs[b], D, A, adjoint, CDZ_AL_RESIDENT);
      D.lowExp = spread_low(h->low_exp, sizeof(T) == 4);
      at += need[b];
      cdz_status s = upload<T>(h, tabs[b], D);
      if (s != CDZ_OK) return s;
      C.t.push_back(&tabs[b]);
      C.D.push_back(D);
      C.A.push_back(A);
    }
    cdz_status s = chunk_forward<T>(h, C);
    if (s != CDZ_OK) return s;
    retries += h->landscape_retries;
    for (int b = start; b < stop; b++) {
      const double *r = &C.res[(size_t)(b - start) * 8];
      if (log_z) log_z[b] = r[0] + r[3] * kLn2;
    }
    if (adjoint) {
      s = chunk_outside<T>(h, C);
      if (s != CDZ_OK) return s;
      for (int b = start; b < stop; b++) {
        const double *r = &C.res[(size_t)(b - start) * 8];
        const DevAdj<T> &A = C.A[b - start];
        s = assemble_marginals(h, tabs[b], A.eta, A.pair, std::exp(r[2] * kLn2 - r[0]),
                               pair ? pair + oo[b].pair : nullptr, base ? base + oo[b].base : nullptr,
                               codon ? codon + oo[b].codon : nullptr,
                               codon_pair ? codon_pair + oo[b].codon_pair : nullptr);
        if (s != CDZ_OK) return s;
      }
    }
    if (sampling) {
      s = sample_batch<T>(h, C.D, seed + (uint64_t)start, N, codons + oo[start].samp_c, pairs + oo[start].samp_p);
      if (s != CDZ_OK) return s;
    }
    start = stop;
  }
  h->landscape_retries = retries;
  return CDZ_OK;
}

}  // namespace

extern "C" cdz_status cdz_workspace_bytes(cdz_handle *h, const cdz_problem *prob, int32_t what, size_t *bytes) {
  if (!h) return CDZ_ERR_ARG;
  if (!prob || !bytes || what < 0 || what > 3) return cdz_fail(h, CDZ_ERR_ARG, "bad argument");
  HostTables t;
  cdz_status s = build_tables(h, prob->n_aa, prob->aa, prob->theta1, prob->theta2, t);
  if (s != CDZ_OK) return s;
  const bool adj = what == CDZ_WS_MARGINALS || what == CDZ_WS_MARGINALS_MIN;
  const bool least = what == CDZ_WS_MARGINALS_MIN || what == CDZ_WS_FORWARD_MIN;
  auto size = [&](int alK) -> size_t {
    size_t b;
    if (h->opt.prec == CDZ_FP64) {
      DevProb<double> D;
      DevAdj<double> A;
      b = carve<double>(nullptr, t, D, A, adj, alK);
    } else {
      DevProb<float> D;
      DevAdj<float> A;
      b = carve<float>(nullptr, t, D, A, adj, alK);
    }
    return (b + 255) / 256 * 256;
  };
  *bytes = size(CDZ_AL_RESIDENT);
  // short sequences: the resident form can be the smaller one
  if (least) *bytes = std::min(*bytes, size(adj ? al_best_k(t.n) : 0));
  return CDZ_OK;
}

// Common entry of the batched calls: forward of every problem, the outside
// pass when a marginal output is given, N samples of each problem when N > 0.
extern "C" cdz_status cdz_batch(cdz_handle *h, const cdz_problem *probs, int32_t count, int32_t n_samples,
                                uint64_t seed, double *log_z, double *pair, double *base, double *codon,
                                double *codon_pair, uint8_t *codons, int32_t *pairs) {
  if (!h) return CDZ_ERR_ARG;
  if (count < 0 || (count > 0 && !probs)) return cdz_fail(h, CDZ_ERR_ARG, "bad problem list");
  if (n_samples < 0) return cdz_fail(h, CDZ_ERR_ARG, "n_samples < 0");
  if (n_samples > 0 && (!codons || !pairs)) return cdz_fail(h, CDZ_ERR_ARG, "null sample output");
  std::vector<HostTables> tabs(count);
  for (int b = 0; b < count; b++) {
    cdz_status s = build_tables(h, probs[b].n_aa, probs[b].aa, probs[b].theta1, probs[b].theta2, tabs[b]);
    if (s != CDZ_OK) {
      h->err = "problem " + std::to_string(b) + ": " + h->err;
      return s;
    }
  }
  // the workspace is about to be overwritten
  h->have_fwd = false;
  for (double &t : h->times) t = 0;
  if (count == 0) return CDZ_OK;
  return h->opt.prec == CDZ_FP64
             ? run_batch<double>(h, tabs, n_samples, seed, log_z, pair, base, codon, codon_pair, codons, pairs)
             : run_batch<float>(h, tabs, n_samples, seed, log_z, pair, base, codon, codon_pair, codons, pairs);
}

extern "C" cdz_status cdz_partition_batch(cdz_handle *h, const cdz_problem *probs, int32_t count, double *log_z) {
  if (!h) return CDZ_ERR_ARG;
  if (!log_z) return cdz_fail(h, CDZ_ERR_ARG, "null argument");
  return cdz_batch(h, probs, count, 0, 0, log_z, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
}

extern "C" cdz_status cdz_marginals_batch(cdz_handle *h, const cdz_problem *probs, int32_t count, double *log_z,
                                          double *pair, double *base, double *codon, double *codon_pair) {
  if (!h) return CDZ_ERR_ARG;
  if (!pair && !base && !codon && !codon_pair) return cdz_fail(h, CDZ_ERR_ARG, "no marginal output");
  return cdz_batch(h, probs, count, 0, 0, log_z, pair, base, codon, codon_pair, nullptr, nullptr);
}

extern "C" cdz_status cdz_sample_batch(cdz_handle *h, const cdz_problem *probs, int32_t count, uint64_t seed,
                                       int32_t n_samples, uint8_t *codons, int32_t *pairs) {
  if (!h) return CDZ_ERR_ARG;
  return cdz_batch(h, probs, count, n_samples, seed, nullptr, nullptr, nullptr, nullptr, nullptr, codons, pairs);
}
