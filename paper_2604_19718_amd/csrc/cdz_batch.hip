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
__global__ void cdz_fwd_diag_batch_fused(const DevProb<T> *probs, const int *off, int count, int dl);
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
__global__ void cdz_out_diag_batch_fused(const DevProb<T> *probs, const DevAdj<T> *adjs, const int *off, int count,
                                         int dl);
template <typename T>
__global__ void cdz_eta_batch(const DevProb<T> *probs, const DevAdj<T> *adjs, const int *off, int count, int lch);
template <typename T>
__global__ void cdz_pairprob(DevProb<T> D, DevAdj<T> A, double r);

// Clears of a chunk's per-problem buffers, as kernels, so that a captured
// sequence holds kernel nodes only.  cdz_clear_fwd: maxb and E of problem
// blockIdx.x, and its scalars res[0..8) when `all`.
template <typename T>
__global__ __launch_bounds__(256) void cdz_clear_fwd(const DevProb<T> *probs, int all) {
  const DevProb<T> D = probs[blockIdx.x];
  for (int k = threadIdx.x; k <= D.n; k += 256) {
    D.maxb[k] = 0u;
    D.E[k] = 0;
  }
  if (all && threadIdx.x < 8) D.res[threadIdx.x] = 0.0;
}

// cdz_clear_out: the accumulators of pushed adjoints (six S x S arrays and
// the two per-edge FP64 arrays) of problem blockIdx.x / per, share
// blockIdx.x % per; every array starts 256-byte aligned and is a multiple of
// 16 bytes long.
template <typename T>
__global__ __launch_bounds__(256) void cdz_clear_out(const DevProb<T> *probs, const DevAdj<T> *adjs, int per) {
  const int b = blockIdx.x / per, part = blockIdx.x % per;
  const DevProb<T> D = probs[b];
  const DevAdj<T> A = adjs[b];
  const uint4 z = make_uint4(0u, 0u, 0u, 0u);
  const size_t q = (size_t)D.ld * D.ld * sizeof(T) / 16, qe = (size_t)D.n * 36 * sizeof(double) / 16;
  uint4 *arr[6] = {(uint4 *)A.UbL, (uint4 *)A.UbR, (uint4 *)A.UbL2, (uint4 *)A.UbR2, (uint4 *)A.DIbL,
                   (uint4 *)A.DIbR};
  const size_t step = (size_t)per * 256, first = (size_t)part * 256 + threadIdx.x;
#pragma unroll 1
  for (int a = 0; a < 6; a++)
    for (size_t k = first; k < q; k += step) arr[a][k] = z;
  for (size_t k = first; k < qe; k += step) {
    ((uint4 *)A.etaV)[k] = z;
    ((uint4 *)A.etaW)[k] = z;
  }
}

namespace {

const double kLn2 = 0.6931471805599453094;

// Enqueue `record(stream)` on the handle's stream through a hipGraph: the
// sequence is captured (on a stream of its own, where nothing runs) the first
// time `key` is seen and replayed on later calls with the same key.  record
// may launch kernels only (no memsets, copies or synchronisation).  With
// graphs switched off it runs directly on the handle's stream.
template <typename F>
cdz_status graph_run(cdz_handle *h, const std::string &key, F record) {
  if (!h->use_graphs) return record(h->stream);
  for (auto &g : h->graphs)
    if (g.key == key) {
      HIPCHK(h, hipGraphLaunch(g.x, h->stream));
      h->graph_replays++;
      return CDZ_OK;
    }
  if (!h->cap_stream) HIPCHK(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
  HIPCHK(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
  const cdz_status s = record(h->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
  if (s != CDZ_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return s != CDZ_OK ? s : cdz_fail(h, CDZ_ERR_HIP, std::string("stream capture failed: ") + hipGetErrorString(e));
  }
  hipGraphExec_t x = nullptr;
  const hipError_t ei = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(g);
    return cdz_fail(h, CDZ_ERR_HIP, std::string("graph instantiation failed: ") + hipGetErrorString(ei));
  }
  if (h->graphs.size() >= 16) {  // a small cache: drop the oldest
    (void)hipGraphExecDestroy(h->graphs.front().x);
    (void)hipGraphDestroy(h->graphs.front().g);
    h->graphs.erase(h->graphs.begin());
  }
  h->graphs.push_back({key, g, x});
  h->graph_captures++;
  HIPCHK(h, hipGraphLaunch(x, h->stream));
  return CDZ_OK;
}

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
// With a grouping function wg(b, l, fused) and a threshold, launch l runs
// fused when its unfused workgroups reach the threshold (fused[l]).
struct Launches {
  int count = 0, nl = 0;
  std::vector<int> off;      // [nl][count + 1]
  std::vector<char> fused;  // [nl]
  template <typename F>
  Launches(int count_, int nl_, F wg) : count(count_), nl(nl_), off((size_t)nl_ * (count_ + 1)), fused(nl_, 0) {
    for (int l = 0; l < nl; l++) {
      int *o = &off[(size_t)l * (count + 1)];
      o[0] = 0;
      for (int b = 0; b < count; b++) o[b + 1] = o[b] + wg(b, l);
    }
  }
  template <typename F>
  Launches(int count_, int nl_, F wg, int fuse_wg)
      : count(count_), nl(nl_), off((size_t)nl_ * (count_ + 1)), fused(nl_, 0) {
    for (int l = 0; l < nl; l++) {
      long long split = 0;
      for (int b = 0; b < count; b++) split += wg(b, l, false);
      fused[l] = split >= fuse_wg;
      int *o = &off[(size_t)l * (count + 1)];
      o[0] = 0;
      for (int b = 0; b < count; b++) o[b + 1] = o[b] + wg(b, l, fused[l] != 0);
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

// key of a captured sequence: phase, precision, the descriptor buffer and
// workspace it points into, and the descriptor image itself
std::string graph_key(const cdz_handle *h, const char *phase, size_t tsize, const Meta &m) {
  std::string k(phase);
  const void *ptrs[2] = {h->bws, h->ws};
  k.append(reinterpret_cast<const char *>(&tsize), sizeof(tsize));
  k.append(reinterpret_cast<const char *>(ptrs), sizeof(ptrs));
  k.append(m.img.data(), m.img.size());
  return k;
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
cdz_status fwd_pass(cdz_handle *h, hipStream_t st, const DevProb<T> *dP, const int *dOff, const Launches &L,
                    size_t shm) {
  for (int l = 0; l < L.nl; l++) {
    const int tot = L.total(l);
    if (tot == 0) continue;
    if (L.fused[l])
      hipLaunchKernelGGL(cdz_fwd_diag_batch_fused<T>, dim3(tot), dim3(CDZ_NT), shm, st, dP, dOff + L.at(l), L.count,
                         l);
    else
      hipLaunchKernelGGL(cdz_fwd_diag_batch<T>, dim3(tot), dim3(CDZ_NT), shm, st, dP, dOff + L.at(l), L.count, l);
  }
  HIPCHK(h, hipGetLastError());
  return CDZ_OK;
}

Launches fwd_launches(const std::vector<int> &n, const std::vector<int> &dlmax, int fuse_wg) {
  int nl = 0;
  for (int x : dlmax) nl = std::max(nl, x + 1);
  return Launches(
      (int)n.size(), nl, [&](int b, int t, bool fu) { return t <= dlmax[b] ? fwd_nblocks(n[b], t, fu) : 0; },
      fuse_wg);
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
  HIPCHK(h, hipFuncSetAttribute((const void *)cdz_fwd_diag_batch_fused<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
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
  long long wmax = 0;
  {
    int nl = 0;
    for (int x : n) nl = std::max(nl, x);
    for (int t = 0; t < nl; t++) {
      long long w = 0;
      for (int b = 0; b < cnt; b++) w += t < n[b] ? fwd_nblocks(n[b], t) : 0;
      wmax = std::max(wmax, w);
    }
  }
  const uint64_t tkey = tune_key(0, true, sizeof(T), wmax);
  tune_begin(h, tkey);
  const Launches Ltr = fwd_launches(n, W, h->fuse_wg), Lex = fwd_launches(n, full, h->fuse_wg);
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
  C.res.assign((size_t)cnt * 8, 0.0);
  // the passes up to the range check: captured once per chunk image, replayed after
  s = graph_run(h, graph_key(h, "forward", sizeof(T), m), [&](hipStream_t gs) -> cdz_status {
    hipLaunchKernelGGL(cdz_clear_fwd<T>, dim3(cnt), dim3(256), 0, gs, dP, 1);
    if (fp32) {
      cdz_status s2 = fwd_pass<T>(h, gs, dP, (const int *)(dev + oTr), Ltr, shm);
      if (s2 != CDZ_OK) return s2;
      hipLaunchKernelGGL(cdz_exterior_scan_batch<T>, dim3(cnt), dim3(CDZ_SCAN_NT), scan_lds_bytes(nmax), gs, dP,
                         (const int *)(dev + oW), (const int *)(dev + oWm1), 1);
      hipLaunchKernelGGL(cdz_exterior_trunc_batch<T>, dim3(cnt), dim3(64), 0, gs, dP, (const int *)(dev + oW));
      hipLaunchKernelGGL(cdz_landscape_batch<T>, dim3(cnt), dim3(1024), 0, gs, dP);
      hipLaunchKernelGGL(cdz_clear_fwd<T>, dim3(cnt), dim3(256), 0, gs, dP, 0);
    }
    cdz_status s2 = fwd_pass<T>(h, gs, dP, (const int *)(dev + oEx), Lex, shm);
    if (s2 != CDZ_OK) return s2;
    hipLaunchKernelGGL(cdz_exterior_scan_batch<T>, dim3(2 * cnt), dim3(CDZ_SCAN_NT), scan_lds_bytes(nmax), gs, dP,
                       (const int *)(dev + oNm1), (const int *)(dev + oNm1), 2);
    // range check of every exact pass: flags res[5] (weak cell), res[6]
    // (non-finite entry); FP32 problems with weak cells repeat the pass once
    // with the landscape of the exact pass and are checked again
    hipLaunchKernelGGL(cdz_spread_check_batch<T>, dim3(Lsp.total(0)), dim3(CDZ_NT), 0, gs, dP,
                       (const int *)(dev + oSp), cnt);
    HIPCHK(h, hipGetLastError());
    return CDZ_OK;
  });
  if (s != CDZ_OK) return s;
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
      const Launches Lr = fwd_launches(rn, rn, h->fuse_wg);
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
      s = fwd_pass<T>(h, st, dR, (const int *)(dev + rO), Lr, shm);
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
  if (h->landscape_retries == 0) tune_end(h, tkey, ms);
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
  HIPCHK(h, hipFuncSetAttribute((const void *)cdz_out_diag_batch_fused<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)shm));
  std::vector<int> n(cnt);
  for (int b = 0; b < cnt; b++) n[b] = C.t[b]->n;
  long long wmax = 0;
  for (int t = 0; t < nmax; t++) {
    long long w = 0;
    for (int b = 0; b < cnt; b++) w += t < n[b] ? out_nblocks(n[b], t) : 0;
    wmax = std::max(wmax, w);
  }
  const uint64_t tkey = tune_key(1, true, sizeof(T), wmax);
  tune_begin(h, tkey);
  const Launches Lo(
      cnt, nmax, [&](int b, int dl, bool fu) { return dl <= n[b] - 1 ? out_nblocks(n[b], dl, fu) : 0; },
      h->fuse_wg);
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
  if (eta_lds_bytes(nmax, sizeof(T)) > (size_t)h->lds_max)
    return cdz_fail(h, CDZ_ERR_ARG, "sequence of " + std::to_string(nmax) + " nt exceeds the LDS layout of the edge kernel");
  HIPCHK(h, hipFuncSetAttribute((const void *)cdz_eta_batch<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)eta_lds_bytes(nmax, sizeof(T))));
  std::vector<double> sc(cnt);
  for (int b = 0; b < cnt; b++) {
    const double *r = &C.res[(size_t)b * 8];
    sc[b] = std::exp(r[2] * kLn2 - r[0]);
  }
  m.put(sc.data(), cnt * sizeof(double));  // part of the key: pairprob takes the scale by value
  HIPCHK(h, hipEventRecord(h->ev[2], st));
  s = graph_run(h, graph_key(h, "outside", sizeof(T), m), [&](hipStream_t gs) -> cdz_status {
    // accumulators of pushed adjoints start at zero
    hipLaunchKernelGGL(cdz_clear_out<T>, dim3(cnt * 64), dim3(256), 0, gs, dP, dA, 64);
    for (int dl = nmax - 1; dl >= 0; dl--) {
      const int tot = Lo.total(dl);
      if (tot == 0) continue;
      if (Lo.fused[dl])
        hipLaunchKernelGGL(cdz_out_diag_batch_fused<T>, dim3(tot), dim3(CDZ_NT), shm, gs, dP, dA,
                           (const int *)(dev + oO) + Lo.at(dl), cnt, dl);
      else
        hipLaunchKernelGGL(cdz_out_diag_batch<T>, dim3(tot), dim3(CDZ_NT), shm, gs, dP, dA,
                           (const int *)(dev + oO) + Lo.at(dl), cnt, dl);
    }
    if (Le.total(0) > 0)
      hipLaunchKernelGGL(cdz_eta_batch<T>, dim3(Le.total(0)), dim3(cdz_eta_nt(sizeof(T))), eta_lds_bytes(nmax, sizeof(T)), gs, dP, dA,
                         (const int *)(dev + oE), cnt, eta_bulge_chunk(nmax, sizeof(T)));
    for (int b = 0; b < cnt; b++) {
      const long long nn = (long long)n[b] * n[b];
      hipLaunchKernelGGL(cdz_pairprob<T>, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, gs, C.D[b], C.A[b],
                         sc[b]);
    }
    HIPCHK(h, hipGetLastError());
    return CDZ_OK;
  });
  if (s != CDZ_OK) return s;
  HIPCHK(h, hipEventRecord(h->ev[3], st));
  HIPCHK(h, hipStreamSynchronize(st));
  float ms = 0;
  HIPCHK(h, hipEventElapsedTime(&ms, h->ev[2], h->ev[3]));
  h->times[1] += ms;
  tune_end(h, tkey, ms);
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
  h->graph_captures = h->graph_replays = 0;
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
