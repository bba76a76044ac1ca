// cdz_host.hip -- C ABI of the codon-constrained partition-function library:
// input validation, per-position tables, device workspace, kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "cdz.h"
#include "cdz_dev.h"
#include "cdz_internal.h"

// ---------------------------------------------------------------------------
// Genetic code: the sense codons of each residue (standard code; start and
// stop codons are not designed, SI S3c).  Slots are the codons sorted by
// spelling under A < C < G < U.
// ---------------------------------------------------------------------------
namespace {
struct AaCodons {
  char aa;
  const char *codons[6];
};
const AaCodons kCode[20] = {
    {'A', {"GCU", "GCC", "GCA", "GCG"}},
    {'R', {"CGU", "CGC", "CGA", "CGG", "AGA", "AGG"}},
    {'N', {"AAU", "AAC"}},
    {'D', {"GAU", "GAC"}},
    {'C', {"UGU", "UGC"}},
    {'Q', {"CAA", "CAG"}},
    {'E', {"GAA", "GAG"}},
    {'G', {"GGU", "GGC", "GGA", "GGG"}},
    {'H', {"CAU", "CAC"}},
    {'I', {"AUU", "AUC", "AUA"}},
    {'L', {"UUA", "UUG", "CUU", "CUC", "CUA", "CUG"}},
    {'K', {"AAA", "AAG"}},
    {'M', {"AUG"}},
    {'F', {"UUU", "UUC"}},
    {'P', {"CCU", "CCC", "CCA", "CCG"}},
    {'S', {"UCU", "UCC", "UCA", "UCG", "AGU", "AGC"}},
    {'T', {"ACU", "ACC", "ACA", "ACG"}},
    {'W', {"UGG"}},
    {'Y', {"UAU", "UAC"}},
    {'V', {"GUU", "GUC", "GUA", "GUG"}},
};

int base_code(char c) {
  switch (c) {
    case 'A': return 0;
    case 'C': return 1;
    case 'G': return 2;
    case 'U': return 3;
  }
  return -1;
}

// slots[aa][s][r] = base; count[aa]
struct CodeTable {
  int count[128];
  signed char base[128][6][3];
  CodeTable() {
    memset(count, 0, sizeof(count));
    memset(base, -1, sizeof(base));
    for (const auto &row : kCode) {
      std::vector<std::string> cs;
      for (const char *c : row.codons)
        if (c) cs.push_back(c);
      std::sort(cs.begin(), cs.end(), [](const std::string &x, const std::string &y) {
        for (int r = 0; r < 3; r++)
          if (x[r] != y[r]) return base_code(x[r]) < base_code(y[r]);
        return false;
      });
      int a = (unsigned char)row.aa;
      count[a] = (int)cs.size();
      for (size_t s = 0; s < cs.size(); s++)
        for (int r = 0; r < 3; r++) base[a][s][r] = (signed char)base_code(cs[s][r]);
    }
  }
};
const CodeTable &code_table() {
  static CodeTable t;
  return t;
}

const char *kStatusText[] = {"ok", "invalid argument", "invalid protein letter",
                             "non-finite input or scaling out of range", "device allocation failed",
                             "memory budget exceeded", "HIP runtime error", "no matching forward pass"};

}  // namespace

// ---------------------------------------------------------------------------
// Handle
// ---------------------------------------------------------------------------
cdz_status cdz_fail(cdz_handle *h, cdz_status s, const std::string &msg) {
  if (h) h->err = msg;
  return s;
}

// the ABI record is 229 doubles: stack 36, hairpin/bulge/interior 3 x 31,
// mismatch 96, ml_a ml_b ml_c extrap 4
static_assert(sizeof(cdz_energy) == 229 * sizeof(double), "cdz_energy must be 229 doubles");

extern "C" const char *cdz_status_string(cdz_status s) {
  int k = (int)s;
  return (k >= 0 && k <= 7) ? kStatusText[k] : "unknown status";
}

extern "C" const char *cdz_last_error(const cdz_handle *h) { return h ? h->err.c_str() : ""; }

extern "C" cdz_status cdz_create(const cdz_energy *energy, const cdz_options *opts,
                                 cdz_handle **out) {
  if (!energy || !out) return CDZ_ERR_ARG;
  *out = nullptr;
  const double *p = reinterpret_cast<const double *>(energy);
  for (size_t k = 0; k < sizeof(cdz_energy) / sizeof(double); k++)
    if (std::isnan(p[k]) || p[k] == -INFINITY) return CDZ_ERR_NUMERIC;
  if (opts && opts->prec != CDZ_FP32_SCALED && opts->prec != CDZ_FP64) return CDZ_ERR_ARG;
  cdz_handle *h = new cdz_handle();
  h->en = *energy;
  if (opts) h->opt = *opts;
  else {
    h->opt.prec = CDZ_FP32_SCALED;
    h->opt.mem_budget_bytes = 0;
    h->opt.hip_stream = nullptr;
  }
  h->stream = reinterpret_cast<hipStream_t>(h->opt.hip_stream);
  if (hipGetDevice(&h->device) != hipSuccess ||
      hipDeviceGetAttribute(&h->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, h->device) != hipSuccess) {
    delete h;
    return CDZ_ERR_HIP;
  }
  for (auto &ev : h->ev)
    if (hipEventCreate(&ev) != hipSuccess) {
      delete h;
      return CDZ_ERR_HIP;
    }
  // device address of the fixed scratch of cdz_sample_noalloc on this device
  if (!noalloc_scratch(h->device)) {
    delete h;
    return CDZ_ERR_HIP;
  }
  *out = h;
  return CDZ_OK;
}

extern "C" void cdz_destroy(cdz_handle *h) {
  if (!h) return;
  if (h->ws) (void)hipFree(h->ws);
  if (h->smp) (void)hipFree(h->smp);
  if (h->bws) (void)hipFree(h->bws);
  for (auto &g : h->graphs) {
    if (g.x) (void)hipGraphExecDestroy(g.x);
    if (g.g) (void)hipGraphDestroy(g.g);
  }
  if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
  for (auto &ev : h->ev)
    if (ev) (void)hipEventDestroy(ev);
  for (auto &ev : h->pev) (void)hipEventDestroy(ev);
  delete h;
}

int codon_count(unsigned char letter) { return letter < 128 ? code_table().count[letter] : 0; }

// ---------------------------------------------------------------------------
// Problem tables
// ---------------------------------------------------------------------------
cdz_status build_tables(cdz_handle *h, int32_t n_aa, const char *aa, const double *theta1,
                        const double *theta2, HostTables &t) {
  if (n_aa < 1 || !aa) return cdz_fail(h, CDZ_ERR_ARG, "n_aa < 1 or aa == NULL");
  const CodeTable &ct = code_table();
  const int m = n_aa, n = 3 * m;
  t.m = m;
  t.n = n;
  t.d.assign(n, 0);
  t.P.assign(n + 1, 0);
  t.nt.assign((size_t)n * 6, -1);
  t.v.assign((size_t)n * 6, 0.0);
  t.e.assign((size_t)n * 36, 0.0);
  t.aa.assign(aa, aa + m);
  for (int a = 0; a < m; a++) {
    unsigned char c = (unsigned char)aa[a];
    if (c >= 128 || ct.count[c] == 0)
      return cdz_fail(h, CDZ_ERR_PROTEIN, std::string("invalid residue letter at ") + std::to_string(a));
    const int cnt = ct.count[c];
    for (int s = 0; s < cnt; s++) {
      if (theta1 && !std::isfinite(theta1[a * 6 + s]))
        return cdz_fail(h, CDZ_ERR_NUMERIC, "non-finite theta1");
      if (theta2 && a >= 1)
        for (int s0 = 0; s0 < ct.count[(unsigned char)aa[a - 1]]; s0++)
          if (!std::isfinite(theta2[(a * 6 + s0) * 6 + s]))
            return cdz_fail(h, CDZ_ERR_NUMERIC, "non-finite theta2");
    }
    for (int r = 0; r < 3; r++) {
      const int p = 3 * a + r;
      t.d[p] = cnt;
      for (int s = 0; s < cnt; s++) {
        t.nt[p * 6 + s] = ct.base[c][s][r];
        t.v[p * 6 + s] = (r == 1 && theta1) ? std::exp(theta1[a * 6 + s]) : 1.0;
      }
    }
  }
  for (int p = 0; p < n; p++) t.P[p + 1] = t.P[p] + t.d[p];
  t.S = t.P[n];
  t.posOf.resize(t.S);
  for (int p = 0; p < n; p++)
    for (int k = t.P[p]; k < t.P[p + 1]; k++) t.posOf[k] = p;
  for (int p = 0; p + 1 < n; p++)
    for (int s = 0; s < t.d[p]; s++)
      for (int u = 0; u < t.d[p + 1]; u++) {
        double w;
        if (p % 3 != 2) w = (s == u) ? 1.0 : 0.0;  // inside a codon: same slot
        else w = theta2 ? std::exp(theta2[((p / 3 + 1) * 6 + s) * 6 + u]) : 1.0;
        t.e[p * 36 + s * 6 + u] = w;
      }
  const cdz_energy &E = h->en;
  t.tab.assign(TB_LEN, 0.0);
  for (int k = 0; k < 36; k++) t.tab[TB_ST + k] = std::exp(-E.stack[k / 6][k % 6]);
  for (int L = 0; L <= 30; L++) {
    t.tab[TB_BU + L] = std::exp(-E.bulge[L]);
    t.tab[TB_IN + L] = std::exp(-E.interior[L]);
  }
  for (int x = 0; x < 4; x++)
    for (int y = 0; y < 4; y++)
      for (int q = 0; q < 6; q++) t.tab[TB_MM + x * 24 + y * 6 + q] = std::exp(-E.mismatch[x][y][q]);
  t.tab[TB_MLAB] = std::exp(-(E.ml_a + E.ml_b));
  t.tab[TB_MLB] = std::exp(-E.ml_b);
  t.tab[TB_MLC] = std::exp(-E.ml_c);
  t.Bhp.assign(n, 0.0);
  for (int L = 3; L < n; L++)
    t.Bhp[L] = L <= 30 ? std::exp(-E.hairpin[L])
                       : std::exp(-(E.hairpin[30] + E.extrap * std::log((double)L / 30.0)));
  // key of the problem, to reuse the forward pass
  uint64_t hsh = 1469598103934665603ull;
  auto mix = [&](const void *p, size_t nb) {
    const unsigned char *b = (const unsigned char *)p;
    for (size_t k = 0; k < nb; k++) hsh = (hsh ^ b[k]) * 1099511628211ull;
  };
  mix(aa, m);
  mix(t.v.data(), t.v.size() * 8);
  mix(t.e.data(), t.e.size() * 8);
  int prec = (int)h->opt.prec;
  mix(&prec, sizeof(prec));
  t.key = hsh;
  return CDZ_OK;
}

// ---------------------------------------------------------------------------
// Workspace: one device allocation carved into tables and S x S arrays
// ---------------------------------------------------------------------------
namespace {
struct Carver {
  size_t off = 0;
  template <typename X>
  X *take(char *base, size_t count) {
    off = (off + 255) / 256 * 256;
    X *p = base ? reinterpret_cast<X *>(base + off) : nullptr;
    off += count * sizeof(X);
    return p;
  }
};
}  // namespace

template <typename T>
size_t carve(char *base, const HostTables &t, DevProb<T> &D, DevAdj<T> &A, bool adjoint, int alK) {
  Carver c;
  const int n = t.n, S = t.S;
  const long long ld = ((long long)S + 31) / 32 * 32;
  const size_t S2 = (size_t)ld * ld;
  D.n = n;
  D.m = t.m;
  D.S = S;
  D.ld = ld;
  D.d = c.take<int>(base, n);
  D.P = c.take<int>(base, n + 1);
  D.posOf = c.take<int>(base, S);
  D.nt = c.take<signed char>(base, (size_t)n * 6);
  D.v = c.take<T>(base, (size_t)n * 6);
  D.e = c.take<T>(base, (size_t)n * 36);
  D.vd = c.take<double>(base, (size_t)n * 6);
  D.ed = c.take<double>(base, (size_t)n * 36);
  D.tab = c.take<T>(base, TB_LEN);
  D.Bhp = c.take<T>(base, n);
  D.E = c.take<int>(base, n + 1);
  D.EX = c.take<int>(base, n + 5);
  D.maxb = c.take<unsigned>(base, n + 1);
  D.Z5 = c.take<double>(base, (size_t)n * 6);
  D.A5 = c.take<double>(base, (size_t)n * 6);
  D.G5 = c.take<int>(base, n);
  D.Z3 = c.take<double>(base, (size_t)n * 6);
  D.H3 = c.take<int>(base, n);
  D.Cl = c.take<int>(base, n);
  D.res = c.take<double>(base, 8);
  T **arrs[] = {&D.U, &D.Qb, &D.G, &D.F, &D.DI, &D.Qm1, &D.Qm1Lr, &D.Qm1Lt,
                &D.Qm1p, &D.QmX, &D.Qm, &D.Qmt, &D.Ut, &D.DIt, &D.Qbt};
  for (T **a : arrs) *a = c.take<T>(base, S2);
  D.ldA = (long long)CDZ_NA * ld;
  D.lowExp = spread_low(0, sizeof(T) == 4);
  D.ALw = nullptr;
  D.ALp = nullptr;
  D.alK = alK;
  if (alK == CDZ_AL_RESIDENT) {
    D.AL = c.take<T>(base, (size_t)CDZ_NA * S2);
    D.ALs = nullptr;
    D.alTop = 0;
    D.alSlots = 0;
  } else {
    D.AL = nullptr;
    D.alTop = al_top(alK, n);
    D.alSlots = al_slots(alK, n);
    D.ALs = c.take<T>(base, (size_t)D.alSlots * n * CDZ_NA * 36);
  }
  if (adjoint) adj_carve<T>(c.off, base, t, A, S2);
  return c.off + 256;
}

template <typename T>
cdz_status upload(cdz_handle *h, const HostTables &t, DevProb<T> &D) {
  std::vector<T> v(t.v.begin(), t.v.end()), e(t.e.begin(), t.e.end()), tab(t.tab.begin(), t.tab.end()),
      bhp(t.Bhp.begin(), t.Bhp.end());
  hipStream_t st = h->stream;
  HIPCHK(h, hipMemcpyAsync((void *)D.d, t.d.data(), t.n * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync((void *)D.P, t.P.data(), (t.n + 1) * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync((void *)D.posOf, t.posOf.data(), t.S * sizeof(int), hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync((void *)D.nt, t.nt.data(), t.nt.size(), hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync((void *)D.v, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync((void *)D.e, e.data(), e.size() * sizeof(T), hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync((void *)D.vd, t.v.data(), t.v.size() * 8, hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync((void *)D.ed, t.e.data(), t.e.size() * 8, hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync((void *)D.tab, tab.data(), tab.size() * sizeof(T), hipMemcpyHostToDevice, st));
  HIPCHK(h, hipMemcpyAsync((void *)D.Bhp, bhp.data(), bhp.size() * sizeof(T), hipMemcpyHostToDevice, st));
  // the staging vectors must outlive the copies
  HIPCHK(h, hipStreamSynchronize(st));
  return CDZ_OK;
}
template size_t carve<float>(char *, const HostTables &, DevProb<float> &, DevAdj<float> &, bool, int);
template size_t carve<double>(char *, const HostTables &, DevProb<double> &, DevAdj<double> &, bool, int);

int al_best_k(int n) {
  int best = 2, cost = INT_MAX;
  for (int K = 2; K <= std::max(2, n); K++) {
    const int c = al_slots(K, n);
    if (c < cost) {
      cost = c;
      best = K;
    }
  }
  return best;
}
template cdz_status upload<float>(cdz_handle *, const HostTables &, DevProb<float> &);
template cdz_status upload<double>(cdz_handle *, const HostTables &, DevProb<double> &);

template <typename T>
__global__ void cdz_fwd_diag(DevProb<T> D, int dl);
template <typename T>
__global__ void cdz_fwd_diag_fused(DevProb<T> D, int dl);


template <typename T>
__global__ void cdz_landscape(DevProb<T> D);
template <typename T>
__global__ void cdz_exterior_trunc(DevProb<T> D, int W);
template <typename T>
__global__ void cdz_exterior_scan(DevProb<T> D, int W, int jend);
template <typename T>
__global__ void cdz_spread_check(DevProb<T> D);


template <typename T>
static cdz_status forward_pass(cdz_handle *h, DevProb<T> &D, size_t shm, bool timed, int dlmax) {
  const int n = D.n;
  hipStream_t st = h->stream;
  HIPCHK(h, hipMemsetAsync(D.maxb, 0, (n + 1) * sizeof(unsigned), st));
  HIPCHK(h, hipMemsetAsync(D.E, 0, (n + 1) * sizeof(int), st));  // E[0] = 0
  DevProb<T> Dl = D;
  for (int t = 0; t <= dlmax && t < n; t++) {
    if (!D.AL) {  // diagonal-major A: the window sums of launch t write diagonal t+1 and read t-1
      Dl.ALw = al_slot_ptr(D, al_slot_fwd(D.alK, D.alTop, t + 1));
      Dl.ALp = al_slot_ptr(D, al_slot_fwd(D.alK, D.alTop, t >= 1 ? t - 1 : 0));
    }
    if (timed) HIPCHK(h, hipEventRecord(h->pev[2 * t], st));
    if (fwd_nblocks(n, t) >= h->fuse_wg)
      hipLaunchKernelGGL(cdz_fwd_diag_fused<T>, dim3(fwd_nblocks(n, t, true)), dim3(CDZ_NT), shm, st, Dl, t);
    else
      hipLaunchKernelGGL(cdz_fwd_diag<T>, dim3(fwd_nblocks(n, t)), dim3(CDZ_NT), shm, st, Dl, t);
    if (timed) HIPCHK(h, hipEventRecord(h->pev[2 * t + 1], st));
  }
  // exterior loops over the finished diagonals: the exact pass runs the
  // prefix and suffix scans (log Z twice); the truncated pass of the FP32
  // landscape the prefix of its first W positions (cdz_exterior_trunc goes on)
  if (dlmax >= n - 1)
    hipLaunchKernelGGL(cdz_exterior_scan<T>, dim3(2), dim3(CDZ_SCAN_NT), scan_lds_bytes(n), st, D, n - 1, n - 1);
  else
    hipLaunchKernelGGL(cdz_exterior_scan<T>, dim3(1), dim3(CDZ_SCAN_NT), scan_lds_bytes(n), st, D, dlmax, dlmax - 1);
  HIPCHK(h, hipGetLastError());
  return CDZ_OK;
}

template <typename T>
static cdz_status launch_forward(cdz_handle *h, DevProb<T> &D) {
  const int n = D.n;
  hipStream_t st = h->stream;
  const size_t shm = fwd_lds_bytes<T>(n);
  if (shm > (size_t)h->lds_max)
    return cdz_fail(h, CDZ_ERR_ARG, "sequence of " + std::to_string(n) + " nt exceeds the LDS layout of the forward kernel");
  HIPCHK(h, hipFuncSetAttribute((const void *)cdz_fwd_diag<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
  HIPCHK(h, hipFuncSetAttribute((const void *)cdz_fwd_diag_fused<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)shm));
  if (scan_lds_bytes(n) > (size_t)h->lds_max)
    return cdz_fail(h, CDZ_ERR_ARG, "sequence of " + std::to_string(n) + " nt exceeds the LDS layout of the exterior scan");
  HIPCHK(h, hipFuncSetAttribute((const void *)cdz_exterior_scan<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)scan_lds_bytes(n)));
  const bool fp32 = std::is_same<T, float>::value;
  long long wmax = 0;
  for (int t = 0; t < n; t++) wmax = std::max<long long>(wmax, fwd_nblocks(n, t));
  const uint64_t tkey = tune_key(0, false, sizeof(T), wmax);
  tune_begin(h, tkey);
  HIPCHK(h, hipMemsetAsync(D.res, 0, 8 * sizeof(double), st));
  if (h->profiling) HIPCHK(h, prof_reserve(h, n + 1));
  HIPCHK(h, hipEventRecord(h->ev[0], st));
  cdz_status s;
  double res[8];
  // range check of the exact pass: flags res[5] (weak cell) and res[6]
  // (non-finite entry), read back into res
  int checks = 0;
  auto range_check = [&]() -> cdz_status {
    HIPCHK(h, hipMemsetAsync(D.res + 5, 0, 3 * sizeof(double), st));
    hipLaunchKernelGGL(cdz_spread_check<T>, dim3(n), dim3(CDZ_NT), 0, st, D);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipMemcpyAsync(res, D.res, sizeof(res), hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipStreamSynchronize(st));
    int deep = 0;
    memcpy(&deep, &res[7], sizeof(int));
    (checks++ == 0 ? h->weakest_first : h->weakest_final) = -deep;
    h->weakest_final = -deep;
    return CDZ_OK;
  };
  h->landscape_retries = 0;
  if (fp32) {
    // FP32: vertex factors rescaled to the free-energy landscape, estimated
    // from a pass truncated to short spans; then the exact pass, and once
    // more with the landscape of the exact pass if its cells still spread
    // too far (see cdz_landscape in cdz_fwd.hip)
    const int W = landscape_span(n, h->span);
    s = forward_pass<T>(h, D, shm, false, W);
    if (s != CDZ_OK) return s;
    hipLaunchKernelGGL(cdz_exterior_trunc<T>, dim3(1), dim3(64), 0, st, D, W);
    hipLaunchKernelGGL(cdz_landscape<T>, dim3(1), dim3(1024), 0, st, D);
    s = forward_pass<T>(h, D, shm, h->profiling, n);
    if (s != CDZ_OK) return s;
    if ((s = range_check()) != CDZ_OK) return s;
    if (res[5] != 0.0 && res[6] == 0.0) {
      h->landscape_retries = 1;
      hipLaunchKernelGGL(cdz_landscape<T>, dim3(1), dim3(1024), 0, st, D);
      s = forward_pass<T>(h, D, shm, false, n);
      if (s != CDZ_OK) return s;
      if ((s = range_check()) != CDZ_OK) return s;
    }
  } else {
    s = forward_pass<T>(h, D, shm, h->profiling, n);
    if (s != CDZ_OK) return s;
    if ((s = range_check()) != CDZ_OK) return s;
  }
  if (res[6] != 0.0)
    return cdz_fail(h, CDZ_ERR_NUMERIC, std::string("non-finite entries in the forward pass (") +
                                            (fp32 ? "FP32-scaled" : "FP64") + " range exceeded)");
  if (res[5] != 0.0)
    return cdz_fail(h, CDZ_ERR_NUMERIC, std::string("cells of the forward pass fell below 2^-") +
                                            std::to_string(D.lowExp) +
                                            (fp32 ? " after the landscape was repeated (FP32 range exceeded)"
                                                  : " (FP64 range exceeded)"));
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipEventRecord(h->ev[1], st));
  HIPCHK(h, hipMemcpyAsync(res, D.res, sizeof(res), hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipStreamSynchronize(st));
  float ms = 0;
  HIPCHK(h, hipEventElapsedTime(&ms, h->ev[0], h->ev[1]));
  h->times[0] = ms;
  if (!h->profiling && h->landscape_retries == 0) tune_end(h, tkey, ms);
  if (h->profiling) {
    double tot = 0;
    for (int dl = 0; dl < n; dl++) {
      float k = 0;
      HIPCHK(h, hipEventElapsedTime(&k, h->pev[2 * dl], h->pev[2 * dl + 1]));
      tot += k;
    }
    h->prof_fwd_ms = tot;
    h->prof_fwd_launches = n;
  }
  if (!std::isfinite(res[0]) || !std::isfinite(res[1]))
    return cdz_fail(h, CDZ_ERR_NUMERIC, "log Z not finite (scaling out of range)");
  const double L2 = 0.6931471805599453094;
  h->logz = res[0] + res[3] * L2;
  h->logz_suffix = res[1] + res[3] * L2;
  h->EZ = res[2];  // exponent of the scaled Z, used by the adjoint
  h->logz_scaled = res[0];
  return CDZ_OK;
}

template <typename T>
static cdz_status forward_impl(cdz_handle *h, const HostTables &t, bool adjoint) {
  DevProb<T> D;
  DevAdj<T> A;
  memset(&D, 0, sizeof(D));
  memset(&A, 0, sizeof(A));
  // A resident for all diagonals when the budget allows, else the
  // memory-bounded form (ring; checkpoints and a recomputed band when the
  // outside pass follows)
  int alK = CDZ_AL_RESIDENT;
  size_t need = carve<T>(nullptr, t, D, A, adjoint, alK);
  // block offsets inside one S x S array are kept in 32-bit integers
  if ((unsigned long long)D.ld * (unsigned long long)D.ld > 0x7fffffffull)
    return cdz_fail(h, CDZ_ERR_ARG, "sequence of " + std::to_string(t.n) + " nt is too long for 32-bit block offsets");
  if (h->al_k_forced >= CDZ_AL_RESIDENT) {
    alK = h->al_k_forced;
    if (adjoint && alK == 0) return cdz_fail(h, CDZ_ERR_ARG, "the outside pass needs checkpoints (K > 0)");
    need = carve<T>(nullptr, t, D, A, adjoint, alK);
  } else if (h->opt.mem_budget_bytes && need > h->opt.mem_budget_bytes) {
    alK = adjoint ? al_best_k(t.n) : 0;
    need = carve<T>(nullptr, t, D, A, adjoint, alK);
    if (need > h->opt.mem_budget_bytes)
      return cdz_fail(h, CDZ_ERR_BUDGET, "workspace of " + std::to_string(need) +
                                             " bytes (checkpointed minimum) exceeds the budget");
  }
  if (need > h->ws_bytes) {
    if (h->ws) HIPCHK(h, hipFree(h->ws));
    h->ws = nullptr;
    h->ws_bytes = 0;
    if (hipMalloc(&h->ws, need) != hipSuccess) {
      h->ws = nullptr;
      (void)hipGetLastError();
      return cdz_fail(h, CDZ_ERR_NOMEM, "hipMalloc of " + std::to_string(need) + " bytes failed");
    }
    h->ws_bytes = need;
  }
  carve<T>((char *)h->ws, t, D, A, adjoint, alK);
  D.lowExp = spread_low(h->low_exp, sizeof(T) == 4);
  h->al_k = alK;
  cdz_status s = upload<T>(h, t, D);
  if (s != CDZ_OK) return s;
  s = launch_forward<T>(h, D);
  if (s != CDZ_OK) return s;
  store_dev(h, D, A);
  return CDZ_OK;
}

cdz_status ensure_forward(cdz_handle *h, const HostTables &t, bool adjoint) {
  if (h->have_fwd && h->fwd_key == t.key && (!adjoint || h->fwd_adjoint)) return CDZ_OK;
  h->have_fwd = false;
  cdz_status s = h->opt.prec == CDZ_FP64 ? forward_impl<double>(h, t, adjoint)
                                         : forward_impl<float>(h, t, adjoint);
  if (s != CDZ_OK) return s;
  h->have_fwd = true;
  h->fwd_key = t.key;
  h->fwd_adjoint = adjoint;
  h->tables = t;
  return CDZ_OK;
}

extern "C" cdz_status cdz_partition(cdz_handle *h, const cdz_problem *prob, double *log_z) {
  if (!h || !prob || !log_z) return cdz_fail(h, CDZ_ERR_ARG, "null argument");
  HostTables t;
  cdz_status s = build_tables(h, prob->n_aa, prob->aa, prob->theta1, prob->theta2, t);
  if (s != CDZ_OK) return s;
  s = ensure_forward(h, t, false);
  if (s != CDZ_OK) return s;
  *log_z = h->logz;
  return CDZ_OK;
}

extern "C" cdz_status cdz_last_timings(cdz_handle *h, double *ms5) {
  if (!h || !ms5) return CDZ_ERR_ARG;
  for (int k = 0; k < 3; k++) ms5[k] = h->times[k];
  ms5[3] = h->prof_fwd_launches ? h->prof_fwd_ms / h->prof_fwd_launches : 0.0;
  ms5[4] = h->prof_fwd_launches;
  return CDZ_OK;
}

extern "C" cdz_status cdz_kernel_timings(cdz_handle *h, double *ms6) {
  if (!h || !ms6) return CDZ_ERR_ARG;
  ms6[0] = h->prof_fwd_ms;
  ms6[1] = h->prof_fwd_launches;
  ms6[2] = h->prof_out_ms;
  ms6[3] = h->prof_out_launches;
  ms6[4] = h->prof_eta_ms;
  ms6[5] = h->prof_smp_ms;
  return CDZ_OK;
}

extern "C" cdz_status cdz_set_profiling(cdz_handle *h, int on) {
  if (!h) return CDZ_ERR_ARG;
  h->profiling = on != 0;
  return CDZ_OK;
}

extern "C" cdz_status cdz_reset(cdz_handle *h) {
  if (!h) return CDZ_ERR_ARG;
  h->have_fwd = false;
  return CDZ_OK;
}

hipError_t prof_reserve(cdz_handle *h, int launches) {
  while ((int)h->pev.size() < 2 * launches) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    h->pev.push_back(e);
  }
  return hipSuccess;
}

// debug/test hook: log Z computed from the suffix exterior pass of the last forward
extern "C" double cdz_debug_logz_suffix(const cdz_handle *h) { return h ? h->logz_suffix : NAN; }
// storage of A in the last forward: -1 all diagonals resident, 0 ring only,
// K > 0 checkpointed with bands of K diagonals
extern "C" int cdz_debug_al_k(const cdz_handle *h) { return h ? h->al_k : -2; }
// span of the truncated pass of the FP32 landscape estimate, and the number of
// exact passes the last forward repeated because cells came too close to
// FP32 underflow
extern "C" int cdz_debug_set_span(cdz_handle *h, int W) {
  if (!h || (W != 0 && W < 4) || W > CDZ_SPAN_MAX) return CDZ_ERR_ARG;
  h->span = W;
  h->have_fwd = false;
  return CDZ_OK;
}
extern "C" int cdz_debug_landscape_retries(const cdz_handle *h) { return h ? h->landscape_retries : -1; }
extern "C" int cdz_debug_weakest(const cdz_handle *h, int *first, int *final_) {
  if (!h || !first || !final_) return CDZ_ERR_ARG;
  *first = h->weakest_first;
  *final_ = h->weakest_final;
  return CDZ_OK;
}
extern "C" int cdz_debug_set_low_exp(cdz_handle *h, int e) {
  if (!h || e < 0 || e > 1074) return CDZ_ERR_ARG;
  h->low_exp = e;
  h->have_fwd = false;
  return CDZ_OK;
}
extern "C" int cdz_debug_set_graphs(cdz_handle *h, int on) {
  if (!h) return CDZ_ERR_ARG;
  h->use_graphs = on != 0;
  return CDZ_OK;
}
extern "C" int cdz_debug_graph_counts(const cdz_handle *h, int *captures, int *replays) {
  if (!h || !captures || !replays) return CDZ_ERR_ARG;
  *captures = h->graph_captures;
  *replays = h->graph_replays;
  return CDZ_OK;
}
extern "C" int cdz_debug_set_fuse(cdz_handle *h, int wg) {
  if (!h || wg < -1) return CDZ_ERR_ARG;
  h->fuse_fixed = wg;
  return CDZ_OK;
}

namespace {
const int kFuseCand[3] = {1 << 30, 16384, 4096};
}
uint64_t tune_key(int pass, bool batch, size_t tsize, long long max_split_wg) {
  int b = 0;
  while (b < 62 && (2ll << b) <= max_split_wg) b++;
  return (uint64_t)pass | (uint64_t)batch << 1 | (uint64_t)(tsize == 8) << 2 | (uint64_t)b << 3;
}
int tune_begin(cdz_handle *h, uint64_t key) {
  if (h->fuse_fixed >= 0) return h->fuse_wg = h->fuse_fixed;
  const cdz_handle::Tune &t = h->tune[key];
  if (t.tried < 0) return h->fuse_wg = kFuseCand[0];
  if (t.tried < 3) return h->fuse_wg = kFuseCand[t.tried];
  int best = 0;
  for (int k = 1; k < 3; k++)
    if (t.ms[k] < t.ms[best]) best = k;
  return h->fuse_wg = kFuseCand[best];
}
void tune_end(cdz_handle *h, uint64_t key, float ms) {
  if (h->fuse_fixed >= 0) return;
  cdz_handle::Tune &t = h->tune[key];
  if (t.tried < 0) t.tried = 0;
  else if (t.tried < 3) t.ms[t.tried++] = ms;
}
// force that storage for the following forward passes (-2: chosen by budget)
extern "C" int cdz_debug_force_al_k(cdz_handle *h, int K) {
  if (!h || K < -2) return CDZ_ERR_ARG;
  h->al_k_forced = K;
  h->have_fwd = false;
  return CDZ_OK;
}
