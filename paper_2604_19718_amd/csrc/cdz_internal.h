// cdz_internal.h -- host-side state shared by the translation units of the
// library (handle, per-problem tables, adjoint workspace description).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "cdz.h"
#include "cdz_dev.h"

// alK of carve: the interior-loop sums A of every diagonal stay resident
#define CDZ_AL_RESIDENT (-1)
// span of the truncated pass that estimates the FP32 landscape: n / 40,
// within [16, 96] (measured: no repeated pass at 300-1200 nt from span 16 up,
// none at 3900 nt with 96), never beyond n - 1; a fixed span when set > 0
#define CDZ_LANDSCAPE_SPAN 96
inline int landscape_span(int n, int fixed) {
  int W = fixed > 0 ? fixed : n / 40;
  if (fixed <= 0) W = W < 16 ? 16 : W > CDZ_LANDSCAPE_SPAN ? CDZ_LANDSCAPE_SPAN : W;
  return W < n - 1 ? W : n - 1;
}
// Range check after the exact pass.  FP32: the pass is repeated once with its
// own landscape when the largest entry of some cell falls below
// 2^-CDZ_SPREAD_LOW (the top of the diagonal sits near 2^0), i.e. within 6
// octaves of the smallest normal float; still weak after that, or any entry
// not finite, the call returns CDZ_ERR_NUMERIC.  FP64 has no landscape: a
// cell below 2^-CDZ_SPREAD_LOW_FP64 or a non-finite entry is an error.
#define CDZ_SPREAD_LOW 120
#define CDZ_SPREAD_LOW_FP64 1020
inline int spread_low(int set, bool fp32) { return set > 0 ? set : fp32 ? CDZ_SPREAD_LOW : CDZ_SPREAD_LOW_FP64; }

// Per-problem host tables (FP64), built before any device work.
struct HostTables {
  int m = 0, n = 0, S = 0;
  std::string aa;
  std::vector<int> d, P, posOf;
  std::vector<signed char> nt;  // [n][6]
  std::vector<double> v, e;     // [n][6], [n][6][6]
  std::vector<double> tab, Bhp;
  uint64_t key = 0;
};

// Adjoint (outside) workspace, S x S arrays in the same block layout.
//   Qbb, Qm1b, Qm1pb, QmXb, Qmb : adjoints of the forward arrays
//   QmXbt                       : QmXb transposed (column gathers)
//   DIb                         : adjoint of DI (block of the inner pair's neighbours)
//   Gb, Fb                      : outer-edge-dressed adjoints of a cell's loop sums,
//                                 at block (i+1, j-1) of the closing pair (i, j)
//   Qm1Lb                       : adjoint of Qm1L (block (i-1, j))
//   UbL, UbR                    : run adjoints pushed by enclosing loops, by
//                                 row (left runs, hairpins) and by column
//                                 (right runs), so no two cells of one
//                                 diagonal write the same element; UbR is
//                                 stored transposed, so that the column a
//                                 cell pushes along is a contiguous row
//   Ub                          : total adjoint of the unpaired runs
template <typename T>
struct DevAdj {
  T *Qbb, *Qm1b, *Qm1pb, *QmXb, *QmXbt, *Qmb, *Qm1Lb, *DIb, *Gb, *Fb, *Ub, *UbL, *UbR;
  T *UbL2, *UbR2;  // run adjoints pushed by bulges (by row, and by column stored transposed)
  T *DIbL, *DIbR;  // DI adjoint pushed along row i+1 / column j-1 of the enclosing cells (DIbR transposed)
  T *ring;         // [3][n][CDZ_NRING][36] interior-loop adjoints by size, last three diagonals
  double *etaV, *etaW;  // [n][36] edge-marginal terms of the size recursion
  double *eta;   // [n][6][6] edge marginals times Z / 2^EZ
  double *pair;  // [n][n] pair probabilities (upper triangle)
  double *out;   // [16] scalars
};

template <typename T>
void adj_carve(size_t &off, char *base, const HostTables &t, DevAdj<T> &A, size_t S2);

struct cdz_handle {
  cdz_energy en;
  cdz_options opt;
  hipStream_t stream = nullptr;
  int device = 0;
  int lds_max = 65536;  // dynamic LDS a workgroup may use on this device
  int landscape_retries = 0;  // FP32: exact passes repeated for range (last forward)
  int al_k = CDZ_AL_RESIDENT;  // storage of A chosen for the last forward (see carve)
  int al_k_forced = -2;        // test hook: storage of A to use regardless of budget (-2: by budget)
  int span = 0;                   // fixed span of the truncated landscape pass (0: by length)
  int low_exp = 0;                // range-check threshold exponent (0: by precision, spread_low)
  int weakest_first = 0, weakest_final = 0;  // binary exponent of the weakest cell: first and last range check
  std::string err;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  void *smp = nullptr;  // sampler workspace (stacks, group sums, outputs)
  size_t smp_bytes = 0;
  void *bws = nullptr;  // batched calls: problem descriptors and launch offset tables
  size_t bws_bytes = 0;
  // captured launch sequences of batch chunks (hipGraph), keyed by the
  // descriptor image and phase they were captured for; replayed when a key
  // recurs (the image holds every device pointer and launch table, so equal
  // keys mean identical launches)
  struct Graph {
    std::string key;
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
  };
  std::vector<Graph> graphs;
  hipStream_t cap_stream = nullptr;  // stream the sequences are captured on (never run)
  bool use_graphs = true;
  // launch grouping: a diagonal launch whose pieces of work would take at
  // least fuse_wg workgroups runs fused (one workgroup per cell index doing
  // every kind in turn) instead of one workgroup per piece.  fuse_wg is set
  // per pass: the caller's fixed threshold (fuse_fixed >= 0), or the choice
  // of the tuner for the pass's class (tune_begin / tune_end)
  int fuse_wg = 1 << 30;
  int fuse_fixed = -1;
  struct Tune {
    int tried = -1;  // -1: the first (warm-up) pass is not timed
    float ms[3] = {0, 0, 0};
  };
  std::map<uint64_t, Tune> tune;
  int graph_captures = 0, graph_replays = 0;  // of the last batched call
  hipEvent_t ev[8] = {};
  double times[5] = {0, 0, 0, 0, 0};
  // per-launch event timing of the diagonal kernels (cdz_set_profiling)
  bool profiling = false;
  std::vector<hipEvent_t> pev;
  double prof_fwd_ms = 0, prof_out_ms = 0, prof_eta_ms = 0, prof_smp_ms = 0;
  int prof_fwd_launches = 0, prof_out_launches = 0;
  // last forward pass
  bool have_fwd = false, fwd_adjoint = false;
  uint64_t fwd_key = 0;
  double logz = 0, logz_suffix = 0, EZ = 0;
  double logz_scaled = 0;  // log of the partition function of the scaled tables
  HostTables tables;
  DevProb<float> pf;
  DevProb<double> pd;
  DevAdj<float> af;
  DevAdj<double> ad;
};

inline void store_dev(cdz_handle *h, const DevProb<float> &D, const DevAdj<float> &A) {
  h->pf = D;
  h->af = A;
}
inline void store_dev(cdz_handle *h, const DevProb<double> &D, const DevAdj<double> &A) {
  h->pd = D;
  h->ad = A;
}

template <typename T>
size_t fwd_lds_bytes(int n);  // dynamic LDS of the forward diagonal kernel
template <typename T>
size_t out_lds_bytes(int n);  // dynamic LDS of the outside diagonal kernel
size_t eta_lds_bytes(int n, int elt);  // dynamic LDS of the edge-marginal kernel (elt = sizeof(T))
// loop sizes of a cell's bulge adjoints staged per round in the edge-marginal
// kernel of an n-nt protein (elt = sizeof(T)): 15 in FP32; in FP64 10 while
// three workgroups still fit a CU (n <= 1100), else 4, so that two do up to
// 3900 nt
__host__ __device__ inline int eta_bulge_chunk(int n, int elt) { return elt == 4 ? 15 : n <= 1100 ? 10 : 4; }

// Storage of the interior-loop sums A (alK of carve):
//   CDZ_AL_RESIDENT (-1): every diagonal in D.AL (block layout)
//   0                   : diagonal-major ring of 3 diagonals (forward only)
//   K > 0               : ring, plus checkpoints of diagonals kK-2, kK-1
//                         (k = 1..top) and a band of K diagonals that the
//                         outside pass recomputes from them
inline int al_top(int K, int n) { return K > 0 && n > 3 ? (n - 3) / K : 0; }
inline int al_slots(int K, int n) { return K > 0 ? 3 + 2 * al_top(K, n) + K : 3; }
// slot holding diagonal x in the forward passes
inline int al_slot_fwd(int K, int top, int x) {
  if (K > 0 && x + 2 >= K) {
    const int k = (x + 2) / K, r = (x + 2) % K;
    if (r < 2 && k <= top) return 3 + 2 * (k - 1) + r;
  }
  return x % 3;
}
// slot holding diagonal x while the outside pass recomputes its band
inline int al_slot_band(int K, int top, int x) { return 3 + 2 * top + x % K; }
template <typename T>
T *al_slot_ptr(const DevProb<T> &D, int slot) {
  return D.ALs + (size_t)slot * D.n * CDZ_NA * 36;
}
// band length with the fewest slots for a sequence of n positions
int al_best_k(int n);

// workspace carve (base == nullptr: only the size) and table upload of one problem
template <typename T>
size_t carve(char *base, const HostTables &t, DevProb<T> &D, DevAdj<T> &A, bool adjoint, int alK);
template <typename T>
cdz_status upload(cdz_handle *h, const HostTables &t, DevProb<T> &D);
// marginal outputs of one problem from its device edge marginals and pair
// probabilities (r = 2^EZ / Z~); any output may be NULL
cdz_status assemble_marginals(cdz_handle *h, const HostTables &t, const double *eta_dev, const double *pair_dev,
                              double r, double *pair, double *base, double *codon, double *codon_pair);

// N samples of each problem of a batch (problem b with seed + b)
template <typename T>
cdz_status sample_batch(cdz_handle *h, const std::vector<DevProb<T>> &Ds, uint64_t seed, int N, uint8_t *codons,
                        int32_t *pairs);

cdz_status cdz_fail(cdz_handle *h, cdz_status s, const std::string &msg);

// Scratch of cdz_sample_noalloc: a file-scope device array of
// CDZ_NOALLOC_SCRATCH_BYTES in cdz_sample.hip.  noalloc_scratch(dev) returns
// its device address on device dev (resolved once per device with dev
// current, by cdz_create), or nullptr if the address cannot be obtained.
#define CDZ_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
void *noalloc_scratch(int device);

// return CDZ_ERR_HIP from the enclosing function when a HIP call fails
#define HIPCHK(h, x)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (x);                                                                      \
    if (e_ != hipSuccess)                                                                     \
      return cdz_fail((h), CDZ_ERR_HIP, std::string(#x " failed: ") + hipGetErrorString(e_)); \
  } while (0)

cdz_status build_tables(cdz_handle *h, int32_t n_aa, const char *aa, const double *theta1,
                        const double *theta2, HostTables &t);
// Launch-grouping tuner.  A class of passes is (forward or outside, single
// problem or batch, precision, log2 of the largest launch's workgroup count
// when split).  Its first pass runs split and is not timed; the next three
// run with the candidate thresholds (never fused, fused from 16384 and from
// 4096 workgroups) and are timed; later passes use the fastest.  Results do
// not depend on the choice.
uint64_t tune_key(int pass, bool batch, size_t tsize, long long max_split_wg);
int tune_begin(cdz_handle *h, uint64_t key);  // threshold for this pass (also set in fuse_wg)
void tune_end(cdz_handle *h, uint64_t key, float ms);
cdz_status ensure_forward(cdz_handle *h, const HostTables &t, bool adjoint);
hipError_t prof_reserve(cdz_handle *h, int launches);
