// cdz_dev.h -- device-side problem description and helpers shared by the
// forward, outside and sampling kernels of the codon-constrained McCaskill
// dynamic program (gfx950 / CDNA4, wave64).
//
// Layout.  Position p (0 <= p < n) carries the codon slot of its residue,
// d[p] <= 6 values.  P[p] = sum_{q<p} d[q] flattens (position, slot) into a
// state index k in [0, S).  Every DP array is an S x S row-major matrix in
// HBM whose block (P[i].., P[j]..) of shape d[i] x d[j] holds the tensor of
// range [i..j] over the slots of its two end positions; this is the block
// layout of the paper's Fig. structures(b) with non-square blocks.  A row of
// blocks is contiguous along the contraction index of the O(n) split sums, so
// the lanes of a wavefront read consecutive addresses there.  Transposed
// copies exist where a split runs down a column.
//
// Scaling.  Every entry of diagonal dl = j - i is stored as true * 2^-E[dl]
// (one integer exponent per diagonal, chosen from the maxima of the two
// previous diagonals); adjoint entries are stored as true * 2^(E[dl] - EZ)
// with EZ = round(log2 Z).  All factors between diagonals are exact powers
// of two.  The exterior loop and log Z are accumulated in FP64 with their own
// per-position exponents.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define CDZ_NT 256      // threads per workgroup of the cell kernels
// threads per workgroup of the edge-marginal kernel (one edge): eight waves in
// FP32; four in FP64, whose registers would leave one eight-wave workgroup a CU
__host__ __device__ constexpr int cdz_eta_nt(int elt) { return elt == 4 ? 512 : 256; }
#define CDZ_MAXLOOP 30  // bulge / interior loop size bound
#define CDZ_NA 27      // interior-loop sizes L = 2..28 kept per cell (the recursion in
                       // L reads L - 2 <= 28; sizes 29, 30 only feed the cell itself)
#define CDZ_NWIN 496    // (l1, l2) pairs with l1 + l2 <= 30, including (0, 0)
#define CDZ_NRING 29    // interior-loop adjoints by size kept per cell by the outside pass (L = 2..30)

// Boltzmann table offsets inside DevProb::tab
#define TB_ST 0      // stack [6][6]
#define TB_BU 36     // bulge [31]
#define TB_IN 67     // interior [31]
#define TB_MM 98     // mismatch [4][4][6]
#define TB_MLAB 194  // exp(-(ml_a + ml_b))
#define TB_MLB 195   // exp(-ml_b)
#define TB_MLC 196   // exp(-ml_c)
#define TB_LEN 197

template <typename T>
struct DevProb {
  int n, m, S;
  long long ld;
  const int *d;            // [n]
  const int *P;            // [n + 1]
  const int *posOf;        // [S] position of state index k
  const signed char *nt;   // [n][6] base of position p in slot s, -1 beyond d
  const T *v;              // [n][6] vertex factors (exp(theta1) at middle bases)
  const T *e;              // [n][6][6] edge factor between p and p+1
  const double *vd, *ed;   // the same in FP64 (exterior loop)
  const T *tab;            // Boltzmann tables, TB_* offsets
  const T *Bhp;            // [n] hairpin factor by loop length L (mismatch excluded)
  // forward arrays, S x S each (see header comment)
  T *U, *Qb, *G, *F, *DI, *Qm1, *Qm1Lr, *Qm1Lt, *Qm1p, *QmX, *Qm, *Qmt;
  T *Ut, *DIt, *Qbt;       // U, DI and Qb transposed (their column strips read as rows)
  // interior-loop sums by loop size: A(i,j,L), L = 2..CDZ_NA+1, for the cell
  // (i,j) at rows P[i+1].. and columns CDZ_NA*P[j-1] + (L-2)*d[j-1] + ..
  T *AL;
  long long ldA;           // CDZ_NA * ld
  // Memory-bounded form (AL == nullptr): A is kept diagonal-major, a diagonal
  // being [n][CDZ_NA][36] (cell i at i * CDZ_NA * 36, blocks padded to 6 x 6)
  // in one of the slots ALs[nslot]; each launch is given the diagonal it
  // writes (ALw) and the diagonal dl - 2 it reads (ALp).  alK > 0: the outside
  // pass recomputes bands of alK diagonals from checkpoints (see cdz_host.hip).
  T *ALs, *ALw;
  const T *ALp;
  int alK, alTop, alSlots;
  int lowExp;              // range check: a cell whose largest entry is below 2^-lowExp
                           // (zero included) is too weak (FP32: the pass is repeated once)
  int *E;                  // [n + 1] diagonal exponents
  int *EX;                 // [n + 5] provisional exponents of the split sums (forward)
  unsigned *maxb;          // [n + 1] float bits of max |entry| per diagonal
  double *Z5;              // [n][6] prefix exterior partition function
  double *A5;              // [n][6] A[k] = Z5[k-1] e_{k-1} (prefix scan)
  int *G5;                 // [n]
  double *Z3;              // [n][6] suffix exterior partition function
  int *H3;                 // [n]
  int *Cl;                 // [n] landscape exponents C[p] (FP32 mode)
  double *res;             // [8] results: [0] log Z~ (prefix), [1] log Z~ (suffix), [2] EZ,
                           // [3] landscape exponent sum, [5] weak cell found, [6] non-finite
                           // entry found (range check flags)
};

__device__ __forceinline__ int cdz_ptype(int x, int y) {
  // nibble (4x + y) of this constant is the pair type, 15 = no pair:
  // AU=0 CG=1 GC=2 UA=3 GU=4 UG=5
  const unsigned long long PT = 0xF5F34F2FF1FF0FFFull;
  if (x < 0 || y < 0) return -1;
  int t = (int)((PT >> (4 * (x * 4 + y))) & 15ull);
  return t == 15 ? -1 : t;
}

// 2^e as a scale factor between diagonals.  Below the smallest subnormal the
// factor is 0 (the term is then below the precision of the cell it feeds,
// whose top sits near 2^0).  Above the largest finite power the factor is
// +inf, never a clamped value: the cell becomes non-finite, which the range
// check after the pass reports as CDZ_ERR_NUMERIC instead of a wrong sum.
template <typename T>
__device__ __forceinline__ T cdz_p2(int e);
template <>
__device__ __forceinline__ float cdz_p2<float>(int e) {
  if (e > 127) return __int_as_float(0x7f800000);
  return e < -149 ? 0.0f : ldexpf(1.0f, e);
}
template <>
__device__ __forceinline__ double cdz_p2<double>(int e) {
  if (e > 1023) return __longlong_as_double(0x7ff0000000000000ll);
  return e < -1074 ? 0.0 : ldexp(1.0, e);
}

// (l1, l2) of window index w: w enumerates l1 = 0..30, then l2 = 0..30-l1
__device__ __forceinline__ void cdz_win(int w, int &l1, int &l2) {
  int a = 0, base = 0;
  while (base + (31 - a) <= w) {
    base += 31 - a;
    a++;
  }
  l1 = a;
  l2 = w - base;
}

__device__ __forceinline__ float cdz_wave_max(float x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, 64));
  return x;
}

// Cells of one diagonal are assigned to workgroups so that each of the 8
// XCDs (workgroups are dealt to them in turn, each XCD has its own L2) runs
// a contiguous range of i: cells with nearby i read each other's rows and
// runs, which then tend to be in the same L2.  Blocks past the last cell exit.
#define CDZ_NXCD 8
// largest span of the truncated pass that estimates the FP32 landscape
#define CDZ_SPAN_MAX 512
__host__ __device__ __forceinline__ int cdz_cells_grid(int ncell) {
  return (ncell + CDZ_NXCD - 1) / CDZ_NXCD * CDZ_NXCD;
}
// 16-byte rounding of LDS region sizes
__host__ __device__ constexpr size_t lds_al(size_t b) { return (b + 15) / 16 * 16; }
// dynamic LDS of the exterior scans: exponents, slot counts, offsets and the
// running exponents of n + 1 positions, then FP64 reduction scratch and sums
#define CDZ_SCAN_NT 1024  // threads per workgroup of the exterior scans
__host__ __device__ constexpr size_t scan_lds_bytes(int n) {
  return lds_al((size_t)4 * (n + 1) * 4) + ((CDZ_SCAN_NT / 64) * 6 + 8) * sizeof(double);
}

// Workgroups of forward launch t (t = 0..n-1) of a sequence of n positions,
// in block order: window sums of diagonal t+1, bulge sums of diagonal t+1
// (both for 4 <= t+1 < n), split of diagonal t+4 (9 <= t+4 < n), finish of
// diagonal t.
__host__ __device__ __forceinline__ void fwd_ranges(int n, int t, int r[4]) {
  r[0] = t + 1 >= 4 && t + 1 < n ? cdz_cells_grid(n - t - 1) : 0;
  r[1] = r[0];
  r[2] = t + 4 >= 9 && t + 4 < n ? cdz_cells_grid(n - t - 4) : 0;
  r[3] = t < n ? cdz_cells_grid(n - t) : 0;
}
// Workgroups of the launch: one per piece of work (split), or, fused, one
// per cell index running every kind that has that block in turn (the kinds
// of a launch never read each other's results, so any order is the same)
__host__ __device__ __forceinline__ int fwd_nblocks(int n, int t, bool fused = false) {
  int r[4];
  fwd_ranges(n, t, r);
  if (fused) return max(max(r[0], r[1]), max(r[2], r[3]));
  return r[0] + r[1] + r[2] + r[3];
}
// Workgroups of outside launch t (t = n-1..0), in block order: interior-loop
// pushes of diagonal t+1 (8 <= t+1 < n), edge terms of the size recursion of
// diagonal t+1 (10 <= t+1 < n), bulge pushes of diagonal t+1 (7 <= t+1 < n),
// bulge gathers of diagonal t-1 (4 <= t-1 <= n-2), split gathers of diagonal
// t-4 (4 <= t-4 <= n-5), finish of diagonal t.
__host__ __device__ __forceinline__ void out_ranges(int n, int t, int r[6]) {
  const int a = t + 1, b = t - 1, c = t - 4;
  r[0] = a >= 8 && a <= n - 1 ? cdz_cells_grid(n - a) : 0;
  r[1] = a >= 10 && a <= n - 1 ? cdz_cells_grid(n - a) : 0;
  r[2] = a >= 7 && a <= n - 1 ? cdz_cells_grid(n - a) : 0;
  r[3] = b >= 4 && b <= n - 2 ? cdz_cells_grid(n - b) : 0;
  r[4] = c >= 4 && c <= n - 5 ? cdz_cells_grid(n - c) : 0;
  r[5] = t >= 0 && t <= n - 1 ? cdz_cells_grid(n - t) : 0;
}
__host__ __device__ __forceinline__ int out_nblocks(int n, int t, bool fused = false) {
  int r[6];
  out_ranges(n, t, r);
  if (fused) return max(max(max(r[0], r[1]), max(r[2], r[3])), max(r[4], r[5]));
  return r[0] + r[1] + r[2] + r[3] + r[4] + r[5];
}
__device__ __forceinline__ int cdz_cell_of_block(int w, int ncell) {
  return (w % CDZ_NXCD) * ((ncell + CDZ_NXCD - 1) / CDZ_NXCD) + w / CDZ_NXCD;
}

// ---- wave-uniform helpers ---------------------------------------------------
__device__ __forceinline__ int cdz_uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
template <typename T>
__device__ __forceinline__ const T *cdz_uni(const T *p) {
  const unsigned long long u = (unsigned long long)p;
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
  return reinterpret_cast<const T *>(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ int cdz_wave_id() { return cdz_uni((int)(threadIdx.x >> 6)); }
// orders the LDS accesses of the lanes of one wavefront (reads of a block by
// some lanes before writes to it by others); LDS serves a wave in order, so
// this only has to stop the compiler from moving them
__device__ __forceinline__ void cdz_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
}

// Batched launches: off[0..count] are prefix sums of the workgroups of each
// problem (off[0] = 0).  Workgroup blk belongs to the largest b with
// off[b] <= blk (problems without workgroups are skipped), as its w-th block.
__device__ __forceinline__ void cdz_batch_locate(const int *off, int count, int blk, int &b, int &w) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= blk) lo = mid;
    else hi = mid - 1;
  }
  b = cdz_uni(lo);
  w = cdz_uni(blk - off[lo]);
}

// Workgroup barrier that orders LDS accesses only: global stores issued
// before it are not drained (a plain __syncthreads waits for every
// outstanding store).  Use __syncthreads where global data written by one
// thread is read by another thread of the workgroup.
__device__ __forceinline__ void cdz_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Maps from a state offset to the position index of the loop window of cell
// (i, j): mapL[k] = q for the states of position i+1+q (q = 0..lmax, offsets
// from lp_P[0]); mapR[k] = q for the states of position j-1-q (q = 0..lmax,
// offsets from rp_P[lmax]).  lp_* / rp_* hold d and P of those positions.
// Threads 0..30 and 32..62 write; the caller synchronises before reading.
__device__ __forceinline__ void cdz_window_maps(unsigned char *mapL, unsigned char *mapR, const int *lp_d,
                                                const int *lp_P, const int *rp_d, const int *rp_P, int lmax) {
  const int tid = threadIdx.x;
  if (tid < 31) {
    if (tid <= lmax)
      for (int c = 0; c < lp_d[tid]; c++) mapL[lp_P[tid] - lp_P[0] + c] = (unsigned char)tid;
  } else if (tid >= 32 && tid < 63) {
    const int q = tid - 32;
    if (q <= lmax)
      for (int c = 0; c < rp_d[q]; c++) mapR[rp_P[q] - rp_P[lmax] + c] = (unsigned char)q;
  }
}

// Copy nblk consecutive 36-value blocks (nblk <= 30) from global src to LDS
// dst, in order or with the block order reversed; every thread issues all of
// its loads before its first store.
template <typename T>
__device__ __forceinline__ void cdz_copy_blocks(T *dst, const T *src, int nblk, bool rev) {
  constexpr int NV = (30 * 36 + CDZ_NT - 1) / CDZ_NT;
  const int count = nblk * 36;
  T v[NV];
#pragma unroll
  for (int k = 0; k < NV; k++) {
    const int f = (int)threadIdx.x + k * CDZ_NT;
    v[k] = f < count ? src[f] : T(0);
  }
#pragma unroll
  for (int k = 0; k < NV; k++) {
    const int f = (int)threadIdx.x + k * CDZ_NT;
    if (f < count) {
      const int b = f / 36;
      dst[(rev ? nblk - 1 - b : b) * 36 + f % 36] = v[k];
    }
  }
}

// Exponents of the diagonals a cell's statements read, into sE at their own
// indices: E[0..31] (short spans: loops of up to 30 unpaired bases) and
// E[c-w .. c+w] (around the cell's diagonal c), both below m; other entries
// of sE are not written.
__device__ __forceinline__ void cdz_copy_exponents(int *sE, const int *E, int m, int c, int w) {
  const int lo = m < 32 ? m : 32;
  const int a = c - w > lo ? c - w : lo, b = c + w + 1 < m ? c + w + 1 : m;
  for (int k = threadIdx.x; k < lo; k += CDZ_NT) sE[k] = E[k];
  for (int k = a + (int)threadIdx.x; k < b; k += CDZ_NT) sE[k] = E[k];
}

// Copy count ints from global src to LDS dst (both 16-byte aligned) with
// 16-byte loads, up to 4 of them in flight per thread.
__device__ __forceinline__ void cdz_copy_ints(int *dst, const int *src, int count) {
  const int n4 = count / 4;
  const int4 *s4 = reinterpret_cast<const int4 *>(src);
  int4 *d4 = reinterpret_cast<int4 *>(dst);
  for (int base = 0; base < n4; base += 4 * CDZ_NT) {
    int4 v[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int f = base + (int)threadIdx.x + k * CDZ_NT;
      v[k] = f < n4 ? s4[f] : make_int4(0, 0, 0, 0);
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int f = base + (int)threadIdx.x + k * CDZ_NT;
      if (f < n4) d4[f] = v[k];
    }
  }
  for (int f = 4 * n4 + (int)threadIdx.x; f < count; f += CDZ_NT) dst[f] = src[f];
}

// Stage count LDS entries: loc(f, d) returns the global address of entry f
// (nullptr: the entry is zero) and sets its index d in dst.  Each thread
// issues NV loads before its stores, so their latencies overlap.
template <int NV, typename T, typename L>
__device__ __forceinline__ void cdz_stage_nv(T *dst, int count, L loc) {
  for (int base = 0; base < count; base += NV * CDZ_NT) {
    T v[NV];
    int di[NV];
#pragma unroll
    for (int k = 0; k < NV; k++) {
      const int f = base + (int)threadIdx.x + k * CDZ_NT;
      const T *p = nullptr;
      di[k] = -1;
      if (f < count) p = loc(f, di[k]);
      v[k] = p ? *p : T(0);
    }
#pragma unroll
    for (int k = 0; k < NV; k++)
      if (di[k] >= 0) dst[di[k]] = v[k];
  }
}

// Zero nblk 36-value blocks at dst (16-byte aligned), 16 bytes a store.
template <typename T>
__device__ __forceinline__ void cdz_zero_blocks(T *dst, int nblk) {
  uint4 *w4 = reinterpret_cast<uint4 *>(dst);
  const int n4 = nblk * 36 * (int)sizeof(T) / 16;
  for (int f = threadIdx.x; f < n4; f += CDZ_NT) w4[f] = make_uint4(0, 0, 0, 0);
}

// ---- workgroup sums by a reduce-scatter butterfly inside each wavefront.
// At level k (k = 5..0) every lane pairs with a partner that differs in lane
// bit k and agrees in the higher bits; the lane with bit k = 0 keeps the
// first half of its values, the partner the second half, and each adds the
// partner's copy of the half it keeps.  After six levels a lane holds
// ceil(R / 64) sums (or none), so R sums cost about R exchanges instead of
// 6R.  Bits 5 and 4 exchange with v_permlane32_swap / v_permlane16_swap,
// bits 3..0 with DPP moves (row_ror:8, row_half_mirror, two quad perms);
// all of them are VALU operations with no LDS round trip.
__device__ __forceinline__ void cdz_swap_words(unsigned &a, unsigned &b, int level) {
  if (level == 5) {
    auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
    a = r[0];
    b = r[1];
  } else {
    auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
    a = r[0];
    b = r[1];
  }
}
__device__ __forceinline__ void cdz_swap(float &a, float &b, int level) {
  unsigned x = __float_as_uint(a), y = __float_as_uint(b);
  cdz_swap_words(x, y, level);
  a = __uint_as_float(x);
  b = __uint_as_float(y);
}
__device__ __forceinline__ void cdz_swap(double &a, double &b, int level) {
  unsigned long long x = (unsigned long long)__double_as_longlong(a), y = (unsigned long long)__double_as_longlong(b);
  unsigned xl = (unsigned)x, xh = (unsigned)(x >> 32), yl = (unsigned)y, yh = (unsigned)(y >> 32);
  cdz_swap_words(xl, yl, level);
  cdz_swap_words(xh, yh, level);
  a = __longlong_as_double((long long)(((unsigned long long)xh << 32) | xl));
  b = __longlong_as_double((long long)(((unsigned long long)yh << 32) | yl));
}
template <int CTRL>
__device__ __forceinline__ float cdz_dpp(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double cdz_dpp(double x) {
  const long long u = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(u & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
// level 5 / 4: pair sums through the permlane swaps
template <int LEVEL, typename T, int N>
__device__ __forceinline__ void cdz_rs_swap(const T (&v)[N], T (&o)[(N + 1) / 2]) {
  constexpr int H = (N + 1) / 2;
#pragma unroll
  for (int q = 0; q < H; q++) {
    T a = v[q], b = H + q < N ? v[H + q] : T(0);
    cdz_swap(a, b, LEVEL);
    o[q] = a + b;
  }
}
// levels 3..0: explicit send / keep through one DPP move per value
template <int CTRL, typename T, int N>
__device__ __forceinline__ void cdz_rs_dpp(const T (&v)[N], T (&o)[(N + 1) / 2], bool bit) {
  constexpr int H = (N + 1) / 2;
#pragma unroll
  for (int q = 0; q < H; q++) {
    const T lo = v[q], hi = H + q < N ? v[H + q] : T(0);
    const T recv = cdz_dpp<CTRL>(bit ? lo : hi);
    o[q] = (bit ? hi : lo) + recv;
  }
}

// Sum R per-thread values over the workgroup of NT threads; result in
// out[0..R) (LDS), visible to all threads after the call.  scratch holds
// (NT/64) * R values.  GLOBAL makes the first barrier a full one, so that
// global stores issued before the call are visible to the workgroup after it.
template <typename T, int R, int NT = CDZ_NT, bool GLOBAL = false>
__device__ __forceinline__ void cdz_block_sum(T (&v)[R], T *scratch, T *out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr int N1 = (R + 1) / 2, N2 = (N1 + 1) / 2, N3 = (N2 + 1) / 2, N4 = (N3 + 1) / 2,
                N5 = (N4 + 1) / 2, N6 = (N5 + 1) / 2;
  T a1[N1], a2[N2], a3[N3], a4[N4], a5[N5], a6[N6];
  cdz_rs_swap<5>(v, a1);
  cdz_rs_swap<4>(a1, a2);
  cdz_rs_dpp<0x128>(a2, a3, (lane >> 3) & 1);  // row_ror:8
  cdz_rs_dpp<0x141>(a3, a4, (lane >> 2) & 1);  // row_half_mirror
  cdz_rs_dpp<0x1B>(a4, a5, (lane >> 1) & 1);   // quad_perm 3,2,1,0
  cdz_rs_dpp<0xB1>(a5, a6, lane & 1);          // quad_perm 1,0,3,2
  // which sums this lane holds: positions base .. base + cnt - 1
  int base = 0, cnt = R, N = R;
#pragma unroll
  for (int k = 5; k >= 0; k--) {
    const int H = (N + 1) / 2;
    if ((lane >> k) & 1) {
      base += H;
      cnt = cnt - H > 0 ? cnt - H : 0;
    } else {
      cnt = cnt < H ? cnt : H;
    }
    N = H;
  }
#pragma unroll
  for (int q = 0; q < N6; q++)
    if (q < cnt) scratch[wv * R + base + q] = a6[q];
  if constexpr (GLOBAL)
    __syncthreads();
  else
    cdz_sync();
  for (int r = threadIdx.x; r < R; r += NT) {
    T s = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; w++) s += scratch[w * R + r];
    out[r] = s;
  }
  cdz_sync();
}
