// cdz_tensor.hip -- sequence-summed free energy of a tensor-based structure
// model (Sections 3b-3c; SI S2b-S2c; Alg. fast-pf of SI S4a).
//
// Q is one dense row-major matrix of the flattened blocks: position p owns
// gamma * Sigma_p consecutive rows and columns starting at off[p] (sigma-major,
// then zeta).  Upper blocks Q_{i,j} (i < j) hold the scaled open-loop sums,
// diagonal blocks the identity, and row block j, left of the diagonal, the
// fold of column j transposed: row off[j] + c, column off[k] + r holds entry
// (r, c) of E_{k,j}, the element spanning [k, j) (the lower triangle of
// eq. dp-short).  Both operands of the propagation are therefore read along
// contiguous rows.
//
// Column j takes two launches:
//   tz_fold (j)  one workgroup per k < j: finishes column j-1 (sums the split-K
//                partials, divides by the column's power of two, writes the
//                blocks back) and builds E_{k,j} -- a pair (k, j-1) folds the
//                block Q_{k+1,j-1} it has just finished (eq. design-fold), the
//                last element is the unpaired base, elements of two or three
//                bases are zero.
//   tz_prop (j)  Y_{[0:j), j} = sum_k Q_{[0:j), k} E_{k,j} on the matrix cores
//                (v_mfma 16x16x4, FP32 or FP64): one workgroup per 64 rows and
//                chunk of k (256 to 2048 wide by column length), its eight
//                waves on eighths of it, summed through LDS in a fixed tree;
//                triangular (a tile starts at the first block its rows own);
//                one partial sum per chunk to a side buffer.
// Scaling: column j is divided by h_{j-1} = 2^e, e the binary exponent of the
// sum over its k chunks of each chunk's largest partial in the row-0 block (at
// least the block's largest entry, at most the chunk count times it), so the
// prefix block stays within a few octaves below 1;
// E_{k,j} of a pair is divided by h_k (the inner block carries the factors of
// k+1 .. j-2 only).  log Z = log Tr[S Q_{0,n}] + ln 2 * sum of the exponents,
// and at each codon boundary j = 3a the same gives log Z of the first a
// residues.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "cdz_internal.h"
#include "cdz_tensor.h"

hipError_t prof_reserve(cdz_handle *h, int launches);

namespace {

// k chunk of one propagation workgroup, chosen per column: the smallest of
// these giving at most TZ_MAXCH chunks (the longest otherwise), so short
// columns get short wave chains and long ones few partial sums
constexpr int TZ_NKC = 4;
constexpr int TZ_KCS[TZ_NKC] = {256, 512, 1024, 2048};
constexpr int TZ_MAXCH = 16;
constexpr int TZ_GRIDCH = 32;  // most chunks a column may have (N <= 32 * 2048 rows)

// the workgroup count of each chunk of one column, passed by value so that
// a workgroup finds its (tile, chunk) without dependent memory loads
struct TzGrid {
  int cnt[TZ_GRIDCH];
};
constexpr int TZ_PW = 8;          // waves of one propagation workgroup
constexpr int TZ_TM = 64;    // rows of one propagation tile (four 16-row MFMA tiles)
constexpr int TZ_WMAX = 64;  // widest column block gamma * Sigma (gamma <= 16, Sigma <= 4)
constexpr int TZ_FT = 256;   // fold workgroup: one item (block row / element)

template <typename T>
struct Mf;
template <>
struct Mf<float> {
  typedef float acc_t __attribute__((ext_vector_type(4)));
  typedef float ld_t __attribute__((ext_vector_type(4)));
  static constexpr int VEC = 4;  // k values per 16-byte load
  static __device__ inline acc_t mac(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of output element v of a lane in k-group q
  static __device__ inline int drow(int q, int v) { return 4 * q + v; }
};
template <>
struct Mf<double> {
  typedef double acc_t __attribute__((ext_vector_type(4)));
  typedef double ld_t __attribute__((ext_vector_type(2)));
  static constexpr int VEC = 2;
  static __device__ inline acc_t mac(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int drow(int q, int v) { return q + 4 * v; }
};

template <typename T>
struct TzDev {
  int n, g, xi;
  int ld;                       // row stride of Q (elements)
  int prow;                     // rows of one chunk of P
  const int *sig;               // [n+1] train dimensions
  const int *off;               // [n+1] first row/column of each position
  const int *rstart;            // [rows] off[] of the position owning the row
  const int *tile_kmin;         // [tiles] rstart of the tile's first row
  const unsigned char *bmask;   // [n] bit phi set if core p is nonzero for base phi
  const T *tc;                  // [n][4][4][4] train cores: p, base, sigma_a, sigma_b
  const T *V;                   // [4][g][g]
  const T *B;                   // [xi][4][4][g][g]
  const T *SB;                  // [xi][4][4][g][g]: S B[rho][x][y]
  const T *S;                   // [g][g]
  unsigned pairmask;            // bit 4x+y: B[rho][x][y] nonzero for some rho
  T *Q;                         // [rows][ld]
  T *P;                         // [chunks][prow][TZ_WMAX] split-K partial sums
  int *colexp;                  // [n+1] exponent of each column's factor
  T *pmax;                      // [n+1][TZ_GRIDCH] largest partial of each chunk in the column's row-0 block
  double *ptr;                  // [m] Tr[S Q_{0,3a}] (scaled) at codon boundaries
};

// sum of the partials of row r, column col of the last propagated column
template <typename T>
__device__ inline T col_sum(const TzDev<T> &D, int r, int col, int nchunks, int kc) {
  const int cf = D.tile_kmin[r / TZ_TM] / kc;
  T y = T(0);
  const T *p = D.P + (size_t)r * TZ_WMAX + col;
  const size_t cs = (size_t)D.prow * TZ_WMAX;
  for (int c0 = cf; c0 < nchunks; c0 += 8) {  // eight loads in flight, added in chunk order
    T v[8];
#pragma unroll
    for (int u = 0; u < 8; u++) v[u] = c0 + u < nchunks ? p[(c0 + u) * cs] : T(0);
#pragma unroll
    for (int u = 0; u < 8; u++) y += v[u];
  }
  return y;
}

// the same for four entries at once (rows r[u], columns col[u], skipped where
// ok[u] is false): up to 32 loads in flight, each sum in chunk order
template <typename T>
__device__ inline void col_sum4(const TzDev<T> &D, const int *r, const int *col, const bool *ok, int nchunks, int kc,
                                T *y) {
  const size_t cs = (size_t)D.prow * TZ_WMAX;
  int cf[4], cmin = nchunks;
  const T *p[4];
#pragma unroll
  for (int u = 0; u < 4; u++) {
    cf[u] = ok[u] ? D.tile_kmin[r[u] / TZ_TM] / kc : nchunks;
    cmin = min(cmin, cf[u]);
    p[u] = D.P + (size_t)(ok[u] ? r[u] : 0) * TZ_WMAX + (ok[u] ? col[u] : 0);
    y[u] = T(0);
  }
  for (int c0 = cmin; c0 < nchunks; c0 += 8) {
    T v[4][8];
#pragma unroll
    for (int u = 0; u < 4; u++)
#pragma unroll
      for (int x = 0; x < 8; x++) v[u][x] = (c0 + x >= cf[u] && c0 + x < nchunks) ? p[u][(c0 + x) * cs] : T(0);
#pragma unroll
    for (int u = 0; u < 4; u++)
#pragma unroll
      for (int x = 0; x < 8; x++) y[u] += v[u][x];
  }
}

__device__ inline int exp_of(double x) {
  int e;
  (void)frexp(x, &e);
  return e - 1;  // x in [2^(e-1), 2^e)
}

template <typename T>
__device__ inline T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
template <typename T>
__device__ inline T wave_max(T v) {
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

// exponent of column jc's factor: binary exponent of the largest entry of its
// row-0 block (rows 0..g-1), summed from the partials (one wave)
template <typename T>
__device__ inline int column_exponent(const TzDev<T> &D, int jc, int nchunks, int kc) {
  const int w = D.g * D.sig[jc];
  T mx = T(0);
  for (int e0 = threadIdx.x & 63; e0 < D.g * w; e0 += 256) {
    int r[4], cc[4];
    bool ok[4];
    T y[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int e = e0 + 64 * u;
      ok[u] = e < D.g * w;
      r[u] = e / w;
      cc[u] = e % w;
    }
    col_sum4(D, r, cc, ok, nchunks, kc, y);
#pragma unroll
    for (int u = 0; u < 4; u++) mx = max(mx, y[u]);
  }
  mx = wave_max(mx);
  return exp_of((double)mx);
}

// ---- propagation: Y_{[0:j), j} on the matrix cores ----------------------
// Lane layout of v_mfma_*_16x16x4 (one block): A row i, k-group q at lane
// i + 16q; B column c, k-group q at lane c + 16q; output column c at lane
// c + 16q, element v holding row 4q + v (f32) or q + 4v (f64).  Each lane loads VEC consecutive k of its row
// (16 bytes) and feeds them to VEC successive instructions, so instruction s
// multiplies k = k0 + VEC q + s for q = 0..3 -- the same set for A and B.
template <typename T, int NTM>
__global__ __launch_bounds__(512, (sizeof(T) == 4 && NTM == 3) ? 4 : 2) void tz_prop(TzDev<T> D, int j, int ntiles, int nchunks,
                                                                                  int kc, TzGrid G) {
  using M = Mf<T>;
  constexpr int VEC = M::VEC, KS = 4 * VEC;
  int b = blockIdx.x, c = 0;
  for (; c < nchunks - 1; c++) {  // chunk-major: chunk c holds the tiles that reach it
    const int cnt = G.cnt[c];
    if (b < cnt) break;
    b -= cnt;
  }
  const int t = b;
  const int R = D.off[j], w = D.g * D.sig[j], ntn = (w + 15) >> 4;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, q = lane >> 4;
  const int r0 = t * TZ_TM;
  const int kw = kc / TZ_PW;  // k range of each wave
  const int kb = max(c * kc + wave * kw, D.tile_kmin[t]) & ~(KS - 1);
  const int ke = min(c * kc + (wave + 1) * kw, R);
  int kst[4];
  // one row pointer per lane for A and one for B; the other row tiles sit a
  // uniform 16 rows further on
  const size_t s16 = (size_t)16 * D.ld;
  const T *arow0 = D.Q + (size_t)(r0 + li) * D.ld;
  const T *brow0 = D.Q + (size_t)(R + li) * D.ld;
#pragma unroll
  for (int m = 0; m < 4; m++) {
    const int row = r0 + 16 * m + li;
    kst[m] = row < R ? D.rstart[row] : INT_MAX;
  }
  typename M::acc_t acc[4][NTM];
#pragma unroll
  for (int m = 0; m < 4; m++)
#pragma unroll
    for (int nn = 0; nn < NTM; nn++) acc[m][nn] = typename M::acc_t{0, 0, 0, 0};
  // rows own k from their block's start: steps below the tile's last start,
  // and the step reaching the chunk end, are masked; the rest are not
  const int kfull = D.rstart[min(r0 + TZ_TM, R) - 1];
  auto load = [&](typename M::ld_t *A_, typename M::ld_t *B_, int k0) {
    const int kk = k0 + VEC * q;
#pragma unroll
    for (int m = 0; m < 4; m++) A_[m] = *reinterpret_cast<const typename M::ld_t *>(arow0 + m * s16 + kk);
#pragma unroll
    for (int nn = 0; nn < NTM; nn++)
      if (nn < ntn) B_[nn] = *reinterpret_cast<const typename M::ld_t *>(brow0 + nn * s16 + kk);
  };
  // B columns past w are rows of later positions, still zero when this
  // column runs (their folds come later), so only the triangle's first steps
  // and the chunk's last step need masks
  auto compute = [&](const typename M::ld_t *A_, const typename M::ld_t *B_, int k0) {
    if (k0 >= kfull && k0 + KS <= ke) {
#pragma unroll
      for (int s = 0; s < VEC; s++)
#pragma unroll
        for (int nn = 0; nn < NTM; nn++)
          if (nn < ntn)
#pragma unroll
            for (int m = 0; m < 4; m++) acc[m][nn] = M::mac(A_[m][s], B_[nn][s], acc[m][nn]);
      return;
    }
    const int kk = k0 + VEC * q;
#pragma unroll
    for (int s = 0; s < VEC; s++) {
      const int k = kk + s;
      T av[4], bs[NTM];
#pragma unroll
      for (int m = 0; m < 4; m++) av[m] = (k >= kst[m] && k < ke) ? A_[m][s] : T(0);
#pragma unroll
      for (int nn = 0; nn < NTM; nn++) bs[nn] = k < ke ? B_[nn][s] : T(0);
#pragma unroll
      for (int nn = 0; nn < NTM; nn++)
        if (nn < ntn)
#pragma unroll
          for (int m = 0; m < 4; m++) acc[m][nn] = M::mac(av[m], bs[nn], acc[m][nn]);
    }
  };
  // operands of two steps in flight: a ring of two register stages (a third
  // stage measured slower: fewer waves fit the registers)
  typename M::ld_t a0[4], b0[NTM], a1[4], b1[NTM];
  if (kb < ke) load(a0, b0, kb);  // a wave whose range lies past the column loads nothing
  if (kb + KS < ke) load(a1, b1, kb + KS);
  for (int k0 = kb; k0 < ke; k0 += 2 * KS) {
    compute(a0, b0, k0);
    if (k0 + 2 * KS < ke) load(a0, b0, k0 + 2 * KS);
    if (k0 + KS >= ke) break;
    compute(a1, b1, k0 + KS);
    if (k0 + 3 * KS < ke) load(a1, b1, k0 + 3 * KS);
  }
  // the eight sums meet through LDS in a fixed tree: w += w + 4 (w < 4),
  // then wave 0 adds waves 1, 2, 3 in order
  extern __shared__ __align__(16) unsigned char tz_plds[];
  typename M::acc_t *red = reinterpret_cast<typename M::acc_t *>(tz_plds);  // [4][4][ntn][64]
  if (wave >= 4)
#pragma unroll
    for (int m = 0; m < 4; m++)
#pragma unroll
      for (int nn = 0; nn < NTM; nn++)
        if (nn < ntn) red[(((wave - 4) * 4 + m) * ntn + nn) * 64 + lane] = acc[m][nn];
  __syncthreads();
  if (wave < 4)
#pragma unroll
    for (int m = 0; m < 4; m++)
#pragma unroll
      for (int nn = 0; nn < NTM; nn++)
        if (nn < ntn) acc[m][nn] += red[((wave * 4 + m) * ntn + nn) * 64 + lane];
  __syncthreads();
  if (wave >= 1 && wave < 4)
#pragma unroll
    for (int m = 0; m < 4; m++)
#pragma unroll
      for (int nn = 0; nn < NTM; nn++)
        if (nn < ntn) red[(((wave - 1) * 4 + m) * ntn + nn) * 64 + lane] = acc[m][nn];
  __syncthreads();
  if (wave != 0) return;
  for (int wv = 1; wv < 4; wv++)
#pragma unroll
    for (int m = 0; m < 4; m++)
#pragma unroll
      for (int nn = 0; nn < NTM; nn++)
        if (nn < ntn) acc[m][nn] += red[(((wv - 1) * 4 + m) * ntn + nn) * 64 + lane];
  T *P = D.P + (size_t)c * D.prow * TZ_WMAX;
#pragma unroll
  for (int m = 0; m < 4; m++)
#pragma unroll
    for (int nn = 0; nn < NTM; nn++)
      if (nn < ntn)
#pragma unroll
        for (int v = 0; v < 4; v++) {
          const int row = r0 + 16 * m + M::drow(q, v), col = 16 * nn + li;
          if (row < R && col < w) P[(size_t)row * TZ_WMAX + col] = acc[m][nn][v];
        }
  // tile 0 (one workgroup in every chunk) records the largest partial of
  // the column's row-0 block in this chunk: the next column's fold takes the
  // column's exponent from their sum, read in one round, instead of summing
  // the block's partials in every workgroup
  if (t == 0) {
    T mx = T(0);
#pragma unroll
    for (int m = 0; m < 4; m++)
#pragma unroll
      for (int nn = 0; nn < NTM; nn++)
        if (nn < ntn)
#pragma unroll
          for (int v = 0; v < 4; v++) {
            const int row = 16 * m + M::drow(q, v), col = 16 * nn + li;
            if (row < D.g && col < w) mx = max(mx, acc[m][nn][v]);
          }
    mx = wave_max(mx);
    if (lane == 0) D.pmax[(size_t)j * TZ_GRIDCH + c] = mx;
  }
}

// ---- fold: finish column j-1, build row block j --------------------------
// One 256-thread workgroup per item q < j: block row q of column j-1 and the
// element E_{q-1,j} (and, for q = j-1, the unpaired base j-1 as well).
// STAGE: the model (S B, B, V) is copied to LDS first; without it (when it
// does not fit beside the item's arrays) the threads read it from memory.
template <typename T, bool STAGE>
__global__ __launch_bounds__(TZ_FT) void tz_fold(TzDev<T> D, int j, int nchunks_prev, int kc_prev) {
  extern __shared__ __align__(16) unsigned char tz_lds[];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int g = D.g, xi = D.xi, G4 = 4 * g;
  const int qi = blockIdx.x;  // block row qi of column j-1, element k = qi - 1
  T *Xs = reinterpret_cast<T *>(tz_lds);  // [g Sigma_q][g Sigma_{j-1}]
  T *ts = Xs + G4 * G4;                  // [combination][sigma_b][sigma_e]
  T *Us = ts + xi * 256;                 // [combination][sigma_k][sigma_j]
  T *tk = Us + xi * 256, *tl = tk + 64;  // cores of the element's two ends
  int *cmb = reinterpret_cast<int *>(tl + 64);
  __shared__ int ncmb;
  const T *sSB = D.SB, *sB = D.B, *sV = D.V;
  if (STAGE) {
    T *l = tk + 192;
    for (int e = tid; e < xi * 16 * g * g; e += TZ_FT) {
      l[e] = D.SB[e];
      l[xi * 16 * g * g + e] = D.B[e];
    }
    for (int e = tid; e < 4 * g * g; e += TZ_FT) l[2 * xi * 16 * g * g + e] = D.V[e];
    sSB = l;
    sB = l + (size_t)xi * 16 * g * g;
    sV = l + (size_t)2 * xi * 16 * g * g;
  }
  const int wp = g * D.sig[j - 1];  // width of column j-1
  const int k = qi - 1, l = j - 1;
  const bool pair = qi >= 1 && l - k >= 4;
  const int sk = pair ? D.sig[k] : 0, sb = pair ? D.sig[k + 1] : 0, se = pair ? D.sig[l] : 0, sj = D.sig[j];
  // 1. loads together: the exponent of column j-1, that of the sum over its
  // chunks (in chunk order) of their largest partials of the row-0 block (an
  // upper bound of the block's largest entry, within a factor of the chunk
  // count; any exact power of two serves as the factor), the sums of block
  // row qi of column j-1 (unscaled, into Xs), the cores of the element's ends
  // and the (rho, phi_k, phi_l) that carry weight (B nonzero, both bases
  // possible), in (rho, phi_k, phi_l) order
  int e_prev = 0;
  if (j >= 2) {
    T sm = T(0);
    for (int c = 0; c < nchunks_prev; c++) sm += D.pmax[(size_t)(j - 1) * TZ_GRIDCH + c];
    e_prev = exp_of((double)sm);
  }
  const int r0 = D.off[qi], rows = g * D.sig[qi];
  if (qi < j - 1) {
    for (int e0 = tid; e0 < rows * wp; e0 += 4 * TZ_FT) {
      int r[4], cc[4];
      bool ok[4];
      T y[4];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const int e = e0 + TZ_FT * u;
        ok[u] = e < rows * wp;
        r[u] = r0 + (ok[u] ? e / wp : 0);
        cc[u] = ok[u] ? e % wp : 0;
      }
      col_sum4(D, r, cc, ok, nchunks_prev, kc_prev, y);
#pragma unroll
      for (int u = 0; u < 4; u++)
        if (ok[u]) Xs[(r[u] - r0) * wp + cc[u]] = y[u];
    }
  }
  if (pair) {
    if (tid < 64) tk[tid] = D.tc[(size_t)k * 64 + tid];
    else if (tid < 128) tl[tid - 64] = D.tc[(size_t)l * 64 + tid - 64];
    if (tid == 128) {
      int na = 0;
      for (int rho = 0; rho < xi; rho++)
        for (int pk = 0; pk < 4; pk++)
          for (int pl = 0; pl < 4; pl++)
            if (((D.pairmask >> (4 * pk + pl)) & 1) && ((D.bmask[k] >> pk) & 1) && ((D.bmask[l] >> pl) & 1))
              cmb[na++] = (rho * 4 + pk) * 4 + pl;
      ncmb = na;
    }
  } else if (qi == j - 1 && tid < 64) {
    tk[tid] = D.tc[(size_t)(j - 1) * 64 + tid];
  }
  __syncthreads();
  // 2. block row qi of column j-1 scaled and written back
  if (tid == 0 && qi == 0 && j >= 2) D.colexp[j - 1] = e_prev;
  if (qi < j - 1) {
    const size_t cbase = (size_t)D.off[j - 1];
    for (int e = tid; e < rows * wp; e += TZ_FT) {
      const int rr = e / wp, col = e % wp;
      const T x = ldexp(Xs[rr * wp + col], -e_prev);
      Xs[rr * wp + col] = x;
      D.Q[(size_t)(r0 + rr) * D.ld + cbase + col] = x;
    }
  }
  __syncthreads();
  if (qi == 0 && (j - 1) % 3 == 0 && j >= 2 && wave == 0) {  // codon boundary: a g x g block, prefix trace
    T tr = T(0);
    for (int e = lane; e < g * g; e += 64) {
      const int x = e / g, y = e % g;
      tr += D.S[x * g + y] * Xs[y * wp + x];
    }
    tr = wave_sum(tr);
    if (lane == 0) D.ptr[(j - 1) / 3 - 1] = (double)tr;
  }
  const int na = pair ? ncmb : 0;
  // 2a. t[a][sigma_b][sigma_e] = Tr[S B_{phi_l, phi_k} X^{sigma_b, sigma_e}] for combination a
  for (int e = tid; e < na * 16; e += TZ_FT) {
    const int a = e >> 4, b = (e >> 2) & 3, ee = e & 3;
    T acc = T(0);
    if (b < sb && ee < se) {
      const int c3 = cmb[a], rho = c3 >> 4, pk = (c3 >> 2) & 3, pl = c3 & 3;
      const T *sbm = sSB + ((((size_t)rho * 4 + pl) * 4 + pk) * g) * g;
      for (int x = 0; x < g; x++)
        for (int y = 0; y < g; y++) acc += sbm[x * g + y] * Xs[(b * g + y) * wp + ee * g + x];
    }
    ts[e] = acc;
  }
  __syncthreads();
  // 2b. U[a][sigma_k][sigma_j] = (T_k^{phi_k} t T_l^{phi_l})[sigma_k][sigma_j]
  for (int e = tid; e < na * 16; e += TZ_FT) {
    const int a = e >> 4, ak = (e >> 2) & 3, cc = e & 3;
    const int c3 = cmb[a], pk = (c3 >> 2) & 3, pl = c3 & 3;
    T u = T(0);
    if (ak < sk && cc < sj)
      for (int b = 0; b < sb; b++)
        for (int ee = 0; ee < se; ee++)
          u += tk[(pk * 4 + ak) * 4 + b] * ts[a * 16 + b * 4 + ee] * tl[(pl * 4 + ee) * 4 + cc];
    Us[e] = u;
  }
  __syncthreads();
  // 2c. E_{k,j} = 2^-e_k sum_a U[a] (x) B_{phi_k, phi_l}, stored transposed
  if (qi >= 1) {
    const int rows = g * D.sig[k], wj = g * sj;
    const size_t rbase = (size_t)D.off[j], cbase = (size_t)D.off[k];
    const int ek = pair ? D.colexp[k + 1] : 0;
    for (int e = tid; e < rows * wj; e += TZ_FT) {
      const int rr = e % rows, cc = e / rows;  // consecutive threads along the stored row
      const int ak = rr / g, za = rr % g, s2 = cc / g, zb = cc % g;
      T f = T(0);
      for (int a = 0; a < na; a++) f += Us[a * 16 + ak * 4 + s2] * sB[(size_t)cmb[a] * g * g + za * g + zb];
      D.Q[(rbase + cc) * D.ld + cbase + rr] = pair ? ldexp(f, -ek) : T(0);
    }
  }
  // 3. the unpaired base j-1
  if (qi == j - 1) {
    const int sa = D.sig[j - 1], rows = g * sa, wj = g * sj;
    const size_t rbase = (size_t)D.off[j], cbase = (size_t)D.off[j - 1];
    for (int e = tid; e < rows * wj; e += TZ_FT) {
      const int rr = e % rows, cc = e / rows;
      const int a = rr / g, za = rr % g, s2 = cc / g, zb = cc % g;
      T f = T(0);
      for (int phi = 0; phi < 4; phi++) f += tk[(phi * 4 + a) * 4 + s2] * sV[(phi * g + za) * g + zb];
      D.Q[(rbase + cc) * D.ld + cbase + rr] = f;
    }
  }
}

// after the last column: its exponent and Tr[S Q_{0,n}] (one wave)
template <typename T>
__global__ __launch_bounds__(64) void tz_final(TzDev<T> D, int nchunks, int kc) {
  const int n = D.n, g = D.g;
  const int e = column_exponent(D, n, nchunks, kc);
  T tr = T(0);
  for (int q = threadIdx.x; q < g * g; q += 64) {
    const int x = q / g, y = q % g;
    tr += D.S[x * g + y] * ldexp(col_sum(D, y, x, nchunks, kc), -e);
  }
  tr = wave_sum(tr);
  if (threadIdx.x == 0) {
    D.colexp[n] = e;
    D.ptr[n / 3 - 1] = (double)tr;
  }
}

// Q = identity (the diagonal blocks), zero elsewhere
template <typename T>
__global__ void tz_init(T *Q, size_t rows, size_t ld, size_t N) {
  const size_t tot = rows * ld;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (size_t)gridDim.x * blockDim.x) {
    const size_t r = e / ld, c = e % ld;
    Q[e] = (r == c && r < N) ? T(1) : T(0);
  }
}

// device workspace released when the call returns (hipFree waits for the device)
struct DevBuf {
  void *p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

struct TzHost {
  int n = 0, m = 0, N = 0, rows = 0, ld = 0, tiles = 0, chunks = 0;
  std::vector<int> sig, off, rstart, tile_kmin;
  std::vector<int> chunk_tiles;  // per chunk size: [chunks of that size] tiles whose first chunk is <= c
  int ct_off[TZ_NKC] = {};       // start of each size's table in chunk_tiles
  std::vector<unsigned char> bmask;
  std::vector<double> tc;  // [n][4][4][4]
};

int kci_of(const TzHost &H, int j) {  // index of column j's chunk size
  for (int i = 0; i < TZ_NKC; i++)
    if ((H.off[j] + TZ_KCS[i] - 1) / TZ_KCS[i] <= TZ_MAXCH) return i;
  return TZ_NKC - 1;
}
int kc_of(const TzHost &H, int j) { return TZ_KCS[kci_of(H, j)]; }
int nchunks_of(const TzHost &H, int j) { return (H.off[j] + kc_of(H, j) - 1) / kc_of(H, j); }
int ntiles_of(const TzHost &H, int j) { return (H.off[j] + TZ_TM - 1) / TZ_TM; }
int prop_grid(const TzHost &H, int j) {
  const int nt = ntiles_of(H, j), nc = nchunks_of(H, j), base = H.ct_off[kci_of(H, j)];
  int tot = 0;
  for (int c = 0; c < nc; c++) tot += c == nc - 1 ? nt : std::min(nt, H.chunk_tiles[base + c]);
  return tot;
}

template <typename T>
cdz_status run_tensor(cdz_handle *h, const TzHost &H, const cdz_tensor_model *md, double *log_z, double *prefix) {
  const int n = H.n, m = H.m, g = md->gamma, xi = md->xi;
  std::vector<T> V((size_t)4 * g * g), B((size_t)xi * 16 * g * g), SB(B.size()), S((size_t)g * g), tc(H.tc.size());
  for (size_t q = 0; q < V.size(); q++) V[q] = (T)md->V[q];
  for (size_t q = 0; q < B.size(); q++) B[q] = (T)md->B[q];
  for (size_t q = 0; q < S.size(); q++) S[q] = (T)md->S[q];
  for (size_t q = 0; q < tc.size(); q++) tc[q] = (T)H.tc[q];
  unsigned pairmask = 0;
  for (int rho = 0; rho < xi; rho++)
    for (int xy = 0; xy < 16; xy++) {
      const double *b = md->B + ((size_t)rho * 16 + xy) * g * g;
      bool nz = false;
      for (int q = 0; q < g * g; q++) nz |= b[q] != 0.0;
      if (nz) pairmask |= 1u << xy;
      for (int x = 0; x < g; x++)
        for (int y = 0; y < g; y++) {
          double acc = 0.0;
          for (int z = 0; z < g; z++) acc += md->S[x * g + z] * b[z * g + y];
          SB[((size_t)rho * 16 + xy) * g * g + x * g + y] = (T)acc;
        }
    }
  // workspace
  size_t at = 0;
  auto take = [&](size_t bytes) {
    const size_t p = (at + 255) / 256 * 256;
    at = p + bytes;
    return p;
  };
  const size_t oQ = take((size_t)H.rows * H.ld * sizeof(T)),
               oP = take((size_t)H.chunks * H.rows * TZ_WMAX * sizeof(T)), oSig = take((n + 1) * 4),
               oOff = take((n + 1) * 4), oRs = take((size_t)H.rows * 4), oTk = take((size_t)H.tiles * 4),
               oBm = take(n), oTc = take(tc.size() * sizeof(T)),
               oV = take(V.size() * sizeof(T)), oB = take(B.size() * sizeof(T)), oSB = take(SB.size() * sizeof(T)),
               oS = take(S.size() * sizeof(T)), oCe = take((n + 1) * 4), oPt = take((size_t)m * 8),
               oPm = take((size_t)(n + 1) * TZ_GRIDCH * sizeof(T));
  DevBuf ws;
  if (hipMalloc(&ws.p, at) != hipSuccess) {
    (void)hipGetLastError();
    ws.p = nullptr;
    return cdz_fail(h, CDZ_ERR_NOMEM, "tensor-model workspace of " + std::to_string(at) + " bytes");
  }
  char *base = (char *)ws.p;
  hipStream_t st = h->stream;
  auto up = [&](size_t o, const void *src, size_t bytes) {
    return hipMemcpyAsync(base + o, src, bytes, hipMemcpyHostToDevice, st);
  };
  HIPCHK(h, up(oSig, H.sig.data(), (n + 1) * 4));
  HIPCHK(h, up(oOff, H.off.data(), (n + 1) * 4));
  HIPCHK(h, up(oRs, H.rstart.data(), (size_t)H.rows * 4));
  HIPCHK(h, up(oTk, H.tile_kmin.data(), (size_t)H.tiles * 4));
  HIPCHK(h, up(oBm, H.bmask.data(), n));
  HIPCHK(h, up(oTc, tc.data(), tc.size() * sizeof(T)));
  HIPCHK(h, up(oV, V.data(), V.size() * sizeof(T)));
  HIPCHK(h, up(oB, B.data(), B.size() * sizeof(T)));
  HIPCHK(h, up(oSB, SB.data(), SB.size() * sizeof(T)));
  HIPCHK(h, up(oS, S.data(), S.size() * sizeof(T)));
  TzDev<T> D;
  D.n = n;
  D.g = g;
  D.xi = xi;
  D.ld = H.ld;
  D.prow = H.rows;
  D.sig = (const int *)(base + oSig);
  D.off = (const int *)(base + oOff);
  D.rstart = (const int *)(base + oRs);
  D.tile_kmin = (const int *)(base + oTk);
  D.bmask = (const unsigned char *)(base + oBm);
  D.tc = (const T *)(base + oTc);
  D.V = (const T *)(base + oV);
  D.B = (const T *)(base + oB);
  D.SB = (const T *)(base + oSB);
  D.S = (const T *)(base + oS);
  D.pairmask = pairmask;
  D.Q = (T *)(base + oQ);
  D.P = (T *)(base + oP);
  D.colexp = (int *)(base + oCe);
  D.pmax = (T *)(base + oPm);
  D.ptr = (double *)(base + oPt);
  const size_t wave_lds = (size_t)(16 * g * g + 2 * xi * 256 + 192) * sizeof(T);
  const size_t model_lds = (size_t)(2 * xi * 16 + 4) * g * g * sizeof(T);
  const bool stage = wave_lds + model_lds <= (size_t)h->lds_max;
  const size_t fold_lds = stage ? wave_lds + model_lds : wave_lds;
  if (wave_lds > (size_t)h->lds_max) return cdz_fail(h, CDZ_ERR_ARG, "gamma too large for the fold's LDS");
  int ntn_max = 1;
  for (int p = 0; p <= n; p++) ntn_max = std::max(ntn_max, (g * H.sig[p] + 15) / 16);
  const size_t prop_lds = (size_t)4 * 4 * ntn_max * 64 * 4 * sizeof(T);
  if (h->profiling) HIPCHK(h, prof_reserve(h, n));
  HIPCHK(h, hipEventRecord(h->ev[0], st));
  tz_init<T><<<2048, 256, 0, st>>>(D.Q, (size_t)H.rows, (size_t)H.ld, (size_t)H.N);
  for (int j = 1; j <= n; j++) {
    const int fgrid = j;
    const int ncp = j >= 2 ? nchunks_of(H, j - 1) : 0, kcp = j >= 2 ? kc_of(H, j - 1) : TZ_KCS[0];
    if (stage) tz_fold<T, true><<<fgrid, TZ_FT, fold_lds, st>>>(D, j, ncp, kcp);
    else tz_fold<T, false><<<fgrid, TZ_FT, fold_lds, st>>>(D, j, ncp, kcp);
    if (h->profiling) HIPCHK(h, hipEventRecord(h->pev[2 * (j - 1)], st));
    TzGrid G{};
    {
      const int nt = ntiles_of(H, j), nc = nchunks_of(H, j), b0 = H.ct_off[kci_of(H, j)];
      for (int c = 0; c < nc; c++) G.cnt[c] = c == nc - 1 ? nt : std::min(nt, H.chunk_tiles[b0 + c]);
    }
    if (ntn_max <= 3) {
      tz_prop<T, 3><<<prop_grid(H, j), 64 * TZ_PW, prop_lds, st>>>(D, j, ntiles_of(H, j), nchunks_of(H, j),
                                                                   kc_of(H, j), G);
    } else {
      tz_prop<T, 4><<<prop_grid(H, j), 64 * TZ_PW, prop_lds, st>>>(D, j, ntiles_of(H, j), nchunks_of(H, j),
                                                                   kc_of(H, j), G);
    }
    if (h->profiling) HIPCHK(h, hipEventRecord(h->pev[2 * (j - 1) + 1], st));
  }
  tz_final<T><<<1, 64, 0, st>>>(D, nchunks_of(H, n), kc_of(H, n));
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipEventRecord(h->ev[1], st));
  std::vector<double> ptr(m);
  std::vector<int> ce(n + 1);
  HIPCHK(h, hipMemcpyAsync(ptr.data(), base + oPt, (size_t)m * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipMemcpyAsync(ce.data(), base + oCe, (n + 1) * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipStreamSynchronize(st));
  float ms = 0;
  HIPCHK(h, hipEventElapsedTime(&ms, h->ev[0], h->ev[1]));
  h->times[0] = ms;
  h->times[1] = h->times[2] = 0;
  h->prof_fwd_ms = 0;
  h->prof_fwd_launches = 0;
  if (h->profiling) {
    double tot = 0;
    for (int j = 0; j < n; j++) {
      float k = 0;
      HIPCHK(h, hipEventElapsedTime(&k, h->pev[2 * j], h->pev[2 * j + 1]));
      tot += k;
    }
    h->prof_fwd_ms = tot;
    h->prof_fwd_launches = n;
  }
  const double L2 = 0.6931471805599453094;
  long esum = 0;
  for (int a = 0; a < m; a++) {
    for (int col = 3 * a + 1; col <= 3 * a + 3; col++) esum += ce[col];
    const double lz = std::log(ptr[a]) + L2 * (double)esum;
    if (!(ptr[a] > 0.0) || !std::isfinite(lz))
      return cdz_fail(h, CDZ_ERR_NUMERIC, "tensor-model prefix " + std::to_string(a) + " not finite");
    if (prefix) prefix[a] = lz;
    if (a == m - 1) *log_z = lz;
  }
  return CDZ_OK;
}

// single-codon train (eq. single-tt): core 3a selects the first base,
// core 3a+1 the codon (first base, middle base, third base) with its bonus,
// core 3a+2 the third base
cdz_status build_train(cdz_handle *h, const HostTables &t, const double *theta1, TzHost &H) {
  H.m = t.m;
  H.n = t.n;
  const int n = H.n;
  H.sig.assign(n + 1, 1);
  H.tc.assign((size_t)n * 64, 0.0);
  H.bmask.assign(n, 0);
  auto TC = [&](int p, int phi, int a, int b) -> double & { return H.tc[(((size_t)p * 4 + phi) * 4 + a) * 4 + b]; };
  for (int a = 0; a < H.m; a++) {
    const int p = 3 * a, d = t.d[p];
    int first[4], third[4], nf = 0, nth = 0;
    for (int b = 0; b < 4; b++) {
      bool hf = false, ht = false;
      for (int s2 = 0; s2 < d; s2++) {
        hf |= t.nt[p * 6 + s2] == b;
        ht |= t.nt[(p + 2) * 6 + s2] == b;
      }
      if (hf) first[nf++] = b;
      if (ht) third[nth++] = b;
    }
    H.sig[p] = 1;
    H.sig[p + 1] = nf;
    H.sig[p + 2] = nth;
    for (int x = 0; x < nf; x++) TC(p, first[x], 0, x) = 1.0;
    for (int s2 = 0; s2 < d; s2++) {
      const int b0 = t.nt[p * 6 + s2], b1 = t.nt[(p + 1) * 6 + s2], b2 = t.nt[(p + 2) * 6 + s2];
      int x = 0, y = 0;
      while (first[x] != b0) x++;
      while (third[y] != b2) y++;
      const double th = theta1 ? theta1[a * 6 + s2] : 0.0;
      if (!std::isfinite(th)) return cdz_fail(h, CDZ_ERR_NUMERIC, "non-finite codon bonus");
      TC(p + 1, b1, x, y) += std::exp(th);
    }
    for (int y = 0; y < nth; y++) TC(p + 2, third[y], y, 0) = 1.0;
  }
  for (int p = 0; p < n; p++)
    for (int phi = 0; phi < 4; phi++)
      for (int q = 0; q < 16; q++)
        if (H.tc[((size_t)p * 4 + phi) * 16 + q] != 0.0) H.bmask[p] |= (unsigned char)(1u << phi);
  return CDZ_OK;
}

// flattened layout of Q and the propagation's tile and chunk tables, then the pass
cdz_status finish_layout(cdz_handle *h, TzHost &H, int g, const cdz_tensor_model *md, double *log_z,
                         double *prefix) {
  const int n = H.n;
  H.off.assign(n + 1, 0);
  int o = 0;
  for (int p = 0; p <= n; p++) {
    H.off[p] = o;
    o += g * H.sig[p];
  }
  H.N = o;
  H.rows = (H.N + TZ_WMAX + TZ_TM - 1) / TZ_TM * TZ_TM;  // room for the widest fold row block past N
  H.ld = H.rows;
  if ((size_t)H.rows * H.ld > ((size_t)1 << 40)) return cdz_fail(h, CDZ_ERR_ARG, "protein too long for Q");
  H.rstart.assign(H.rows, H.N);
  for (int p = 0; p <= n; p++)
    for (int r = H.off[p]; r < H.off[p] + g * H.sig[p]; r++) H.rstart[r] = H.off[p];
  H.tiles = (H.N + TZ_TM - 1) / TZ_TM;
  H.tile_kmin.resize(H.tiles);
  for (int ti = 0; ti < H.tiles; ti++) H.tile_kmin[ti] = H.rstart[ti * TZ_TM];
  H.chunk_tiles.clear();
  for (int i = 0; i < TZ_NKC; i++) {
    const int kc = TZ_KCS[i], nch = (H.N + kc - 1) / kc;
    H.ct_off[i] = (int)H.chunk_tiles.size();
    for (int c = 0; c < nch; c++) {
      int cnt = 0;
      for (int ti = 0; ti < H.tiles; ti++) cnt += H.tile_kmin[ti] / kc <= c;
      H.chunk_tiles.push_back(cnt);
    }
  }
  H.chunks = 1;  // partial-sum slots: the most chunks any column uses
  for (int j = 1; j <= n; j++) H.chunks = std::max(H.chunks, nchunks_of(H, j));
  if (H.chunks > TZ_GRIDCH) return cdz_fail(h, CDZ_ERR_ARG, "protein too long for the propagation grid");
  if (h->opt.prec == CDZ_FP64) return run_tensor<double>(h, H, md, log_z, prefix);
  return run_tensor<float>(h, H, md, log_z, prefix);
}

}  // namespace

extern "C" cdz_status cdz_tensor_logz(cdz_handle *h, const cdz_tensor_model *md, const cdz_problem *prob,
                                      double *log_z, double *prefix) {
  if (!h || !md || !prob || !log_z) return cdz_fail(h, CDZ_ERR_ARG, "null argument");
  if (prob->theta2) return cdz_fail(h, CDZ_ERR_ARG, "the single-codon train takes no codon-pair weights");
  const int g = md->gamma, xi = md->xi;
  if (g < 1 || g > 16 || xi < 1 || xi > 4 || !md->V || !md->B || !md->S)
    return cdz_fail(h, CDZ_ERR_ARG, "tensor model: gamma in 1..16, xi in 1..4, V, B, S given");
  auto ok = [](const double *p, size_t cnt) {
    for (size_t q = 0; q < cnt; q++)
      if (!(p[q] >= 0.0) || !std::isfinite(p[q])) return false;
    return true;
  };
  if (!ok(md->V, (size_t)4 * g * g) || !ok(md->B, (size_t)xi * 16 * g * g) || !ok(md->S, (size_t)g * g))
    return cdz_fail(h, CDZ_ERR_NUMERIC, "tensor model entries must be finite and non-negative");
  HostTables t;
  cdz_status s = build_tables(h, prob->n_aa, prob->aa, prob->theta1, nullptr, t);
  if (s != CDZ_OK) return s;
  TzHost H;
  s = build_train(h, t, prob->theta1, H);
  if (s != CDZ_OK) return s;
  return finish_layout(h, H, g, md, log_z, prefix);
}

extern "C" cdz_status cdz_tensor_dims(const cdz_problem *prob, int32_t *sig) {
  if (!prob || !sig || prob->n_aa < 1 || !prob->aa) return CDZ_ERR_ARG;
  cdz_handle tmp;
  HostTables t;
  cdz_status s = build_tables(&tmp, prob->n_aa, prob->aa, nullptr, nullptr, t);
  if (s != CDZ_OK) return s;
  TzHost H;
  s = build_train(&tmp, t, nullptr, H);
  if (s != CDZ_OK) return s;
  for (int p = 0; p <= H.n; p++) sig[p] = H.sig[p];
  return CDZ_OK;
}
