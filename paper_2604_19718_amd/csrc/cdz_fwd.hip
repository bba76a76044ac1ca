// cdz_fwd.hip -- forward (inside) pass of the codon-constrained McCaskill
// dynamic program: one launch per anti-diagonal dl = j - i, one workgroup
// per cell (i, i+dl) plus one workgroup for the FP64 exterior loop.
//
// What a cell computes (tensors over the codon slots of the two end
// positions; e_p = backbone edge factor between p and p+1, v_p = vertex
// factor; sequence-summed fold of the paper's Section 3c applied to
// nearest-neighbour loops):
//   U    unpaired run [i..j]
//   Qb   pair (i,j) closing a hairpin, a stack/bulge/interior loop (window of
//        inner pairs with l1 + l2 <= 30) or a multiloop
//   Qm1  one multiloop branch starting at i, unpaired tail
//   Qm1p unpaired prefix, then one branch
//   QmX  >= 2 branches: sum_u Qm[i][u-1] e_{u-1} Qm1[u][j]  (the O(n) split)
//   Qm   >= 1 branch = QmX + Qm1p
// plus derived blocks consumed by later diagonals: DI (Qb dressed as the
// inner pair of an interior loop), Qm1L (Qm1 with its left edge, in row and
// column orientation), Qmt (Qm transposed), and G/F (the bulge and interior
// loop sums of the cell, kept for the adjoint).
#include <algorithm>

#include "cdz_dev.h"

namespace {

}  // namespace

// LDS stage of one cell: every small block the O(1) recurrences of the cell
// read, fetched by one parallel load phase.
template <typename T>
struct CellStage {
  T tab[TB_LEN];
  T eIm1[36], eI[36], eJm1[36], eJ[36];  // edge factors e_{i-1}, e_i, e_{j-1}, e_j
  T vI[6], vJ[6];
  T Uin[36];   // U[i+1][j-1]
  T Xin[36];   // QmX[i+1][j-1]
  T Bin[36];   // Qb[i+1][j-1]
  T M1l[36];   // Qm1[i][j-1]
  T M1pr[36];  // Qm1p[i+1][j]
  T Ul[36];    // U[i][j-1]
  T split[36], gf[72], qb[36], qm1[36];
  T eI1[36], eJm2[36], vI1[6], vJm1[6];  // e_{i+1}, e_{j-2}, v_{i+1}, v_{j-1}
  signed char nt[6][6];  // bases of positions i-1, i, i+1, j-1, j, j+1
  int d[6], P[6];
  int wd[64], wP[64];    // d, P of positions i+1+q ([q]) and j-1-q ([32+q])
  unsigned char mapL[192], mapR[192];  // state offset -> position index (window staging)
};

// Blocks of 36 values of the window kind (a_window: runs U[i+1][i+l] 30,
// U[j-l][j-1] 30, DI strips 29 + 28, A of the inner cell 27, A of the cell
// for L = 2..30 29) and of the bulge kind (runs 2 x 30, edges 2 x 30, inner
// pairs 2 x 30)
#define CDZ_FWD_WBLK 173
#define CDZ_BUL_BLK 180



// Interior-loop sums A(i,j,L), L = 2..lmax, of cell (i, j) into AC by the
// loop-size recursion, staging on the way UR1 = U[i+1][i+l] and UC1 =
// U[j-l][j-1] (l = 1..lmax), which the bulge sums of the forward read next.
// The forward and the recomputation of A for the memory-bounded outside pass
// both run this code, so they produce the same bits.  A(i+1, j-1, .) comes
// from D.AL (all diagonals resident) or from D.ALp (diagonal dl - 2, stored
// diagonal-major).
template <typename T>
__device__ __forceinline__ void a_window(const DevProb<T> &D, CellStage<T> &C, const int *sE, T *W, int i,
                                         int j, int dl, int lmax, int Ed) {
  const int tid = threadIdx.x;
  const long long ld = D.ld;
  const int d1 = C.d[2], dm = C.d[3], P1 = C.P[2], Pm = C.P[3];
  T *UR1 = W;              // [l-1] U[i+1][i+l]
  T *UC1 = W + 30 * 36;    // [l-1] U[j-l][j-1]
  T *X = W + 60 * 36;      // phase-dependent blocks
  T *DIrow = X;            // [L-2] DI[i+1][j-L+1]
  T *DIcol = X + 29 * 36;  // [L-3] DI[i+L-1][j-1]
  T *AP = X + 57 * 36;     // [L-2] A(i+1,j-1,L), then A(i+1,j-1,L) . W
  T *AC = X + 84 * 36;     // [L-2] A(i,j,L)
  const int *lp_d = C.wd, *lp_P = C.wP, *rp_d = C.wd + 32, *rp_P = C.wP + 32;
  const int nAP = lmax - 3 > 0 ? lmax - 3 : 0;  // L = 2..lmax-2
  if (lmax >= 1) {
    // Every region is read as contiguous row segments (the column strips
    // U[j-l][j-1] and DI[i+L-1][j-1] as rows of the transposed arrays), lanes
    // walking the row so that the loads coalesce; a map from state offset to
    // position places each value in its 6 x 6 block, zeroed first for the
    // padding.  Left states: positions i+1.. (lp index q), from lp_P[0];
    // right states: positions j-lmax..j-1 (rp index q), from rp_P[lmax-1].
    const int baseL = lp_P[0], baseR = rp_P[lmax];
    cdz_window_maps(C.mapL, C.mapR, lp_d, lp_P, rp_d, rp_P, lmax);
    {  // clear UR1, UC1, DIrow, DIcol and the AP blocks in use, 16 bytes a store
      uint4 *w4 = reinterpret_cast<uint4 *>(W);
      const int n4 = (117 + nAP) * 36 * (int)sizeof(T) / 16;
      for (int idx = tid; idx < n4; idx += CDZ_NT) w4[idx] = make_uint4(0, 0, 0, 0);
    }
    cdz_sync();
    const int KU = lp_P[lmax] - baseL;                           // end states of U[i+1][i+1..i+lmax]
    const int endR = rp_P[0] + rp_d[0] - baseR;                  // right map: positions j-1-lmax..j-1
    const int oC = rp_P[lmax - 1] - baseR, KC = endR - oC;       // start states of U[j-lmax..j-1][j-1]
    const int oD = lmax >= 2 ? rp_P[lmax - 2] - baseR : endR;    // DI[i+1][j-lmax+1..j-1]
    const int KD = endR - oD;
    const int oL = lp_P[1] - baseL;                              // DI[i+2..i+lmax-1][j-1]: part of KU
    const int KL = lmax >= 3 ? lp_P[lmax - 1] - lp_P[1] : 0;
    const int dA = lp_d[1], dB = rp_d[1], KA = nAP * dB;         // A(i+1, j-1, L), L = 2..lmax-2
    const int nU = d1 * KU, nC = dm * KC, nD = d1 * KD, nL = dm * KL;
    const int nA = D.AL ? dA * KA : nAP * 36;
    const int e1 = nU, e2 = e1 + nC, e3 = e2 + nD, e4 = e3 + nL;
    // W offsets: UR1 0, UC1 30*36, DIrow 60*36, DIcol 89*36, AP 117*36
    cdz_stage_nv<4, T>(W, e4 + nA, [&](int idx, int &d) -> const T * {
      if (idx < e1) {  // U[i+1][i+l]: row P1 + r of U
        const int r = idx / KU, k = idx % KU, qq = C.mapL[k], c = k - (lp_P[qq] - baseL);
        d = qq * 36 + r * 6 + c;
        return D.U + (long long)(P1 + r) * ld + baseL + k;
      }
      if (idx < e2) {  // U[j-l][j-1]: row Pm + c of Ut, l = qq + 1
        const int t = idx - e1, c = t / KC, k = t % KC + oC, qq = C.mapR[k], r = k - (rp_P[qq] - baseR);
        d = (30 + qq) * 36 + r * 6 + c;
        return D.Ut + (long long)(Pm + c) * ld + baseR + k;
      }
      if (idx < e3) {  // DI[i+1][j-L+1]: row P1 + r of DI, L = qq + 2
        const int t = idx - e2, r = t / KD, k = t % KD + oD, qq = C.mapR[k], c = k - (rp_P[qq] - baseR);
        d = (60 + qq) * 36 + r * 6 + c;
        return D.DI + (long long)(P1 + r) * ld + baseR + k;
      }
      if (idx < e4) {  // DI[i+L-1][j-1]: row Pm + c of DIt, L = qq + 2
        const int t = idx - e3, c = t / KL, k = t % KL + oL, qq = C.mapL[k], r = k - (lp_P[qq] - baseL);
        d = (89 + qq - 1) * 36 + r * 6 + c;
        return D.DIt + (long long)(Pm + c) * ld + baseL + k;
      }
      const int t = idx - e4;
      if (D.AL) {
        const int r = t / KA, k = t % KA;
        d = (117 + k / dB) * 36 + r * 6 + k % dB;
        return D.AL + (long long)(lp_P[1] + r) * D.ldA + (long long)CDZ_NA * rp_P[1] + k;
      }
      d = 117 * 36 + t;
      return D.ALp + (long long)(i + 1) * (CDZ_NA * 36) + t;
    });
  }
  cdz_sync();
  // AP <- AP . W (in place: every output is read into registers first)
  {
    T t4[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int idx = tid + u * CDZ_NT;
      t4[u] = 0;
      if (idx < nAP * 36) {
        const int b = idx / 36, q = idx % 36, a2 = q / 6, dd = q % 6;
        T s = 0;
#pragma unroll
        for (int d2 = 0; d2 < 6; d2++) s += AP[b * 36 + a2 * 6 + d2] * C.eJm2[d2 * 6 + dd];
        t4[u] = s * C.vJm1[dd];
      }
    }
    cdz_sync();
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const int idx = tid + u * CDZ_NT;
      if (idx < nAP * 36) AP[idx] = t4[u];
    }
  }
  cdz_sync();
  // A(i,j,L), L = 2..lmax
  const T frec = cdz_p2<T>(sE[dl >= 2 ? dl - 2 : 0] - Ed);
  for (int idx = tid; idx < (lmax - 1) * 36; idx += CDZ_NT) {
    const int L = idx / 36 + 2, q = idx % 36, a = q / 6, dd = q % 6;
    const T fb = cdz_p2<T>(sE[dl - L - 2] + sE[L - 2] - Ed);
    T rec = 0, b1 = 0, b2 = 0;
    if (L >= 4) {
#pragma unroll
      for (int a2 = 0; a2 < 6; a2++) rec += C.eI1[a * 6 + a2] * AP[(L - 4) * 36 + a2 * 6 + dd];
    }
#pragma unroll
    for (int c = 0; c < 6; c++) b1 += DIrow[(L - 2) * 36 + a * 6 + c] * UC1[(L - 2) * 36 + c * 6 + dd];
    if (L >= 3) {
#pragma unroll
      for (int b = 0; b < 6; b++) b2 += UR1[(L - 2) * 36 + a * 6 + b] * DIcol[(L - 3) * 36 + b * 6 + dd];
    }
    AC[(L - 2) * 36 + q] = C.vI1[a] * (rec * frec + b1 * fb) + b2 * C.vJm1[dd] * fb;
  }
  cdz_sync();
}

// Store A(i,j,L), L = 2..CDZ_NA+1, of cell (i, j) (zero where no inner pair
// fits): into D.AL at rows P[i+1].., or, diagonal-major, into D.ALw at cell i
// (all 36 entries of each block, padding zero).
template <typename T>
__device__ __forceinline__ void a_store(const DevProb<T> &D, const CellStage<T> &C, int i, int lmax, const T *AC) {
  const int d1 = C.d[2], dm = C.d[3], P1 = C.P[2], Pm = C.P[3];
  for (int idx = threadIdx.x; idx < CDZ_NA * 36; idx += CDZ_NT) {
    const int L = idx / 36 + 2, qq = idx % 36, a = qq / 6, dd = qq % 6;
    const T v = (L <= lmax && a < d1 && dd < dm) ? AC[(L - 2) * 36 + qq] : T(0);
    if (D.AL) {
      if (a < d1 && dd < dm) D.AL[(long long)(P1 + a) * D.ldA + (long long)CDZ_NA * Pm + (L - 2) * dm + dd] = v;
    } else {
      D.ALw[(long long)i * (CDZ_NA * 36) + idx] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// One launch per step t = 0..n.  The work of a diagonal is split by what it
// reads, and each piece runs in the earliest launch where its inputs are
// final, as its own workgroups; the pieces of one launch never read each
// other's results:
//   window   (diagonal t+1)  interior-loop sums by size A(i,j,L) and F: reads
//                            U, DI and A of diagonals <= t-1
//   bulges   (diagonal t+1)  bulge sums G: reads Qb of diagonals <= t-2
//   split    (diagonal t+4)  QmX, the O(n) multiloop split: reads Qm and Qm1L
//                            of diagonals <= t-1; stored under a provisional
//                            exponent EX[t+4] that the finish converts
//   finish   (diagonal t)    U, Qb, Qm1, DI, Qm1L, Qm1p, QmX, Qm of every cell:
//                            O(1) blocks of diagonals t-1, t-2 and the sums
//                            above
// The FP64 exterior loops run after the last launch (exterior_scan_body).
// Exponents.  E[t+1] and EX[t+4] are chosen in launch t from the maxima of
// the last complete diagonals, extrapolated; every workgroup of the launch
// that needs them computes the same values and the first finish workgroup
// stores them.  E[0] = 0 (set by the host).
// ---------------------------------------------------------------------------

// Exponent for diagonal `target`, chosen in launch t (t >= 0): the log2 of
// the largest entry of diagonal t-1, extrapolated with the growth per
// diagonal averaged over diagonals t-5..t-1 (over t-2..t-1 early on), so that
// the short, irregular diagonals at the start do not make it overshoot
template <typename T>
__device__ __forceinline__ int exponent_ahead(const DevProb<T> &D, int t, int target) {
  if (t <= 0) return 0;
  const int E1 = D.E[t - 1];
  const float m1 = __uint_as_float(D.maxb[t - 1]);
  if (!(m1 > 0.f)) return E1;
  const double L1 = E1 + log2((double)m1);
  double slope = 0;
  const int back = t >= 5 ? 4 : t >= 2 ? 1 : 0;
  if (back > 0) {
    const float mb = __uint_as_float(D.maxb[t - 1 - back]);
    if (mb > 0.f) slope = fmin(fmax((L1 - (D.E[t - 1 - back] + log2((double)mb))) / back, -16.0), 16.0);
  }
  return (int)rint(L1 + (target - (t - 1)) * slope);
}

// LDS of the finish: every operand of the O(1) recurrences of a cell
template <typename T>
struct FinStage {
  T tab[TB_LEN];
  T eIm1[36], eI[36], eJm1[36], eJ[36];  // edge factors e_{i-1}, e_i, e_{j-1}, e_j
  T vI[6], vJ[6];
  T Uin[36], Xin[36], Bin[36];  // U, QmX, Qb of (i+1, j-1)
  T M1l[36];                    // Qm1[i][j-1]
  T M1pr[36];                   // Qm1p[i+1][j]
  T Ul[36];                     // U[i][j-1]
  T G[36], F[36];               // bulge and interior sums of the cell (block (i+1, j-1))
  T X[36];                      // split sum of the cell, provisional exponent
  T qb[36], qm1[36];
  signed char nt[6][6];  // bases of positions i-1, i, i+1, j-1, j, j+1
  int d[6], P[6];
};

// LDS of the bulge sums of a cell
struct BulStage {
  int d[6], P[6];
  int wd[64], wP[64];  // d, P of positions i+1+q ([q]) and j-1-q ([32+q])
  unsigned char mapL[192], mapR[192];
};

// LDS layouts of the workgroup kinds, byte offsets from the start of the
// dynamic LDS.  The kernels carve their LDS with these and the launch size
// (fwd_lds_bytes) is the largest end among them, so the two cannot drift.
__host__ __device__ constexpr size_t lds_se(int n) { return lds_al((size_t)(n + 1) * 4); }  // E[0..n]
template <typename T>
struct WinLayout {  // window kind and the outside's recomputation of A
  static __host__ __device__ size_t stage(int n) { return lds_se(n); }
  static __host__ __device__ size_t blocks(int n) { return stage(n) + lds_al(sizeof(CellStage<T>)); }
  static __host__ __device__ size_t end(int n) { return blocks(n) + (size_t)CDZ_FWD_WBLK * 36 * sizeof(T); }
};
template <typename T>
struct BulLayout {  // bulge kind: exponents, stage, 32 bulge weights, blocks
  static __host__ __device__ size_t stage(int n) { return lds_se(n); }
  static __host__ __device__ size_t weights(int n) { return stage(n) + lds_al(sizeof(BulStage)); }
  static __host__ __device__ size_t blocks(int n) { return weights(n) + 32 * sizeof(T); }
  static __host__ __device__ size_t end(int n) { return blocks(n) + (size_t)CDZ_BUL_BLK * 36 * sizeof(T); }
};
template <typename T>
struct SplLayout {  // split kind: exponents, reduction scratch, 36 sums
  static __host__ __device__ size_t red(int n) { return lds_se(n); }
  static __host__ __device__ size_t out(int n) { return red(n) + (CDZ_NT / 64) * 36 * sizeof(T); }
  static __host__ __device__ size_t end(int n) { return out(n) + 36 * sizeof(T); }
};
template <typename T>
struct FinLayout {  // finish kind: 216 partial sums, stage
  static __host__ __device__ size_t stage(int) { return lds_al(216 * sizeof(T)); }
  static __host__ __device__ size_t end(int n) { return stage(n) + sizeof(FinStage<T>); }
};

template <typename T>
__device__ __forceinline__ void stage_block(T *dst, const T *A, long long ld, int r0, int c0, int dr,
                                            int dc, int q) {
  const int r = q / 6, c = q % 6;
  dst[q] = (r < dr && c < dc) ? A[(long long)(r0 + r) * ld + c0 + c] : T(0);
}

// positions i-1, i, i+1, j-1, j, j+1 (d = 0, P = 0 where absent), by threads 0..5
template <typename T>
__device__ __forceinline__ void load_positions(const DevProb<T> &D, int i, int j, int *d, int *P,
                                               signed char (*nt)[6]) {
  const int tid = threadIdx.x, n = D.n;
  if (tid < 6) {
    const int pos[6] = {i - 1, i, i + 1, j - 1, j, j + 1};
    const int p = pos[tid];
    const bool ok = p >= 0 && p < n;
    d[tid] = ok ? D.d[p] : 0;
    P[tid] = ok ? D.P[p] : 0;
    if (nt)
#pragma unroll
      for (int s = 0; s < 6; s++) nt[tid][s] = ok ? D.nt[p * 6 + s] : (signed char)-1;
  }
}
// window positions i+1+q ([q]) and j-1-q ([32+q]), q = 0..31, by threads 64..127
template <typename T>
__device__ __forceinline__ void load_window_positions(const DevProb<T> &D, int i, int j, int *wd, int *wP) {
  const int tid = threadIdx.x, n = D.n;
  if (tid >= 64 && tid < 128) {
    const int q = tid - 64;
    const int p = q < 32 ? i + 1 + q : j - 1 - (q - 32);
    const bool ok = p >= 0 && p < n;
    wd[q] = ok ? D.d[p] : 0;
    wP[q] = ok ? D.P[p] : 0;
  }
}

// ---- window: A(i,j,L) and F of the cells of diagonal dl (launch dl - 1)
template <typename T>
__device__ __forceinline__ void fwd_window(const DevProb<T> &D, int t, int dl, int blk) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int *sE = reinterpret_cast<int *>(smem_raw);  // [n + 1]
  CellStage<T> &C = *reinterpret_cast<CellStage<T> *>(smem_raw + WinLayout<T>::stage(D.n));
  T *W = reinterpret_cast<T *>(smem_raw + WinLayout<T>::blocks(D.n));
  const int n = D.n, tid = threadIdx.x, ncell = n - dl;
  const int i = cdz_cell_of_block(blk, ncell), j = i + dl;
  if (i >= ncell) return;
  const int Ed = exponent_ahead(D, t, dl);
  cdz_copy_exponents(sE, D.E, dl, dl, 34);  // the spans the window reads; E[dl] below
  load_positions(D, i, j, C.d, C.P, (signed char(*)[6]) nullptr);
  load_window_positions(D, i, j, C.wd, C.wP);
  if (tid >= 128 && tid < 164) {
    const int q = tid - 128;
    C.eI1[q] = i + 1 < n ? D.e[(i + 1) * 36 + q] : T(0);
    C.eJm2[q] = j >= 2 ? D.e[(j - 2) * 36 + q] : T(0);
    if (q < 6) {
      C.vI1[q] = i + 1 < n ? D.v[(i + 1) * 6 + q] : T(0);
      C.vJm1[q] = j >= 1 ? D.v[(j - 1) * 6 + q] : T(0);
    }
  } else if (tid >= 164 && tid < 164 + 31) {
    C.tab[TB_IN + tid - 164] = D.tab[TB_IN + tid - 164];
  }
  if (tid == 0) sE[dl] = Ed;
  cdz_sync();
  const int lmax = min(CDZ_MAXLOOP, dl - 6);
  a_window<T>(D, C, sE, W, i, j, dl, lmax, Ed);
  T *AC = W + 60 * 36 + 84 * 36;
  if (tid < 36) {
    const int a = tid / 6, dd = tid % 6;
    T f = 0;
    for (int L = 2; L <= lmax; L++) f += C.tab[TB_IN + L] * AC[(L - 2) * 36 + tid];
    if (a < C.d[2] && dd < C.d[3]) D.F[(long long)(C.P[2] + a) * D.ld + C.P[3] + dd] = f;
  }
  // keep A(i,j,L), L = 2..CDZ_NA+1, for the cells of diagonal dl + 2 and the
  // outside pass (zero where no inner pair fits)
  a_store<T>(D, C, i, lmax, AC);
}

// ---- bulges: G of the cells of diagonal dl (launch dl - 1).  Left bulge l:
//      run i+1..k-1, inner pair (k, j-1), k = i+1+l; right bulge l: inner pair
//      (i+1, l'), run l'+1..j-1, l' = j-1-l; l = 1..lmax.  The edge between
//      run and inner pair is folded into one side per term first (M below), so
//      each term is two 6x6x6 products.
template <typename T>
__device__ __forceinline__ void fwd_bulges(const DevProb<T> &D, int t, int dl, int blk) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int *sE = reinterpret_cast<int *>(smem_raw);  // [n + 1]
  BulStage &C = *reinterpret_cast<BulStage *>(smem_raw + BulLayout<T>::stage(D.n));
  T *tb = reinterpret_cast<T *>(smem_raw + BulLayout<T>::weights(D.n));  // bulge weights by length
  T *X = reinterpret_cast<T *>(smem_raw + BulLayout<T>::blocks(D.n));
  T *UR1 = X, *UC1 = X + 30 * 36, *EL = X + 60 * 36, *ER = X + 90 * 36, *QL = X + 120 * 36, *QR = X + 150 * 36;
  T *GP = UR1;  // 7 x 36 partial sums, after the products have used UR1
  const int n = D.n, tid = threadIdx.x, ncell = n - dl;
  const long long ld = D.ld;
  const int i = cdz_cell_of_block(blk, ncell), j = i + dl;
  if (i >= ncell) return;
  const int Ed = exponent_ahead(D, t, dl);
  const int lmax = min(CDZ_MAXLOOP, dl - 6);
  cdz_copy_exponents(sE, D.E, dl, dl, 34);  // the spans the bulges read
  load_positions(D, i, j, C.d, C.P, (signed char(*)[6]) nullptr);
  load_window_positions(D, i, j, C.wd, C.wP);
  if (tid >= 128 && tid < 128 + 31) tb[tid - 128] = D.tab[TB_BU + tid - 128];
  cdz_sync();
  const int d1 = C.d[2], dm = C.d[3], P1 = C.P[2], Pm = C.P[3];
  T g = 0;
  if (lmax >= 1) {
    const int *lp_d = C.wd, *lp_P = C.wP, *rp_d = C.wd + 32, *rp_P = C.wP + 32;
    cdz_window_maps(C.mapL, C.mapR, lp_d, lp_P, rp_d, rp_P, lmax);
    {  // clear the blocks the staging places values into (padding stays zero)
      uint4 *w4 = reinterpret_cast<uint4 *>(X);
      const int n4 = 180 * 36 * (int)sizeof(T) / 16;
      for (int idx = tid; idx < n4; idx += CDZ_NT) w4[idx] = make_uint4(0, 0, 0, 0);
    }
    cdz_sync();
    // one staging round: e blocks (contiguous in D.e), the two runs, the two
    // inner-pair strips, each a set of contiguous row segments placed by the
    // window maps
    cdz_copy_blocks<T>(EL, D.e + (long long)(i + 1) * 36, lmax, false);       // e_{i+l}
    cdz_copy_blocks<T>(ER, D.e + (long long)(j - 1 - lmax) * 36, lmax, true);  // e_{j-1-l}
    const int baseL = lp_P[0], baseR = rp_P[lmax];
    const int KU = lp_P[lmax] - baseL;                        // U[i+1][i+1..i+lmax]: row P1 + r of U
    const int endR = rp_P[0] + rp_d[0] - baseR;
    const int oC = rp_P[lmax - 1] - baseR, KC = endR - oC;    // U[j-lmax..j-1][j-1]: row Pm + c of Ut
    const int oq = lp_P[1] - baseL, KQ = lp_P[lmax + 1] - lp_P[1];  // Qb[i+2..i+1+lmax][j-1]: rows of Qbt
    const int KR = rp_P[1] + rp_d[1] - baseR;                 // Qb[i+1][j-1-lmax..j-2]: row P1 + r of Qb
    const int e1 = d1 * KU, e2 = e1 + dm * KC, e3 = e2 + dm * KQ, e4 = e3 + d1 * KR;
    cdz_stage_nv<3, T>(X, e4, [&](int idx, int &d) -> const T * {
      if (idx < e1) {  // U[i+1][i+l](r, c), block l - 1
        const int r = idx / KU, k = idx % KU, q = C.mapL[k], c = k - (lp_P[q] - baseL);
        d = q * 36 + r * 6 + c;
        return D.U + (long long)(P1 + r) * ld + baseL + k;
      }
      if (idx < e2) {  // U[j-l][j-1](r, c), block 30 + l - 1
        const int s = idx - e1, c = s / KC, k = s % KC + oC, q = C.mapR[k], r = k - (rp_P[q] - baseR);
        d = (30 + q) * 36 + r * 6 + c;
        return D.Ut + (long long)(Pm + c) * ld + baseR + k;
      }
      if (idx < e3) {  // Qb[i+1+l][j-1](x, c), block 120 + l - 1
        const int s = idx - e2, c = s / KQ, k = s % KQ + oq, l = C.mapL[k], x = k - (lp_P[l] - baseL);
        d = (120 + l - 1) * 36 + x * 6 + c;
        return D.Qbt + (long long)(Pm + c) * ld + baseL + k;
      }
      // Qb[i+1][j-1-l](r, c), block 150 + l - 1
      const int s = idx - e3, r = s / KR, k = s % KR, l = C.mapR[k], c = k - (rp_P[l] - baseR);
      d = (150 + l - 1) * 36 + r * 6 + c;
      return D.Qb + (long long)(P1 + r) * ld + baseR + k;
    });
    cdz_sync();
    // per term, in place: left M = e_{k-1} . Qb[k][j-1] (into EL), right
    // M = e_{l'} . U[l'+1][j-1] (into ER); a wave per term
    {
      const int lane = tid & 63, r = lane / 6, c = lane % 6;
      for (int b = cdz_wave_id(); b < 2 * lmax; b += CDZ_NT / 64) {
        const bool left = b < lmax;
        const int l = (left ? b : b - lmax) + 1;
        T *ek = (left ? EL : ER) + (l - 1) * 36;
        const T *o = left ? QL + (l - 1) * 36 : UC1 + (l - 1) * 36;
        T v = 0;
        if (lane < 36) {
#pragma unroll
          for (int x = 0; x < 6; x++) v += ek[r * 6 + x] * o[x * 6 + c];
        }
        cdz_wave_sync();
        if (lane < 36) ek[lane] = v;
      }
    }
    cdz_sync();
    // G(a, c) = sum_l f_l (sum_b U[i+1][i+l](a,b) M_l(b,c) + sum_y Qb[i+1][l'](a,y) M'_l(y,c));
    // thread (grp, q) sums the terms grp, grp + 7, .. of output q
    const int q = tid % 36, grp = tid / 36, a = q / 6, c = q % 6;
    if (grp < 7) {
      for (int term = grp; term < 2 * lmax; term += 7) {
        const bool left = term < lmax;
        const int l = (left ? term : term - lmax) + 1;
        const T f = tb[l] * cdz_p2<T>(sE[l - 1] + sE[dl - 2 - l] - Ed);
        const T *u = left ? UR1 + (l - 1) * 36 : QR + (l - 1) * 36;
        const T *mm = (left ? EL : ER) + (l - 1) * 36;
        T sm = 0;
#pragma unroll
        for (int b = 0; b < 6; b++) sm += u[a * 6 + b] * mm[b * 6 + c];
        g += f * sm;
      }
    }
    cdz_sync();  // UR1 is reused for the partial sums
    if (grp < 7) GP[grp * 36 + q] = g;
    cdz_sync();
    if (tid < 36) {
      g = 0;
#pragma unroll
      for (int gg = 0; gg < 7; gg++) g += GP[gg * 36 + tid];
    }
  }
  if (tid < 36) {
    const int a = tid / 6, c = tid % 6;
    if (a < d1 && c < dm) D.G[(long long)(P1 + a) * ld + Pm + c] = g;
  }
}

// ---- split: QmX[i][j] = sum_k Qm[i][k] f(k) Qm1Lt[j][k], k over the states of
//      positions i+4 .. j-5 (u - 1 = pos(k)), for the cells of diagonal dl
//      (launch dl - 4), stored as true * 2^-EX[dl]
template <typename T>
__device__ __forceinline__ void fwd_split(const DevProb<T> &D, int t, int dl, int blk) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int *sE = reinterpret_cast<int *>(smem_raw);  // [n + 1]
  T *red = reinterpret_cast<T *>(smem_raw + SplLayout<T>::red(D.n));
  T *out = reinterpret_cast<T *>(smem_raw + SplLayout<T>::out(D.n));
  const int n = D.n, tid = threadIdx.x, ncell = n - dl;
  const long long ld = D.ld;
  const int i = cdz_cell_of_block(blk, ncell), j = i + dl;
  if (i >= ncell) return;
  const int EX = exponent_ahead(D, t, dl);
  const int di = D.d[i], dj = D.d[j], Pi = D.P[i], Pj = D.P[j];
  const int K0 = D.P[i + 4], K1 = D.P[j - 4];
  cdz_copy_ints(sE, D.E, dl - 4);  // spans 0..dl-5
  cdz_sync();
  constexpr int UN = sizeof(T) == 4 ? 4 : 1;
  T acc[36];
#pragma unroll
  for (int r = 0; r < 36; r++) acc[r] = 0;
  for (int k0 = K0 + tid; k0 < K1; k0 += UN * CDZ_NT) {
    T a[UN][6], b[UN][6];
    int pp[UN];
#pragma unroll
    for (int u = 0; u < UN; u++) {
      const int k = k0 + u * CDZ_NT;
      const bool ok = k < K1;
      pp[u] = ok ? D.posOf[k] : i + 4;
#pragma unroll
      for (int s = 0; s < 6; s++) a[u][s] = (ok && s < di) ? D.Qm[(Pi + s) * ld + k] : T(0);
#pragma unroll
      for (int c = 0; c < 6; c++) b[u][c] = (ok && c < dj) ? D.Qm1Lt[(Pj + c) * ld + k] : T(0);
    }
#pragma unroll
    for (int u = 0; u < UN; u++) {
      const T f = cdz_p2<T>(sE[pp[u] - i] + sE[j - pp[u] - 1] - EX);
#pragma unroll
      for (int s = 0; s < 6; s++) {
        const T as = a[u][s] * f;
#pragma unroll
        for (int c = 0; c < 6; c++) acc[s * 6 + c] = fma(as, b[u][c], acc[s * 6 + c]);
      }
    }
  }
  cdz_block_sum<T, 36>(acc, red, out);
  if (tid < 36) {
    const int s = tid / 6, c = tid % 6;
    if (s < di && c < dj) D.QmX[(long long)(Pi + s) * ld + Pj + c] = out[tid];
  }
}

// ---- finish: the O(1) recurrences of the cells of diagonal dl (launch dl)
template <typename T>
__device__ __forceinline__ void fwd_finish(const DevProb<T> &D, int dl, int blk) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *red = reinterpret_cast<T *>(smem_raw);  // 216 partial sums
  FinStage<T> &C = *reinterpret_cast<FinStage<T> *>(smem_raw + FinLayout<T>::stage(D.n));
  const int n = D.n, tid = threadIdx.x, ncell = n - dl;
  const long long ld = D.ld;
  const int i = cdz_cell_of_block(blk, ncell), j = i + dl;
  if (i >= ncell) return;
  const int Ed = D.E[dl];
  const int E1 = dl >= 1 ? D.E[dl - 1] : 0, E2 = dl >= 2 ? D.E[dl - 2] : 0;
  const int EXd = dl >= 9 ? D.EX[dl] : 0;
  const T hp = dl >= 4 ? D.Bhp[dl - 1] : T(0);
  // round 1: positions, tables, edge and vertex factors (indexed by position)
  load_positions(D, i, j, C.d, C.P, C.nt);
  for (int q = tid; q < TB_LEN; q += CDZ_NT) C.tab[q] = D.tab[q];
  if (tid >= 32 && tid < 32 + 144) {
    const int w = (tid - 32) / 36, q = (tid - 32) % 36;
    const int p = w == 0 ? i - 1 : w == 1 ? i : w == 2 ? j - 1 : j;
    T *dst = w == 0 ? C.eIm1 : w == 1 ? C.eI : w == 2 ? C.eJm1 : C.eJ;
    dst[q] = (p >= 0 && p < n) ? D.e[p * 36 + q] : T(0);
  } else if (tid >= 176 && tid < 188) {
    const int q = tid - 176;
    if (q < 6) C.vI[q] = D.v[i * 6 + q];
    else C.vJ[q - 6] = D.v[j * 6 + q - 6];
  }
  cdz_sync();
  const int di = C.d[1], dj = C.d[4], Pi = C.P[1], Pj = C.P[4];
  const int d1 = C.d[2], dm = C.d[3], P1 = C.P[2], Pm = C.P[3];
  // round 2: the blocks of the cell's neighbours and its loop and split sums
  for (int idx = tid; idx < 9 * 36; idx += CDZ_NT) {
    const int g = idx / 36, q = idx % 36;
    switch (g) {
      case 0: if (dl >= 2) stage_block(C.Uin, D.U, ld, P1, Pm, d1, dm, q); else C.Uin[q] = 0; break;
      case 1: if (dl >= 2) stage_block(C.Xin, D.QmX, ld, P1, Pm, d1, dm, q); else C.Xin[q] = 0; break;
      case 2: if (dl >= 2) stage_block(C.Bin, D.Qb, ld, P1, Pm, d1, dm, q); else C.Bin[q] = 0; break;
      case 3: if (dl >= 1) stage_block(C.M1l, D.Qm1, ld, Pi, Pm, di, dm, q); else C.M1l[q] = 0; break;
      case 4: if (dl >= 1) stage_block(C.M1pr, D.Qm1p, ld, P1, Pj, d1, dj, q); else C.M1pr[q] = 0; break;
      case 5: if (dl >= 1) stage_block(C.Ul, D.U, ld, Pi, Pm, di, dm, q); else C.Ul[q] = 0; break;
      case 6: if (dl >= 4) stage_block(C.G, D.G, ld, P1, Pm, d1, dm, q); else C.G[q] = 0; break;
      case 7: if (dl >= 4) stage_block(C.F, D.F, ld, P1, Pm, d1, dm, q); else C.F[q] = 0; break;
      case 8: if (dl >= 9) stage_block(C.X, D.QmX, ld, Pi, Pj, di, dj, q); else C.X[q] = 0; break;
      default: break;
    }
  }
  cdz_sync();
  float vmax = 0.f;
  const T *tab = C.tab;
  // ---- unpaired run U[i][j]; Qb partial sums: thread (a, o) takes the terms
  //      of output o = (s, s2) whose slot at i+1 is a
  if (tid < 36) {
    const int s = tid / 6, c = tid % 6;
    if (s < di && c < dj) {
      T u = 0;
      if (dl == 0) {
        u = (s == c) ? C.vI[s] : T(0);
      } else {
        T a = 0;
#pragma unroll
        for (int x = 0; x < 6; x++) a += C.Ul[s * 6 + x] * C.eJm1[x * 6 + c];
        u = a * C.vJ[c] * cdz_p2<T>(E1 - Ed);
      }
      D.U[(Pi + s) * ld + Pj + c] = u;
      D.Ut[(Pj + c) * ld + Pi + s] = u;
      vmax = fmaxf(vmax, (float)fabs(u));
      if (dl < 4) {
        const long long o = (Pi + s) * ld + Pj + c;
        D.Qb[o] = 0;
        D.Qbt[(Pj + c) * ld + Pi + s] = 0;
        D.Qm1[o] = 0;
        D.Qm1p[o] = 0;
        D.QmX[o] = 0;
        D.Qm[o] = 0;
        D.Qmt[(Pj + c) * ld + Pi + s] = 0;
      }
    }
  }
  if (dl >= 4) {
    if (tid < 216) {
      const int a = tid / 36, o = tid % 36, s = o / 6, s2 = o % 6;
      T part = 0;
      if (s < di && s2 < dj && a < d1) {
        const int ty = cdz_ptype(C.nt[1][s], C.nt[4][s2]);
        if (ty >= 0) {
          const int na = C.nt[2][a];
          const T ea = C.eI[s * 6 + a];
          T acc = 0, hpa = 0, st = 0, ml = 0;
#pragma unroll
          for (int b = 0; b < 6; b++) {
            if (b >= dm) continue;
            const int nb = C.nt[3][b];
            const T w = ea * C.eJm1[b * 6 + s2];
            const T mmo = tab[TB_MM + na * 24 + nb * 6 + ty];
            const int o2 = a * 6 + b;
            hpa += w * C.Uin[o2] * mmo;
            acc += w * (C.G[o2] + C.F[o2] * mmo);
            ml += w * C.Xin[o2];
            const int t2 = cdz_ptype(na, nb);
            if (dl - 2 >= 4 && t2 >= 0) st += w * C.Bin[o2] * tab[TB_ST + ty * 6 + t2];
          }
          part = acc + (hpa * hp + st + ml * tab[TB_MLAB]) * cdz_p2<T>(E2 - Ed);
        }
      }
      red[a * 36 + o] = part;
    }
    cdz_sync();
    if (tid < 36) {
      const int s = tid / 6, s2 = tid % 6;
      T qb = 0, q1 = 0;
      if (s < di && s2 < dj) {
        T acc = 0;
#pragma unroll
        for (int a = 0; a < 6; a++) acc += red[a * 36 + tid];
        qb = C.vI[s] * C.vJ[s2] * acc;
        D.Qb[(Pi + s) * ld + Pj + s2] = qb;
        D.Qbt[(Pj + s2) * ld + Pi + s] = qb;
        vmax = fmaxf(vmax, (float)fabs(qb));
        T a = 0;
#pragma unroll
        for (int x = 0; x < 6; x++) a += C.M1l[s * 6 + x] * C.eJm1[x * 6 + s2];
        q1 = a * C.vJ[s2] * tab[TB_MLC] * cdz_p2<T>(E1 - Ed) + qb * tab[TB_MLB];
        D.Qm1[(Pi + s) * ld + Pj + s2] = q1;
        vmax = fmaxf(vmax, (float)fabs(q1));
      }
      C.qb[tid] = qb;
      C.qm1[tid] = q1;
    }
    cdz_sync();
    // ---- DI (Qb dressed as an interior loop's inner pair), thread (x, o)
    //      summing over the slot y of j for output o = (b, c)
    const bool hasDI = i >= 1 && j + 1 < n;
    if (hasDI && tid < 216) {
      const int x = tid / 36, o = tid % 36, b = o / 6, c = o % 6;
      T part = 0;
      if (x < di && b < C.d[0] && c < C.d[5]) {
        const int nb = C.nt[0][b], nc = C.nt[5][c];
        const T eb = C.eIm1[b * 6 + x];
#pragma unroll
        for (int y = 0; y < 6; y++) {
          const T q = C.qb[x * 6 + y];
          const int t2 = cdz_ptype(C.nt[4][y], C.nt[1][x]);
          if (q != T(0) && t2 >= 0) part += eb * q * C.eJ[y * 6 + c] * tab[TB_MM + nc * 24 + nb * 6 + t2];
        }
      }
      red[x * 36 + o] = part;
    }
    cdz_sync();
    // ---- DI, Qm1L, Qm1p, QmX (split sum converted to E[dl]), Qm
    if (tid < 36) {
      const int s = tid / 6, s2 = tid % 6;
      if (hasDI && s < C.d[0] && s2 < C.d[5]) {
        T a = 0;
#pragma unroll
        for (int x = 0; x < 6; x++) a += red[x * 36 + tid];
        D.DI[(C.P[0] + s) * ld + C.P[5] + s2] = a;
        D.DIt[(C.P[5] + s2) * ld + C.P[0] + s] = a;
      }
      if (i >= 1 && s < C.d[0] && s2 < dj) {
        T a = 0;
#pragma unroll
        for (int x = 0; x < 6; x++) a += C.eIm1[s * 6 + x] * C.qm1[x * 6 + s2];
        D.Qm1Lr[(C.P[0] + s) * ld + Pj + s2] = a;
        D.Qm1Lt[(Pj + s2) * ld + C.P[0] + s] = a;
      }
      if (s < di && s2 < dj) {
        T a = 0;
#pragma unroll
        for (int x = 0; x < 6; x++) a += C.eI[s * 6 + x] * C.M1pr[x * 6 + s2];
        const T qp = C.qm1[tid] + tab[TB_MLC] * C.vI[s] * cdz_p2<T>(E1 - Ed) * a;
        const T qx = dl >= 9 ? C.X[tid] * cdz_p2<T>(EXd - Ed) : T(0);
        const T qm = qx + qp;
        const long long o = (Pi + s) * ld + Pj + s2;
        D.Qm1p[o] = qp;
        D.QmX[o] = qx;
        D.Qm[o] = qm;
        D.Qmt[(Pj + s2) * ld + Pi + s] = qm;
        vmax = fmaxf(vmax, fmaxf((float)fabs(qp), (float)fabs(qm)));
      }
    }
  }
  // ---- per-diagonal maximum for the exponents of later diagonals
  if (tid < 64) {
    vmax = fminf(cdz_wave_max(vmax), 3.0e38f);
    if (tid == 0 && vmax > 0.f) atomicMax(&D.maxb[dl], __float_as_uint(vmax));
  }
}

// One workgroup of launch t; w is its index among this problem's workgroups.
// Split (FUSED false): the kinds' blocks are numbered one kind after the
// other and the workgroup runs one of them.  Fused: it runs block w of every
// kind that has one, in turn (LDS is reused, hence the barriers).  The two
// are separate kernels, so each holds one copy of every kind.
template <typename T, bool FUSED>
__device__ __forceinline__ void fwd_block(const DevProb<T> &D, int t, int w) {
  int r[4], wk[4];
  fwd_ranges(D.n, t, r);
  int base = 0;
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int x = FUSED ? w : w - base;
    wk[k] = x >= 0 && x < r[k] ? x : -1;
    base += r[k];
  }
  if (wk[0] >= 0) {
    fwd_window<T>(D, t, t + 1, wk[0]);
    if (FUSED) __syncthreads();
    else return;
  }
  if (wk[1] >= 0) {
    fwd_bulges<T>(D, t, t + 1, wk[1]);
    if (FUSED) __syncthreads();
    else return;
  }
  if (wk[2] >= 0) {
    fwd_split<T>(D, t, t + 4, wk[2]);
    if (FUSED) __syncthreads();
    else return;
  }
  if (wk[3] >= 0) {
    if (wk[3] == 0 && threadIdx.x == 0) {  // the exponents chosen in this launch
      if (t + 1 <= D.n) D.E[t + 1] = exponent_ahead(D, t, t + 1);
      D.EX[t + 4] = exponent_ahead(D, t, t + 4);
    }
    fwd_finish<T>(D, t, wk[3]);
  }
}

// dynamic LDS of a forward launch: the largest of its workgroup kinds
template <typename T>
size_t fwd_lds_bytes(int n) {
  return std::max(std::max(WinLayout<T>::end(n), BulLayout<T>::end(n)),
                  std::max(SplLayout<T>::end(n), FinLayout<T>::end(n)));
}
template size_t fwd_lds_bytes<float>(int);
template size_t fwd_lds_bytes<double>(int);

// ---------------------------------------------------------------------------
// FP64 exterior loops, after the diagonal launches, as two scans over
// positions (eq. complex-logq: the exterior loop sums the pairs that close
// it, with nothing between them):
//   prefix   Z5[j](t) = Z5[j-1] e_{j-1} v_j (t)                 j unpaired
//                     + sum_{k>=1} 2^(..) A[k] Qb[k][j](., t)    k pairs j
//                     + 2^(..) sum_x Qb[0][j](x, t)              0 pairs j
//            A[k] = Z5[k-1] e_{k-1};  log Z = ln sum_t Z5[n-1](t)
//   suffix   Z3[p](s) = sum_x e_p(s, x) w(x),
//            w(x) = v_{p+1}(x) Z3[p+1](x) + sum_jj 2^(..) Qb[p+1][jj](x, .) Z3[jj]
// Each step reads pairs of every span up to the step's position, so it runs
// once every diagonal is final.  One workgroup per direction: the pair items
// of a step are spread over its threads and summed, thread 0 renormalises
// (Z5[j] = true 2^-G5[j] with the largest entry in [1, 2), likewise Z3/H3).
// Pairs are limited to spans <= W (the truncated pass of the FP32 landscape
// estimate); the prefix stops after position jend.
// ---------------------------------------------------------------------------
// Both recurrences are sequential in the position; each step's pair terms
// (up to W of them) are spread over the CDZ_SCAN_NT threads, one pair per
// thread at the workload sizes.  None of a step's loads depends on the
// previous step: in FP32 the block of Qb and the A[k] (or Z3[jj]) of a
// thread's first pair of step j + 1 are issued as soon as the thread has used
// those of step j, so they arrive while the workgroup sums step j (the vectors
// read were stored at least three steps, and barriers, earlier), and a step
// costs about one workgroup sum; FP64 loads them in the step.  The per-step factors v and e are fetched a step ahead
// by the threads that use them, and every thread derives the step's exponent
// from the sums, so no extra barrier orders it.
template <typename T>
__device__ __forceinline__ void exterior_scan_body(const DevProb<T> &D, int W, int jend, int dir) {
  constexpr int NT = CDZ_SCAN_NT;
  // FP32 only: the 72 registers of an FP64 block would spill at 1024 threads
  constexpr bool PRE = sizeof(T) == 4;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = D.n, tid = threadIdx.x;
  int *sE = reinterpret_cast<int *>(smem_raw);  // [n + 1] diagonal exponents
  int *sd = sE + (n + 1), *sP = sd + (n + 1);   // [n + 1] slot counts and offsets
  int *sX = sP + (n + 1);                       // [n + 1] G5 (prefix) or H3 (suffix)
  double *red = reinterpret_cast<double *>(smem_raw + lds_al((size_t)4 * (n + 1) * 4));  // [NT/64][6]
  double *tot = red + (NT / 64) * 6;                                                      // [6]
  const long long ld = D.ld;
  for (int k = tid; k <= n; k += NT) {
    sE[k] = D.E[k];
    sd[k] = k < n ? D.d[k] : 0;
    sP[k] = D.P[k];
  }
  __syncthreads();
  const double L2 = 0.6931471805599453094;
  // exponent of the largest of six sums (0 for all zero or non-finite)
  auto step_exponent = [&](int cnt) __attribute__((always_inline)) {
    double mx = 0;
#pragma unroll
    for (int t = 0; t < 6; t++)
      if (t < cnt) mx = fmax(mx, fabs(tot[t]));
    return (mx > 0 && isfinite(mx)) ? ilogb(mx) : 0;
  };
  if (dir == 0) {
    // thread x < 6: column x of e_j, v_j(x) and A[j](x)
    double ecol[6] = {0, 0, 0, 0, 0, 0}, vx = 0, ax = 0;
    if (tid < 6) {
      vx = D.vd[tid];
#pragma unroll
      for (int q = 0; q < 6; q++) ecol[q] = D.ed[q * 6 + tid];
    }
    int R = 0;  // exponent of Z5[j-1]
    // this thread's first pair (k, j) of step j, k = max(0, j - W) + tid:
    // Qb(k, j) and A[k], zero outside the slots
    T fq[6][6];
    double fa[6];
    auto issue_first = [&](int jj) __attribute__((always_inline)) {
      const int k0 = jj - W > 0 ? jj - W : 0, nk = jj - 4 - k0 + 1;
      if (jj < 4 || jj > jend || tid >= nk) return;
      const int k = k0 + tid, dk = sd[k], Pk = sP[k], dq = sd[jj], Pq = sP[jj];
#pragma unroll
      for (int x = 0; x < 6; x++) fa[x] = (k >= 1 && x < dk) ? D.A5[k * 6 + x] : 0.0;
#pragma unroll
      for (int t = 0; t < 6; t++)
#pragma unroll
        for (int x = 0; x < 6; x++)
          fq[x][t] = (t < dq && x < dk) ? D.Qbt[(long long)(Pq + t) * ld + Pk + x] : T(0);
    };
    if (PRE) issue_first(4);
    for (int j = 0; j <= jend; j++) {
      const int dj = sd[j], Pj = sP[j];
      double enx[6] = {0, 0, 0, 0, 0, 0}, vnx = 0;
      if (tid < 6 && j + 1 < n) {
        vnx = D.vd[(j + 1) * 6 + tid];
#pragma unroll
        for (int q = 0; q < 6; q++) enx[q] = D.ed[(j + 1) * 36 + q * 6 + tid];
      }
      double part[6] = {0, 0, 0, 0, 0, 0};
      // position j unpaired: A[j](x) v_j(x) (A[0] = 1)
      const double own = j == 0 ? vx : ax * vx;
#pragma unroll
      for (int x = 0; x < 6; x++)
        if (x == tid && x < dj) part[x] = own;
      if (j >= 4) {  // j paired with k: A[k] Qb(k, j), Qb read along rows of Qbt
        const int k0 = j - W > 0 ? j - W : 0, nk = j - 4 - k0 + 1;
        if (PRE && tid < nk) {  // the first pair, loaded a step ahead
          const int k = k0 + tid, dk = sd[k];
          double a[6];
          if (k == 0) {
            const double sc = ldexp(1.0, sE[j] - R);
#pragma unroll
            for (int x = 0; x < 6; x++) a[x] = sc;
          } else {
            const double sc = ldexp(1.0, sX[k - 1] + sE[j - k] - R);
#pragma unroll
            for (int x = 0; x < 6; x++) a[x] = fa[x] * sc;
          }
#pragma unroll
          for (int t = 0; t < 6; t++) {
            if (t >= dj) break;
            double sm = 0;
#pragma unroll
            for (int x = 0; x < 6; x++)
              if (x < dk) sm += a[x] * (double)fq[x][t];
            part[t] += sm;
          }
        }
        for (int it = PRE ? tid + NT : tid; it < nk; it += NT) {
          const int k = k0 + it, dk = sd[k], Pk = sP[k];
          double a[6];
          if (k == 0) {
            const double sc = ldexp(1.0, sE[j] - R);
#pragma unroll
            for (int x = 0; x < 6; x++) a[x] = sc;
          } else {
            const double sc = ldexp(1.0, sX[k - 1] + sE[j - k] - R);
#pragma unroll
            for (int x = 0; x < 6; x++) a[x] = D.A5[k * 6 + x] * sc;
          }
#pragma unroll
          for (int t = 0; t < 6; t++) {
            if (t >= dj) break;
            double sm = 0;
#pragma unroll
            for (int x = 0; x < 6; x++)
              if (x < dk) sm += a[x] * (double)D.Qbt[(long long)(Pj + t) * ld + Pk + x];
            part[t] += sm;
          }
        }
      }
      if (PRE) issue_first(j + 1);
      // the full first barrier makes the A[.] stored a step earlier visible
      cdz_block_sum<double, 6, NT, true>(part, red, tot);
      const int e = step_exponent(dj);
      R += e;
      if (tid == 0) {
        sX[j] = R;
        D.G5[j] = R;
      }
      if (tid < 6) {
        double z[6];
#pragma unroll
        for (int q = 0; q < 6; q++) z[q] = q < dj ? ldexp(tot[q], -e) : 0.0;
        double zt = 0;
#pragma unroll
        for (int q = 0; q < 6; q++)
          if (q == tid) zt = z[q];
        D.Z5[j * 6 + tid] = zt;
        if (j + 1 < n) {  // A[j+1](x) = sum_q Z5[j](q) e_j(q, x)
          double acc = 0;
#pragma unroll
          for (int q = 0; q < 6; q++) acc += z[q] * ecol[q];
          ax = acc;
          D.A5[(j + 1) * 6 + tid] = acc;
        }
#pragma unroll
        for (int q = 0; q < 6; q++) ecol[q] = enx[q];
        vx = vnx;
      }
    }
    __syncthreads();
    if (tid == 0 && jend == n - 1) {
      double z5 = 0;
      for (int t = 0; t < 6; t++) z5 += D.Z5[(n - 1) * 6 + t];
      const double lz5 = log(z5) + sX[n - 1] * L2;
      D.res[0] = lz5;
      D.res[2] = rint(lz5 / L2);  // EZ, the adjoint scale exponent
    }
    return;
  }
  // ---- suffix.  Thread s < 6: row s of e_p, v_{p+1}(s) and Z3[p+1](s).
  double erow[6] = {0, 0, 0, 0, 0, 0}, vs = 0, zs = 0;
  const int dlast = sd[n - 1];
  if (tid < 6) {
    zs = tid < dlast ? 1.0 : 0.0;
    D.Z3[(n - 1) * 6 + tid] = zs;
    vs = D.vd[(n - 1) * 6 + tid];
    if (n >= 2) {
#pragma unroll
      for (int x = 0; x < 6; x++) erow[x] = D.ed[(n - 2) * 36 + tid * 6 + x];
    }
  }
  if (tid == 0) {
    sX[n - 1] = 0;
    D.H3[n - 1] = 0;
  }
  int R = 0;  // exponent of Z3[p+1]
  // this thread's first pair (p+1, jj) of step p, jj = p + 5 + tid: Qb(p+1, jj)
  // and Z3[jj], zero outside the slots
  T fq[6][6];
  double fz[6];
  auto issue_first = [&](int pp) __attribute__((always_inline)) {
    const int j1 = pp + 1 + W < n - 1 ? pp + 1 + W : n - 1, nj = j1 - (pp + 5) + 1;
    if (pp < 0 || tid >= nj) return;
    const int jj = pp + 5 + tid, dq = sd[jj], Pq = sP[jj], d1 = sd[pp + 1], P1 = sP[pp + 1];
#pragma unroll
    for (int t = 0; t < 6; t++) fz[t] = t < dq ? D.Z3[jj * 6 + t] : 0.0;
#pragma unroll
    for (int x = 0; x < 6; x++)
#pragma unroll
      for (int t = 0; t < 6; t++)
        fq[x][t] = (x < d1 && t < dq) ? D.Qb[(long long)(P1 + x) * ld + Pq + t] : T(0);
  };
  if (PRE) issue_first(n - 2);
  for (int p = n - 2; p >= 0; p--) {
    const int dp = sd[p], d1 = sd[p + 1], P1 = sP[p + 1];
    double enx[6] = {0, 0, 0, 0, 0, 0}, vnx = 0;
    if (tid < 6) {
      vnx = D.vd[p * 6 + tid];
      if (p >= 1) {
#pragma unroll
        for (int x = 0; x < 6; x++) enx[x] = D.ed[(p - 1) * 36 + tid * 6 + x];
      }
    }
    // w(x) over the slots x of position p+1: p+1 unpaired, or paired with jj
    double w[6] = {0, 0, 0, 0, 0, 0};
    const double own = vs * zs;
#pragma unroll
    for (int x = 0; x < 6; x++)
      if (x == tid && x < d1) w[x] = own;
    const int j1 = p + 1 + W < n - 1 ? p + 1 + W : n - 1, nj = j1 - (p + 5) + 1;
    if (PRE && tid < nj) {  // the first pair, loaded a step ahead
      const int jj = p + 5 + tid, dq = sd[jj];
      const double sc = ldexp(1.0, sE[jj - p - 1] + sX[jj] - R);
      double z3[6];
#pragma unroll
      for (int t = 0; t < 6; t++) z3[t] = fz[t] * sc;
#pragma unroll
      for (int x = 0; x < 6; x++) {
        if (x >= d1) break;
        double sm = 0;
#pragma unroll
        for (int t = 0; t < 6; t++)
          if (t < dq) sm += (double)fq[x][t] * z3[t];
        w[x] += sm;
      }
    }
    if (PRE) issue_first(p - 1);
    for (int it = PRE ? tid + NT : tid; it < nj; it += NT) {
      const int jj = p + 5 + it, dq = sd[jj], Pq = sP[jj];
      const double sc = ldexp(1.0, sE[jj - p - 1] + sX[jj] - R);
      double z3[6];
#pragma unroll
      for (int t = 0; t < 6; t++) z3[t] = D.Z3[jj * 6 + t] * sc;
#pragma unroll
      for (int x = 0; x < 6; x++) {
        if (x >= d1) break;
        double sm = 0;
#pragma unroll
        for (int t = 0; t < 6; t++)
          if (t < dq) sm += (double)D.Qb[(long long)(P1 + x) * ld + Pq + t] * z3[t];
        w[x] += sm;
      }
    }
    cdz_block_sum<double, 6, NT, true>(w, red, tot);
    // Z3[p](s) = sum_x e_p(s, x) w(x): every thread forms all six for the exponent
    double mx = 0, zown = 0;
    if (tid < 64) {  // the first wavefront: lane s < 6 holds row s
      double z = 0;
#pragma unroll
      for (int x = 0; x < 6; x++) z += erow[x] * tot[x];
      z = tid < dp ? z : 0.0;
      zown = z;
      mx = fabs(z);
#pragma unroll
      for (int off = 4; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
      if (tid == 0) red[0] = mx;  // published for the other wavefronts below
    }
    __syncthreads();
    mx = red[0];
    const int e = (mx > 0 && isfinite(mx)) ? ilogb(mx) : 0;
    R += e;
    if (tid == 0) {
      sX[p] = R;
      D.H3[p] = R;
    }
    if (tid < 6) {
      zs = ldexp(zown, -e);
      D.Z3[p * 6 + tid] = zs;
#pragma unroll
      for (int x = 0; x < 6; x++) erow[x] = enx[x];
      vs = vnx;
    }
  }
  __syncthreads();
  // total from the suffix: position 0 unpaired, or 0 pairs jj
  {
    double part[6] = {0, 0, 0, 0, 0, 0};
    if (tid == 0)
      for (int s = 0; s < 6; s++) part[0] += D.vd[s] * D.Z3[s];
    const int d0 = sd[0];
    for (int jj = 4 + tid; jj < n; jj += NT) {
      const int dq = sd[jj], Pq = sP[jj];
      double a = 0;
      for (int x = 0; x < d0; x++)
        for (int t = 0; t < dq; t++) a += (double)D.Qb[(long long)x * ld + Pq + t] * D.Z3[jj * 6 + t];
      part[0] += a * ldexp(1.0, sE[jj] + sX[jj] - sX[0]);
    }
    cdz_block_sum<double, 6, NT, true>(part, red, tot);
    if (tid == 0) D.res[1] = log(tot[0]) + sX[0] * L2;
  }
}

// ---- FP32: the free-energy landscape of the sequence ---------------------
// With C[p] = round(log2 Z5[p]) (prefix exterior partition function, C[-1]
// = 0), multiplying every vertex factor v_p by 2^-(C[p] - C[p-1]) multiplies
// every quantity over a span [a..b] by the exact power of two
// 2^-(C[b] - C[a-1]).  Cells of one diagonal then stay within a few octaves
// of each other, even where strong and weak regions of the sequence differ
// by more than 2^120 (beyond the FP32 range); probabilities do not change
// and log Z is restored exactly from sum_p (C[p] - C[p-1]) = C[n-1].
//
// The landscape is estimated before the exact pass from a truncated one:
// the dynamic program over spans <= W only, then the exterior prefix with
// pairs of span <= W (cdz_exterior_trunc).  Any landscape gives exact
// results; its quality only decides how far cells spread, which
// cdz_spread_check verifies after the exact pass.

// Z5[j], j = W..n-1, from pairs (k, j) with j - k <= W (Z5[0..W-1] are the
// exact values of the truncated pass).  One workgroup, positions in turn.
// One wavefront (64 lanes, no workgroup barriers) steps the truncated exterior
// prefix through j = W..n-1:
//   Z5[j] = A[j] v_j  +  sum_{k = max(0, j-W)}^{j-4} 2^(..) A[k] Qb[k][j],
//   A[k] = Z5[k-1] e_{k-1}  (A[0] = the unit row),
// lanes take the pair items k of a step, a butterfly of lane exchanges sums
// them, lane 0 renormalises, and lanes 0..5 form A[j+1] once Z5[j] is known
// (each A is used by up to W steps).  Qb[k][j] is read from Qbt, where the
// items of a step lie along one row.
template <typename T>
__device__ __forceinline__ void exterior_trunc_body(const DevProb<T> &D, int W) {
  // the recurrence reaches back at most W + 1 positions: Z5, G5, A, d and P
  // of positions j - W - 1 .. j live in an LDS ring, the exponents E[0..W]
  // too, so each step waits on LDS rather than on global memory.  The ring
  // holds 64 positions more, and the new Z5, G5 go to global memory 64
  // positions at a time (a store in every step would hold up the next step's
  // loads, which complete in order behind it).
  constexpr int RMAX = CDZ_SPAN_MAX + 2 + 64;
  __shared__ double zr[RMAX * 6], ar[RMAX * 6];
  __shared__ int gr[RMAX], dr[RMAX], Pr[RMAX], sE[CDZ_SPAN_MAX + 1];
  const int n = D.n, lane = threadIdx.x, R = W + 2 + 64;
  const long long ld = D.ld;
  int flushed = W;  // positions W.. not yet written to D.Z5 / D.G5
  if (W > CDZ_SPAN_MAX) {
    if (lane == 0) D.res[0] = NAN;  // caller error: log Z reports it
    return;
  }
  for (int k = lane; k <= W && k < n; k += 64) {
#pragma unroll
    for (int q = 0; q < 6; q++) zr[(k % R) * 6 + q] = D.Z5[k * 6 + q];
    gr[k % R] = D.G5[k];
    dr[k % R] = D.d[k];
    Pr[k % R] = D.P[k];
    sE[k] = D.E[k];
  }
  cdz_wave_sync();
  for (int k = 1 + lane; k <= W && k < n; k += 64) {  // A of positions 1..W
#pragma unroll
    for (int x = 0; x < 6; x++) {
      double a = 0;
#pragma unroll
      for (int q = 0; q < 6; q++) a += zr[((k - 1) % R) * 6 + q] * D.ed[(k - 1) * 36 + q * 6 + x];
      ar[(k % R) * 6 + x] = a;
    }
  }
  cdz_wave_sync();
  // The global operands of a step do not depend on the recurrence: those of
  // step j + 1 (the Qb of this lane's first item, v_{j+1}, e_{j+1}) are
  // issued at the start of step j into the other of two operand sets and
  // waited on at j + 1; d and P enter the ring 64 positions ahead of the
  // steps (slot p % R of position p is free once step p - R + W + 1 has
  // passed, as R = W + 66).  The items k of step jj
  // are k0 .. jj - 4, k0 = max(0, jj - W); the loads of a lane without an
  // item, or outside the item's states, read a valid element in its place
  // and are masked where they are used.
  struct Ops {
    T q[6][6];
    int dk, ok;
    double v, e[6];
  };
  auto load_qb = [&](T(&q)[6][6], int Pj, int dj, int k) __attribute__((always_inline)) {
    const int dk = dr[k % R], Pk = Pr[k % R];
#pragma unroll
    for (int t = 0; t < 6; t++)
#pragma unroll
      for (int x = 0; x < 6; x++) {
        const int tc = t < dj ? t : dj - 1, xc = x < dk ? x : dk - 1;
        q[x][t] = D.Qbt[(Pj + tc) * ld + Pk + xc];
      }
  };
  auto issue = [&](int jj, int djj, int Pjj, Ops &o) __attribute__((always_inline)) {
    const int k0 = jj - W > 0 ? jj - W : 0, k = k0 + lane;
    o.ok = k <= jj - 4;
    const int kc = o.ok ? k : k0;
    o.dk = o.ok ? dr[kc % R] : 0;
    load_qb(o.q, Pjj, djj, kc);
    const int ls = lane < 6 ? lane : 0;
    o.v = D.vd[jj * 6 + ls];
#pragma unroll
    for (int c = 0; c < 6; c++) o.e[c] = D.ed[jj * 36 + c * 6 + ls];
  };
  auto step = [&](int j, const Ops &cur, Ops &nxt) __attribute__((always_inline)) {
    const int sj = j % R, sm1 = (j - 1) % R;
    if ((j - W) % 64 == 0) {  // d, P of positions j + 1 .. j + 64 into the ring
      const int p = j + 1 + lane;
      if (p < n) {
        dr[p % R] = D.d[p];
        Pr[p % R] = D.P[p];
      }
      cdz_wave_sync();
    }
    const int G = gr[sm1], dj = dr[sj];
    // every step issues the same loads (the count of loads in flight stays
    // fixed); the last one loads a set for position n - 1 that is not used
    const int jn = j + 1 < n ? j + 1 : j;
    issue(jn, dr[jn % R], Pr[jn % R], nxt);
    double part[6] = {0, 0, 0, 0, 0, 0};
    const int k0 = j - W > 0 ? j - W : 0;  // first pair start
    const int nk = j - 4 - k0 + 1 > 0 ? j - 4 - k0 + 1 : 0;  // pair items k = k0..j-4
    auto add_item = [&](int k, int dk, const T(&q)[6][6]) __attribute__((always_inline)) {
      double a[6];
      if (k == 0) {
        const double sc = ldexp(1.0, sE[j] - G);
#pragma unroll
        for (int x = 0; x < 6; x++) a[x] = sc;
      } else {
        const double sc = ldexp(1.0, gr[(k - 1) % R] + sE[j - k] - G);
#pragma unroll
        for (int x = 0; x < 6; x++) a[x] = ar[(k % R) * 6 + x] * sc;
      }
#pragma unroll
      for (int x = 0; x < 6; x++) {
        if (x >= dk) break;
#pragma unroll
        for (int t = 0; t < 6; t++)
          if (t < dj) part[t] += a[x] * (double)q[x][t];
      }
    };
    if (cur.ok) add_item(k0 + lane, cur.dk, cur.q);
    for (int it = lane + 64; it < nk; it += 64) {  // spans above 67: items beyond the first 64
      const int k = k0 + it;
      T q[6][6];
      load_qb(q, Pr[sj], dj, k);
      add_item(k, dr[k % R], q);
    }
    // j unpaired: lane t adds A[j](t) v_j(t)
#pragma unroll
    for (int t = 0; t < 6; t++)
      if (t == lane && t < dj) part[t] += ar[sj * 6 + t] * cur.v;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
      for (int t = 0; t < 6; t++) part[t] += __shfl_xor(part[t], off, 64);
    if (lane == 0) {
      double mx = 0;
      for (int t = 0; t < 6; t++) mx = fmax(mx, fabs(part[t]));
      const int e = (mx > 0 && isfinite(mx)) ? ilogb(mx) : 0;
      for (int t = 0; t < 6; t++) zr[sj * 6 + t] = t < dj ? ldexp(part[t], -e) : 0.0;
      gr[sj] = G + e;
    }
    cdz_wave_sync();  // Z5[j] is read by lanes 0..5 below, the ring at j + 1
    if (lane < 6 && j + 1 < n) {  // A[j+1](x = lane) = sum_q Z5[j](q) e_j(q, x)
      double a = 0;
#pragma unroll
      for (int q = 0; q < 6; q++) a += zr[sj * 6 + q] * cur.e[q];
      ar[((j + 1) % R) * 6 + lane] = a;
    }
    if (j - flushed == 63 || j == n - 1) {
      const int p = flushed + lane;
      if (p <= j) {
#pragma unroll
        for (int t = 0; t < 6; t++) D.Z5[p * 6 + t] = zr[(p % R) * 6 + t];
        D.G5[p] = gr[p % R];
      }
      flushed = j + 1;
    }
    cdz_wave_sync();  // A[j+1] is read at j + 1
  };
  Ops o0, o1;
  if (W < n) issue(W, dr[W % R], Pr[W % R], o0);
  for (int j = W; j < n; j += 2) {  // two steps per turn: the operand sets swap roles
    step(j, o0, o1);
    if (j + 1 < n) step(j + 1, o1, o0);
  }
}

// C[p] from the current Z5, v and vd rescaled by it; res[3] accumulates
// C[n-1] over the rescalings (log Z = log Z~ + res[3] ln 2).
template <typename T>
__device__ __forceinline__ void landscape_body(const DevProb<T> &D) {
  const int n = D.n;
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
    double z = 0;
    for (int t = 0; t < 6; t++) z += D.Z5[p * 6 + t];
    D.Cl[p] = (z > 0 && isfinite(z)) ? (int)llrint(D.G5[p] + log2(z)) : 0;
  }
  __syncthreads();  // C is read across threads below (global memory)
  double *vd = const_cast<double *>(D.vd);
  T *v = const_cast<T *>(D.v);
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
    const int g = D.Cl[p] - (p >= 1 ? D.Cl[p - 1] : 0);
    for (int s = 0; s < 6; s++) {
      vd[p * 6 + s] = ldexp(vd[p * 6 + s], -g);
      v[p * 6 + s] = (T)ldexp((double)v[p * 6 + s], -g);
    }
  }
  if (threadIdx.x == 0) D.res[3] += D.Cl[n - 1];
}

// Range check after the exact pass, over the cells of diagonal dl:
//   res[5] = 1 if the largest entry of some cell lies below 2^-lowExp, zero
//          included (the unpaired run U of every cell is positive in exact
//          arithmetic, so an all-zero cell has underflowed); FP32 then
//          repeats the pass once with the landscape of the exact pass
//   res[6] = 1 if some entry is not finite (a scale factor overflowed)
//   res[7] (as an int) = -(binary exponent) of the weakest cell's largest entry
template <typename T>
__device__ __forceinline__ void spread_check_body(const DevProb<T> &D, int dl) {
  const int n = D.n, ncell = n - dl;
  const long long ld = D.ld;
  T *const full[6] = {D.U, D.Qb, D.Qm1, D.Qm1p, D.QmX, D.Qm};
  const T low = (T)ldexp(1.0, -D.lowExp);
  bool weak = false, bad = false;
  int deep = 0;  // -(binary exponent) of the weakest cell maximum seen, 1100 for a zero cell
  for (int i = threadIdx.x; i < ncell; i += CDZ_NT) {
    const int j = i + dl, di = D.d[i], dj = D.d[j], Pi = D.P[i], Pj = D.P[j];
    T m = 0;
    for (int a = 0; a < 6; a++)
      for (int r = 0; r < di; r++)
        for (int c = 0; c < dj; c++) {
          const T x = fabs(full[a][(long long)(Pi + r) * ld + Pj + c]);
          bad = bad || !isfinite(x);
          m = fmax(m, x);
        }
    weak = weak || !(m >= low);
    deep = max(deep, m > T(0) && isfinite(m) ? -ilogb(m) : (m > T(0) ? 0 : 1100));
  }
  if (__any(weak) && (threadIdx.x & 63) == 0) D.res[5] = 1.0;
  if (__any(bad) && (threadIdx.x & 63) == 0) D.res[6] = 1.0;
  // res[7] holds an int: the largest -(exponent) over all cells (memset to 0)
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) deep = max(deep, __shfl_xor(deep, o, 64));
  if ((threadIdx.x & 63) == 0 && deep > 0) atomicMax(reinterpret_cast<int *>(D.res + 7), deep);
}

// Recompute the interior-loop sums A of the cells of diagonal dl (>= 4) into
// D.ALw, from the stored U, DI and exponents of the final forward pass: the
// memory-bounded outside pass rebuilds a band of diagonals this way from its
// checkpoints.  Same LDS layout and window code as the forward.
template <typename T>
__global__ __launch_bounds__(CDZ_NT) void cdz_arec_diag(DevProb<T> D, int dl) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // the LDS layout of the window kind of the forward (fwd_window)
  int *sE = reinterpret_cast<int *>(smem_raw);  // [n + 1]
  CellStage<T> &C = *reinterpret_cast<CellStage<T> *>(smem_raw + WinLayout<T>::stage(D.n));
  T *W = reinterpret_cast<T *>(smem_raw + WinLayout<T>::blocks(D.n));
  const int n = D.n, tid = threadIdx.x, ncell = n - dl;
  const int i = cdz_cell_of_block(blockIdx.x, ncell), j = i + dl;
  if (i >= ncell) return;
  for (int k = tid; k <= dl; k += CDZ_NT) sE[k] = D.E[k];
  if (tid < 6) {
    const int pos[6] = {i - 1, i, i + 1, j - 1, j, j + 1};
    const int p = pos[tid];
    const bool ok = p >= 0 && p < n;
    C.d[tid] = ok ? D.d[p] : 0;
    C.P[tid] = ok ? D.P[p] : 0;
  } else if (tid >= 64 && tid < 128) {
    const int q = tid - 64;
    const int p = q < 32 ? i + 1 + q : j - 1 - (q - 32);
    const bool ok = p >= 0 && p < n;
    C.wd[q] = ok ? D.d[p] : 0;
    C.wP[q] = ok ? D.P[p] : 0;
  } else if (tid >= 128 && tid < 164) {
    const int q = tid - 128;
    C.eI1[q] = i + 1 < n ? D.e[(i + 1) * 36 + q] : T(0);
    C.eJm2[q] = j >= 2 ? D.e[(j - 2) * 36 + q] : T(0);
    if (q < 6) {
      C.vI1[q] = i + 1 < n ? D.v[(i + 1) * 6 + q] : T(0);
      C.vJm1[q] = j >= 1 ? D.v[(j - 1) * 6 + q] : T(0);
    }
  }
  cdz_sync();
  const int lmax = min(CDZ_MAXLOOP, dl - 6);
  a_window<T>(D, C, sE, W, i, j, dl, lmax, sE[dl]);
  a_store<T>(D, C, i, lmax, W + 60 * 36 + 84 * 36);
}

template <typename T>
__global__ __launch_bounds__(CDZ_NT) void cdz_fwd_diag(DevProb<T> D, int t) {
  fwd_block<T, false>(D, t, blockIdx.x);
}
template <typename T>
__global__ __launch_bounds__(CDZ_NT) void cdz_fwd_diag_fused(DevProb<T> D, int t) {
  fwd_block<T, true>(D, t, blockIdx.x);
}

// Batched wavefront: one launch runs diagonal dl of every problem of a batch.
// off[0..count] are the prefix sums of the workgroups per problem for this
// launch (problems without work on dl have none).
template <typename T>
__global__ __launch_bounds__(CDZ_NT) void cdz_fwd_diag_batch(const DevProb<T> *probs, const int *off, int count,
                                                            int dl) {
  int b, w;
  cdz_batch_locate(off, count, blockIdx.x, b, w);
  const DevProb<T> D = probs[b];
  fwd_block<T, false>(D, dl, w);
}
template <typename T>
__global__ __launch_bounds__(CDZ_NT) void cdz_fwd_diag_batch_fused(const DevProb<T> *probs, const int *off,
                                                                  int count, int dl) {
  int b, w;
  cdz_batch_locate(off, count, blockIdx.x, b, w);
  const DevProb<T> D = probs[b];
  fwd_block<T, true>(D, dl, w);
}

// per problem b of a batch: the span-truncated exterior prefix (span W[b]),
// the landscape, and the spread check over off (n_b workgroups per problem)
template <typename T>
__global__ __launch_bounds__(64) void cdz_exterior_trunc_batch(const DevProb<T> *probs, const int *W) {
  const int b = blockIdx.x;
  exterior_trunc_body<T>(probs[b], W[b]);
}
template <typename T>
__global__ __launch_bounds__(1024) void cdz_landscape_batch(const DevProb<T> *probs) {
  landscape_body<T>(probs[blockIdx.x]);
}
template <typename T>
__global__ __launch_bounds__(CDZ_NT) void cdz_spread_check_batch(const DevProb<T> *probs, const int *off, int count) {
  int b, w;
  cdz_batch_locate(off, count, blockIdx.x, b, w);
  spread_check_body<T>(probs[b], w);
}

template <typename T>
__global__ __launch_bounds__(CDZ_SCAN_NT) void cdz_exterior_scan(DevProb<T> D, int W, int jend) {
  exterior_scan_body<T>(D, W, jend, blockIdx.x);
}
template <typename T>
__global__ __launch_bounds__(CDZ_SCAN_NT) void cdz_exterior_scan_batch(const DevProb<T> *probs, const int *W,
                                                                 const int *jend, int per) {
  const int b = blockIdx.x / per;
  exterior_scan_body<T>(probs[b], W[b], jend[b], blockIdx.x % per);
}
template <typename T>
__global__ __launch_bounds__(64) void cdz_exterior_trunc(DevProb<T> D, int W) {
  exterior_trunc_body<T>(D, W);
}
template <typename T>
__global__ __launch_bounds__(1024) void cdz_landscape(DevProb<T> D) {
  landscape_body<T>(D);
}
template <typename T>
__global__ __launch_bounds__(CDZ_NT) void cdz_spread_check(DevProb<T> D) {
  spread_check_body<T>(D, blockIdx.x);
}

template __global__ void cdz_exterior_scan<float>(DevProb<float>, int, int);
template __global__ void cdz_exterior_scan<double>(DevProb<double>, int, int);
template __global__ void cdz_exterior_scan_batch<float>(const DevProb<float> *, const int *, const int *, int);
template __global__ void cdz_exterior_scan_batch<double>(const DevProb<double> *, const int *, const int *, int);
template __global__ void cdz_exterior_trunc<float>(DevProb<float>, int);
template __global__ void cdz_exterior_trunc<double>(DevProb<double>, int);
template __global__ void cdz_landscape<float>(DevProb<float>);
template __global__ void cdz_landscape<double>(DevProb<double>);
template __global__ void cdz_spread_check<float>(DevProb<float>);
template __global__ void cdz_spread_check<double>(DevProb<double>);
template __global__ void cdz_arec_diag<float>(DevProb<float>, int);
template __global__ void cdz_arec_diag<double>(DevProb<double>, int);
template __global__ void cdz_fwd_diag<float>(DevProb<float>, int);
template __global__ void cdz_fwd_diag<double>(DevProb<double>, int);
template __global__ void cdz_fwd_diag_fused<float>(DevProb<float>, int);
template __global__ void cdz_fwd_diag_fused<double>(DevProb<double>, int);
template __global__ void cdz_fwd_diag_batch<float>(const DevProb<float> *, const int *, int, int);
template __global__ void cdz_fwd_diag_batch<double>(const DevProb<double> *, const int *, int, int);
template __global__ void cdz_fwd_diag_batch_fused<float>(const DevProb<float> *, const int *, int, int);
template __global__ void cdz_fwd_diag_batch_fused<double>(const DevProb<double> *, const int *, int, int);
template __global__ void cdz_exterior_trunc_batch<float>(const DevProb<float> *, const int *);
template __global__ void cdz_exterior_trunc_batch<double>(const DevProb<double> *, const int *);
template __global__ void cdz_landscape_batch<float>(const DevProb<float> *);
template __global__ void cdz_landscape_batch<double>(const DevProb<double> *);
template __global__ void cdz_spread_check_batch<float>(const DevProb<float> *, const int *, int);
template __global__ void cdz_spread_check_batch<double>(const DevProb<double> *, const int *, int);
