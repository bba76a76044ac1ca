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
#include "cdz_dev.h"

namespace {

template <typename T>
__device__ int choose_exponent(const DevProb<T> &D, int dl, const int *sE) {
  if (dl == 0) return 0;
  float m1 = __uint_as_float(D.maxb[dl - 1]);
  if (dl >= 2) {
    float m2 = __uint_as_float(D.maxb[dl - 2]);
    if (m1 > 0.f && m2 > 0.f) {
      double L1 = sE[dl - 1] + log2((double)m1);
      double L2 = sE[dl - 2] + log2((double)m2);
      double slope = fmin(fmax(L1 - L2, -16.0), 16.0);
      return (int)rint(L1 + slope);
    }
  }
  if (m1 > 0.f) return (int)rint(sE[dl - 1] + log2((double)m1));
  return sE[dl - 1];
}

// FP64 exterior loop, one step each way:
//   Z5[j](t) = prefix [0..j] with slot t at j
//   Z3[p](s) = suffix [p+1..n-1] given slot s at p, edge e_p included
// Every term is evaluated by its own thread with fully unrolled slot loops,
// so the loads of a step are issued together.
template <typename T>
__device__ void exterior_step(const DevProb<T> &D, int dl, const int *sE, double *red) {
  const int n = D.n, tid = threadIdx.x;
  const long long ld = D.ld;
  double *tot = red + (CDZ_NT / 64) * 6;
  // ---- prefix Z5[j], j = dl - 1
  int j = dl - 1;
  if (j == 0) {
    if (tid < 6) D.Z5[tid] = tid < D.d[0] ? D.vd[tid] : 0.0;
    if (tid == 0) D.G5[0] = 0;
  } else if (j > 0 && j < n) {
    const int R = D.G5[j - 1], dj = D.d[j], Pj = D.P[j];
    double part[6] = {0, 0, 0, 0, 0, 0};
    // item 0: j unpaired; item 1: 0 pairs j; item k >= 2: (k-1) pairs j
    const int nit = j >= 3 ? j - 2 : 1;  // item 0 always; items 1.. need j >= 4
    for (int it = tid; it < nit; it += CDZ_NT) {
      if (it == 0) {
        double z[6];
#pragma unroll
        for (int s = 0; s < 6; s++) z[s] = D.Z5[(j - 1) * 6 + s];
#pragma unroll
        for (int t = 0; t < 6; t++) {
          double a = 0;
#pragma unroll
          for (int s = 0; s < 6; s++) a += z[s] * D.ed[(j - 1) * 36 + s * 6 + t];
          part[t] += t < dj ? a * D.vd[j * 6 + t] : 0.0;
        }
      } else if (it == 1) {
        if (j >= 4) {
          const double sc = ldexp(1.0, sE[j] - R);
          const int d0 = D.d[0];
#pragma unroll
          for (int t = 0; t < 6; t++) {
            double a = 0;
#pragma unroll
            for (int x = 0; x < 6; x++)
              if (x < d0 && t < dj) a += (double)D.Qb[x * ld + Pj + t];
            part[t] += a * sc;
          }
        }
      } else {
        const int k = it - 1;  // 1 <= k <= j-4
        const int dk = D.d[k], Pk = D.P[k];
        const double sc = ldexp(1.0, D.G5[k - 1] + sE[j - k] - R);
        double z[6];
#pragma unroll
        for (int s = 0; s < 6; s++) z[s] = D.Z5[(k - 1) * 6 + s];
        // one slot x of k at a time (keeps the register count of the kernel low)
#pragma unroll 1
        for (int x = 0; x < dk; x++) {
          double a = 0;
#pragma unroll
          for (int s = 0; s < 6; s++) a += z[s] * D.ed[(k - 1) * 36 + s * 6 + x];
          a *= sc;
#pragma unroll
          for (int t = 0; t < 6; t++)
            if (t < dj) part[t] += a * (double)D.Qb[(Pk + x) * ld + Pj + t];
        }
      }
    }
    cdz_block_sum<double, 6>(part, red, tot);
    if (tid == 0) {
      double mx = 0;
      for (int t = 0; t < 6; t++) mx = fmax(mx, fabs(tot[t]));
      const int e = (mx > 0 && isfinite(mx)) ? ilogb(mx) : 0;
      for (int t = 0; t < 6; t++) D.Z5[j * 6 + t] = t < dj ? ldexp(tot[t], -e) : 0.0;
      D.G5[j] = R + e;
    }
    cdz_sync();
  }
  // ---- suffix Z3[p], p = n - 1 - dl
  int p = n - 1 - dl;
  if (p == n - 1) {
    if (tid < 6) D.Z3[p * 6 + tid] = tid < D.d[p] ? 1.0 : 0.0;
    if (tid == 0) D.H3[p] = 0;
  } else if (p >= 0) {
    const int R = D.H3[p + 1], dp = D.d[p], d1 = D.d[p + 1], P1 = D.P[p + 1];
    double part[6] = {0, 0, 0, 0, 0, 0};
    // item 0: p+1 unpaired; item it >= 1: p+1 pairs jj = p + 4 + it
    const int nit = n - 5 - p >= 0 ? n - 4 - p : 1;  // item 0 always
    for (int it = tid; it < nit; it += CDZ_NT) {
      double w[6];
      if (it == 0) {
#pragma unroll
        for (int t = 0; t < 6; t++) w[t] = D.vd[(p + 1) * 6 + t] * D.Z3[(p + 1) * 6 + t];
      } else {
        const int jj = p + 4 + it, dq = D.d[jj], Pq = D.P[jj];
        const double sc = ldexp(1.0, sE[jj - p - 1] + D.H3[jj] - R);
        double z3[6];
#pragma unroll
        for (int t = 0; t < 6; t++) z3[t] = D.Z3[jj * 6 + t];
#pragma unroll 1
        for (int x = 0; x < 6; x++) {
          double a = 0;
#pragma unroll
          for (int t = 0; t < 6; t++)
            if (x < d1 && t < dq) a += (double)D.Qb[(P1 + x) * ld + Pq + t] * z3[t];
          w[x] = a * sc;
        }
      }
#pragma unroll
      for (int s = 0; s < 6; s++) {
        double a = 0;
#pragma unroll
        for (int x = 0; x < 6; x++) a += D.ed[p * 36 + s * 6 + x] * w[x];
        part[s] += s < dp ? a : 0.0;
      }
    }
    cdz_block_sum<double, 6>(part, red, tot);
    if (tid == 0) {
      double mx = 0;
      for (int s = 0; s < 6; s++) mx = fmax(mx, fabs(tot[s]));
      const int e = (mx > 0 && isfinite(mx)) ? ilogb(mx) : 0;
      for (int s = 0; s < 6; s++) D.Z3[p * 6 + s] = s < dp ? ldexp(tot[s], -e) : 0.0;
      D.H3[p] = R + e;
    }
    cdz_sync();
  }
  // ---- totals after the last diagonal
  if (dl == n) {
    double part[2] = {0, 0};
    const int nit = n >= 4 ? n - 3 : 1;  // item 0 always
    for (int it = tid; it < nit; it += CDZ_NT) {
      if (it == 0) {
        double a = 0;
#pragma unroll
        for (int s = 0; s < 6; s++) a += D.vd[s] * D.Z3[s];
        part[0] += a;
      } else {
        const int jj = 3 + it, dq = D.d[jj], Pq = D.P[jj], d0 = D.d[0];
        double a = 0;
#pragma unroll
        for (int x = 0; x < 6; x++)
#pragma unroll
          for (int t = 0; t < 6; t++)
            if (x < d0 && t < dq) a += (double)D.Qb[x * ld + Pq + t] * D.Z3[jj * 6 + t];
        part[0] += a * ldexp(1.0, sE[jj] + D.H3[jj] - D.H3[0]);
      }
    }
    cdz_block_sum<double, 2>(part, red, tot);
    if (tid == 0) {
      double z5 = 0;
      for (int t = 0; t < 6; t++) z5 += D.Z5[(n - 1) * 6 + t];
      const double L2 = 0.6931471805599453094;
      const double lz5 = log(z5) + D.G5[n - 1] * L2;
      const double lz3 = log(tot[0]) + D.H3[0] * L2;
      D.res[0] = lz5;
      D.res[1] = lz3;
      D.res[2] = rint(lz5 / L2);  // EZ, the adjoint scale exponent
    }
  }
}

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

// Blocks of 36 values staged for the loops closed by a cell (after the stage)
#define CDZ_FWD_WBLK 173

template <typename T>
size_t fwd_lds_bytes(int n) {
  const size_t head = ((size_t)(n + 1) * 4 + 15) / 16 * 16 + (size_t)((CDZ_NT / 64) * 72) * sizeof(T);
  const size_t st = (sizeof(CellStage<T>) + 15) / 16 * 16;
  return head + st + (size_t)CDZ_FWD_WBLK * 36 * sizeof(T);
}
template size_t fwd_lds_bytes<float>(int);
template size_t fwd_lds_bytes<double>(int);

template <typename T>
__device__ __forceinline__ void stage_block(T *dst, const T *A, long long ld, int r0, int c0, int dr,
                                            int dc, int q) {
  const int r = q / 6, c = q % 6;
  dst[q] = (r < dr && c < dc) ? A[(long long)(r0 + r) * ld + c0 + c] : T(0);
}

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

// One cell (or the exterior step) of diagonal dl; blk is the workgroup's index
// among the workgroups of this problem's diagonal.
template <typename T>
__device__ __forceinline__ void fwd_cell(const DevProb<T> &D, int dl, int blk) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int *sE = reinterpret_cast<int *>(smem_raw);  // [n + 1]
  T *red = reinterpret_cast<T *>(smem_raw + ((size_t)(D.n + 1) * 4 + 15) / 16 * 16);
  CellStage<T> &C = *reinterpret_cast<CellStage<T> *>(red + (CDZ_NT / 64) * 72);
  T *W = reinterpret_cast<T *>(reinterpret_cast<unsigned char *>(&C) + (sizeof(CellStage<T>) + 15) / 16 * 16);
  const int n = D.n, tid = threadIdx.x;
  const long long ld = D.ld;
  cdz_copy_ints(sE, D.E, dl < n + 1 ? dl : n + 1);
  cdz_sync();
  const int Ed = choose_exponent(D, dl, sE);
  if (tid == 0) sE[dl] = Ed;
  if (blk == 0 && tid == 0) D.E[dl] = Ed;
  cdz_sync();
  const int ncell = n - dl > 0 ? n - dl : 0;
  if (blk == cdz_cells_grid(ncell)) {
    exterior_step<T>(D, dl, sE, reinterpret_cast<double *>(red));
    return;
  }
  const int i = cdz_cell_of_block(blk, ncell), j = i + dl;
  if (i >= ncell) return;

  // ---- stage: positions i-1, i, i+1, j-1, j, j+1 (clamped; unused when absent)
  if (tid < 6) {
    const int pos[6] = {i - 1, i, i + 1, j - 1, j, j + 1};
    const int p = pos[tid];
    const bool ok = p >= 0 && p < n;
    C.d[tid] = ok ? D.d[p] : 0;
    C.P[tid] = ok ? D.P[p] : 0;
#pragma unroll
    for (int s = 0; s < 6; s++) C.nt[tid][s] = ok ? D.nt[p * 6 + s] : (signed char)-1;
  }
  for (int q = tid; q < TB_LEN; q += CDZ_NT) C.tab[q] = D.tab[q];
  if (tid >= 64 && tid < 128) {
    const int q = tid - 64;
    const int p = q < 32 ? i + 1 + q : j - 1 - (q - 32);
    const bool ok = p >= 0 && p < n;
    C.wd[q] = ok ? D.d[p] : 0;
    C.wP[q] = ok ? D.P[p] : 0;
  }
  cdz_sync();
  const int di = C.d[1], dj = C.d[4], Pi = C.P[1], Pj = C.P[4];
  const int d1 = C.d[2], dm = C.d[3], P1 = C.P[2], Pm = C.P[3];
  {
    const int g = tid / 36, q = tid % 36;
    switch (g) {
      case 0:
        if (dl >= 2) stage_block(C.Uin, D.U, ld, P1, Pm, d1, dm, q);
        else C.Uin[q] = 0;
        break;
      case 1:
        if (dl >= 2) stage_block(C.Xin, D.QmX, ld, P1, Pm, d1, dm, q);
        else C.Xin[q] = 0;
        break;
      case 2:
        if (dl >= 2) stage_block(C.Bin, D.Qb, ld, P1, Pm, d1, dm, q);
        else C.Bin[q] = 0;
        break;
      case 3:
        if (dl >= 1) stage_block(C.M1l, D.Qm1, ld, Pi, Pm, di, dm, q);
        else C.M1l[q] = 0;
        break;
      case 4:
        if (dl >= 1) stage_block(C.M1pr, D.Qm1p, ld, P1, Pj, d1, dj, q);
        else C.M1pr[q] = 0;
        break;
      case 5:
        if (dl >= 1) stage_block(C.Ul, D.U, ld, Pi, Pm, di, dm, q);
        else C.Ul[q] = 0;
        break;
      case 6:
        C.eIm1[q] = i >= 1 ? D.e[(i - 1) * 36 + q] : T(0);
        C.eI[q] = D.e[i * 36 + q];
        C.eJm1[q] = j >= 1 ? D.e[(j - 1) * 36 + q] : T(0);
        C.eJ[q] = D.e[j * 36 + q];
        C.eI1[q] = i + 1 < n ? D.e[(i + 1) * 36 + q] : T(0);
        C.eJm2[q] = j >= 2 ? D.e[(j - 2) * 36 + q] : T(0);
        if (q < 6) {
          C.vI[q] = D.v[i * 6 + q];
          C.vJ[q] = D.v[j * 6 + q];
          C.vI1[q] = i + 1 < n ? D.v[(i + 1) * 6 + q] : T(0);
          C.vJm1[q] = j >= 1 ? D.v[(j - 1) * 6 + q] : T(0);
        }
        break;
    }
  }
  cdz_sync();
  float vmax = 0.f;

  // ---- unpaired run U[i][j]
  if (tid < 36) {
    const int s = tid / 6, t = tid % 6;
    if (s < di && t < dj) {
      T u = 0;
      if (dl == 0) {
        u = (s == t) ? C.vI[s] : T(0);
      } else {
        T a = 0;
#pragma unroll
        for (int c = 0; c < 6; c++) a += C.Ul[s * 6 + c] * C.eJm1[c * 6 + t];
        u = a * C.vJ[t] * cdz_p2<T>(sE[dl - 1] - Ed);
      }
      D.U[(Pi + s) * ld + Pj + t] = u;
      D.Ut[(Pj + t) * ld + Pi + s] = u;
      vmax = fmaxf(vmax, (float)fabs(u));
      if (dl < 4) {
        const long long o = (Pi + s) * ld + Pj + t;
        D.Qb[o] = 0;
        D.Qbt[(Pj + t) * ld + Pi + s] = 0;
        D.Qm1[o] = 0;
        D.Qm1p[o] = 0;
        D.QmX[o] = 0;
        D.Qm[o] = 0;
        D.Qmt[(Pj + t) * ld + Pi + s] = 0;
      }
    }
  }
  if (dl >= 4) {
    // ---- split: QmX[i][j] = sum_k Qm[i][k] f(k) Qm1Lt[j][k], k over the
    //      states of positions i+4 .. j-5 (u - 1 = pos(k)); the stream is
    //      unrolled so that the loads of several k are in flight together
    {
      constexpr int UN = sizeof(T) == 4 ? 4 : 1;
      T acc[36];
#pragma unroll
      for (int r = 0; r < 36; r++) acc[r] = 0;
      const int K0 = D.P[i + 4], K1 = D.P[j - 4];
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
          for (int t = 0; t < 6; t++) b[u][t] = (ok && t < dj) ? D.Qm1Lt[(Pj + t) * ld + k] : T(0);
        }
#pragma unroll
        for (int u = 0; u < UN; u++) {
          const T f = cdz_p2<T>(sE[pp[u] - i] + sE[j - pp[u] - 1] - Ed);
#pragma unroll
          for (int s = 0; s < 6; s++) {
            const T as = a[u][s] * f;
#pragma unroll
            for (int t = 0; t < 6; t++) acc[s * 6 + t] = fma(as, b[u][t], acc[s * 6 + t]);
          }
        }
      }
      cdz_block_sum<T, 36>(acc, red, C.split);
    }
    // ---- bulge and interior loops closed by (i, j), indices (a, dd) = slots
    //      of positions i+1 and j-1, outer edges and outer mismatch not
    //      applied: G = bulges, F = interior loops.
    //
    //      Interior loops use the loop-size recursion (Lyngso's observation,
    //      valid because the interior-loop energy depends on l1 + l2 and the
    //      end mismatches only): with A(i,j,L) the sum over inner pairs at
    //      total loop size L = l1 + l2 of U[i+1][k-1] . DI[k][l] . U[l+1][j-1],
    //        A(i,j,L) = V . A(i+1,j-1,L-2) . W          (l1, l2 >= 2)
    //                 + diag v_{i+1} . DI . U[j-L+1][j-1]  (l1 = 1)
    //                 + U[i+1][i+L-1] . DI . diag v_{j-1}  (l2 = 1, L >= 3)
    //      with V = v_{i+1} e_{i+1}, W = e_{j-2} v_{j-1}; F = sum_L w_int(L) A.
    //      Every term needs an inner pair at distance >= 4, i.e. L <= dl - 6.
    {
      const int lmax = min(CDZ_MAXLOOP, dl - 6);
      T *UR1 = W;              // [l-1] U[i+1][i+l]
      T *UC1 = W + 30 * 36;    // [l-1] U[j-l][j-1]
      T *X = W + 60 * 36;      // phase-dependent blocks
      T *AC = X + 84 * 36;     // [L-2] A(i,j,L)
      const int *lp_d = C.wd, *lp_P = C.wP, *rp_d = C.wd + 32, *rp_P = C.wP + 32;
      a_window<T>(D, C, sE, W, i, j, dl, lmax, Ed);
      if (tid < 36) {
        T f = 0;
        for (int L = 2; L <= lmax; L++) f += C.tab[TB_IN + L] * AC[(L - 2) * 36 + tid];
        C.gf[36 + tid] = f;
      }
      cdz_sync();
      // bulges: left (run i+1..k-1, inner pair (k, j-1)), right (inner pair
      // (i+1, l), run l+1..j-1), l = 1..lmax; one side after the other, each
      // thread summing the terms term = g, g + 7, .. of output q
      T *EB = X, *QB = X + 30 * 36;
      T *GP = red;  // 7 x 36 partial sums (the reduction scratch is free here)
      const int q = tid % 36, g = tid / 36, r = q / 6, c = q % 6;
      T gacc = 0;
      for (int side = 0; side < 2; side++) {
        // e blocks (contiguous in D.e), then the Qb blocks of the inner pairs:
        // the left side's column strip as contiguous rows of Qbt, the right
        // side's row strip as one contiguous row segment of Qb, each placed by
        // the window map of its side into blocks cleared first
        // e_{k-1}, k = i+1+l (left: positions i+1..i+lmax) / e_l, l = j-1-l2
        // (right: positions j-2 down to j-1-lmax), block l-1
        if (side == 0) cdz_copy_blocks<T>(EB, D.e + (long long)(i + 1) * 36, lmax, false);
        else cdz_copy_blocks<T>(EB, D.e + (long long)(j - 1 - lmax) * 36, lmax, true);
        cdz_zero_blocks<T>(QB, lmax);
        cdz_sync();
        if (side == 0 && lmax >= 1) {  // Qb[i+1+l][j-1](x, c) = Qbt row Pm + c, states of positions i+2..i+1+lmax
          const int o = lp_P[1] - lp_P[0], K = lp_P[lmax + 1] - lp_P[1];
          for (int idx = tid; idx < dm * K; idx += CDZ_NT) {
            const int c = idx / K, k = idx % K + o, l = C.mapL[k], x = k - (lp_P[l] - lp_P[0]);
            QB[(l - 1) * 36 + x * 6 + c] = D.Qbt[(long long)(Pm + c) * ld + lp_P[0] + k];
          }
        } else if (lmax >= 1) {  // Qb[i+1][j-1-l] = row P1 + r of Qb, states of positions
                                 // j-1-lmax..j-2, placed by the right window map
          const int baseR = rp_P[lmax], K = rp_P[1] + rp_d[1] - baseR;
          for (int idx = tid; idx < d1 * K; idx += CDZ_NT) {
            const int r = idx / K, k = idx % K, l = C.mapR[k], c = k - (rp_P[l] - baseR);
            QB[(l - 1) * 36 + r * 6 + c] = D.Qb[(long long)(P1 + r) * ld + baseR + k];
          }
        }
        cdz_sync();
        if (g < 7) {
          for (int l = g + 1; l <= lmax; l += 7) {
            const T f = C.tab[TB_BU + l] * cdz_p2<T>(sE[l - 1] + sE[dl - 2 - l] - Ed);
            const T *ek = EB + (l - 1) * 36, *qk = QB + (l - 1) * 36;
            T sm = 0;
            if (side == 0) {  // output (a, y) = (r, c): U[i+1][k-1] e_{k-1} Qb[k][j-1]
              const T *ul = UR1 + (l - 1) * 36;
#pragma unroll
              for (int b = 0; b < 6; b++) {
                T m = 0;
#pragma unroll
                for (int x = 0; x < 6; x++) m += ek[b * 6 + x] * qk[x * 6 + c];
                sm += ul[r * 6 + b] * m;
              }
            } else {  // output (x, dd) = (r, c): Qb[i+1][l] e_l U[l+1][j-1]
              const T *ur = UC1 + (l - 1) * 36;
#pragma unroll
              for (int y = 0; y < 6; y++) {
                T m = 0;
#pragma unroll
                for (int cc = 0; cc < 6; cc++) m += ek[y * 6 + cc] * ur[cc * 6 + c];
                sm += qk[r * 6 + y] * m;
              }
            }
            gacc += f * sm;
          }
        }
        cdz_sync();
      }
      if (g < 7) GP[g * 36 + q] = gacc;
      cdz_sync();
      if (tid < 36) {
        T gs = 0;
#pragma unroll
        for (int gg = 0; gg < 7; gg++) gs += GP[gg * 36 + tid];
        C.gf[tid] = gs;
      }
      // keep A(i,j,L), L = 2..CDZ_NA+1, for the cells of diagonal dl + 2 and
      // the outside pass (zero where no inner pair fits); stored after the
      // loads above so that none of them waits behind these stores
      a_store<T>(D, C, i, lmax, AC);
      cdz_sync();
    }
    const T *tab = C.tab;
    // ---- Qb: thread (a, o) sums the terms of output o = (s, s2) whose slot
    //      at i+1 is a; the six partial sums are added afterwards
    if (tid < 216) {
      const int a = tid / 36, o = tid % 36, s = o / 6, s2 = o % 6;
      T part = 0;
      if (s < di && s2 < dj && a < d1) {
        const int t = cdz_ptype(C.nt[1][s], C.nt[4][s2]);
        if (t >= 0) {
          const int na = C.nt[2][a];
          const T ea = C.eI[s * 6 + a];
          T acc = 0, hp = 0, st = 0, ml = 0;
#pragma unroll
          for (int b = 0; b < 6; b++) {
            if (b >= dm) continue;
            const int nb = C.nt[3][b];
            const T w = ea * C.eJm1[b * 6 + s2];
            const T mmo = tab[TB_MM + na * 24 + nb * 6 + t];
            const int o2 = a * 6 + b;
            hp += w * C.Uin[o2] * mmo;
            acc += w * (C.gf[o2] + C.gf[36 + o2] * mmo);
            ml += w * C.Xin[o2];
            const int t2 = cdz_ptype(na, nb);
            if (dl - 2 >= 4 && t2 >= 0) st += w * C.Bin[o2] * tab[TB_ST + t * 6 + t2];
          }
          part = acc + (hp * D.Bhp[dl - 1] + st + ml * tab[TB_MLAB]) * cdz_p2<T>(sE[dl - 2] - Ed);
        }
      }
      red[a * 36 + o] = part;
    }
    cdz_sync();
    if (tid < 36) {
      const int s = tid / 6, s2 = tid % 6;
      T qb = 0;
      if (s < di && s2 < dj) {
        T acc = 0;
#pragma unroll
        for (int a = 0; a < 6; a++) acc += red[a * 36 + tid];
        qb = C.vI[s] * C.vJ[s2] * acc;
        D.Qb[(Pi + s) * ld + Pj + s2] = qb;
        D.Qbt[(Pj + s2) * ld + Pi + s] = qb;
        vmax = fmaxf(vmax, (float)fabs(qb));
      }
      C.qb[tid] = qb;
      // keep the window sums of this cell for the adjoint (block (i+1, j-1))
      if (s < d1 && s2 < dm) {
        D.G[(P1 + s) * ld + Pm + s2] = C.gf[tid];
        D.F[(P1 + s) * ld + Pm + s2] = C.gf[36 + tid];
      }
    }
    cdz_sync();
    // ---- Qm1, and DI (Qb dressed as an interior loop's inner pair) with
    //      thread (x, o) summing over the slot y of j for output o = (b, c)
    if (tid < 36) {
      const int s = tid / 6, s2 = tid % 6;
      T q1 = 0;
      if (s < di && s2 < dj) {
        T a = 0;
#pragma unroll
        for (int t = 0; t < 6; t++) a += C.M1l[s * 6 + t] * C.eJm1[t * 6 + s2];
        q1 = a * C.vJ[s2] * tab[TB_MLC] * cdz_p2<T>(sE[dl - 1] - Ed) + C.qb[tid] * tab[TB_MLB];
        D.Qm1[(Pi + s) * ld + Pj + s2] = q1;
        vmax = fmaxf(vmax, (float)fabs(q1));
      }
      C.qm1[tid] = q1;
    }
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
    // ---- DI, Qm1L, Qm1p, QmX, Qm
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
        for (int t = 0; t < 6; t++) a += C.eIm1[s * 6 + t] * C.qm1[t * 6 + s2];
        D.Qm1Lr[(C.P[0] + s) * ld + Pj + s2] = a;
        D.Qm1Lt[(Pj + s2) * ld + C.P[0] + s] = a;
      }
      if (s < di && s2 < dj) {
        T a = 0;
#pragma unroll
        for (int t = 0; t < 6; t++) a += C.eI[s * 6 + t] * C.M1pr[t * 6 + s2];
        const T qp = C.qm1[tid] + tab[TB_MLC] * C.vI[s] * cdz_p2<T>(sE[dl - 1] - Ed) * a;
        const T qx = C.split[tid];
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
  // ---- per-diagonal maximum for the next exponents
  if (tid < 64) {
    vmax = fminf(cdz_wave_max(vmax), 3.0e38f);
    if (tid == 0 && vmax > 0.f) atomicMax(&D.maxb[dl], __float_as_uint(vmax));
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
template <typename T>
__device__ __forceinline__ void spread_check_body(const DevProb<T> &D, int dl) {
  const int n = D.n, ncell = n - dl;
  const long long ld = D.ld;
  T *const full[6] = {D.U, D.Qb, D.Qm1, D.Qm1p, D.QmX, D.Qm};
  const T low = (T)ldexp(1.0, -D.lowExp);
  bool weak = false, bad = false;
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
  }
  if (__any(weak) && (threadIdx.x & 63) == 0) D.res[5] = 1.0;
  if (__any(bad) && (threadIdx.x & 63) == 0) D.res[6] = 1.0;
}

// Recompute the interior-loop sums A of the cells of diagonal dl (>= 4) into
// D.ALw, from the stored U, DI and exponents of the final forward pass: the
// memory-bounded outside pass rebuilds a band of diagonals this way from its
// checkpoints.  Same LDS layout and window code as the forward.
template <typename T>
__global__ __launch_bounds__(CDZ_NT) void cdz_arec_diag(DevProb<T> D, int dl) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int *sE = reinterpret_cast<int *>(smem_raw);  // [n + 1]
  T *red = reinterpret_cast<T *>(smem_raw + ((size_t)(D.n + 1) * 4 + 15) / 16 * 16);
  CellStage<T> &C = *reinterpret_cast<CellStage<T> *>(red + (CDZ_NT / 64) * 72);
  T *W = reinterpret_cast<T *>(reinterpret_cast<unsigned char *>(&C) + (sizeof(CellStage<T>) + 15) / 16 * 16);
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
__global__ __launch_bounds__(CDZ_NT) void cdz_fwd_diag(DevProb<T> D, int dl) {
  fwd_cell<T>(D, dl, blockIdx.x);
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
  fwd_cell<T>(D, dl, w);
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
template __global__ void cdz_fwd_diag_batch<float>(const DevProb<float> *, const int *, int, int);
template __global__ void cdz_fwd_diag_batch<double>(const DevProb<double> *, const int *, int, int);
template __global__ void cdz_exterior_trunc_batch<float>(const DevProb<float> *, const int *);
template __global__ void cdz_exterior_trunc_batch<double>(const DevProb<double> *, const int *);
template __global__ void cdz_landscape_batch<float>(const DevProb<float> *);
template __global__ void cdz_landscape_batch<double>(const DevProb<double> *);
template __global__ void cdz_spread_check_batch<float>(const DevProb<float> *, const int *, int);
template __global__ void cdz_spread_check_batch<double>(const DevProb<double> *, const int *, int);
