// cdz_out.hip -- outside pass: the hand-written adjoint of the forward
// recursions (reverse mode, pull form), then the marginals.
//
// The adjoint X' of a forward entry X is dZ/dX.  Cells are processed in
// decreasing anti-diagonal order, one launch per diagonal, one workgroup per
// cell; every adjoint of a cell is gathered from cells on larger diagonals
// (no atomics).  Stored adjoints are true * 2^(E[dl] - EZ); with that choice
// every adjoint term carries exactly the power-of-two factor of the forward
// term it reverses.
//
// Marginals (Section 2c of the paper): every derivation uses each backbone
// edge factor e_p exactly once, so eta_p(s,t) = e_p(s,t) dZ/de_p(s,t) / Z is
// the joint probability of slots (s, t) at positions (p, p+1).  Codon
// marginals are eta at the edge inside a codon, codon-pair marginals eta at
// the edge between two codons (equal to d log Z / d theta1 and d theta2),
// and pair probabilities are sum Qb * Qb' / Z.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "cdz_internal.h"

template <typename T>
void adj_carve(size_t &off, char *base, const HostTables &t, DevAdj<T> &A, size_t S2) {
  auto take = [&](size_t bytes) -> char * {
    off = (off + 255) / 256 * 256;
    char *p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  T **arrs[] = {&A.Qbb, &A.Qm1b, &A.Qm1pb, &A.QmXb, &A.QmXbt, &A.Qmb, &A.Qm1Lb, &A.DIb, &A.Gb,
                &A.Fb, &A.Ub, &A.UbL, &A.UbR, &A.UbL2, &A.UbR2, &A.DIbL, &A.DIbR};
  for (T **a : arrs) *a = reinterpret_cast<T *>(take(S2 * sizeof(T)));
  A.ring = reinterpret_cast<T *>(take((size_t)3 * t.n * CDZ_NRING * 36 * sizeof(T)));
  A.etaV = reinterpret_cast<double *>(take((size_t)t.n * 36 * sizeof(double)));
  A.etaW = reinterpret_cast<double *>(take((size_t)t.n * 36 * sizeof(double)));
  A.eta = reinterpret_cast<double *>(take((size_t)t.n * 36 * sizeof(double)));
  A.pair = reinterpret_cast<double *>(take((size_t)t.n * t.n * sizeof(double)));
  A.out = reinterpret_cast<double *>(take(16 * sizeof(double)));
}
template void adj_carve<float>(size_t &, char *, const HostTables &, DevAdj<float> &, size_t);
template void adj_carve<double>(size_t &, char *, const HostTables &, DevAdj<double> &, size_t);

// LDS stage of one cell of the outside pass (see cdz_fwd.hip for the idea):
// all small operands of the cell's O(1) adjoint statements, fetched by one
// parallel load phase.
template <typename T>
struct OutStage {
  T tab[TB_LEN];
  T eIm1[36], eI[36], eJm1[36], eJ[36], eI1[36], eJm2[36];
  T vIm1[6], vI[6], vJ[6], vJp1[6], vI1[6], vJm1[6];
  T m1pUp[36];   // Qm1p'[i-1][j]
  T m1Right[36]; // Qm1'[i][j+1]
  T qbOut[36];   // Qb'[i-1][j+1]
  T gbOut[36];   // Gb at block (i, j): dressed adjoint of the enclosing pair
  T ubRight[36]; // U'[i][j+1]
  T ubl[36], ubr[36];  // run adjoints of [i..j] pushed by interior loops and hairpins
  T ubl2[36], ubr2[36];  // run adjoints of [i..j] pushed by bulges
  T acc[72], w[72], qm1pb[36], qm1lb[36], qm1b[36], qbb[36], gb[36], fb[36];
  double z5[6], z3[6], edm1[36];
  signed char nt[6][6];
  int d[6], P[6];
  // d, P of positions i+1+q ([q]), j-1-q ([32+q]), i-1-q ([64+q]), j+1+q ([96+q])
  int wd[128], wP[128];
  unsigned char mapL[192], mapR[192];  // state offset -> position index (window staging)
};

// Blocks of 36 values for the loop terms of a cell: the adjoints of the
// interior-loop sums by size (29) and one phase-dependent region (127).
#define CDZ_OUT_WBLK (29 + 127)

template <typename T>
size_t out_lds_bytes(int n) {
  const size_t head = ((size_t)(n + 1) * 4 + 15) / 16 * 16 + (size_t)((CDZ_NT / 64) * 72) * sizeof(T);
  const size_t st = (sizeof(OutStage<T>) + 15) / 16 * 16;
  return head + st + (size_t)CDZ_OUT_WBLK * 36 * sizeof(T);
}
template size_t out_lds_bytes<float>(int);
template size_t out_lds_bytes<double>(int);

template <typename T>
__device__ __forceinline__ void ostage(T *dst, const T *A, long long ld, int r0, int c0, int dr, int dc,
                                       int q, bool ok) {
  const int r = q / 6, c = q % 6;
  dst[q] = (ok && r < dr && c < dc) ? A[(long long)(r0 + r) * ld + c0 + c] : T(0);
}
// the same block from an array stored transposed (element (r, c) at [c][r])
template <typename T>
__device__ __forceinline__ void ostage_t(T *dst, const T *At, long long ld, int r0, int c0, int dr, int dc,
                                         int q, bool ok) {
  const int r = q / 6, c = q % 6;
  dst[q] = (ok && r < dr && c < dc) ? At[(long long)(c0 + c) * ld + r0 + r] : T(0);
}

// ring of interior-loop adjoints: diagonal dl, cell i, size L (2..30)
template <typename T>
__device__ __forceinline__ T *ring_at(const DevAdj<T> &A, int n, int dl, int i, int L) {
  return A.ring + (((long long)(dl % 3) * n + i) * CDZ_NRING + (L - 2)) * 36;
}

// ---------------------------------------------------------------------------
// One launch per step t = n-1..0.  The adjoint of a cell is split by what it
// reads, and each piece runs as its own workgroups in the launch where its
// inputs are final (adjoints flow from longer to shorter spans); the pieces
// of one launch never read each other's results:
//   interior pushes (diagonal t+1)  the size-recursion boundary terms of the
//                                   cell's interior loops: DI' and run
//                                   adjoints pushed to shorter spans
//   edge terms      (diagonal t+1)  the uses of e_{i+1} and e_{j-2} inside the
//                                   size recursion (eta)
//   bulge pushes    (diagonal t+1)  run adjoints of the cell's bulges, into
//                                   their own accumulators (UbL2, UbR2)
//   bulge gathers   (diagonal t-1)  the part of Qb' from the enclosing bulges
//                                   (reads Gb of spans >= t+1)
//   split gathers   (diagonal t-4)  Qm' and Qm1L' (read QmX' of spans >= t+1)
//   finish          (diagonal t)    the O(1) adjoint statements, Qb' (with the
//                                   gathered parts), Gb, Fb, the adjoints of
//                                   the interior-loop sums by size (ring),
//                                   the hairpin run push, the run total Ub
// ---------------------------------------------------------------------------

// ---- split gathers of the cells of diagonal dl (launch dl + 4): Qm'[i][j]
//      and Qm1L'[i-1][j], complete (no other statement reaches them)
template <typename T>
__device__ __forceinline__ void out_split(const DevProb<T> &D, const DevAdj<T> &A, int dl, int blk) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = D.n, tid = threadIdx.x;
  const long long ld = D.ld;
  int *sE = reinterpret_cast<int *>(smem_raw);
  T *red = reinterpret_cast<T *>(smem_raw + ((size_t)(n + 1) * 4 + 15) / 16 * 16);
  OutStage<T> &C = *reinterpret_cast<OutStage<T> *>(red + (CDZ_NT / 64) * 72);
  T *AB = reinterpret_cast<T *>(reinterpret_cast<unsigned char *>(&C) + (sizeof(OutStage<T>) + 15) / 16 * 16);
  T *X = AB + 29 * 36;
  cdz_copy_ints(sE, D.E, n);
  const int EZ = (int)D.res[2];
  const int i = cdz_cell_of_block(blk, n - dl), j = i + dl;
  if (i >= n - dl) return;
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
  if (tid >= 128) {
    const int q = tid - 128, grp = q / 32, o = q % 32;
    const int p = grp == 0 ? i + 1 + o : grp == 1 ? j - 1 - o : grp == 2 ? i - 1 - o : j + 1 + o;
    const bool ok = p >= 0 && p < n;
    C.wd[q] = ok ? D.d[p] : 0;
    C.wP[q] = ok ? D.P[p] : 0;
  }
  cdz_sync();
  const int di = C.d[1], dj = C.d[4], Pi = C.P[1], Pj = C.P[4];
  const int dim1 = C.d[0], Pim1 = C.P[0], djp1 = C.d[5], Pjp1 = C.P[5];
  const int d1 = C.d[2], dm = C.d[3], P1 = C.P[2], Pm = C.P[3];
  const bool hasL = i >= 1, hasR = j + 1 <= n - 1;
  const int *lp_d = C.wd, *lp_P = C.wP, *rp_d = C.wd + 32, *rp_P = C.wP + 32;
  const int *ll_d = C.wd + 64, *ll_P = C.wP + 64, *rr_d = C.wd + 96, *rr_P = C.wP + 96;
    // ---- split gathers: Qm'[i][j] along row i, Qm1L'[i][j] down column j
    {
      constexpr int UN = 2;
      T acc[72];
#pragma unroll
      for (int r = 0; r < 72; r++) acc[r] = 0;
      if (j + 5 <= n - 1) {
        const int K0 = D.P[j + 5], K1 = D.P[n];
        for (int k0 = K0 + tid; k0 < K1; k0 += UN * CDZ_NT) {
          T a[UN][6], b[UN][6];
          int pp[UN];
#pragma unroll
          for (int u = 0; u < UN; u++) {
            const int k = k0 + u * CDZ_NT;
            const bool ok = k < K1;
            pp[u] = ok ? D.posOf[k] : j + 5;
#pragma unroll
            for (int s = 0; s < 6; s++) a[u][s] = (ok && s < di) ? A.QmXb[(Pi + s) * ld + k] : T(0);
#pragma unroll
            for (int t = 0; t < 6; t++) b[u][t] = (ok && t < dj) ? D.Qm1Lr[(Pj + t) * ld + k] : T(0);
          }
#pragma unroll
          for (int u = 0; u < UN; u++) {
            const T f = cdz_p2<T>(sE[dl] + sE[pp[u] - j - 1] - sE[pp[u] - i]);
#pragma unroll
            for (int s = 0; s < 6; s++) {
              const T as = a[u][s] * f;
#pragma unroll
              for (int t = 0; t < 6; t++) acc[s * 6 + t] = fma(as, b[u][t], acc[s * 6 + t]);
            }
          }
        }
      }
      if (i >= 5) {
        const int K1 = D.P[i - 4];
        for (int k0 = tid; k0 < K1; k0 += UN * CDZ_NT) {
          T a[UN][6], c[UN][6];
          int pp[UN];
#pragma unroll
          for (int u = 0; u < UN; u++) {
            const int k = k0 + u * CDZ_NT;
            const bool ok = k < K1;
            pp[u] = ok ? D.posOf[k] : 0;
#pragma unroll
            for (int b = 0; b < 6; b++) a[u][b] = (ok && b < dim1) ? D.Qmt[(Pim1 + b) * ld + k] : T(0);
#pragma unroll
            for (int s2 = 0; s2 < 6; s2++) c[u][s2] = (ok && s2 < dj) ? A.QmXbt[(Pj + s2) * ld + k] : T(0);
          }
#pragma unroll
          for (int u = 0; u < UN; u++) {
            const T f = cdz_p2<T>(sE[i - 1 - pp[u]] + sE[dl] - sE[j - pp[u]]);
#pragma unroll
            for (int b = 0; b < 6; b++) {
              const T ab = a[u][b] * f;
#pragma unroll
              for (int s2 = 0; s2 < 6; s2++) acc[36 + b * 6 + s2] = fma(ab, c[u][s2], acc[36 + b * 6 + s2]);
            }
          }
        }
      }
      cdz_block_sum<T, 72>(acc, red, C.acc);
    }
  if (tid < 36) {
    const int s = tid / 6, t = tid % 6;
    if (s < di && t < dj) A.Qmb[(Pi + s) * ld + Pj + t] = C.acc[tid];
    if (hasL && s < dim1 && t < dj) A.Qm1Lb[(Pim1 + s) * ld + Pj + t] = C.acc[36 + tid];
  }
}

// ---- bulge gathers of the cells of diagonal dl (launch dl + 1): the part of
//      Qb'[i][j] from the bulges that enclose (i, j), into Qbb (completed by
//      the finish of the cell)
template <typename T>
__device__ __forceinline__ void out_bulge_gather(const DevProb<T> &D, const DevAdj<T> &A, int dl, int blk) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = D.n, tid = threadIdx.x;
  const long long ld = D.ld;
  int *sE = reinterpret_cast<int *>(smem_raw);
  T *red = reinterpret_cast<T *>(smem_raw + ((size_t)(n + 1) * 4 + 15) / 16 * 16);
  OutStage<T> &C = *reinterpret_cast<OutStage<T> *>(red + (CDZ_NT / 64) * 72);
  T *AB = reinterpret_cast<T *>(reinterpret_cast<unsigned char *>(&C) + (sizeof(OutStage<T>) + 15) / 16 * 16);
  T *X = AB + 29 * 36;
  cdz_copy_exponents(sE, D.E, n, dl, 34);
  const int EZ = (int)D.res[2];
  const int i = cdz_cell_of_block(blk, n - dl), j = i + dl;
  if (i >= n - dl) return;
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
  if (tid >= 128) {
    const int q = tid - 128, grp = q / 32, o = q % 32;
    const int p = grp == 0 ? i + 1 + o : grp == 1 ? j - 1 - o : grp == 2 ? i - 1 - o : j + 1 + o;
    const bool ok = p >= 0 && p < n;
    C.wd[q] = ok ? D.d[p] : 0;
    C.wP[q] = ok ? D.P[p] : 0;
  }
  if (tid < 36) {
    C.eIm1[tid] = i >= 1 ? D.e[(i - 1) * 36 + tid] : T(0);
    C.eJ[tid] = D.e[j * 36 + tid];
  }
  cdz_sync();
  const int di = C.d[1], dj = C.d[4], Pi = C.P[1], Pj = C.P[4];
  const int dim1 = C.d[0], Pim1 = C.P[0], djp1 = C.d[5], Pjp1 = C.P[5];
  const int d1 = C.d[2], dm = C.d[3], P1 = C.P[2], Pm = C.P[3];
  const bool hasL = i >= 1, hasR = j + 1 <= n - 1;
  const int *lp_d = C.wd, *lp_P = C.wP, *rp_d = C.wd + 32, *rp_P = C.wP + 32;
  const int *ll_d = C.wd + 64, *ll_P = C.wP + 64, *rr_d = C.wd + 96, *rr_P = C.wP + 96;
  const T *tab = C.tab;
    // ---- bulges enclosing the pair (i, j): the bulge part of Qb'[i][j].
    //      Left bulge (i-l1-1, j+1): run i-l1..i-1; right bulge
    //      (i-1, j+l2+1): run j+1..j+l2.
    {
      const int nl = hasR ? min(CDZ_MAXLOOP, i - 1) : 0;
      const int nr = hasL ? min(CDZ_MAXLOOP, n - 2 - j) : 0;
      T *Ulc = X, *Gbc = X + 30 * 36, *Urr = X + 60 * 36, *Gbr = X + 90 * 36, *GP = X + 120 * 36;
      // X offsets: Ulc 0, Gbc 30*36, Urr 60*36, Gbr 90*36
      cdz_stage_nv<3, T>(X, 2 * (nl + nr) * 36, [&](int idx, int &d) -> const T * {
        const int b = idx / 36, q = idx % 36, r = q / 6, c = q % 6;
        if (b < 2 * nl) {
          const int kind = b / nl, l1 = b % nl + 1, pa = l1 - 1;  // position i - l1
          d = (kind * 30 + l1 - 1) * 36 + q;
          if (kind == 0)  // U[i-l1][i-1], a column strip read along a row of Ut
            return (r < ll_d[pa] && c < dim1) ? D.Ut + (long long)(Pim1 + c) * ld + ll_P[pa] + r : nullptr;
          // Gb at block (i-l1, j)
          return (r < ll_d[pa] && c < dj) ? A.Gb + (long long)(ll_P[pa] + r) * ld + Pj + c : nullptr;
        }
        const int bb = b - 2 * nl, kind = bb / nr, l2 = bb % nr + 1, pz = l2 - 1;  // position j + l2
        d = ((2 + kind) * 30 + l2 - 1) * 36 + q;
        if (kind == 0)  // U[j+1][j+l2]
          return (r < djp1 && c < rr_d[pz]) ? D.U + (long long)(Pjp1 + r) * ld + rr_P[pz] + c : nullptr;
        // Gb at block (i, j+l2)
        return (r < di && c < rr_d[pz]) ? A.Gb + (long long)(Pi + r) * ld + rr_P[pz] + c : nullptr;
      });
      cdz_sync();
      // per term, once: Ulc . e_{i-1} (left) and e_j . Urr (right), in place
      {
        const int lane = tid & 63, r = lane / 6, c = lane % 6;
        for (int b = cdz_wave_id(); b < nl + nr; b += CDZ_NT / 64) {
          T *blk = b < nl ? Ulc + b * 36 : Urr + (b - nl) * 36;
          T v = 0;
          if (lane < 36) {
            if (b < nl) {  // (Ulc . e_{i-1})(a, x) = sum_b U[i-l1][i-1](a,b) e_{i-1}(b,x)
#pragma unroll
              for (int k = 0; k < 6; k++) v += blk[r * 6 + k] * C.eIm1[k * 6 + c];
            } else {  // (e_j . Urr)(y, dd) = sum_c e_j(y,c) U[j+1][j+l2](c,dd)
#pragma unroll
              for (int k = 0; k < 6; k++) v += C.eJ[r * 6 + k] * blk[k * 6 + c];
            }
          }
          cdz_wave_sync();
          if (lane < 36) blk[lane] = v;
        }
      }
      cdz_sync();
      const int q = tid % 36, g = tid / 36, x = q / 6, y = q % 6;
      if (g < 7) {
        T acc = 0;
        for (int term = g; term < nl + nr; term += 7) {
          if (term < nl) {
            const int l1 = term + 1;
            const T f = tab[TB_BU + l1] * cdz_p2<T>(sE[l1 - 1] + sE[dl] - sE[dl + l1 + 2]);
            const T *m = Ulc + (l1 - 1) * 36, *gg = Gbc + (l1 - 1) * 36;
            T sm = 0;
#pragma unroll
            for (int a = 0; a < 6; a++) sm += m[a * 6 + x] * gg[a * 6 + y];
            acc += f * sm;
          } else {
            const int l2 = term - nl + 1;
            const T f = tab[TB_BU + l2] * cdz_p2<T>(sE[dl] + sE[l2 - 1] - sE[dl + l2 + 2]);
            const T *m = Urr + (l2 - 1) * 36, *gg = Gbr + (l2 - 1) * 36;
            T sm = 0;
#pragma unroll
            for (int dd = 0; dd < 6; dd++) sm += gg[x * 6 + dd] * m[y * 6 + dd];
            acc += f * sm;
          }
        }
        GP[g * 36 + q] = acc;
      }
      cdz_sync();
      if (tid < 36) {
        T s = 0;
#pragma unroll
        for (int gg = 0; gg < 7; gg++) s += GP[gg * 36 + tid];
        C.w[36 + tid] = s;
      }
      cdz_sync();
    }
  if (tid < 36) {
    const int s = tid / 6, t = tid % 6;
    if (s < di && t < dj) A.Qbb[(Pi + s) * ld + Pj + t] = C.w[36 + tid];
  }
}

// ---- finish of the cells of diagonal dl (launch dl)
template <typename T>
__device__ __forceinline__ void out_finish(const DevProb<T> &D, const DevAdj<T> &A, int dl, int blk) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = D.n, tid = threadIdx.x;
  const long long ld = D.ld;
  int *sE = reinterpret_cast<int *>(smem_raw);
  T *red = reinterpret_cast<T *>(smem_raw + ((size_t)(n + 1) * 4 + 15) / 16 * 16);
  OutStage<T> &C = *reinterpret_cast<OutStage<T> *>(red + (CDZ_NT / 64) * 72);
  T *AB = reinterpret_cast<T *>(reinterpret_cast<unsigned char *>(&C) + (sizeof(OutStage<T>) + 15) / 16 * 16);
  T *X = AB + 29 * 36;
  cdz_copy_exponents(sE, D.E, n, dl, 34);
  const int EZ = (int)D.res[2];
  const int i = cdz_cell_of_block(blk, n - dl), j = i + dl;
  if (i >= n - dl) return;
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
  if (tid >= 128) {
    const int q = tid - 128, grp = q / 32, o = q % 32;
    const int p = grp == 0 ? i + 1 + o : grp == 1 ? j - 1 - o : grp == 2 ? i - 1 - o : j + 1 + o;
    const bool ok = p >= 0 && p < n;
    C.wd[q] = ok ? D.d[p] : 0;
    C.wP[q] = ok ? D.P[p] : 0;
  }
  cdz_sync();
  const int di = C.d[1], dj = C.d[4], Pi = C.P[1], Pj = C.P[4];
  const int dim1 = C.d[0], Pim1 = C.P[0], djp1 = C.d[5], Pjp1 = C.P[5];
  const int d1 = C.d[2], dm = C.d[3], P1 = C.P[2], Pm = C.P[3];
  const bool hasL = i >= 1, hasR = j + 1 <= n - 1;
  const int *lp_d = C.wd, *lp_P = C.wP, *rp_d = C.wd + 32, *rp_P = C.wP + 32;
  const int *ll_d = C.wd + 64, *ll_P = C.wP + 64, *rr_d = C.wd + 96, *rr_P = C.wP + 96;
  {
    for (int idx = tid; idx < 8 * 36; idx += CDZ_NT) {
    const int g = idx / 36, q = idx % 36;
    switch (g) {
      case 0:
        ostage(C.m1pUp, A.Qm1pb, ld, Pim1, Pj, dim1, dj, q, hasL);
        ostage(C.m1Right, A.Qm1b, ld, Pi, Pjp1, di, djp1, q, hasR);
        break;
      case 1:
        ostage(C.qbOut, A.Qbb, ld, Pim1, Pjp1, dim1, djp1, q, hasL && hasR);
        ostage(C.gbOut, A.Gb, ld, Pi, Pj, di, dj, q, hasL && hasR);
        break;
      case 2:
        ostage(C.ubRight, A.Ub, ld, Pi, Pjp1, di, djp1, q, hasR);
        ostage(C.ubl, A.UbL, ld, Pi, Pj, di, dj, q, true);
        ostage_t(C.ubr, A.UbR, ld, Pi, Pj, di, dj, q, true);
        break;
      case 3:
        C.eIm1[q] = hasL ? D.e[(i - 1) * 36 + q] : T(0);
        C.eI[q] = D.e[i * 36 + q];
        C.eJm1[q] = j >= 1 ? D.e[(j - 1) * 36 + q] : T(0);
        C.eJ[q] = D.e[j * 36 + q];
        C.eI1[q] = i + 1 < n ? D.e[(i + 1) * 36 + q] : T(0);
        C.eJm2[q] = j >= 2 ? D.e[(j - 2) * 36 + q] : T(0);
        break;
      case 4:
        C.edm1[q] = hasL ? D.ed[(i - 1) * 36 + q] : 0.0;
        if (q < 6) {
          C.vIm1[q] = hasL ? D.v[(i - 1) * 6 + q] : T(0);
          C.vI[q] = D.v[i * 6 + q];
          C.vJ[q] = D.v[j * 6 + q];
          C.vJp1[q] = hasR ? D.v[(j + 1) * 6 + q] : T(0);
          C.vI1[q] = i + 1 < n ? D.v[(i + 1) * 6 + q] : T(0);
          C.vJm1[q] = j >= 1 ? D.v[(j - 1) * 6 + q] : T(0);
          C.z5[q] = hasL ? D.Z5[(i - 1) * 6 + q] : 0.0;
          C.z3[q] = D.Z3[j * 6 + q];
        }
        break;
      case 5: {
        // adjoint of DI at block (i-1, j+1): pushed by the enclosing loops
        T v = 0;
        const int r = q / 6, c = q % 6;
        if (hasL && hasR && r < dim1 && c < djp1) {
          const long long o = (long long)(Pim1 + r) * ld + Pjp1 + c, ot = (long long)(Pjp1 + c) * ld + Pim1 + r;
          v = A.DIbL[o] + A.DIbR[ot];
        }
        C.w[q] = v;
        break;
      }
      case 6: {  // split gathers of the cell, stored by out_split (diagonals 4..n-5)
        const bool sp = dl >= 4 && dl <= n - 5;
        ostage(C.acc, A.Qmb, ld, Pi, Pj, di, dj, q, sp);
        ostage(C.acc + 36, A.Qm1Lb, ld, Pim1, Pj, dim1, dj, q, sp && hasL);
        break;
      }
      case 7:  // bulge part of Qb' (out_bulge_gather, diagonals 4..n-2); bulge-pushed runs
        ostage(C.w + 36, A.Qbb, ld, Pi, Pj, di, dj, q, dl >= 4 && dl <= n - 2);
        ostage(C.ubl2, A.UbL2, ld, Pi, Pj, di, dj, q, true);
        ostage_t(C.ubr2, A.UbR2, ld, Pi, Pj, di, dj, q, true);
        break;
    }
    }
  }

  cdz_sync();
  const T *tab = C.tab;
  if (dl >= 4) {
    const int lmax = min(CDZ_MAXLOOP, dl - 6);
    const int s = tid / 6, t = tid % 6;
    // ---- Qm', QmX', Qm1p', Qm1L', DI' (all operands in LDS)
    if (tid < 36) {
      T qlb = 0;
      if (hasL && s < dim1 && t < dj) {
        qlb = C.acc[36 + tid];
        A.Qm1Lb[(Pim1 + s) * ld + Pj + t] = qlb;
      }
      C.qm1lb[tid] = qlb;
      if (hasL && hasR && s < dim1 && t < djp1) A.DIb[(Pim1 + s) * ld + Pjp1 + t] = C.w[tid];
      T qpb = 0;
      if (s < di && t < dj) {
        const T qmb = C.acc[tid];
        T qxb = qmb;
        if (hasL && hasR) qxb += tab[TB_MLAB] * cdz_p2<T>(sE[dl] - sE[dl + 2]) * C.gbOut[tid];
        qpb = qmb;
        if (hasL) {
          T a = 0;
#pragma unroll
          for (int q = 0; q < 6; q++) a += C.m1pUp[q * 6 + t] * C.vIm1[q] * C.eIm1[q * 6 + s];
          qpb += tab[TB_MLC] * cdz_p2<T>(sE[dl] - sE[dl + 1]) * a;
        }
        const long long o = (Pi + s) * ld + Pj + t;
        A.Qmb[o] = qmb;
        A.QmXb[o] = qxb;
        A.QmXbt[(Pj + t) * ld + Pi + s] = qxb;
        A.Qm1pb[o] = qpb;
      }
      C.qm1pb[tid] = qpb;
    }
    cdz_sync();
    // ---- Qm1'
    if (tid < 36) {
      T q1b = 0;
      if (s < di && t < dj) {
        q1b = C.qm1pb[tid];
#pragma unroll
        for (int b = 0; b < 6; b++) q1b += C.eIm1[b * 6 + s] * C.qm1lb[b * 6 + t];
        if (hasR) {
          T a = 0;
#pragma unroll
          for (int q = 0; q < 6; q++) a += C.m1Right[s * 6 + q] * C.vJp1[q] * C.eJ[t * 6 + q];
          q1b += tab[TB_MLC] * cdz_p2<T>(sE[dl] - sE[dl + 1]) * a;
        }
        A.Qm1b[(Pi + s) * ld + Pj + t] = q1b;
      }
      C.qm1b[tid] = q1b;
    }
    cdz_sync();
    // ---- Qb': thread (b, o) adds the interior-loop terms with outer slot b
    //      at i-1 and the stack terms with slot b at i-1 of output o = (x, y)
    if (tid < 216) {
      const int b = tid / 36, o = tid % 36, x = o / 6, y = o % 6;
      T part = 0;
      if (x < di && y < dj && hasL && hasR && b < dim1) {
        const int nx = C.nt[1][x], ny = C.nt[4][y];
        const int tin = cdz_ptype(ny, nx);  // inner pair read in loop order (j, i)
        const T eb = C.eIm1[b * 6 + x];
        if (tin >= 0) {
#pragma unroll
          for (int c = 0; c < 6; c++)
            if (c < djp1)
              part += C.w[b * 6 + c] * eb * C.eJ[y * 6 + c] * tab[TB_MM + C.nt[5][c] * 24 + C.nt[0][b] * 6 + tin];
        }
        const int txy = cdz_ptype(nx, ny);
        if (txy >= 0) {  // stacked under (i-1, j+1)
          const T f2 = cdz_p2<T>(sE[dl] - sE[dl + 2]);
#pragma unroll
          for (int r = 0; r < 6; r++) {
            const int to = cdz_ptype(C.nt[0][b], C.nt[5][r]);
            if (r < djp1 && to >= 0)
              part += C.qbOut[b * 6 + r] * C.vIm1[b] * C.vJp1[r] * eb * C.eJ[y * 6 + r] * tab[TB_ST + to * 6 + txy] * f2;
          }
        }
      }
      red[b * 36 + o] = part;
    }
    cdz_sync();
    if (tid < 36) {
      const int x = s, y = t;
      T qbb = 0;
      if (x < di && y < dj) {
        qbb = C.qm1b[tid] * tab[TB_MLB] + C.w[36 + tid];
#pragma unroll
        for (int b = 0; b < 6; b++) qbb += red[b * 36 + tid];
        {  // exterior loop: prefix before i, suffix after j (FP64)
          double zl = 1.0;
          int G = 0;
          if (hasL) {
            zl = 0;
#pragma unroll
            for (int q = 0; q < 6; q++) zl += C.z5[q] * C.edm1[q * 6 + x];
            G = D.G5[i - 1];
          }
          qbb += (T)(zl * C.z3[y] * ldexp(1.0, G + D.H3[j] + sE[dl] - EZ));
        }
        A.Qbb[(Pi + x) * ld + Pj + y] = qbb;
      }
      C.qbb[tid] = qbb;
    }
    cdz_sync();
    // ---- outer-edge-dressed adjoints of this cell's loop sums, block (i+1, j-1):
    //      thread (q, o) sums over the slot r of j for output o = (a, dd)
    if (tid < 216) {
      const int q = tid / 36, o = tid % 36, a = o / 6, dd = o % 6;
      T gb = 0, fb = 0;
      if (a < d1 && dd < dm && q < di) {
        const int na = C.nt[2][a], nd = C.nt[3][dd];
        const T wq = C.vI[q] * C.eI[q * 6 + a];
#pragma unroll
        for (int r = 0; r < 6; r++) {
          const int to = cdz_ptype(C.nt[1][q], C.nt[4][r]);
          if (r < dj && to >= 0) {
            const T w = C.qbb[q * 6 + r] * wq * C.vJ[r] * C.eJm1[dd * 6 + r];
            gb += w;
            fb += w * tab[TB_MM + na * 24 + nd * 6 + to];
          }
        }
      }
      X[q * 36 + o] = gb;
      X[216 + q * 36 + o] = fb;
    }
    cdz_sync();
    if (tid < 36) {
      const int a = s, dd = t;
      T gb = 0, fb = 0;
#pragma unroll
      for (int q = 0; q < 6; q++) {
        gb += X[q * 36 + tid];
        fb += X[216 + q * 36 + tid];
      }
      if (a < d1 && dd < dm) {
        A.Gb[(P1 + a) * ld + Pm + dd] = gb;
        A.Fb[(P1 + a) * ld + Pm + dd] = fb;
      }
      C.gb[tid] = gb;
      C.fb[tid] = fb;
    }
    cdz_sync();
    // ---- adjoints of the interior-loop sums by size, AB[L-2] = A'(i,j,L):
    //      from F (F = sum_L w_int(L) A) and, through the size recursion,
    //      from the enclosing cell (i-1, j+1) at size L + 2 (kept in a ring
    //      of three diagonals)
    const bool pull = hasL && hasR && lmax >= 2;
    {
      T *APV = X, *TB = X + 27 * 36;
      const int npull = pull ? min(lmax, 28) - 1 : 0;  // L = 2..min(lmax, 28)
      for (int idx = tid; idx < npull * 36; idx += CDZ_NT) {
        const int b = idx / 36, q = idx % 36;
        APV[idx] = ring_at(A, n, dl + 2, i - 1, b + 4)[q];
      }
      cdz_sync();
      // TB(a, d') = sum_dd A'(i-1,j+1,L+2)(a,dd) e_{j-1}(d',dd) v_j(dd)
      for (int idx = tid; idx < npull * 36; idx += CDZ_NT) {
        const int b = idx / 36, q = idx % 36, a = q / 6, d2 = q % 6;
        T v = 0;
#pragma unroll
        for (int dd = 0; dd < 6; dd++) v += APV[b * 36 + a * 6 + dd] * C.eJm1[d2 * 6 + dd] * C.vJ[dd];
        TB[idx] = v;
      }
      cdz_sync();
      const T frA = pull ? cdz_p2<T>(sE[dl] - sE[dl + 2]) : T(0);
      for (int idx = tid; idx < 29 * 36; idx += CDZ_NT) {
        const int L = idx / 36 + 2, q = idx % 36, a2 = q / 6, d2 = q % 6;
        T v = 0;
        if (L <= lmax) {
          v = tab[TB_IN + L] * C.fb[q];
          if (L - 2 < npull) {
            T r = 0;
#pragma unroll
            for (int a = 0; a < 6; a++) r += C.vI[a] * C.eI[a * 6 + a2] * TB[(L - 2) * 36 + a * 6 + d2];
            v += frA * r;
          }
        }
        AB[idx] = v;
        ring_at(A, n, dl, i, L)[q] = v;
      }
      cdz_sync();
    }
    // hairpin closed by (i, j): its run i+1..j-1 (block distinct from the runs above)
    if (tid < 36 && s < d1 && t < dm)
      A.UbL[(P1 + s) * ld + Pm + t] += D.Bhp[dl - 1] * cdz_p2<T>(sE[dl - 2] - sE[dl]) * C.fb[tid];
  } else if (tid < 36) {
    const int s = tid / 6, t = tid % 6;
    if (s < di && t < dj) {
      const long long o = (Pi + s) * ld + Pj + t;
      A.Qbb[o] = 0;
      A.Qm1b[o] = 0;
      A.Qm1pb[o] = 0;
      A.QmXb[o] = 0;
      A.Qmb[o] = 0;
      A.QmXbt[(Pj + t) * ld + Pi + s] = 0;
    }
  }
  // ---- total adjoint of the unpaired run [i..j]: the runs pushed into by
  //      enclosing interior loops (UbL, UbR), bulges (UbL2, UbR2) and
  //      hairpins (UbL), and the run extended by j + 1
  if (tid < 36) {
    const int a = tid / 6, c = tid % 6;
    if (a < di && c < dj) {
      T u = C.ubl[tid] + C.ubr[tid] + C.ubl2[tid] + C.ubr2[tid];
      if (hasR) {
        T sm = 0;
#pragma unroll
        for (int b = 0; b < 6; b++) sm += C.ubRight[a * 6 + b] * C.eJ[c * 6 + b] * C.vJp1[b];
        u += sm * cdz_p2<T>(sE[dl] - sE[dl + 1]);
      }
      A.Ub[(Pi + a) * ld + Pj + c] = u;
    }
  }
}


// ---- interior-loop pushes of the cells of diagonal dl (launch dl - 1), from
//      the adjoints by size that the finish of the cell left in the ring
template <typename T>
__device__ __forceinline__ void out_int_push(const DevProb<T> &D, const DevAdj<T> &A, int dl, int blk) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = D.n, tid = threadIdx.x;
  const long long ld = D.ld;
  int *sE = reinterpret_cast<int *>(smem_raw);
  T *red = reinterpret_cast<T *>(smem_raw + ((size_t)(n + 1) * 4 + 15) / 16 * 16);
  OutStage<T> &C = *reinterpret_cast<OutStage<T> *>(red + (CDZ_NT / 64) * 72);
  T *AB = reinterpret_cast<T *>(reinterpret_cast<unsigned char *>(&C) + (sizeof(OutStage<T>) + 15) / 16 * 16);
  T *X = AB + 29 * 36;
  cdz_copy_exponents(sE, D.E, n, dl, 34);
  const int EZ = (int)D.res[2];
  const int i = cdz_cell_of_block(blk, n - dl), j = i + dl;
  if (i >= n - dl) return;
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
  if (tid >= 128) {
    const int q = tid - 128, grp = q / 32, o = q % 32;
    const int p = grp == 0 ? i + 1 + o : grp == 1 ? j - 1 - o : grp == 2 ? i - 1 - o : j + 1 + o;
    const bool ok = p >= 0 && p < n;
    C.wd[q] = ok ? D.d[p] : 0;
    C.wP[q] = ok ? D.P[p] : 0;
  }
  if (tid < 36) {
    C.eI1[tid] = i + 1 < n ? D.e[(i + 1) * 36 + tid] : T(0);
    C.eJm2[tid] = j >= 2 ? D.e[(j - 2) * 36 + tid] : T(0);
    if (tid < 6) {
      C.vI1[tid] = i + 1 < n ? D.v[(i + 1) * 6 + tid] : T(0);
      C.vJm1[tid] = j >= 1 ? D.v[(j - 1) * 6 + tid] : T(0);
    }
  }
  const int lmax = min(CDZ_MAXLOOP, dl - 6);
  for (int idx = tid; idx < (lmax - 1) * 36; idx += CDZ_NT) AB[idx] = ring_at(A, n, dl, i, idx / 36 + 2)[idx % 36];
  cdz_sync();
  const int di = C.d[1], dj = C.d[4], Pi = C.P[1], Pj = C.P[4];
  const int dim1 = C.d[0], Pim1 = C.P[0], djp1 = C.d[5], Pjp1 = C.P[5];
  const int d1 = C.d[2], dm = C.d[3], P1 = C.P[2], Pm = C.P[3];
  const bool hasL = i >= 1, hasR = j + 1 <= n - 1;
  const int *lp_d = C.wd, *lp_P = C.wP, *rp_d = C.wd + 32, *rp_P = C.wP + 32;
  const int *ll_d = C.wd + 64, *ll_P = C.wP + 64, *rr_d = C.wd + 96, *rr_P = C.wP + 96;
    if (lmax >= 2) {
      // ---- interior loops closed by (i, j): adjoints of the blocks the size
      //      recursion reads directly (the l1 = 1 and l2 = 1 terms)
      T *UR1 = X, *UC1 = X + 30 * 36, *DIrow = X + 60 * 36, *DIcol = X + 89 * 36;
      {
        // the forward's window staging: contiguous rows (U, DI, and their
        // transposes for the column strips), placed by state-to-position maps
        // into blocks cleared first for the padding
        const int baseL = lp_P[0], baseR = rp_P[lmax];
        cdz_window_maps(C.mapL, C.mapR, lp_d, lp_P, rp_d, rp_P, lmax);
        uint4 *w4 = reinterpret_cast<uint4 *>(X);
        for (int idx = tid; idx < 118 * 36 * (int)sizeof(T) / 16; idx += CDZ_NT) w4[idx] = make_uint4(0, 0, 0, 0);
        cdz_sync();
        const int KU = lp_P[lmax] - baseL;                        // end states of U[i+1][i+1..i+lmax]
        const int endR = rp_P[0] + rp_d[0] - baseR;               // right map: positions j-1-lmax..j-1
        const int oC = rp_P[lmax - 1] - baseR, KC = endR - oC;    // start states of U[j-lmax..j-1][j-1]
        const int oD = rp_P[lmax - 2] - baseR, KD = endR - oD;    // DI[i+1][j-lmax+1..j-1]
        const int oL = lp_P[1] - baseL;                           // DI[i+2..i+lmax-1][j-1]
        const int KL = lmax >= 3 ? lp_P[lmax - 1] - lp_P[1] : 0;
        const int e1 = d1 * KU, e2 = e1 + dm * KC, e3 = e2 + d1 * KD, e4 = e3 + dm * KL;
        // X offsets: UR1 0, UC1 30*36, DIrow 60*36, DIcol 89*36
        cdz_stage_nv<3, T>(X, e4, [&](int idx, int &d) -> const T * {
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
          // DI[i+L-1][j-1]: row Pm + c of DIt, L = qq + 2
          const int t = idx - e3, c = t / KL, k = t % KL + oL, qq = C.mapL[k], r = k - (lp_P[qq] - baseL);
          d = (89 + qq) * 36 + r * 6 + c;
          return D.DIt + (long long)(Pm + c) * ld + baseL + k;
        });
      }
      cdz_sync();
      // every target block is updated by exactly one thread; all old values
      // are fetched first so that the loads are in flight together
      constexpr int NPT = (4 * 29 * 36 + CDZ_NT - 1) / CDZ_NT;
      // targets first, so that the old values are in flight while the pushed
      // values are formed from LDS
      int off[NPT];
#pragma unroll
      for (int m = 0; m < NPT; m++) {
        const int idx = tid + m * CDZ_NT;
        off[m] = -1;
        if (idx >= 4 * 29 * 36) continue;
        const int kind = idx / (29 * 36), rem = idx % (29 * 36), L = rem / 36 + 2, q = rem % 36;
        const int r = q / 6, c = q % 6;
        if (L > lmax || (L < 3 && (kind == 1 || kind == 3))) continue;
        if (kind == 0) {  // DI'[i+1][j-L+1](a, c)
          if (r < d1 && c < rp_d[L - 2]) off[m] = (P1 + r) * (int)ld + rp_P[L - 2] + c;
        } else if (kind == 1) {  // DI'[i+L-1][j-1](b, dd), DIbR stored transposed
          if (r < lp_d[L - 2] && c < dm) off[m] = (Pm + c) * (int)ld + lp_P[L - 2] + r;
        } else if (kind == 2) {  // U'[j-L+1][j-1](c, dd), run of L - 1, UbR stored transposed
          if (r < rp_d[L - 2] && c < dm) off[m] = (Pm + c) * (int)ld + rp_P[L - 2] + r;
        } else {  // U'[i+1][i+L-1](a, b), run of L - 1
          if (r < d1 && c < lp_d[L - 2]) off[m] = (P1 + r) * (int)ld + lp_P[L - 2] + c;
        }
      }
      auto target = [&](int m) -> T * {
        const int kind = (tid + m * CDZ_NT) / (29 * 36);
        T *base = kind == 0 ? A.DIbL : kind == 1 ? A.DIbR : kind == 2 ? A.UbR : A.UbL;
        return base + off[m];
      };
      T old[NPT];
#pragma unroll
      for (int m = 0; m < NPT; m++) old[m] = off[m] >= 0 ? *target(m) : T(0);
#pragma unroll
      for (int m = 0; m < NPT; m++) {
        if (off[m] < 0) continue;
        const int idx = tid + m * CDZ_NT;
        const int kind = idx / (29 * 36), rem = idx % (29 * 36), L = rem / 36 + 2, q = rem % 36;
        const int r = q / 6, c = q % 6;
        const T fb = cdz_p2<T>(sE[dl - L - 2] + sE[L - 2] - sE[dl]);
        const T *ab = AB + (L - 2) * 36;
        T v = 0, val;
        if (kind == 0) {
#pragma unroll
          for (int dd = 0; dd < 6; dd++) v += ab[r * 6 + dd] * UC1[(L - 2) * 36 + c * 6 + dd];
          val = fb * C.vI1[r] * v;
        } else if (kind == 1) {
#pragma unroll
          for (int a = 0; a < 6; a++) v += UR1[(L - 2) * 36 + a * 6 + r] * ab[a * 6 + c];
          val = fb * C.vJm1[c] * v;
        } else if (kind == 2) {
#pragma unroll
          for (int a = 0; a < 6; a++) v += C.vI1[a] * DIrow[(L - 2) * 36 + a * 6 + r] * ab[a * 6 + c];
          val = fb * v;
        } else {
#pragma unroll
          for (int dd = 0; dd < 6; dd++) v += ab[r * 6 + dd] * C.vJm1[dd] * DIcol[(L - 2) * 36 + c * 6 + dd];
          val = fb * v;
        }
        *target(m) = old[m] + val;
      }
      __syncthreads();  // the bulge pushes below update some of the same runs
    }
}

// ---- edge terms of the size recursion of the cells of diagonal dl (launch
//      dl - 1): the uses of e_{i+1} in V and e_{j-2} in W, from the cell's
//      adjoints by size (ring) and A of the inner cell, into etaV / etaW
template <typename T>
__device__ __forceinline__ void out_edge_terms(const DevProb<T> &D, const DevAdj<T> &A, int dl, int blk) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = D.n, tid = threadIdx.x;
  const long long ld = D.ld;
  int *sE = reinterpret_cast<int *>(smem_raw);
  T *red = reinterpret_cast<T *>(smem_raw + ((size_t)(n + 1) * 4 + 15) / 16 * 16);
  OutStage<T> &C = *reinterpret_cast<OutStage<T> *>(red + (CDZ_NT / 64) * 72);
  T *AB = reinterpret_cast<T *>(reinterpret_cast<unsigned char *>(&C) + (sizeof(OutStage<T>) + 15) / 16 * 16);
  T *X = AB + 29 * 36;
  cdz_copy_exponents(sE, D.E, n, dl, 34);
  const int EZ = (int)D.res[2];
  const int i = cdz_cell_of_block(blk, n - dl), j = i + dl;
  if (i >= n - dl) return;
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
  if (tid >= 128) {
    const int q = tid - 128, grp = q / 32, o = q % 32;
    const int p = grp == 0 ? i + 1 + o : grp == 1 ? j - 1 - o : grp == 2 ? i - 1 - o : j + 1 + o;
    const bool ok = p >= 0 && p < n;
    C.wd[q] = ok ? D.d[p] : 0;
    C.wP[q] = ok ? D.P[p] : 0;
  }
  if (tid < 36) {
    C.eI1[tid] = i + 1 < n ? D.e[(i + 1) * 36 + tid] : T(0);
    C.eJm2[tid] = j >= 2 ? D.e[(j - 2) * 36 + tid] : T(0);
    if (tid < 6) {
      C.vI1[tid] = i + 1 < n ? D.v[(i + 1) * 6 + tid] : T(0);
      C.vJm1[tid] = j >= 1 ? D.v[(j - 1) * 6 + tid] : T(0);
    }
  }
  const int lmax = min(CDZ_MAXLOOP, dl - 6);
  for (int idx = tid; idx < (lmax - 1) * 36; idx += CDZ_NT) AB[idx] = ring_at(A, n, dl, i, idx / 36 + 2)[idx % 36];
  cdz_sync();
  const int di = C.d[1], dj = C.d[4], Pi = C.P[1], Pj = C.P[4];
  const int dim1 = C.d[0], Pim1 = C.P[0], djp1 = C.d[5], Pjp1 = C.P[5];
  const int d1 = C.d[2], dm = C.d[3], P1 = C.P[2], Pm = C.P[3];
  const bool hasL = i >= 1, hasR = j + 1 <= n - 1;
  const int *lp_d = C.wd, *lp_P = C.wP, *rp_d = C.wd + 32, *rp_P = C.wP + 32;
  const int *ll_d = C.wd + 64, *ll_P = C.wP + 64, *rr_d = C.wd + 96, *rr_P = C.wP + 96;
    if (lmax >= 4) {
      // ---- edges e_{i+1} (in V) and e_{j-2} (in W) of the size recursion:
      //      their share of the edge marginals
      T *AP = X, *TM = X + 27 * 36, *SM = X + 54 * 36;
      const int nAP = lmax - 3;  // A(i+1, j-1, L'), L' = 2..lmax-2
      for (int idx = tid; idx < nAP * 36; idx += CDZ_NT) {
        const int b = idx / 36, q = idx % 36, r = q / 6, c = q % 6;
        T v = 0;
        if (r < lp_d[1] && c < rp_d[1])
          v = D.AL ? D.AL[(long long)(lp_P[1] + r) * D.ldA + (long long)CDZ_NA * rp_P[1] + b * rp_d[1] + c]
                   : D.ALp[(long long)(i + 1) * (CDZ_NA * 36) + b * 36 + q];
        AP[idx] = v;
      }
      cdz_sync();
      for (int idx = tid; idx < nAP * 36; idx += CDZ_NT) {
        const int b = idx / 36, q = idx % 36, r = q / 6, c = q % 6;
        T tm = 0, sm = 0;
#pragma unroll
        for (int u = 0; u < 6; u++) {
          tm += AP[b * 36 + r * 6 + u] * C.eJm2[u * 6 + c];
          sm += C.eI1[r * 6 + u] * AP[b * 36 + u * 6 + c];
        }
        TM[idx] = tm * C.vJm1[c];  // (A . W)(a', dd)
        SM[idx] = C.vI1[r] * sm;   // (V . A)(a, d')
      }
      cdz_sync();
      const T frec = cdz_p2<T>(sE[dl - 2] - sE[dl]);
      if (tid < 72) {
        const int q = tid % 36, r = q / 6, c = q % 6;
        T v = 0;
        if (tid < 36) {  // e_{i+1}(a, a') with (a, a') = (r, c)
          for (int L = 4; L <= lmax; L++)
#pragma unroll
            for (int dd = 0; dd < 6; dd++) v += AB[(L - 2) * 36 + r * 6 + dd] * TM[(L - 4) * 36 + c * 6 + dd];
          v *= frec * C.vI1[r] * C.eI1[q];
          A.etaV[(long long)(i + 1) * 36 + q] += (double)v;
        } else {  // e_{j-2}(d', dd) with (d', dd) = (r, c)
          for (int L = 4; L <= lmax; L++)
#pragma unroll
            for (int a = 0; a < 6; a++) v += AB[(L - 2) * 36 + a * 6 + c] * SM[(L - 4) * 36 + a * 6 + r];
          v *= frec * C.eJm2[q] * C.vJm1[c];
          A.etaW[(long long)(j - 2) * 36 + q] += (double)v;
        }
      }
      cdz_sync();
    }
}

// ---- bulge pushes of the cells of diagonal dl (launch dl - 1): run adjoints
//      of the bulges closed by (i, j), from the cell's Gb, into UbL2 / UbR2
template <typename T>
__device__ __forceinline__ void out_bulge_push(const DevProb<T> &D, const DevAdj<T> &A, int dl, int blk) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int n = D.n, tid = threadIdx.x;
  const long long ld = D.ld;
  int *sE = reinterpret_cast<int *>(smem_raw);
  T *red = reinterpret_cast<T *>(smem_raw + ((size_t)(n + 1) * 4 + 15) / 16 * 16);
  OutStage<T> &C = *reinterpret_cast<OutStage<T> *>(red + (CDZ_NT / 64) * 72);
  T *AB = reinterpret_cast<T *>(reinterpret_cast<unsigned char *>(&C) + (sizeof(OutStage<T>) + 15) / 16 * 16);
  T *X = AB + 29 * 36;
  cdz_copy_exponents(sE, D.E, n, dl, 34);
  const int EZ = (int)D.res[2];
  const int i = cdz_cell_of_block(blk, n - dl), j = i + dl;
  if (i >= n - dl) return;
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
  if (tid >= 128) {
    const int q = tid - 128, grp = q / 32, o = q % 32;
    const int p = grp == 0 ? i + 1 + o : grp == 1 ? j - 1 - o : grp == 2 ? i - 1 - o : j + 1 + o;
    const bool ok = p >= 0 && p < n;
    C.wd[q] = ok ? D.d[p] : 0;
    C.wP[q] = ok ? D.P[p] : 0;
  }
  {
    const int P1g = D.P[i + 1], Pmg = D.P[j - 1], d1g = D.d[i + 1], dmg = D.d[j - 1];
    if (tid < 36) ostage(C.gb, A.Gb, ld, P1g, Pmg, d1g, dmg, tid, true);
  }
  cdz_sync();
  const int di = C.d[1], dj = C.d[4], Pi = C.P[1], Pj = C.P[4];
  const int dim1 = C.d[0], Pim1 = C.P[0], djp1 = C.d[5], Pjp1 = C.P[5];
  const int d1 = C.d[2], dm = C.d[3], P1 = C.P[2], Pm = C.P[3];
  const bool hasL = i >= 1, hasR = j + 1 <= n - 1;
  const int *lp_d = C.wd, *lp_P = C.wP, *rp_d = C.wd + 32, *rp_P = C.wP + 32;
  const int *ll_d = C.wd + 64, *ll_P = C.wP + 64, *rr_d = C.wd + 96, *rr_P = C.wP + 96;
  const T *tab = C.tab;
  const int lmax = min(CDZ_MAXLOOP, dl - 6);
    if (lmax >= 1) {
      // ---- bulges closed by (i, j): adjoints of their runs. Left bulge
      //      l1: run i+1..i+l1, inner pair (i+l1+1, j-1); right bulge l2:
      //      inner pair (i+1, j-1-l2), run j-l2..j-1.
      T *EL = X, *ER = X + 30 * 36, *QL = X + 60 * 36, *QR = X + 90 * 36;
      // e blocks (contiguous in D.e); the Qb blocks of the inner pairs, the
      // left column strip as contiguous rows of Qbt and the right row strip as
      // one contiguous segment of a row of Qb, placed by the window maps into
      // blocks cleared first
      cdz_window_maps(C.mapL, C.mapR, lp_d, lp_P, rp_d, rp_P, lmax);
      cdz_copy_blocks<T>(EL, D.e + (long long)(i + 1) * 36, lmax, false);       // e_{i+l}
      cdz_copy_blocks<T>(ER, D.e + (long long)(j - 1 - lmax) * 36, lmax, true);  // e_{j-1-l}
      cdz_zero_blocks<T>(QL, lmax);
      cdz_zero_blocks<T>(QR, lmax);
      cdz_sync();
      {
        const int oq = lp_P[1] - lp_P[0], KQ = lp_P[lmax + 1] - lp_P[1];  // positions i+2..i+1+lmax
        const int baseR = rp_P[lmax], KR = rp_P[1] + rp_d[1] - baseR;     // positions j-1-lmax..j-2
        const int e1 = dm * KQ;
        for (int idx = tid; idx < e1 + d1 * KR; idx += CDZ_NT) {
          if (idx < e1) {  // Qb[i+1+l][j-1](x, c): row Pm + c of Qbt
            const int c = idx / KQ, k = idx % KQ + oq, l = C.mapL[k], x = k - (lp_P[l] - lp_P[0]);
            QL[(l - 1) * 36 + x * 6 + c] = D.Qbt[(long long)(Pm + c) * ld + lp_P[0] + k];
          } else {  // Qb[i+1][j-1-l](r, c): row P1 + r of Qb
            const int t = idx - e1, r = t / KR, k = t % KR, l = C.mapR[k], c = k - (rp_P[l] - baseR);
            QR[(l - 1) * 36 + r * 6 + c] = D.Qb[(long long)(P1 + r) * ld + baseR + k];
          }
        }
      }
      cdz_sync();
      // per term, once and in place: R(a, x) = sum_y Gb(a,y) Qb[k][j-1](x,y)
      // (left) and S(y, dd) = sum_x Qb[i+1][l](x,y) Gb(x,dd) (right)
      {
        const int lane = tid & 63, r = lane / 6, c = lane % 6;
        for (int b = cdz_wave_id(); b < 2 * lmax; b += CDZ_NT / 64) {
          T *blk = b < lmax ? QL + b * 36 : QR + (b - lmax) * 36;
          T v = 0;
          if (lane < 36) {
            if (b < lmax) {
#pragma unroll
              for (int k = 0; k < 6; k++) v += C.gb[r * 6 + k] * blk[c * 6 + k];
            } else {
#pragma unroll
              for (int k = 0; k < 6; k++) v += blk[k * 6 + r] * C.gb[k * 6 + c];
            }
          }
          cdz_wave_sync();
          if (lane < 36) blk[lane] = v;
        }
      }
      cdz_sync();
      constexpr int NPB = (2 * 30 * 36 + CDZ_NT - 1) / CDZ_NT;
      // targets first (their old values in flight while the pushes are formed)
      int off[NPB];
#pragma unroll
      for (int m = 0; m < NPB; m++) {
        const int idx = tid + m * CDZ_NT;
        off[m] = -1;
        if (idx >= 2 * lmax * 36) continue;
        const int b = idx / 36, q = idx % 36, r = q / 6, c = q % 6;
        const int side = b / lmax, l = b % lmax + 1;
        if (side == 0) {  // U'[i+1][i+l](a, b)
          if (r < d1 && c < lp_d[l - 1]) off[m] = (P1 + r) * (int)ld + lp_P[l - 1] + c;
        } else {  // U'[j-l][j-1](c, dd), UbR stored transposed
          if (r < rp_d[l - 1] && c < dm) off[m] = (Pm + c) * (int)ld + rp_P[l - 1] + r;
        }
      }
      T old[NPB];
#pragma unroll
      for (int m = 0; m < NPB; m++) {
        const bool left = (tid + m * CDZ_NT) / 36 < lmax;
        old[m] = off[m] >= 0 ? (left ? A.UbL2 : A.UbR2)[off[m]] : T(0);
      }
#pragma unroll
      for (int m = 0; m < NPB; m++) {
        if (off[m] < 0) continue;
        const int idx = tid + m * CDZ_NT;
        const int b = idx / 36, q = idx % 36, r = q / 6, c = q % 6;
        const int side = b / lmax, l = b % lmax + 1;
        const T *el = (side == 0 ? EL : ER) + (l - 1) * 36, *qk = (side == 0 ? QL : QR) + (l - 1) * 36;
        const T f = tab[TB_BU + l] * cdz_p2<T>(sE[l - 1] + sE[dl - 2 - l] - sE[dl]);
        T v = 0;
        if (side == 0) {  // U'[i+1][i+l](a, b) = sum_x e_{k-1}(b,x) R(a,x)
#pragma unroll
          for (int x = 0; x < 6; x++) v += el[c * 6 + x] * qk[r * 6 + x];
        } else {  // U'[j-l][j-1](c, dd) = sum_y e_l(y,c) S(y,dd)
#pragma unroll
          for (int y = 0; y < 6; y++) v += el[y * 6 + r] * qk[y * 6 + c];
        }
        (side == 0 ? A.UbL2 : A.UbR2)[off[m]] = old[m] + f * v;
      }
    }
}

// One workgroup of outside launch t; w is its index among this problem's workgroups
template <typename T, bool FUSED>
__device__ __forceinline__ void out_block(const DevProb<T> &D, const DevAdj<T> &A, int t, int w) {
  // split: one block of one kind (kinds numbered in turn); fused: block w of
  // every kind that has one, in turn (LDS is reused); separate kernels
  int r[6], wk[6];
  out_ranges(D.n, t, r);
  int base = 0;
#pragma unroll
  for (int k = 0; k < 6; k++) {
    const int x = FUSED ? w : w - base;
    wk[k] = x >= 0 && x < r[k] ? x : -1;
    base += r[k];
  }
  if (wk[0] >= 0) {
    out_int_push<T>(D, A, t + 1, wk[0]);
    if (FUSED) __syncthreads();
    else return;
  }
  if (wk[1] >= 0) {
    out_edge_terms<T>(D, A, t + 1, wk[1]);
    if (FUSED) __syncthreads();
    else return;
  }
  if (wk[2] >= 0) {
    out_bulge_push<T>(D, A, t + 1, wk[2]);
    if (FUSED) __syncthreads();
    else return;
  }
  if (wk[3] >= 0) {
    out_bulge_gather<T>(D, A, t - 1, wk[3]);
    if (FUSED) __syncthreads();
    else return;
  }
  if (wk[4] >= 0) {
    out_split<T>(D, A, t - 4, wk[4]);
    if (FUSED) __syncthreads();
    else return;
  }
  if (wk[5] >= 0) out_finish<T>(D, A, t, wk[5]);
}


// ---------------------------------------------------------------------------
// Edge marginals: one workgroup per backbone edge p (between p and p+1)
// gathers every term of dZ/de_p * e_p.  Terms come from the cells whose
// statements use e_p: row p (edge right after a closing base), row p+1
// (edge right before a pair / run start), column p+1 and column p.
// ---------------------------------------------------------------------------
// Edge marginals of edge p (between positions p and p+1): the cells whose
// loops or runs use e_p, i.e. (p+1, j) and (p, j) to the right and (i, p+1),
// (i, p) to the left, plus the exterior step over the edge.  One workgroup
// per edge; each wavefront takes one cell at a time and lane q < 36 owns
// output (u, w) = (q / 6, q % 6), the slots of positions p and p+1.
template <typename T>
__device__ __forceinline__ void eta_edge(const DevProb<T> &D, const DevAdj<T> &A, int p, int LCH) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  constexpr int ENT = cdz_eta_nt(sizeof(T));
  const int n = D.n, tid = threadIdx.x, lane = tid & 63, wv = cdz_wave_id();
  const long long ld = D.ld;
  // LDS: exponents, slot counts and offsets of every position (so that the
  // loops below issue one level of global loads), then reduction scratch;
  // LCH = eta_bulge_chunk of the length the launch's LDS was sized for
  int *sE = reinterpret_cast<int *>(smem_raw);
  int *sd = sE + (n + 1), *sP = sd + (n + 1);
  double *red = reinterpret_cast<double *>(smem_raw + ((size_t)3 * (n + 1) * 4 + 15) / 16 * 16);
  double *Mw = red + (ENT / 64) * 36 + wv * 36;  // per-wave bulge partial products
  // the unpaired runs of the bulges through this edge, shared by its cells:
  // Ubl[l1 - 1](a, b) = U(p + 1 - l1 slot a, p slot b) (left bulges of the
  // cells (p+1, j)), Ubr[l2 - 1](q, c) = U(p+1 slot c, p + l2 slot q) (right
  // bulges of the cells (i, p)), zero outside the slots
  T *Ubl = reinterpret_cast<T *>(red + 2 * (ENT / 64) * 36);
  T *Ubr = Ubl + CDZ_MAXLOOP * 36;
  T *Gw = Ubr + CDZ_MAXLOOP * 36 + wv * LCH * 36;  // per wave: LCH loop sizes of a cell's bulge adjoints
  T *tab = Ubr + CDZ_MAXLOOP * 36 + (ENT / 64) * LCH * 36;  // [TB_LEN] Boltzmann tables
  // per wave: U, QmX, Qb, G, F of an inner block, then the edge factors e of
  // the position a cell's dressing sums over
  T *Xw = tab + (TB_LEN + 7) / 8 * 8 + wv * 6 * 36;
  T *Ew = Xw + 5 * 36;
  int *Nw = reinterpret_cast<int *>(tab + (TB_LEN + 7) / 8 * 8 + (ENT / 64) * 6 * 36) + wv * 12;
  for (int k = tid; k < n; k += ENT) {
    sE[k] = D.E[k];
    sd[k] = D.d[k];
    sP[k] = D.P[k];
  }
  for (int k = tid; k < TB_LEN; k += ENT) tab[k] = D.tab[k];
  const int dp = D.d[p], dq = D.d[p + 1], Pp = D.P[p], Pq = D.P[p + 1];
  const int l1top = min(CDZ_MAXLOOP, p), l2top = min(CDZ_MAXLOOP, n - 2 - p);
  for (int k = tid; k < CDZ_MAXLOOP * 36; k += ENT) {
    const int l = k / 36 + 1, r1 = (k % 36) / 6, r2 = k % 6;
    T xl = 0, xr = 0;
    if (l <= l1top && r2 < dp) {  // (a, b) = (r1, r2)
      const int pa = p + 1 - l;
      if (r1 < D.d[pa]) xl = D.Ut[(long long)(Pp + r2) * ld + D.P[pa] + r1];
    }
    if (l <= l2top && r2 < dq) {  // (q, c) = (r1, r2)
      const int pz = p + l;
      if (r1 < D.d[pz]) xr = D.U[(long long)(Pq + r2) * ld + D.P[pz] + r1];
    }
    Ubl[k] = xl;
    Ubr[k] = xr;
  }
  __syncthreads();
  const int EZ = (int)D.res[2];
  const T *ep = D.e + p * 36;
  // The wave stages block (i+1, j-1) of the loop closed by (i, j) (lane q =
  // (a, dd)), the bases of positions i+1 and j-1 and the edge factors e_pe;
  // inner(a, dd, to) is then the inner part of that loop for outer pair type
  // to: hairpin, stack, multiloop, bulge and interior terms with the outer
  // edges removed, in the units of the cell (i, j).
  auto stage_inner = [&](int i, int j, int pe) {
    if (lane < 36) {
      const int a = lane / 6, dd = lane % 6;
      const bool ok = a < sd[i + 1] && dd < sd[j - 1];
      const long long o = (long long)(sP[i + 1] + a) * ld + sP[j - 1] + dd;
      Xw[lane] = ok ? D.U[o] : T(0);
      Xw[36 + lane] = ok ? D.QmX[o] : T(0);
      Xw[72 + lane] = ok ? D.Qb[o] : T(0);
      Xw[108 + lane] = ok ? D.G[o] : T(0);
      Xw[144 + lane] = ok ? D.F[o] : T(0);
      Ew[lane] = D.e[pe * 36 + lane];
    } else if (lane < 48) {
      const int q = lane - 36;
      Nw[q] = q < 6 ? D.nt[(i + 1) * 6 + q] : D.nt[(j - 1) * 6 + q - 6];
    }
    cdz_wave_sync();
  };
  auto inner = [&](int a, int dd, int to, int dl) -> T {
    const int q = a * 6 + dd, na = Nw[a], nd = Nw[6 + dd];
    const T mm = tab[TB_MM + na * 24 + nd * 6 + to];
    T x = D.Bhp[dl - 1] * Xw[q] * mm + tab[TB_MLAB] * Xw[36 + q];
    if (dl - 2 >= 4) {
      const int t2 = cdz_ptype(na, nd);
      if (t2 >= 0) x += Xw[72 + q] * tab[TB_ST + to * 6 + t2];
    }
    return x * cdz_p2<T>(sE[dl - 2] - sE[dl]) + Xw[108 + q] + Xw[144 + q] * mm;
  };
  const int u = lane / 6, w = lane % 6;
  const bool own = lane < 36 && u < dp && w < dq;  // this lane's output exists
  double acc = 0;
  const int nR1 = n - p - 5 > 0 ? n - p - 5 : 0;  // cells (p+1, j), j >= p+5
  const int nR0 = n - p - 4 > 0 ? n - p - 4 : 0;  // cells (p, j), j >= p+4
  const int nC1 = p + 2;                          // cells (i, p+1), i <= p+1
  const int nC0 = p - 3 > 0 ? p - 3 : 0;          // cells (i, p), i <= p-4
  const int total = nR1 + nR0 + nC1 + nC0;
  for (int it = wv; it < total; it += ENT / 64) {
    int k = it;
    if (k < nR1) {
      // ---- cell (i, j) = (p+1, j): the edge before its first base;
      //      output (b, x) = (u, w), x a slot of i
      const int i = p + 1, j = p + 5 + k, dl = j - i, di = dq, dj = sd[j], Pj = sP[j];
      const long long Pi = Pq;
      const int b = u, x = w;
      if (j + 1 <= n - 1) {
        const T ev = lane < 36 ? D.e[j * 36 + lane] : T(0);  // e_j, into Ew with M
        // left bulges with inner pair (i, j): lane (b, y) forms
        // M(b, y) = sum_l1 f sum_a Gb(a, y) U(a, b) for the wave, the
        // adjoints Gb(i - l1 slot a, j slot y) staged LCH loop sizes at a time
        // (one round of loads each), the runs U from Ubl
        {
          const int y = w, l1max = min(CDZ_MAXLOOP, i - 1);
          T M = 0;
          for (int l0 = 1; l0 <= l1max; l0 += LCH) {
            for (int e = lane; e < LCH * 36; e += 64) {
              const int l1 = l0 + e / 36, a = (e % 36) / 6, yy = e % 6;
              T g = 0;
              if (l1 <= l1max && yy < dj) {
                const int pa = i - l1;
                if (a < sd[pa]) g = A.Gb[(long long)(sP[pa] + a) * ld + Pj + yy];
              }
              Gw[e] = g;
            }
            cdz_wave_sync();
            if (lane < 36 && b < dp && y < dj) {
              const int lend = min(LCH, l1max - l0 + 1);
              for (int l = 0; l < lend; l++) {
                const int l1 = l0 + l;
                const T f = tab[TB_BU + l1] * cdz_p2<T>(sE[l1 - 1] + sE[dl] - sE[dl + l1 + 2]);
                T sm = 0;
#pragma unroll
                for (int a = 0; a < 6; a++) sm += Gw[l * 36 + a * 6 + y] * Ubl[(l1 - 1) * 36 + a * 6 + b];
                M += f * sm;
              }
            }
            cdz_wave_sync();
          }
          if (lane < 36) {
            Mw[lane] = (double)M;
            Ew[lane] = ev;
          }
          cdz_wave_sync();
        }
        if (own) {
          // DI dressing (every operand of a loop over at most 6 slots is
          // loaded before the loop, absent slots as 0, so the loads overlap)
          const int dc = sd[j + 1], Pc = sP[j + 1];
          const T epx = ep[b * 6 + x];
          const int nix = D.nt[i * 6 + x], npb = D.nt[p * 6 + b];
          T qbr[6], dib[6];
          int ntj[6], ncr[6];
#pragma unroll
          for (int y = 0; y < 6; y++) {
            qbr[y] = y < dj ? D.Qb[(Pi + x) * ld + Pj + y] : T(0);
            ntj[y] = y < dj ? D.nt[j * 6 + y] : 0;
            dib[y] = y < dc ? A.DIb[(Pp + b) * ld + Pc + y] : T(0);
            ncr[y] = y < dc ? D.nt[(j + 1) * 6 + y] : 0;
          }
#pragma unroll
          for (int y = 0; y < 6; y++) {
            if (y >= dj || qbr[y] == T(0)) continue;
            const int tin = cdz_ptype(ntj[y], nix);
            T er[6];
#pragma unroll
            for (int c = 0; c < 6; c++) er[c] = c < dc ? Ew[y * 6 + c] : T(0);
#pragma unroll
            for (int c = 0; c < 6; c++) {
              if (c >= dc) break;
              const T wyc = qbr[y] * er[c];
              acc += (double)(dib[c] * epx * wyc * tab[TB_MM + ncr[c] * 24 + npb * 6 + tin]);
            }
          }
          // the bulges: sum_y Qb(x, y) M(b, y)
          T sm = 0;
#pragma unroll
          for (int y = 0; y < 6; y++)
            if (y < dj) sm += qbr[y] * (T)Mw[b * 6 + y];
          acc += (double)(sm * epx);
        }
        cdz_wave_sync();
      }
      if (own) {
        T lb[6], q1[6], qb[6];
        double z3[6];
#pragma unroll
        for (int s2 = 0; s2 < 6; s2++) {
          lb[s2] = s2 < dj ? A.Qm1Lb[(Pp + b) * ld + Pj + s2] : T(0);
          q1[s2] = s2 < dj ? D.Qm1[(Pi + x) * ld + Pj + s2] : T(0);
          qb[s2] = s2 < dj ? D.Qb[(Pi + x) * ld + Pj + s2] : T(0);
          z3[s2] = s2 < dj ? D.Z3[j * 6 + s2] : 0.0;
        }
        // Qm1L dressing
        T sm = 0;
#pragma unroll
        for (int s2 = 0; s2 < 6; s2++)
          if (s2 < dj) sm += lb[s2] * q1[s2];
        acc += (double)(sm * ep[b * 6 + x]);
        // exterior loop: pair (i, j) right after the prefix [0..p]
        const double sc = ldexp(1.0, D.G5[p] + sE[dl] + D.H3[j] - EZ);
        double sz = 0;
#pragma unroll
        for (int t = 0; t < 6; t++)
          if (t < dj) sz += (double)qb[t] * z3[t];
        acc += D.Z5[p * 6 + b] * D.ed[p * 36 + b * 6 + x] * (sz * sc);
      }
      continue;
    }
    k -= nR1;
    if (k < nR0) {
      // ---- cell (p, j): the edge after its first base; output (s, a) = (u, w)
      const int i = p, j = p + 4 + k, dl = j - i, di = dp, dj = sd[j], Pj = sP[j];
      const long long Pi = Pp;
      const int dm = sd[j - 1], s = u, a = w;
      stage_inner(i, j, j - 1);
      if (own) {
        const T eps = ep[s * 6 + a], vis = D.v[i * 6 + s];
        const int nis = D.nt[i * 6 + s];
        T ac[6], mp[6], qp[6];
        int ntj[6];
#pragma unroll
        for (int s2 = 0; s2 < 6; s2++) {
          ntj[s2] = s2 < dj ? D.nt[j * 6 + s2] : 0;
          ac[s2] = s2 < dj ? A.Qbb[(Pi + s) * ld + Pj + s2] * vis * D.v[j * 6 + s2] : T(0);
          mp[s2] = s2 < dj ? A.Qm1pb[(Pi + s) * ld + Pj + s2] : T(0);
          qp[s2] = s2 < dj ? D.Qm1p[(Pq + a) * ld + Pj + s2] : T(0);
        }
#pragma unroll
        for (int s2 = 0; s2 < 6; s2++) {
          if (s2 >= dj) break;
          const int to = cdz_ptype(nis, ntj[s2]);
          if (to < 0 || ac[s2] == T(0) || eps == T(0)) continue;
          T em[6];
#pragma unroll
          for (int dd = 0; dd < 6; dd++) em[dd] = dd < dm ? Ew[dd * 6 + s2] : T(0);
          T sm = 0;
#pragma unroll
          for (int dd = 0; dd < 6; dd++)
            if (dd < dm) sm += inner(a, dd, to, dl) * em[dd];
          acc += (double)(ac[s2] * eps * sm);
        }
        // multiloop unpaired prefix base i
        const T f = tab[TB_MLC] * cdz_p2<T>(sE[dl - 1] - sE[dl]);
        T sm = 0;
#pragma unroll
        for (int s2 = 0; s2 < 6; s2++)
          if (s2 < dj) sm += mp[s2] * qp[s2];
        acc += (double)(sm * f * vis * eps);
      }
      cdz_wave_sync();
      (void)di;
      continue;
    }
    k -= nR0;
    if (k < nC1) {
      // ---- cell (i, p+1): the edge before its last base; output (dd, s2) = (u, w)
      const int i = k, j = p + 1, dl = j - i, di = sd[i];
      const long long Pi = sP[i], Pj = Pq;
      const int dd = u, s2 = w;
      if (dl >= 4) stage_inner(i, j, i);
      const T eps = own ? ep[dd * 6 + s2] : T(0), vjs = own ? D.v[j * 6 + s2] : T(0);
      if (own && dl >= 4) {
        const int d1 = sd[i + 1], njs = D.nt[j * 6 + s2];
        T ac[6], mb[6], q1[6];
        int nti[6];
#pragma unroll
        for (int s = 0; s < 6; s++) {
          nti[s] = s < di ? D.nt[i * 6 + s] : 0;
          ac[s] = s < di ? A.Qbb[(Pi + s) * ld + Pj + s2] * D.v[i * 6 + s] * vjs : T(0);
          mb[s] = s < di ? A.Qm1b[(Pi + s) * ld + Pj + s2] : T(0);
          q1[s] = s < di ? D.Qm1[(Pi + s) * ld + Pp + dd] : T(0);
        }
        if (eps != T(0)) {
#pragma unroll
          for (int s = 0; s < 6; s++) {
            if (s >= di) break;
            const int to = cdz_ptype(nti[s], njs);
            if (to < 0 || ac[s] == T(0)) continue;
            T ei[6];
#pragma unroll
            for (int a = 0; a < 6; a++) ei[a] = a < d1 ? Ew[s * 6 + a] : T(0);
            T sm = 0;
#pragma unroll
            for (int a = 0; a < 6; a++)
              if (a < d1) sm += ei[a] * inner(a, dd, to, dl);
            acc += (double)(ac[s] * eps * sm);
          }
        }
        // multiloop unpaired tail base j
        const T f = tab[TB_MLC] * cdz_p2<T>(sE[dl - 1] - sE[dl]);
        T sm = 0;
#pragma unroll
        for (int s = 0; s < 6; s++)
          if (s < di) sm += mb[s] * q1[s];
        acc += (double)(sm * f * eps * vjs);
      }
      if (dl >= 4) cdz_wave_sync();
      if (own && dl >= 1) {
        // unpaired run [i..p+1] extended from [i..p]
        const T f = cdz_p2<T>(sE[dl - 1] - sE[dl]);
        T ub[6], uu[6];
#pragma unroll
        for (int a = 0; a < 6; a++) {
          ub[a] = a < di ? A.Ub[(Pi + a) * ld + Pj + s2] : T(0);
          uu[a] = a < di ? D.U[(Pi + a) * ld + Pp + dd] : T(0);
        }
        T sm = 0;
#pragma unroll
        for (int a = 0; a < 6; a++)
          if (a < di) sm += ub[a] * uu[a];
        acc += (double)(sm * f * eps * vjs);
      }
      continue;
    }
    k -= nC1;
    {
      // ---- cell (i, p): the edge after its last base; output (y, c) = (u, w)
      const int i = k, j = p, dl = j - i, di = sd[i];
      const long long Pi = sP[i], Pj = Pp;
      if (i >= 1) {
        const T ev = lane < 36 ? D.e[(i - 1) * 36 + lane] : T(0);  // e_{i-1}, into Ew with M
        // right bulges with inner pair (i, p): lane (x, c) forms
        // M(x, c) = sum_l2 f sum_dd U(c, dd) Gb(x, dd) for the wave, the
        // adjoints Gb(i slot x, p + l2 slot dd) staged LCH loop sizes at a
        // time, the runs U from Ubr
        {
          const int x = u, c = w, l2max = l2top;
          T M = 0;
          for (int l0 = 1; l0 <= l2max; l0 += LCH) {
            for (int e = lane; e < LCH * 36; e += 64) {
              const int l2 = l0 + e / 36, xx = (e % 36) / 6, q = e % 6;
              T g = 0;
              if (l2 <= l2max && xx < di) {
                const int pz = p + l2;
                if (q < sd[pz]) g = A.Gb[(Pi + xx) * ld + sP[pz] + q];
              }
              Gw[e] = g;
            }
            cdz_wave_sync();
            if (lane < 36 && x < di && c < dq) {
              const int lend = min(LCH, l2max - l0 + 1);
              for (int l = 0; l < lend; l++) {
                const int l2 = l0 + l;
                const T f = tab[TB_BU + l2] * cdz_p2<T>(sE[dl] + sE[l2 - 1] - sE[dl + l2 + 2]);
                T sm = 0;
#pragma unroll
                for (int q = 0; q < 6; q++) sm += Ubr[(l2 - 1) * 36 + q * 6 + c] * Gw[l * 36 + x * 6 + q];
                M += f * sm;
              }
            }
            cdz_wave_sync();
          }
          if (lane < 36) {
            Mw[lane] = (double)M;
            Ew[lane] = ev;
          }
          cdz_wave_sync();
        }
        if (own) {
          const int y = u, c = w;
          // DI dressing
          const int db = sd[i - 1], Pb = sP[i - 1];
          const T epc = ep[y * 6 + c];
          const int njy = D.nt[j * 6 + y], nqc = D.nt[(p + 1) * 6 + c];
          T qbc[6], dib[6];
          int nti[6], nbr[6];
#pragma unroll
          for (int x = 0; x < 6; x++) {
            qbc[x] = x < di ? D.Qb[(Pi + x) * ld + Pj + y] : T(0);
            nti[x] = x < di ? D.nt[i * 6 + x] : 0;
            dib[x] = x < db ? A.DIb[(Pb + x) * ld + Pq + c] : T(0);
            nbr[x] = x < db ? D.nt[(i - 1) * 6 + x] : 0;
          }
#pragma unroll
          for (int x = 0; x < 6; x++) {
            if (x >= di || qbc[x] == T(0)) continue;
            const int tin = cdz_ptype(njy, nti[x]);
            T eb[6];
#pragma unroll
            for (int b = 0; b < 6; b++) eb[b] = b < db ? Ew[b * 6 + x] : T(0);
#pragma unroll
            for (int b = 0; b < 6; b++) {
              if (b >= db) break;
              const T wb = eb[b] * qbc[x];
              if (wb == T(0)) continue;
              acc += (double)(dib[b] * wb * epc * tab[TB_MM + nqc * 24 + nbr[b] * 6 + tin]);
            }
          }
          // the bulges: sum_x Qb(x, y) M(x, c)
          T sm = 0;
#pragma unroll
          for (int x = 0; x < 6; x++)
            if (x < di) sm += qbc[x] * (T)Mw[x * 6 + c];
          acc += (double)(sm * epc);
        }
        cdz_wave_sync();
      }
    }
  }
  // ---- exterior loop: base p+1 unpaired right after the prefix [0..p]
  if (wv == 0 && own) {
    const double sc = ldexp(1.0, D.G5[p] + D.H3[p + 1] - EZ);
    acc += D.Z5[p * 6 + u] * D.ed[p * 36 + u * 6 + w] * D.vd[(p + 1) * 6 + w] * D.Z3[(p + 1) * 6 + w] * sc;
  }
  if (lane < 36) red[wv * 36 + lane] = acc;
  __syncthreads();
  // plus the uses of e_p as V (e_{i+1}) and W (e_{j-2}) in the interior-loop
  // size recursion, accumulated by the outside pass
  if (tid < 36) {
    double t = 0;
    for (int v = 0; v < ENT / 64; v++) t += red[v * 36 + tid];
    A.eta[p * 36 + tid] = t + A.etaV[p * 36 + tid] + A.etaW[p * 36 + tid];
  }
}

template <typename T>
__global__ __launch_bounds__(CDZ_NT) void cdz_out_diag(DevProb<T> D, DevAdj<T> A, int dl) {
  out_block<T, false>(D, A, dl, blockIdx.x);
}
template <typename T>
__global__ __launch_bounds__(CDZ_NT) void cdz_out_diag_fused(DevProb<T> D, DevAdj<T> A, int dl) {
  out_block<T, true>(D, A, dl, blockIdx.x);
}
template <typename T>
__global__ __launch_bounds__(cdz_eta_nt(sizeof(T))) void cdz_eta(DevProb<T> D, DevAdj<T> A, int lch) {
  eta_edge<T>(D, A, blockIdx.x, lch);
}
// batched forms (see cdz_fwd_diag_batch): one launch for diagonal dl / for the
// edges of every problem of a batch
template <typename T>
__global__ __launch_bounds__(CDZ_NT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) void cdz_out_diag_batch(const DevProb<T> *probs, const DevAdj<T> *adjs,
                                                            const int *off, int count, int dl) {
  int b, w;
  cdz_batch_locate(off, count, blockIdx.x, b, w);
  const DevProb<T> D = probs[b];
  const DevAdj<T> A = adjs[b];
  out_block<T, false>(D, A, dl, w);
}
template <typename T>
__global__ __launch_bounds__(CDZ_NT) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) void cdz_out_diag_batch_fused(const DevProb<T> *probs, const DevAdj<T> *adjs,
                                                            const int *off, int count, int dl) {
  int b, w;
  cdz_batch_locate(off, count, blockIdx.x, b, w);
  const DevProb<T> D = probs[b];
  const DevAdj<T> A = adjs[b];
  out_block<T, true>(D, A, dl, w);
}
template <typename T>
__global__ __launch_bounds__(cdz_eta_nt(sizeof(T))) void cdz_eta_batch(const DevProb<T> *probs, const DevAdj<T> *adjs,
                                                       const int *off, int count, int lch) {
  int b, w;
  cdz_batch_locate(off, count, blockIdx.x, b, w);
  const DevProb<T> D = probs[b];
  const DevAdj<T> A = adjs[b];
  eta_edge<T>(D, A, w, lch);
}

// pair probabilities P[i][j] = r * sum Qb~ Qb'~ over cells with j - i >= 4
template <typename T>
__global__ void cdz_pairprob(DevProb<T> D, DevAdj<T> A, double r) {
  const long long n = D.n, ld = D.ld;
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n * n) return;
  const int i = (int)(c / n), j = (int)(c % n);
  double v = 0;
  if (j >= i + 4) {
    const int di = D.d[i], dj = D.d[j], Pi = D.P[i], Pj = D.P[j];
    for (int s = 0; s < di; s++)
      for (int t = 0; t < dj; t++)
        v += (double)D.Qb[(Pi + s) * ld + Pj + t] * (double)A.Qbb[(Pi + s) * ld + Pj + t];
    v *= r;
  }
  A.pair[c] = v;
}

// d log Z / d theta from the edge marginals (device outputs, scaled by g)
__global__ void cdz_grad_theta(const double *eta, const int *d, int m, double scale,
                               double *dth1, double *dth2) {
  const int a = blockIdx.x, q = threadIdx.x;  // one thread per (x, y) slot pair
  if (a >= m || q >= 36) return;
  const int da = d[3 * a], x = q / 6, y = q % 6;
  if (q < 6) dth1[a * 6 + q] = q < da ? scale * eta[(3 * a) * 36 + q * 6 + q] : 0.0;
  if (dth2) {
    double v = 0;
    if (a >= 1 && x < d[3 * a - 1] && y < da) v = scale * eta[(3 * a - 1) * 36 + x * 6 + y];
    dth2[(a * 6 + x) * 6 + y] = v;
  }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
size_t eta_lds_bytes(int n, int elt) {
  // d, P, E of every position; reduction and bulge scratch; the runs of the
  // edge's bulges and the per-wave bulge adjoints; tables; per-wave inner
  // blocks and bases
  const int lch = eta_bulge_chunk(n, elt);
  const int nw = cdz_eta_nt(elt) / 64;
  return ((size_t)3 * (n + 1) * 4 + 15) / 16 * 16 + (size_t)(2 * nw * 36) * 8 +
         ((size_t)2 * CDZ_MAXLOOP * 36 + (size_t)nw * lch * 36 + (TB_LEN + 7) / 8 * 8 + nw * 6 * 36) * elt +
         nw * 12 * 4;
}

template <typename T>
__global__ void cdz_arec_diag(DevProb<T> D, int dl);

template <typename T>
static cdz_status run_outside(cdz_handle *h, DevProb<T> &D, DevAdj<T> &A) {
  const int n = D.n;
  hipStream_t st = h->stream;
  const size_t S2b = (size_t)D.ld * D.ld * sizeof(T);
  const size_t shm = out_lds_bytes<T>(n);
  if (shm > (size_t)h->lds_max)
    return cdz_fail(h, CDZ_ERR_ARG, "sequence of " + std::to_string(n) + " nt exceeds the LDS layout of the outside kernel");
  HIPCHK(h, hipFuncSetAttribute((const void *)cdz_out_diag<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
  HIPCHK(h, hipFuncSetAttribute((const void *)cdz_out_diag_fused<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)shm));
  long long wmax = 0;
  for (int t = 0; t < n; t++) wmax = std::max<long long>(wmax, out_nblocks(n, t));
  const uint64_t tkey = tune_key(1, false, sizeof(T), wmax);
  tune_begin(h, tkey);
  HIPCHK(h, hipEventRecord(h->ev[2], st));
  // accumulators of pushed adjoints start at zero
  HIPCHK(h, hipMemsetAsync(A.UbL, 0, S2b, st));
  HIPCHK(h, hipMemsetAsync(A.UbR, 0, S2b, st));
  HIPCHK(h, hipMemsetAsync(A.UbL2, 0, S2b, st));
  HIPCHK(h, hipMemsetAsync(A.UbR2, 0, S2b, st));
  HIPCHK(h, hipMemsetAsync(A.DIbL, 0, S2b, st));
  HIPCHK(h, hipMemsetAsync(A.DIbR, 0, S2b, st));
  HIPCHK(h, hipMemsetAsync(A.etaV, 0, (size_t)n * 36 * sizeof(double), st));
  HIPCHK(h, hipMemsetAsync(A.etaW, 0, (size_t)n * 36 * sizeof(double), st));
  if (h->profiling) HIPCHK(h, prof_reserve(h, n + 1));
  // memory-bounded form: the interior pushes of diagonal t + 1 (launch t)
  // read A of diagonal t - 1 (when t + 1 >= 10); the band of K diagonals
  // holding it is rebuilt from its two checkpoint diagonals the first time
  // the pass reaches it
  DevProb<T> Dl = D;
  int band = -1;
  const int K = D.alK, top = D.alTop;
  if (!D.AL) {
    if (K <= 0) return cdz_fail(h, CDZ_ERR_STATE, "forward kept no checkpoints for the outside pass");
    const size_t shf = fwd_lds_bytes<T>(n);
    HIPCHK(h, hipFuncSetAttribute((const void *)cdz_arec_diag<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)shf));
  }
  for (int dl = n - 1; dl >= 0; dl--) {
    if (!D.AL && dl + 1 >= 10 && dl + 1 <= n - 1) {
      const int x = dl - 1, k = x / K;
      if (k != band) {
        DevProb<T> Dr = D;
        for (int y = std::max(4, k * K); y <= x; y++) {
          Dr.ALw = al_slot_ptr(D, al_slot_band(K, top, y));
          Dr.ALp = al_slot_ptr(D, y - 2 >= k * K ? al_slot_band(K, top, y - 2) : al_slot_fwd(K, top, y - 2));
          hipLaunchKernelGGL(cdz_arec_diag<T>, dim3(cdz_cells_grid(n - y)), dim3(CDZ_NT), fwd_lds_bytes<T>(n), st,
                             Dr, y);
        }
        band = k;
      }
      Dl.ALp = al_slot_ptr(D, al_slot_band(K, top, x));
    }
    if (h->profiling) HIPCHK(h, hipEventRecord(h->pev[2 * dl], st));
    const bool fu = out_nblocks(n, dl) >= h->fuse_wg;
    if (fu)
      hipLaunchKernelGGL(cdz_out_diag_fused<T>, dim3(out_nblocks(n, dl, true)), dim3(CDZ_NT), shm, st, Dl, A, dl);
    else
      hipLaunchKernelGGL(cdz_out_diag<T>, dim3(out_nblocks(n, dl)), dim3(CDZ_NT), shm, st, Dl, A, dl);
    if (h->profiling) HIPCHK(h, hipEventRecord(h->pev[2 * dl + 1], st));
  }
  HIPCHK(h, hipGetLastError());
  if (n >= 2) {
    const size_t shm2 = eta_lds_bytes(n, sizeof(T));
    if (shm2 > (size_t)h->lds_max)
      return cdz_fail(h, CDZ_ERR_ARG, "sequence of " + std::to_string(n) + " nt exceeds the LDS layout of the edge kernel");
    HIPCHK(h, hipFuncSetAttribute((const void *)cdz_eta<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm2));
    if (h->profiling) HIPCHK(h, hipEventRecord(h->pev[2 * n], st));
    hipLaunchKernelGGL(cdz_eta<T>, dim3(n - 1), dim3(cdz_eta_nt(sizeof(T))), shm2, st, D, A, eta_bulge_chunk(n, sizeof(T)));
    if (h->profiling) HIPCHK(h, hipEventRecord(h->pev[2 * n + 1], st));
  }
  const double r = std::exp(h->EZ * 0.6931471805599453094 - h->logz_scaled);
  const long long nn = (long long)n * n;
  hipLaunchKernelGGL(cdz_pairprob<T>, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, st, D, A, r);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipEventRecord(h->ev[3], st));
  HIPCHK(h, hipStreamSynchronize(st));
  float ms = 0;
  HIPCHK(h, hipEventElapsedTime(&ms, h->ev[2], h->ev[3]));
  h->times[1] = ms;
  if (!h->profiling) tune_end(h, tkey, ms);
  if (h->profiling) {
    double tot = 0;
    for (int dl = 0; dl < n; dl++) {
      float k = 0;
      HIPCHK(h, hipEventElapsedTime(&k, h->pev[2 * dl], h->pev[2 * dl + 1]));
      tot += k;
    }
    h->prof_out_ms = tot;
    h->prof_out_launches = n;
    float k = 0;
    if (n >= 2) HIPCHK(h, hipEventElapsedTime(&k, h->pev[2 * n], h->pev[2 * n + 1]));
    h->prof_eta_ms = k;
  }
  return CDZ_OK;
}

static cdz_status outside(cdz_handle *h) {
  return h->opt.prec == CDZ_FP64 ? run_outside<double>(h, h->pd, h->ad)
                                 : run_outside<float>(h, h->pf, h->af);
}

static const double *eta_dev(cdz_handle *h) { return h->opt.prec == CDZ_FP64 ? h->ad.eta : h->af.eta; }
static const double *pair_dev(cdz_handle *h) { return h->opt.prec == CDZ_FP64 ? h->ad.pair : h->af.pair; }
static const int *d_dev(cdz_handle *h) { return h->opt.prec == CDZ_FP64 ? h->pd.d : h->pf.d; }

extern "C" cdz_status cdz_marginals(cdz_handle *h, const cdz_problem *prob, double *log_z,
                                    double *pair, double *base, double *codon, double *codon_pair) {
  if (!h || !prob) return cdz_fail(h, CDZ_ERR_ARG, "null argument");
  HostTables t;
  cdz_status s = build_tables(h, prob->n_aa, prob->aa, prob->theta1, prob->theta2, t);
  if (s != CDZ_OK) return s;
  s = ensure_forward(h, t, true);
  if (s != CDZ_OK) return s;
  s = outside(h);
  if (s != CDZ_OK) return s;
  if (log_z) *log_z = h->logz;
  const double r = std::exp(h->EZ * 0.6931471805599453094 - h->logz_scaled);
  return assemble_marginals(h, t, eta_dev(h), pair_dev(h), r, pair, base, codon, codon_pair);
}

// the edge marginals the outside pass writes (edges p = 0..n-2, slots below
// d[p] x d[p+1]; the padding of each 6 x 6 block is never written) are finite
static bool edge_marginals_finite(const HostTables &t, const std::vector<double> &eta) {
  for (int p = 0; p + 1 < t.n; p++)
    for (int u = 0; u < t.d[p]; u++)
      for (int w = 0; w < t.d[p + 1]; w++)
        if (!std::isfinite(eta[(size_t)p * 36 + u * 6 + w])) return false;
  return true;
}

cdz_status assemble_marginals(cdz_handle *h, const HostTables &t, const double *eta_dev, const double *pair_dev,
                              double r, double *pair, double *base, double *codon, double *codon_pair) {
  const int n = t.n, m = t.m;
  std::vector<double> eta((size_t)n * 36);
  HIPCHK(h, hipMemcpy(eta.data(), eta_dev, eta.size() * 8, hipMemcpyDeviceToHost));
  if (!edge_marginals_finite(t, eta))
    return cdz_fail(h, CDZ_ERR_NUMERIC, "non-finite edge marginals (outside pass out of range)");
  std::vector<double> cod((size_t)m * 6, 0.0);
  for (int a = 0; a < m; a++)
    for (int c = 0; c < t.d[3 * a]; c++) cod[a * 6 + c] = r * eta[(size_t)(3 * a) * 36 + c * 6 + c];
  if (codon) memcpy(codon, cod.data(), cod.size() * 8);
  if (codon_pair) {
    for (int k = 0; k < m * 36; k++) codon_pair[k] = 0.0;
    for (int a = 1; a < m; a++)
      for (int x = 0; x < t.d[3 * a - 1]; x++)
        for (int y = 0; y < t.d[3 * a]; y++)
          codon_pair[a * 36 + x * 6 + y] = r * eta[(size_t)(3 * a - 1) * 36 + x * 6 + y];
  }
  if (base) {
    for (int p = 0; p < n; p++) {
      for (int b = 0; b < 4; b++) base[p * 4 + b] = 0.0;
      for (int c = 0; c < t.d[p]; c++) base[p * 4 + t.nt[p * 6 + c]] += cod[(p / 3) * 6 + c];
    }
  }
  if (pair) {
    HIPCHK(h, hipMemcpy(pair, pair_dev, (size_t)n * n * 8, hipMemcpyDeviceToHost));
    for (int i = 0; i < n; i++)
      for (int j = i + 1; j < n; j++)
        if (!std::isfinite(pair[(size_t)i * n + j]))
          return cdz_fail(h, CDZ_ERR_NUMERIC, "non-finite pair probabilities (outside pass out of range)");
    for (int i = 0; i < n; i++)
      for (int j = i + 1; j < n; j++) pair[(size_t)j * n + i] = pair[(size_t)i * n + j];
    for (int i = 0; i < n; i++) {
      double sm = 0;
      for (int j = 0; j < n; j++)
        if (j != i) sm += pair[(size_t)i * n + j];
      pair[(size_t)i * n + i] = 1.0 - sm;
    }
  }
  return CDZ_OK;
}

extern "C" cdz_status cdz_forward_dev(cdz_handle *h, int32_t n_aa, const char *aa,
                                      const double *theta1_dev, const double *theta2_dev,
                                      double *log_z) {
  if (!h || !aa || !theta1_dev || !log_z || n_aa < 1) return cdz_fail(h, CDZ_ERR_ARG, "null argument");
  std::vector<double> t1((size_t)n_aa * 6), t2;
  HIPCHK(h, hipMemcpyAsync(t1.data(), theta1_dev, t1.size() * 8, hipMemcpyDeviceToHost, h->stream));
  if (theta2_dev) {
    t2.resize((size_t)n_aa * 36);
    HIPCHK(h, hipMemcpyAsync(t2.data(), theta2_dev, t2.size() * 8, hipMemcpyDeviceToHost, h->stream));
  }
  HIPCHK(h, hipStreamSynchronize(h->stream));
  HostTables t;
  cdz_status s = build_tables(h, n_aa, aa, t1.data(), theta2_dev ? t2.data() : nullptr, t);
  if (s != CDZ_OK) return s;
  s = ensure_forward(h, t, true);
  if (s != CDZ_OK) return s;
  *log_z = h->logz;
  return CDZ_OK;
}

extern "C" cdz_status cdz_backward_dev(cdz_handle *h, double grad_logz, double *dtheta1_dev,
                                       double *dtheta2_dev) {
  if (!h || !dtheta1_dev) return cdz_fail(h, CDZ_ERR_ARG, "null argument");
  if (!h->have_fwd || !h->fwd_adjoint) return cdz_fail(h, CDZ_ERR_STATE, "no forward pass to differentiate");
  cdz_status s = outside(h);
  if (s != CDZ_OK) return s;
  {
    std::vector<double> eta((size_t)h->tables.n * 36);
    HIPCHK(h, hipMemcpy(eta.data(), eta_dev(h), eta.size() * 8, hipMemcpyDeviceToHost));
    if (!edge_marginals_finite(h->tables, eta))
      return cdz_fail(h, CDZ_ERR_NUMERIC, "non-finite edge marginals (outside pass out of range)");
  }
  const double r = std::exp(h->EZ * 0.6931471805599453094 - h->logz_scaled);
  hipLaunchKernelGGL(cdz_grad_theta, dim3(h->tables.m), dim3(64), 0, h->stream, eta_dev(h), d_dev(h),
                     h->tables.m, grad_logz * r, dtheta1_dev, dtheta2_dev);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return CDZ_OK;
}

// Diagnostic copy of one workspace array of the last pass to the host:
// which = 0..11 forward (U Qb G F DI Qm1 Qm1Lr Qm1Lt Qm1p QmX Qm Qmt),
// 12..24 adjoint (Qbb Qm1b Qm1pb QmXb QmXbt Qmb Qm1Lb DIb Gb Fb Ub UbL UbR; UbR
// transposed),
// 25 diagonal exponents (int32, n + 1).  Element type is the handle's
// precision; ld x ld elements.
template <typename T>
static cdz_status debug_copy(cdz_handle *h, const DevProb<T> &D, const DevAdj<T> &A, int which,
                             void *dst, size_t bytes) {
  const T *fw[] = {D.U, D.Qb, D.G, D.F, D.DI, D.Qm1, D.Qm1Lr, D.Qm1Lt, D.Qm1p, D.QmX, D.Qm, D.Qmt};
  const T *bw[] = {A.Qbb, A.Qm1b, A.Qm1pb, A.QmXb, A.QmXbt, A.Qmb, A.Qm1Lb, A.DIb, A.Gb, A.Fb, A.Ub, A.UbL, A.UbR};
  const void *src = nullptr;
  size_t need = (size_t)D.ld * D.ld * sizeof(T);
  if (which >= 0 && which < 12) src = fw[which];
  else if (which >= 12 && which < 25) src = h->fwd_adjoint ? bw[which - 12] : nullptr;
  else if (which == 25) {
    src = D.E;
    need = (size_t)(D.n + 1) * sizeof(int);
  }
  if (!src || bytes < need) return cdz_fail(h, CDZ_ERR_ARG, "bad debug copy request");
  HIPCHK(h, hipMemcpy(dst, src, need, hipMemcpyDeviceToHost));
  return CDZ_OK;
}

extern "C" cdz_status cdz_debug_copy(cdz_handle *h, int which, void *dst, size_t bytes, long long *ld) {
  if (!h || !dst || !h->have_fwd) return cdz_fail(h, CDZ_ERR_STATE, "no forward pass");
  if (ld) *ld = h->opt.prec == CDZ_FP64 ? h->pd.ld : h->pf.ld;
  return h->opt.prec == CDZ_FP64 ? debug_copy<double>(h, h->pd, h->ad, which, dst, bytes)
                                 : debug_copy<float>(h, h->pf, h->af, which, dst, bytes);
}

template __global__ void cdz_out_diag<float>(DevProb<float>, DevAdj<float>, int);
template __global__ void cdz_out_diag<double>(DevProb<double>, DevAdj<double>, int);
template __global__ void cdz_out_diag_fused<float>(DevProb<float>, DevAdj<float>, int);
template __global__ void cdz_out_diag_fused<double>(DevProb<double>, DevAdj<double>, int);
template __global__ void cdz_out_diag_batch<float>(const DevProb<float> *, const DevAdj<float> *, const int *, int,
                                                    int);
template __global__ void cdz_out_diag_batch<double>(const DevProb<double> *, const DevAdj<double> *, const int *,
                                                     int, int);
template __global__ void cdz_out_diag_batch_fused<float>(const DevProb<float> *, const DevAdj<float> *, const int *,
                                                          int, int);
template __global__ void cdz_out_diag_batch_fused<double>(const DevProb<double> *, const DevAdj<double> *,
                                                           const int *, int, int);
template __global__ void cdz_eta_batch<float>(const DevProb<float> *, const DevAdj<float> *, const int *, int, int);
template __global__ void cdz_eta_batch<double>(const DevProb<double> *, const DevAdj<double> *, const int *, int, int);
template __global__ void cdz_pairprob<float>(DevProb<float>, DevAdj<float>, double);
template __global__ void cdz_pairprob<double>(DevProb<double>, DevAdj<double>, double);
