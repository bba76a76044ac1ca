// cdz_mfe.hip -- minimum free energy over codon sequences and structures
// (Section 4d; the (min, +) algebra of SI S2c), with an argmin traceback.
//
// The recursions are those of the partition function with every sum over
// decompositions replaced by a minimum and every product of factors by a sum
// of energies (kT): a vertex carries -theta1 on the middle base of a codon,
// an edge inside a codon 0 (same slot) or +inf, an edge across a codon
// boundary -theta2, a loop its energy; +inf marks what cannot occur.  The
// entries are FP64 n x n arrays of 6 x 6 blocks (cell (i, j) at
// ((i n + j) * 36), slot of i by slot of j): the unpaired run U, the pair Qb,
// the interior-loop inner pair DI (Qb[i][j] with the edges to i-1, j+1 and the
// inner mismatch), one multiloop branch Qm1, a branch after an unpaired prefix
// Qm1p, two or more branches QmX, and Qm = min(QmX, Qm1p).
//
// One launch per anti-diagonal, one 256-thread workgroup per cell.  A cell
// enumerates its bulge and interior windows (l1 + l2 <= 30) directly:
// threads take (slot a of i+1, slot dd of j-1) and a seventh of the windows,
// with the run blocks of both window sides staged in LDS.  Every quantity is
// added in one fixed order, so the traceback, which evaluates the same
// expressions, finds exactly the values the forward pass kept.
//
// The argmin traceback runs in one workgroup: a stack of fragments in device
// memory, each decision's alternatives evaluated by all threads and reduced to
// the first of smallest value in the documented order.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "cdz_internal.h"
#include "cdz_mfe.h"

namespace {

constexpr int MT = 256;  // threads per workgroup
constexpr int MAXW = 30;

struct MfeDev {
  int n;
  const int *d;           // [n] slots of the residue of position p
  const signed char *nt;  // [n][6] base under slot s
  const double *v;        // [n][6] vertex energy
  const double *e;        // [n][36] edge energy p -> p+1
  const double *hp;       // [n + 1] hairpin energy by unpaired length (+inf below 3)
  const double *stack;    // [6][6]
  const double *bulge, *interior;  // [31]
  const double *mm;       // [4][4][6]
  double ml_ab, ml_b, ml_c;  // multiloop closing (a + b), per branch, per unpaired base
  double *U, *Qb, *DI, *Qm1, *Qm1p, *QmX, *Qm;
  double *Z5;   // [n][6]
  int *slot;    // [n]
  int *pt;      // [n]
  int *stk;     // [cap][5]
  int cap;
  double *out;  // [1] minimum
  int *err;     // [1] traceback stack overflow
};

__device__ __forceinline__ double *blk(double *A, int n, int i, int j) { return A + ((size_t)i * n + j) * 36; }
__device__ __forceinline__ const double *cblk(const double *A, int n, int i, int j) {
  return A + ((size_t)i * n + j) * 36;
}
__device__ __forceinline__ int bpair(int x, int y) {  // AU CG GC UA GU UG = 0..5, -1 if none
  const int code = x * 4 + y;
  switch (code) {
    case 3: return 0;   // A-U
    case 6: return 1;   // C-G
    case 9: return 2;   // G-C
    case 12: return 3;  // U-A
    case 11: return 4;  // G-U
    case 14: return 5;  // U-G
  }
  return -1;
}
__device__ __forceinline__ double E(const MfeDev &D, int p, int s, int t) { return D.e[p * 36 + s * 6 + t]; }
__device__ __forceinline__ int NT(const MfeDev &D, int p, int s) { return D.nt[p * 6 + s]; }
__device__ __forceinline__ double MM(const MfeDev &D, int x, int y, int t) { return D.mm[(x * 4 + y) * 6 + t]; }

// (l1, l2) of window index w = l1 * 31 + l2, valid when l1 + l2 <= 30, not
// both zero, and the inner pair spans at least 4 (l1 + l2 <= dl - 6)
__device__ __forceinline__ bool window_of(int w, int dl, int &l1, int &l2) {
  l1 = w / 31;
  l2 = w % 31;
  return l1 + l2 <= MAXW && (l1 | l2) != 0 && l1 + l2 <= dl - 6;
}

// interior windows (l1, l2 >= 1, l1 + l2 <= 30) in enumeration order
struct WinTab {
  unsigned char l1[435], l2[435];
};
constexpr WinTab make_wintab() {
  WinTab t{};
  int m = 0;
  for (int a = 1; a <= MAXW - 1; a++)
    for (int b = 1; a + b <= MAXW; b++) {
      t.l1[m] = (unsigned char)a;
      t.l2[m] = (unsigned char)b;
      m++;
    }
  return t;
}
__constant__ WinTab kWin = make_wintab();
constexpr int NIW = 435;  // interior windows
constexpr int CH = 32;    // interior windows staged per round

// dynamic LDS of mfe_diag (doubles): runs of both window sides, the bulges'
// inner pairs and edges, a chunk of interior inner pairs, then the window
// minima per thread group and the small blocks of the cell
struct MfeLds {
  static constexpr int UL = 0, UR = UL + MAXW * 36, QL = UR + MAXW * 36, QR = QL + MAXW * 36, EL = QR + MAXW * 36,
                       ER = EL + MAXW * 36, DI = ER + MAXW * 36, W = DI + CH * 36, G = W + 7 * 3 * 36,
                       QB = G + 3 * 36, Q1P = QB + 36, SP = Q1P + 36, SM = SP + 6 * 36, MMT = SM + 10 * 36,
                       END = MMT + 96 + 36;
  static constexpr size_t bytes = (size_t)END * sizeof(double);
};

// per window, at outer slots (a of i+1, dd of j-1): the minimum over the
// parts' inner slots, plus the loop energy; no outer edges, no outer mismatch
__device__ double window_value(const MfeDev &D, int i, int j, int l1, int l2, int a, int dd, const double *ul,
                               const double *ur) {
  const int n = D.n, k = i + 1 + l1, l = j - 1 - l2;
  double best = INFINITY;
  if (l2 == 0) {  // left bulge: run i+1..k-1 (ul), pair (k, j-1)
    const double *q = cblk(D.Qb, n, k, j - 1);
    for (int b = 0; b < D.d[k - 1]; b++)
      for (int x = 0; x < D.d[k]; x++) best = fmin(best, ul[a * 6 + b] + E(D, k - 1, b, x) + q[x * 6 + dd]);
    return D.bulge[l1] + best;
  }
  if (l1 == 0) {  // right bulge: pair (i+1, l), run l+1..j-1 (ur)
    const double *q = cblk(D.Qb, n, i + 1, l);
    for (int y = 0; y < D.d[l]; y++)
      for (int c = 0; c < D.d[l + 1]; c++) best = fmin(best, q[a * 6 + y] + E(D, l, y, c) + ur[c * 6 + dd]);
    return D.bulge[l2] + best;
  }
  const double *di = cblk(D.DI, n, k, l);  // interior loop
  for (int c = 0; c < D.d[l + 1]; c++) {
    double T = INFINITY;
    for (int b = 0; b < D.d[k - 1]; b++) T = fmin(T, ul[a * 6 + b] + di[b * 6 + c]);
    best = fmin(best, T + ur[c * 6 + dd]);
  }
  return D.interior[l1 + l2] + best;
}

__device__ __forceinline__ double hairpin_term(const MfeDev &D, int i, int j, int s, int s2, int t, int a, int b) {
  return E(D, i, s, a) + cblk(D.U, D.n, i + 1, j - 1)[a * 6 + b] + E(D, j - 1, b, s2) +
         MM(D, NT(D, i + 1, a), NT(D, j - 1, b), t);
}
__device__ __forceinline__ double stack_term(const MfeDev &D, int i, int j, int s, int s2, int t, int x, int y) {
  const double q = cblk(D.Qb, D.n, i + 1, j - 1)[x * 6 + y];
  if (q == INFINITY) return INFINITY;
  const int t2 = bpair(NT(D, i + 1, x), NT(D, j - 1, y));
  return E(D, i, s, x) + q + E(D, j - 1, y, s2) + D.stack[t * 6 + t2];
}
__device__ __forceinline__ double ml_term(const MfeDev &D, int i, int j, int s, int s2, int x, int y) {
  return E(D, i, s, x) + cblk(D.QmX, D.n, i + 1, j - 1)[x * 6 + y] + E(D, j - 1, y, s2);
}
__device__ __forceinline__ double di_term(const MfeDev &D, const double *qb, int i, int j, int b, int c, int x,
                                          int y) {
  const double q = qb[x * 6 + y];
  if (q == INFINITY) return INFINITY;
  const int t2 = bpair(NT(D, j, y), NT(D, i, x));
  return E(D, i - 1, b, x) + q + E(D, j, y, c) + MM(D, NT(D, j + 1, c), NT(D, i - 1, b), t2);
}
__device__ __forceinline__ double outer_term(const MfeDev &D, int i, int j, int s, int s2, int a, int dd,
                                             double w) {
  return E(D, i, s, a) + E(D, j - 1, dd, s2) + w;
}

__global__ __launch_bounds__(256) void mfe_fill(double *p, size_t count) {
  for (size_t k = (size_t)blockIdx.x * 256 + threadIdx.x; k < count; k += (size_t)gridDim.x * 256) p[k] = INFINITY;
}

__global__ __launch_bounds__(64) void mfe_init_runs(MfeDev D) {
  const int p = blockIdx.x, a = threadIdx.x;
  if (a < D.d[p]) blk(D.U, D.n, p, p)[a * 6 + a] = D.v[p * 6 + a];
}

// cell (i, i + dl), dl >= 1
__global__ __launch_bounds__(MT) void mfe_diag(MfeDev D, int dl) {
  extern __shared__ __align__(16) double lds[];
  double(*sUL)[36] = reinterpret_cast<double(*)[36]>(lds + MfeLds::UL);  // U[i+1][i+l], l = 1..30
  double(*sUR)[36] = reinterpret_cast<double(*)[36]>(lds + MfeLds::UR);  // U[j-l][j-1]
  double(*sQL)[36] = reinterpret_cast<double(*)[36]>(lds + MfeLds::QL);  // Qb[i+1+l][j-1] (left bulge l)
  double(*sQR)[36] = reinterpret_cast<double(*)[36]>(lds + MfeLds::QR);  // Qb[i+1][j-1-l] (right bulge l)
  double(*sEL)[36] = reinterpret_cast<double(*)[36]>(lds + MfeLds::EL);  // e_{i+l}
  double(*sER)[36] = reinterpret_cast<double(*)[36]>(lds + MfeLds::ER);  // e_{j-1-l}
  double(*sDI)[36] = reinterpret_cast<double(*)[36]>(lds + MfeLds::DI);  // DI of a chunk of interior windows
  double(*sW)[3][36] = reinterpret_cast<double(*)[3][36]>(lds + MfeLds::W);
  double(*sG)[36] = reinterpret_cast<double(*)[36]>(lds + MfeLds::G);
  double *sQb = lds + MfeLds::QB, *sQ1p = lds + MfeLds::Q1P;
  double(*sSp)[36] = reinterpret_cast<double(*)[36]>(lds + MfeLds::SP);  // split minima per wavefront
  // the cell's small blocks: 0 U[i+1][j-1], 1 e_i, 2 e_{j-1}, 3 Qb[i+1][j-1], 4 QmX[i+1][j-1], 5 e_{i-1},
  // 6 e_j, 7 Qm1[i][j-1], 8 Qm1p[i+1][j]; then the mismatch and stack tables
  double(*sB)[36] = reinterpret_cast<double(*)[36]>(lds + MfeLds::SM);
  double *sMM = lds + MfeLds::MMT, *sST = sMM + 96;
  const int n = D.n, i = blockIdx.x, j = i + dl, tid = threadIdx.x;
  if (j >= n) return;
  // unpaired run [i..j]
  if (tid < 36) {
    const int a = tid / 6, b = tid % 6;
    if (a < D.d[i] && b < D.d[j]) {
      const double *ul = cblk(D.U, n, i, j - 1);
      double best = INFINITY;
      for (int c = 0; c < D.d[j - 1]; c++) best = fmin(best, ul[a * 6 + c] + E(D, j - 1, c, b));
      blk(D.U, n, i, j)[tid] = best + D.v[j * 6 + b];
    }
  }
  if (dl < 4) return;
  // ---- bulge and interior windows: minima GL (left bulges), GR (right), FI (interior)
  for (int q = tid; q < MAXW * 36; q += MT) {
    const int r = q / 36, x = q % 36, l = r + 1;
    sUL[r][x] = i + l <= n - 1 ? cblk(D.U, n, i + 1, i + l)[x] : INFINITY;
    sUR[r][x] = j - l >= 0 ? cblk(D.U, n, j - l, j - 1)[x] : INFINITY;
    sQL[r][x] = i + 1 + l <= j - 1 ? cblk(D.Qb, n, i + 1 + l, j - 1)[x] : INFINITY;
    sQR[r][x] = j - 1 - l >= i + 1 ? cblk(D.Qb, n, i + 1, j - 1 - l)[x] : INFINITY;
    sEL[r][x] = i + l <= n - 2 ? D.e[(size_t)(i + l) * 36 + x] : INFINITY;
    sER[r][x] = j - 1 - l >= 0 ? D.e[(size_t)(j - 1 - l) * 36 + x] : INFINITY;
  }
  for (int q = tid; q < 9 * 36 + 96 + 36; q += MT) {
    const int r = q / 36, x = q % 36;
    double val = INFINITY;
    if (q >= 9 * 36) {
      const int z = q - 9 * 36;
      val = z < 96 ? D.mm[z] : D.stack[z - 96];
      sMM[z] = val;
      continue;
    }
    switch (r) {
      case 0: val = cblk(D.U, n, i + 1, j - 1)[x]; break;
      case 1: val = D.e[(size_t)i * 36 + x]; break;
      case 2: val = D.e[(size_t)(j - 1) * 36 + x]; break;
      case 3: val = cblk(D.Qb, n, i + 1, j - 1)[x]; break;
      case 4: val = cblk(D.QmX, n, i + 1, j - 1)[x]; break;
      case 5: val = i >= 1 ? D.e[(size_t)(i - 1) * 36 + x] : INFINITY; break;
      case 6: val = j + 1 < n ? D.e[(size_t)j * 36 + x] : INFINITY; break;
      case 7: val = cblk(D.Qm1, n, i, j - 1)[x]; break;
      case 8: val = cblk(D.Qm1p, n, i + 1, j)[x]; break;
    }
    sB[r][x] = val;
  }
  __syncthreads();
  const int q = tid % 36, g = tid / 36, a = q / 6, dd = q % 6;
  const bool act = g < 7 && a < D.d[i + 1] && dd < D.d[j - 1];
  double mL = INFINITY, mR = INFINITY, mI = INFINITY;
  if (act) {
    // bulges: the same sums as window_value, from the staged blocks
    for (int l = 1 + g; l <= MAXW && l <= dl - 6; l += 7) {
      const int k = i + 1 + l, r = l - 1;
      double best = INFINITY;
      for (int b = 0; b < D.d[k - 1]; b++)
        for (int x = 0; x < D.d[k]; x++) best = fmin(best, sUL[r][a * 6 + b] + sEL[r][b * 6 + x] + sQL[r][x * 6 + dd]);
      mL = fmin(mL, D.bulge[l] + best);
      const int lr = j - 1 - l;
      best = INFINITY;
      for (int y = 0; y < D.d[lr]; y++)
        for (int c = 0; c < D.d[lr + 1]; c++) best = fmin(best, sQR[r][a * 6 + y] + sER[r][y * 6 + c] + sUR[r][c * 6 + dd]);
      mR = fmin(mR, D.bulge[l] + best);
    }
  }
  // interior windows, CH at a time: stage their DI blocks, then reduce
  for (int c0 = 0; c0 < NIW; c0 += CH) {
    __syncthreads();
    for (int z = tid; z < CH * 36; z += MT) {
      const int m = c0 + z / 36, x = z % 36;
      double val = INFINITY;
      if (m < NIW) {
        const int l1 = kWin.l1[m], l2 = kWin.l2[m];
        if (l1 + l2 <= dl - 6) val = cblk(D.DI, n, i + 1 + l1, j - 1 - l2)[x];
      }
      sDI[z / 36][x] = val;
    }
    __syncthreads();
    if (act)
      for (int mm = g; mm < CH && c0 + mm < NIW; mm += 7) {
        const int m = c0 + mm, l1 = kWin.l1[m], l2 = kWin.l2[m];
        if (l1 + l2 > dl - 6) continue;
        const int k = i + 1 + l1, l = j - 1 - l2;
        const double *ul = sUL[l1 - 1], *ur = sUR[l2 - 1], *di = sDI[mm];
        double best = INFINITY;
        for (int c = 0; c < D.d[l + 1]; c++) {
          double T = INFINITY;
          for (int b = 0; b < D.d[k - 1]; b++) T = fmin(T, ul[a * 6 + b] + di[b * 6 + c]);
          best = fmin(best, T + ur[c * 6 + dd]);
        }
        mI = fmin(mI, D.interior[l1 + l2] + best);
      }
  }
  if (g < 7) {
    sW[g][0][q] = mL;
    sW[g][1][q] = mR;
    sW[g][2][q] = mI;
  }
  __syncthreads();
  if (tid < 3 * 36) {
    const int k = tid / 36, q = tid % 36;
    double m = INFINITY;
    for (int g = 0; g < 7; g++) m = fmin(m, sW[g][k][q]);
    sG[k][q] = m;
  }
  __syncthreads();
  // ---- the pair (i, j), from the staged blocks (the same sums as hairpin_term,
  // stack_term, outer_term and ml_term)
  const int di = D.d[i], dj = D.d[j], d1 = D.d[i + 1], dm = D.d[j - 1];
  if (tid < 36) {
    const int s = tid / 6, s2 = tid % 6;
    double qb = INFINITY;
    const int t = s < di && s2 < dj ? bpair(NT(D, i, s), NT(D, j, s2)) : -1;
    if (t >= 0) {
      int n1[6], nm[6];
      for (int a = 0; a < 6; a++) {
        n1[a] = a < d1 ? NT(D, i + 1, a) : 0;
        nm[a] = a < dm ? NT(D, j - 1, a) : 0;
      }
      const double *eI = sB[1], *eJ = sB[2], *u = sB[0], *qin = sB[3], *qx = sB[4];
      double h = INFINITY;
      for (int a = 0; a < d1; a++)
        for (int b = 0; b < dm; b++)
          h = fmin(h, eI[s * 6 + a] + u[a * 6 + b] + eJ[b * 6 + s2] + sMM[(n1[a] * 4 + nm[b]) * 6 + t]);
      double acc = fmin(INFINITY, D.hp[j - i - 1] + h);
      if ((j - 1) - (i + 1) >= 4)
        for (int x = 0; x < d1; x++)
          for (int y = 0; y < dm; y++) {
            const double qq = qin[x * 6 + y];
            if (qq == INFINITY) continue;
            const int t2 = bpair(n1[x], nm[y]);
            acc = fmin(acc, eI[s * 6 + x] + qq + eJ[y * 6 + s2] + sST[t * 6 + t2]);
          }
      for (int a = 0; a < d1; a++)
        for (int dd = 0; dd < dm; dd++) {
          const int q = a * 6 + dd;
          acc = fmin(acc, eI[s * 6 + a] + eJ[dd * 6 + s2] +
                              fmin(fmin(sG[0][q], sG[1][q]), sG[2][q] + sMM[(n1[a] * 4 + nm[dd]) * 6 + t]));
        }
      double mlv = INFINITY;
      for (int x = 0; x < d1; x++)
        for (int y = 0; y < dm; y++) mlv = fmin(mlv, eI[s * 6 + x] + qx[x * 6 + y] + eJ[y * 6 + s2]);
      acc = fmin(acc, D.ml_ab + mlv);
      qb = D.v[i * 6 + s] + D.v[j * 6 + s2] + acc;
      blk(D.Qb, n, i, j)[tid] = qb;
    }
    sQb[tid] = qb;
  }
  __syncthreads();
  if (tid < 36) {
    const int a = tid / 6, b = tid % 6;
    // DI[i][j](b', c'): (i, j) as the inner pair of an interior loop (di_term)
    if (i >= 1 && j + 1 < n && a < D.d[i - 1] && b < D.d[j + 1]) {
      const double *eL = sB[5], *eR = sB[6];
      const int nl = NT(D, i - 1, a), nr = NT(D, j + 1, b);
      double best = INFINITY;
      for (int x = 0; x < di; x++)
        for (int y = 0; y < dj; y++) {
          const double qq = sQb[x * 6 + y];
          if (qq == INFINITY) continue;
          const int t2 = bpair(NT(D, j, y), NT(D, i, x));
          best = fmin(best, eL[a * 6 + x] + qq + eR[y * 6 + b] + sMM[(nr * 4 + nl) * 6 + t2]);
        }
      blk(D.DI, n, i, j)[tid] = best;
    }
    // one branch with an unpaired tail, then with an unpaired prefix
    const int s = a, s2 = b;
    double q1p = INFINITY;
    if (s < di && s2 < dj) {
      const double *q1l = sB[7], *q1pr = sB[8], *eI = sB[1], *eJ = sB[2];
      double tail = INFINITY;
      for (int t = 0; t < dm; t++) tail = fmin(tail, q1l[s * 6 + t] + eJ[t * 6 + s2]);
      const double q1 = fmin(sQb[tid] + D.ml_b, tail + D.v[j * 6 + s2] + D.ml_c);
      blk(D.Qm1, n, i, j)[tid] = q1;
      double pre = INFINITY;
      for (int t = 0; t < d1; t++) pre = fmin(pre, eI[s * 6 + t] + q1pr[t * 6 + s2]);
      q1p = fmin(q1, D.v[i * 6 + s] + D.ml_c + pre);
      blk(D.Qm1p, n, i, j)[tid] = q1p;
    }
    sQ1p[tid] = q1p;
  }
  // ---- two or more branches: the split over u = i+5..j-4, threads over u
  // (each thread all 36 outputs for its u), then minima across the workgroup
  double part[36];
#pragma unroll
  for (int q = 0; q < 36; q++) part[q] = INFINITY;
  for (int u = i + 5 + tid; u <= j - 4; u += MT) {
    const double *qm = cblk(D.Qm, n, i, u - 1), *q1 = cblk(D.Qm1, n, u, j);
    const int du1 = D.d[u - 1], du = D.d[u];
    for (int t = 0; t < du1; t++)
      for (int t2 = 0; t2 < du; t2++) {
        const double et = E(D, u - 1, t, t2);
        double qv[6];
#pragma unroll
        for (int s2 = 0; s2 < 6; s2++) qv[s2] = s2 < dj ? q1[t2 * 6 + s2] : INFINITY;
#pragma unroll
        for (int s = 0; s < 6; s++)
          if (s < di) {
            const double ae = qm[s * 6 + t] + et;
#pragma unroll
            for (int s2 = 0; s2 < 6; s2++) part[s * 6 + s2] = fmin(part[s * 6 + s2], ae + qv[s2]);
          }
      }
  }
#pragma unroll
  for (int q = 0; q < 36; q++) {
    double m = part[q];
    for (int off = 32; off >= 1; off >>= 1) m = fmin(m, __shfl_xor(m, off, 64));
    part[q] = m;
  }
  if ((tid & 63) == 0)
    for (int q = 0; q < 36; q++) sSp[tid >> 6][q] = part[q];
  __syncthreads();
  if (tid < 36) {
    const int s = tid / 6, s2 = tid % 6;
    if (s < di && s2 < dj) {
      double x = INFINITY;
      for (int w = 0; w < MT / 64; w++) x = fmin(x, sSp[w][tid]);
      blk(D.QmX, n, i, j)[tid] = x;
      blk(D.Qm, n, i, j)[tid] = fmin(x, sQ1p[tid]);
    }
  }
}

// first-of-smallest reduction over a workgroup: (value, order index); an
// alternative of value +inf is never chosen
struct Pick {
  double v;
  int idx;
};
__device__ __forceinline__ bool better(double v, int idx, const Pick &p) {
  return v < p.v || (v == p.v && v != INFINITY && idx < p.idx);
}
__device__ Pick pick_reduce(Pick p, double *sv, int *si) {
  const int tid = threadIdx.x;
  __syncthreads();
  sv[tid] = p.v;
  si[tid] = p.idx;
  __syncthreads();
  for (int w = MT / 2; w >= 1; w >>= 1) {
    if (tid < w) {
      const double ov = sv[tid + w];
      const int oi = si[tid + w];
      if (better(ov, oi, Pick{sv[tid], si[tid]})) {
        sv[tid] = ov;
        si[tid] = oi;
      }
    }
    __syncthreads();
  }
  const Pick r{sv[0], si[0]};
  __syncthreads();
  return r;
}

// exterior prefix: Z5[j](t) over the structures of [0..j] with slot t at j
__global__ __launch_bounds__(MT) void mfe_exterior(MfeDev D) {
  __shared__ double sP[MT / 64][6];
  const int n = D.n, tid = threadIdx.x;
  if (tid < 6) D.Z5[tid] = tid < D.d[0] ? D.v[tid] : INFINITY;
  __syncthreads();
  for (int j = 1; j < n; j++) {
    // k pairs j, k = 1..j-4: minima over (k, slot of k-1, slot of k) per slot
    // t of j; a thread takes whole k, all its operands loaded at once (entries
    // beyond a position's slots are +inf and drop out of the minima)
    double part[6];
#pragma unroll
    for (int t = 0; t < 6; t++) part[t] = INFINITY;
    const int dj = D.d[j];
    for (int k = 1 + tid; k <= j - 4; k += MT) {
      const double *z = D.Z5 + (k - 1) * 6, *eb = D.e + (size_t)(k - 1) * 36, *qb = cblk(D.Qb, n, k, j);
      double zz[6], ee[36], qq[36];
#pragma unroll
      for (int q = 0; q < 6; q++) zz[q] = z[q];
#pragma unroll
      for (int q = 0; q < 36; q++) {
        ee[q] = eb[q];
        qq[q] = qb[q];
      }
#pragma unroll
      for (int s = 0; s < 6; s++)
#pragma unroll
        for (int x = 0; x < 6; x++) {
          const double ze = zz[s] + ee[s * 6 + x];
#pragma unroll
          for (int t = 0; t < 6; t++) part[t] = fmin(part[t], ze + qq[x * 6 + t]);
        }
    }
#pragma unroll
    for (int t = 0; t < 6; t++)
      for (int off = 32; off >= 1; off >>= 1) part[t] = fmin(part[t], __shfl_xor(part[t], off, 64));
    if ((tid & 63) == 0)
      for (int t = 0; t < 6; t++) sP[tid >> 6][t] = part[t];
    __syncthreads();
    if (tid < 6) {
      const int t = tid;
      double best = INFINITY;
      if (t < dj) {
        double un = INFINITY;
        for (int s = 0; s < D.d[j - 1]; s++) un = fmin(un, D.Z5[(j - 1) * 6 + s] + E(D, j - 1, s, t));
        best = un + D.v[j * 6 + t];
        if (j >= 4)
          for (int x = 0; x < D.d[0]; x++) best = fmin(best, cblk(D.Qb, n, 0, j)[x * 6 + t]);
        for (int w = 0; w < MT / 64; w++) best = fmin(best, sP[w][t]);
      }
      D.Z5[j * 6 + t] = best;
    }
    __syncthreads();
  }
  if (tid == 0) {
    double m = INFINITY;
    for (int t = 0; t < D.d[n - 1]; t++) m = fmin(m, D.Z5[(n - 1) * 6 + t]);
    D.out[0] = m;
  }
}

enum { K_EXT = 0, K_PAIR, K_RUN, K_QM1, K_QM1P, K_QM, K_QMX };

// ---- argmin traceback, one workgroup
__global__ __launch_bounds__(MT) void mfe_traceback(MfeDev D) {
  __shared__ double sv[MT];
  __shared__ int si[MT];
  __shared__ int top;
  __shared__ int frag[5];
  const int n = D.n, tid = threadIdx.x;
  auto push = [&](int kind, int i, int j, int s, int s2) {  // thread 0 only
    if (top >= D.cap) {
      D.err[0] = 1;
      return;
    }
    int *f = D.stk + top * 5;
    f[0] = kind;
    f[1] = i;
    f[2] = j;
    f[3] = s;
    f[4] = s2;
    top++;
  };
  if (tid == 0) {
    top = 0;
    D.err[0] = 0;
    int bt = -1;
    double bv = INFINITY;
    for (int t = 0; t < D.d[n - 1]; t++)
      if (D.Z5[(n - 1) * 6 + t] < bv) {
        bv = D.Z5[(n - 1) * 6 + t];
        bt = t;
      }
    push(K_EXT, n - 1, 0, bt, 0);
  }
  for (int p = tid; p < n; p += MT) {
    D.slot[p] = -1;
    D.pt[p] = -1;
  }
  __syncthreads();
  while (true) {
    if (tid == 0) {
      if (top > 0 && D.err[0] == 0) {
        top--;
        for (int k = 0; k < 5; k++) frag[k] = D.stk[top * 5 + k];
      } else {
        frag[0] = -1;
      }
    }
    __syncthreads();
    const int kind = frag[0], i = frag[1], j = frag[2], s = frag[3], s2 = frag[4];
    __syncthreads();
    if (kind < 0) break;
    if (kind == K_EXT) {
      // exterior at (j = i here, slot s): j unpaired [s'], 0 pairs j [100 + x], k pairs j [1000 + ...]
      const int jj = i, t = s;
      if (tid == 0) D.slot[jj] = t;
      if (jj == 0) continue;
      Pick p{INFINITY, 0x7fffffff};
      for (int k = 1 + tid; k <= jj - 4; k += MT) {  // whole k per thread, (s, x) ascending
        const double *z = D.Z5 + (k - 1) * 6, *eb = D.e + (size_t)(k - 1) * 36, *qb = cblk(D.Qb, n, k, jj);
        double zz[6], ee[36], qq[6];
#pragma unroll
        for (int q = 0; q < 6; q++) {
          zz[q] = z[q];
          qq[q] = qb[q * 6 + t];
        }
#pragma unroll
        for (int q = 0; q < 36; q++) ee[q] = eb[q];
#pragma unroll
        for (int sp = 0; sp < 6; sp++)
#pragma unroll
          for (int x = 0; x < 6; x++) {
            const double val = zz[sp] + ee[sp * 6 + x] + qq[x];
            const int idx = 1000 + (k * 6 + sp) * 6 + x;
            if (better(val, idx, p)) p = Pick{val, idx};
          }
      }
      if (tid == 0) {
        for (int sp = 0; sp < D.d[jj - 1]; sp++) {
          const double val = (D.Z5[(jj - 1) * 6 + sp] + E(D, jj - 1, sp, t)) + D.v[jj * 6 + t];
          if (better(val, sp, p)) p = Pick{val, sp};
        }
        if (jj >= 4)
          for (int x = 0; x < D.d[0]; x++) {
            const double val = cblk(D.Qb, n, 0, jj)[x * 6 + t];
            if (better(val, 100 + x, p)) p = Pick{val, 100 + x};
          }
      }
      p = pick_reduce(p, sv, si);
      if (tid == 0) {
        if (p.v == INFINITY) {
          D.err[0] = 2;  // no finite alternative: the stored minimum cannot be reproduced
        } else if (p.idx < 100) {
          push(K_EXT, jj - 1, 0, p.idx, 0);
        } else if (p.idx < 1000) {
          push(K_PAIR, 0, jj, p.idx - 100, t);
        } else {
          const int r = p.idx - 1000, x = r % 6, sp = (r / 6) % 6, k = r / 36;
          push(K_EXT, k - 1, 0, sp, 0);
          push(K_PAIR, k, jj, x, t);
        }
      }
    } else if (kind == K_RUN) {
      if (tid == 0) {
        D.slot[j] = s2;
        if (i != j) {
          const double *ul = cblk(D.U, n, i, j - 1);
          int bc = -1;
          double bv = INFINITY;
          for (int c = 0; c < D.d[j - 1]; c++) {
            const double val = ul[s * 6 + c] + E(D, j - 1, c, s2);
            if (val < bv) {
              bv = val;
              bc = c;
            }
          }
          if (bc < 0) D.err[0] = 2;
          else push(K_RUN, i, j - 1, s, bc);
        }
      }
    } else if (kind == K_PAIR) {
      if (tid == 0) {
        D.slot[i] = s;
        D.slot[j] = s2;
        D.pt[i] = j;
        D.pt[j] = i;
      }
      const int t = bpair(NT(D, i, s), NT(D, j, s2)), dl = j - i;
      // level 1: hairpin [0], stack [1], windows [2 + l1 * 31 + l2], multiloop [2000]
      Pick p{INFINITY, 0x7fffffff};
      for (int w = tid; w < 31 * 31; w += MT) {
        int l1, l2;
        if (!window_of(w, dl, l1, l2)) continue;
        const double *ul = l1 > 0 ? cblk(D.U, n, i + 1, i + l1) : nullptr;
        const double *ur = l2 > 0 ? cblk(D.U, n, j - l2, j - 1) : nullptr;
        double best = INFINITY;
        for (int a = 0; a < D.d[i + 1]; a++)
          for (int dd = 0; dd < D.d[j - 1]; dd++) {
            double wv = window_value(D, i, j, l1, l2, a, dd, ul, ur);
            if (l1 > 0 && l2 > 0) wv = wv + MM(D, NT(D, i + 1, a), NT(D, j - 1, dd), t);
            best = fmin(best, outer_term(D, i, j, s, s2, a, dd, wv));
          }
        if (better(best, 2 + w, p)) p = Pick{best, 2 + w};
      }
      if (tid == 0) {
        double h = INFINITY;
        for (int a = 0; a < D.d[i + 1]; a++)
          for (int b = 0; b < D.d[j - 1]; b++) h = fmin(h, hairpin_term(D, i, j, s, s2, t, a, b));
        const double hv = D.hp[j - i - 1] + h;
        if (better(hv, 0, p)) p = Pick{hv, 0};
        if ((j - 1) - (i + 1) >= 4) {
          double st = INFINITY;
          for (int x = 0; x < D.d[i + 1]; x++)
            for (int y = 0; y < D.d[j - 1]; y++) st = fmin(st, stack_term(D, i, j, s, s2, t, x, y));
          if (better(st, 1, p)) p = Pick{st, 1};
        }
        double mlv = INFINITY;
        for (int x = 0; x < D.d[i + 1]; x++)
          for (int y = 0; y < D.d[j - 1]; y++) mlv = fmin(mlv, ml_term(D, i, j, s, s2, x, y));
        const double mv = D.ml_ab + mlv;
        if (better(mv, 2000, p)) p = Pick{mv, 2000};
      }
      p = pick_reduce(p, sv, si);
      if (tid == 0 && p.v == INFINITY) D.err[0] = 2;
      if (tid == 0 && p.v != INFINITY) {
        auto first6 = [&](auto f, int da, int db) {  // first (x, y) of smallest f(x, y); -1 if none
          int bi = -1;
          double bv = INFINITY;
          for (int x = 0; x < da; x++)
            for (int y = 0; y < db; y++) {
              const double val = f(x, y);
              if (val < bv) {
                bv = val;
                bi = x * 6 + y;
              }
            }
          if (bi < 0) D.err[0] = 2;
          return bi < 0 ? 0 : bi;
        };
        if (p.idx == 0) {
          const int c = first6([&](int a, int b) { return hairpin_term(D, i, j, s, s2, t, a, b); }, D.d[i + 1],
                               D.d[j - 1]);
          push(K_RUN, i + 1, j - 1, c / 6, c % 6);
        } else if (p.idx == 1) {
          const int c = first6([&](int x, int y) { return stack_term(D, i, j, s, s2, t, x, y); }, D.d[i + 1],
                               D.d[j - 1]);
          push(K_PAIR, i + 1, j - 1, c / 6, c % 6);
        } else if (p.idx == 2000) {
          const int c = first6([&](int x, int y) { return ml_term(D, i, j, s, s2, x, y); }, D.d[i + 1],
                               D.d[j - 1]);
          push(K_QMX, i + 1, j - 1, c / 6, c % 6);
        } else {
          const int w = p.idx - 2, l1 = w / 31, l2 = w % 31, k = i + 1 + l1, l = j - 1 - l2;
          const double *ul = l1 > 0 ? cblk(D.U, n, i + 1, i + l1) : nullptr;
          const double *ur = l2 > 0 ? cblk(D.U, n, j - l2, j - 1) : nullptr;
          const int c = first6(
              [&](int a, int dd) {
                double wv = window_value(D, i, j, l1, l2, a, dd, ul, ur);
                if (l1 > 0 && l2 > 0) wv = wv + MM(D, NT(D, i + 1, a), NT(D, j - 1, dd), t);
                return outer_term(D, i, j, s, s2, a, dd, wv);
              },
              D.d[i + 1], D.d[j - 1]);
          const int a = c / 6, dd = c % 6;
          if (l2 == 0) {  // left bulge: (b, x)
            const double *q = cblk(D.Qb, n, k, j - 1);
            const int g = first6([&](int b, int x) { return ul[a * 6 + b] + E(D, k - 1, b, x) + q[x * 6 + dd]; },
                                 D.d[k - 1], D.d[k]);
            push(K_RUN, i + 1, k - 1, a, g / 6);
            push(K_PAIR, k, j - 1, g % 6, dd);
          } else if (l1 == 0) {  // right bulge: (y, c)
            const double *q = cblk(D.Qb, n, i + 1, l);
            const int g = first6([&](int y, int cc) { return q[a * 6 + y] + E(D, l, y, cc) + ur[cc * 6 + dd]; },
                                 D.d[l], D.d[l + 1]);
            push(K_PAIR, i + 1, l, a, g / 6);
            push(K_RUN, l + 1, j - 1, g % 6, dd);
          } else {  // interior: c, then b, then the inner pair's slots
            const double *di = cblk(D.DI, n, k, l);
            int cc = -1;
            double bv = INFINITY;
            for (int c2 = 0; c2 < D.d[l + 1]; c2++) {
              double T = INFINITY;
              for (int b = 0; b < D.d[k - 1]; b++) T = fmin(T, ul[a * 6 + b] + di[b * 6 + c2]);
              const double val = T + ur[c2 * 6 + dd];
              if (val < bv) {
                bv = val;
                cc = c2;
              }
            }
            if (cc < 0) {
              D.err[0] = 2;
              cc = 0;
            }
            int bb = -1;
            bv = INFINITY;
            for (int b = 0; b < D.d[k - 1]; b++) {
              const double val = ul[a * 6 + b] + di[b * 6 + cc];
              if (val < bv) {
                bv = val;
                bb = b;
              }
            }
            if (bb < 0) {
              D.err[0] = 2;
              bb = 0;
            }
            const double *qk = cblk(D.Qb, n, k, l);
            const int g = first6([&](int x, int y) { return di_term(D, qk, k, l, bb, cc, x, y); }, D.d[k], D.d[l]);
            push(K_RUN, i + 1, k - 1, a, bb);
            push(K_PAIR, k, l, g / 6, g % 6);
            push(K_RUN, l + 1, j - 1, cc, dd);
          }
        }
      }
    } else if (kind == K_QM || kind == K_QMX) {
      Pick p{INFINITY, 0x7fffffff};
      for (int u = i + 5 + tid; u <= j - 4; u += MT) {
        const double *qm = cblk(D.Qm, n, i, u - 1), *q1 = cblk(D.Qm1, n, u, j);
        for (int t = 0; t < D.d[u - 1]; t++)
          for (int t2 = 0; t2 < D.d[u]; t2++) {
            const double val = qm[s * 6 + t] + E(D, u - 1, t, t2) + q1[t2 * 6 + s2];
            const int idx = (u * 6 + t) * 6 + t2;
            if (better(val, idx, p)) p = Pick{val, idx};
          }
      }
      if (tid == 0 && kind == K_QM) {  // the one-branch form, last in order
        const double val = cblk(D.Qm1p, n, i, j)[s * 6 + s2];
        if (better(val, 0x7ffffffe, p)) p = Pick{val, 0x7ffffffe};
      }
      p = pick_reduce(p, sv, si);
      if (tid == 0) {
        if (p.v == INFINITY) {
          D.err[0] = 2;
        } else if (p.idx == 0x7ffffffe) {
          push(K_QM1P, i, j, s, s2);
        } else {
          const int t2 = p.idx % 6, t = (p.idx / 6) % 6, u = p.idx / 36;
          push(K_QM, i, u - 1, s, t);
          push(K_QM1, u, j, t2, s2);
        }
      }
    } else if (kind == K_QM1) {
      if (tid == 0) {
        double bv = cblk(D.Qb, n, i, j)[s * 6 + s2] + D.ml_b;
        int bi = -2;
        for (int t = 0; t < D.d[j - 1]; t++) {
          const double val = (cblk(D.Qm1, n, i, j - 1)[s * 6 + t] + E(D, j - 1, t, s2)) + D.v[j * 6 + s2] + D.ml_c;
          if (val < bv) {
            bv = val;
            bi = t;
          }
        }
        if (bi == -2) {
          push(K_PAIR, i, j, s, s2);
        } else {
          D.slot[j] = s2;
          push(K_QM1, i, j - 1, s, bi);
        }
      }
    } else if (kind == K_QM1P) {
      if (tid == 0) {
        double bv = cblk(D.Qm1, n, i, j)[s * 6 + s2];
        int bi = -2;
        for (int t = 0; t < D.d[i + 1]; t++) {
          const double val = D.v[i * 6 + s] + D.ml_c + (E(D, i, s, t) + cblk(D.Qm1p, n, i + 1, j)[t * 6 + s2]);
          if (val < bv) {
            bv = val;
            bi = t;
          }
        }
        if (bi == -2) {
          push(K_QM1, i, j, s, s2);
        } else {
          D.slot[i] = s;
          push(K_QM1P, i + 1, j, bi, s2);
        }
      }
    }
    __syncthreads();
  }
}

// ---- suboptimal enumeration (SI S4d) ------------------------------------
// Every state within gap of the minimum, by a depth-first search over the
// traceback's decisions.  A partial state is a stack of pending fragments and
// a bound: the energy decided so far plus the minimum (the DP entry) of every
// pending fragment.  Expanding fragment f by an alternative of value V (its
// own energy plus the entries of the fragments it leaves) gives the bound
// (bound - entry(f)) + V; alternatives whose bound exceeds the threshold are
// dropped, the others are tried in the traceback's order.  One workgroup runs
// the search: thread 0 keeps the levels, and all threads evaluate a
// fragment's candidate alternatives, kept in enumeration order by a
// workgroup prefix sum.  A pair's windows are first screened at the level of
// their outer slots (the window's minimum is a lower bound of its children).

struct SubAlt {
  double V;
  int nsub, nas;
  int sub[3][5];
  int as[3][3];  // position, slot, partner (-1 unpaired)
};
struct SubLevel {
  int f[5];  // fragment expanded here (kind -1 at the root)
  int flen0;  // pending length after f was taken off
  int a0, na, next;
  double b0;  // bound before f was expanded
};
struct SubDev {
  double thr;
  int max_states, cap_alts, cap_lv;
  SubAlt *alts;
  SubLevel *lv;
  int *pend;          // [cap_lv][5]
  int *pk;            // [n + 1] prefix sums of d[k-1] d[k] over k (k >= 1)
  int *wlist;         // [496 * 36] screened (window, a, dd) of the pair being expanded
  double *energies;   // [max_states]
  unsigned char *codons;  // [max_states][m]
  int *pairs;         // [max_states][n]
  int *status;        // [0] states, [1] 0 done / 1 more states / 2 alternatives / 3 levels / 4 inconsistent
};

__device__ double frag_entry(const MfeDev &D, const int *f) {
  const int n = D.n, i = f[1], j = f[2], s = f[3], s2 = f[4];
  switch (f[0]) {
    case K_EXT: return D.Z5[i * 6 + s];
    case K_PAIR: return cblk(D.Qb, n, i, j)[s * 6 + s2];
    case K_RUN: return cblk(D.U, n, i, j)[s * 6 + s2];
    case K_QM1: return cblk(D.Qm1, n, i, j)[s * 6 + s2];
    case K_QM1P: return cblk(D.Qm1p, n, i, j)[s * 6 + s2];
    case K_QM: return cblk(D.Qm, n, i, j)[s * 6 + s2];
    default: return cblk(D.QmX, n, i, j)[s * 6 + s2];
  }
}

__device__ __forceinline__ void alt_sub(SubAlt &a, int kind, int i, int j, int s, int s2) {
  int *q = a.sub[a.nsub++];
  q[0] = kind;
  q[1] = i;
  q[2] = j;
  q[3] = s;
  q[4] = s2;
}
__device__ __forceinline__ void alt_as(SubAlt &a, int p, int s, int partner) {
  a.as[a.nas][0] = p;
  a.as[a.nas][1] = s;
  a.as[a.nas][2] = partner;
  a.nas++;
}

// exclusive prefix of one count per thread over the workgroup; returns the total
__device__ int block_scan_count(int cnt, int &pos, int *wsum) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  int inc = cnt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  __syncthreads();
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int off = 0, tot = 0;
  for (int q = 0; q < MT / 64; q++) {
    if (q < w) off += wsum[q];
    tot += wsum[q];
  }
  pos = off + inc - cnt;
  __syncthreads();
  return tot;
}

// candidates per thread and round: each thread takes EPT consecutive indices,
// so one workgroup prefix sum orders MT * EPT of them
constexpr int EPT = 8;

// append, in index order, the candidates idx < cnt that gen() builds and
// whose bound base + V stays within the threshold (the few that pass are
// built a second time when they are written out)
template <typename G>
__device__ void emit(const SubDev &S, int cnt, double base, G gen, int *wsum, int *nalts) {
  for (int c0 = 0; c0 < cnt; c0 += MT * EPT) {
    const int first = c0 + (int)threadIdx.x * EPT;
    unsigned mask = 0;
    int mine = 0;
    for (int u = 0; u < EPT; u++) {
      const int idx = first + u;
      if (idx < cnt) {
        SubAlt a;
        a.nsub = a.nas = 0;
        gen(idx, a);
        if (base + a.V <= S.thr) {
          mask |= 1u << u;
          mine++;
        }
      }
    }
    int pos;
    const int tot = block_scan_count(mine, pos, wsum);
    const int at = *nalts;
    for (int u = 0, q = 0; u < EPT && mask; u++)
      if ((mask >> u) & 1) {
        SubAlt a;
        a.nsub = a.nas = 0;
        gen(first + u, a);
        if (at + pos + q < S.cap_alts) S.alts[at + pos + q] = a;
        q++;
      }
    __syncthreads();
    if (threadIdx.x == 0) *nalts = at + tot;
    __syncthreads();
  }
}

// bulge and interior windows (l1, l2), l1 + l2 <= 30 and not both zero, in
// enumeration order (l1 ascending, then l2 ascending)
struct AllWin {
  unsigned char l1[495], l2[495];
};
constexpr AllWin make_allwin() {
  AllWin t{};
  int m = 0;
  for (int a = 0; a <= MAXW; a++)
    for (int b = 0; a + b <= MAXW; b++) {
      if (a == 0 && b == 0) continue;
      t.l1[m] = (unsigned char)a;
      t.l2[m] = (unsigned char)b;
      m++;
    }
  return t;
}
__constant__ AllWin kAllWin = make_allwin();

// index of the last k with pk[k] <= idx, searching k in [lo, hi)
__device__ __forceinline__ int pk_find(const int *pk, int lo, int hi, int idx) {
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pk[mid] <= idx) lo = mid;
    else hi = mid;
  }
  return lo;
}

__device__ void sub_alternatives(const MfeDev &D, const SubDev &S, const int *f, double base, int *wsum, int *nalts,
                                 int *wcount) {
  const int n = D.n, kind = f[0], i = f[1], j = f[2], s = f[3], s2 = f[4];
  if (kind == K_EXT) {
    const int jj = i, t = s;
    if (jj == 0) {
      emit(S, 1, base, [&](int, SubAlt &a) {
        a.V = D.Z5[t];
        alt_as(a, 0, t, -1);
      }, wsum, nalts);
      return;
    }
    const int c1 = D.d[jj - 1], c2 = jj >= 4 ? D.d[0] : 0;
    const int c3 = jj >= 5 ? S.pk[jj - 3] - S.pk[1] : 0;  // k = 1..jj-4
    emit(S, c1 + c2 + c3, base, [&](int idx, SubAlt &a) {
      if (idx < c1) {
        const int sp = idx;
        a.V = (D.Z5[(jj - 1) * 6 + sp] + E(D, jj - 1, sp, t)) + D.v[jj * 6 + t];
        alt_as(a, jj, t, -1);
        alt_sub(a, K_EXT, jj - 1, 0, sp, 0);
      } else if (idx < c1 + c2) {
        const int x = idx - c1;
        a.V = cblk(D.Qb, n, 0, jj)[x * 6 + t];
        alt_sub(a, K_PAIR, 0, jj, x, t);
      } else {
        const int r = idx - c1 - c2 + S.pk[1];
        const int k = pk_find(S.pk, 1, jj - 3, r), q = r - S.pk[k];
        const int sp = q / D.d[k], x = q % D.d[k];
        a.V = D.Z5[(k - 1) * 6 + sp] + E(D, k - 1, sp, x) + cblk(D.Qb, n, k, jj)[x * 6 + t];
        alt_sub(a, K_EXT, k - 1, 0, sp, 0);
        alt_sub(a, K_PAIR, k, jj, x, t);
      }
    }, wsum, nalts);
    return;
  }
  if (kind == K_RUN) {
    if (i == j) {
      emit(S, 1, base, [&](int, SubAlt &a) {
        a.V = cblk(D.U, n, i, i)[s * 6 + s2];
        alt_as(a, i, s2, -1);
      }, wsum, nalts);
      return;
    }
    emit(S, D.d[j - 1], base, [&](int c, SubAlt &a) {
      a.V = (cblk(D.U, n, i, j - 1)[s * 6 + c] + E(D, j - 1, c, s2)) + D.v[j * 6 + s2];
      alt_as(a, j, s2, -1);
      alt_sub(a, K_RUN, i, j - 1, s, c);
    }, wsum, nalts);
    return;
  }
  if (kind == K_QM1) {
    emit(S, 1 + D.d[j - 1], base, [&](int idx, SubAlt &a) {
      if (idx == 0) {
        a.V = cblk(D.Qb, n, i, j)[s * 6 + s2] + D.ml_b;
        alt_sub(a, K_PAIR, i, j, s, s2);
      } else {
        const int t = idx - 1;
        a.V = (cblk(D.Qm1, n, i, j - 1)[s * 6 + t] + E(D, j - 1, t, s2)) + D.v[j * 6 + s2] + D.ml_c;
        alt_as(a, j, s2, -1);
        alt_sub(a, K_QM1, i, j - 1, s, t);
      }
    }, wsum, nalts);
    return;
  }
  if (kind == K_QM1P) {
    emit(S, 1 + D.d[i + 1], base, [&](int idx, SubAlt &a) {
      if (idx == 0) {
        a.V = cblk(D.Qm1, n, i, j)[s * 6 + s2];
        alt_sub(a, K_QM1, i, j, s, s2);
      } else {
        const int t = idx - 1;
        a.V = D.v[i * 6 + s] + D.ml_c + (E(D, i, s, t) + cblk(D.Qm1p, n, i + 1, j)[t * 6 + s2]);
        alt_as(a, i, s, -1);
        alt_sub(a, K_QM1P, i + 1, j, t, s2);
      }
    }, wsum, nalts);
    return;
  }
  if (kind == K_QM || kind == K_QMX) {
    // splits u = i+5 .. j-4 by (slot t of u-1, slot t2 of u), then (Qm only) Qm1p
    const int cs = j - 4 >= i + 5 ? S.pk[j - 3] - S.pk[i + 5] : 0;
    emit(S, cs + (kind == K_QM ? 1 : 0), base, [&](int idx, SubAlt &a) {
      if (idx < cs) {
        const int r = idx + S.pk[i + 5];
        const int u = pk_find(S.pk, i + 5, j - 3, r), q = r - S.pk[u];
        const int t = q / D.d[u], t2 = q % D.d[u];
        a.V = cblk(D.Qm, n, i, u - 1)[s * 6 + t] + E(D, u - 1, t, t2) + cblk(D.Qm1, n, u, j)[t2 * 6 + s2];
        alt_sub(a, K_QM, i, u - 1, s, t);
        alt_sub(a, K_QM1, u, j, t2, s2);
      } else {
        a.V = cblk(D.Qm1p, n, i, j)[s * 6 + s2];
        alt_sub(a, K_QM1P, i, j, s, s2);
      }
    }, wsum, nalts);
    return;
  }
  // K_PAIR: every alternative's value is (v_i + v_j) + its term
  const double vv = D.v[i * 6 + s] + D.v[j * 6 + s2];
  const int t = bpair(NT(D, i, s), NT(D, j, s2));
  const int da = D.d[i + 1], db = D.d[j - 1];
  const double bh = D.hp[j - i - 1];
  emit(S, da * db, base, [&](int idx, SubAlt &a) {  // hairpin by the end slots of its run
    const int x = idx / db, y = idx % db;
    a.V = vv + (bh + hairpin_term(D, i, j, s, s2, t, x, y));
    alt_as(a, i, s, j);
    alt_as(a, j, s2, i);
    alt_sub(a, K_RUN, i + 1, j - 1, x, y);
  }, wsum, nalts);
  if ((j - 1) - (i + 1) >= 4)
    emit(S, da * db, base, [&](int idx, SubAlt &a) {  // stack
      const int x = idx / db, y = idx % db;
      a.V = vv + stack_term(D, i, j, s, s2, t, x, y);
      alt_as(a, i, s, j);
      alt_as(a, j, s2, i);
      alt_sub(a, K_PAIR, i + 1, j - 1, x, y);
    }, wsum, nalts);
  // bulge and interior windows, l1 then l2 ascending: screen every
  // (window, a, dd) by the window's minimum, keep the survivors in order
  {
    const int nwin = 495 * 36;
    if (threadIdx.x == 0) *wcount = 0;
    __syncthreads();
    for (int c0 = 0; c0 < nwin; c0 += MT * EPT) {
      const int first = c0 + (int)threadIdx.x * EPT;
      unsigned mask = 0;
      int mine = 0;
      int code[EPT];
      for (int u = 0; u < EPT; u++) {
        const int e = first + u;
        code[u] = 0;
        if (e >= nwin) continue;
        const int wi = e / 36, a = (e % 36) / 6, dd = e % 6, l1 = kAllWin.l1[wi], l2 = kAllWin.l2[wi];
        const int k = i + 1 + l1, l = j - 1 - l2;
        if (l - k >= 4 && a < da && dd < db) {
          const bool inter = l1 > 0 && l2 > 0;
          const double wv0 = window_value(D, i, j, l1, l2, a, dd, cblk(D.U, n, i + 1, k - 1),
                                          cblk(D.U, n, l + 1, j - 1));
          const double wv = inter ? wv0 + MM(D, NT(D, i + 1, a), NT(D, j - 1, dd), t) : wv0;
          if (base + (vv + outer_term(D, i, j, s, s2, a, dd, wv)) <= S.thr) {
            mask |= 1u << u;
            mine++;
            code[u] = (l1 * 31 + l2) * 36 + a * 6 + dd;
          }
        }
      }
      int pos;
      const int tot = block_scan_count(mine, pos, wsum);
      const int at = *wcount;
      for (int u = 0, q = 0; u < EPT; u++)
        if ((mask >> u) & 1) S.wlist[at + pos + q++] = code[u];
      __syncthreads();
      if (threadIdx.x == 0) *wcount = at + tot;
      __syncthreads();
    }
  }
  const int nw = *wcount;
  for (int q = 0; q < nw; q++) {
    const int e = S.wlist[q], w = e / 36, a = (e % 36) / 6, dd = e % 6, l1 = w / 31, l2 = w % 31;
    const int k = i + 1 + l1, l = j - 1 - l2;
    if (l2 == 0) {  // left bulge: run i+1..k-1 (a, b), edge (b, x), pair (k, j-1) (x, dd)
      const int dx = D.d[k];
      emit(S, D.d[k - 1] * dx, base, [&](int idx, SubAlt &al) {
        const int b = idx / dx, x = idx % dx;
        const double wv = D.bulge[l1] + (cblk(D.U, n, i + 1, k - 1)[a * 6 + b] + E(D, k - 1, b, x) +
                                         cblk(D.Qb, n, k, j - 1)[x * 6 + dd]);
        al.V = vv + outer_term(D, i, j, s, s2, a, dd, wv);
        alt_as(al, i, s, j);
        alt_as(al, j, s2, i);
        alt_sub(al, K_RUN, i + 1, k - 1, a, b);
        alt_sub(al, K_PAIR, k, j - 1, x, dd);
      }, wsum, nalts);
    } else if (l1 == 0) {  // right bulge: pair (i+1, l) (a, y), edge (y, c), run l+1..j-1 (c, dd)
      const int dc = D.d[l + 1];
      emit(S, D.d[l] * dc, base, [&](int idx, SubAlt &al) {
        const int y = idx / dc, c = idx % dc;
        const double wv = D.bulge[l2] + (cblk(D.Qb, n, i + 1, l)[a * 6 + y] + E(D, l, y, c) +
                                         cblk(D.U, n, l + 1, j - 1)[c * 6 + dd]);
        al.V = vv + outer_term(D, i, j, s, s2, a, dd, wv);
        alt_as(al, i, s, j);
        alt_as(al, j, s2, i);
        alt_sub(al, K_PAIR, i + 1, l, a, y);
        alt_sub(al, K_RUN, l + 1, j - 1, c, dd);
      }, wsum, nalts);
    } else {  // interior: (slot c of l+1, slot b of k-1, inner pair slots x, y)
      const int dc = D.d[l + 1], dbk = D.d[k - 1], dx = D.d[k], dy = D.d[l];
      const double mm = MM(D, NT(D, i + 1, a), NT(D, j - 1, dd), t);
      const double *qb = cblk(D.Qb, n, k, l);
      emit(S, dc * dbk * dx * dy, base, [&](int idx, SubAlt &al) {
        const int y = idx % dy, x = (idx / dy) % dx, b = (idx / (dy * dx)) % dbk, c = idx / (dy * dx * dbk);
        const double dt = di_term(D, qb, k, l, b, c, x, y);
        const double wv = D.interior[l1 + l2] +
                          ((cblk(D.U, n, i + 1, k - 1)[a * 6 + b] + dt) + cblk(D.U, n, l + 1, j - 1)[c * 6 + dd]);
        al.V = vv + outer_term(D, i, j, s, s2, a, dd, wv + mm);
        alt_as(al, i, s, j);
        alt_as(al, j, s2, i);
        alt_sub(al, K_RUN, i + 1, k - 1, a, b);
        alt_sub(al, K_PAIR, k, l, x, y);
        alt_sub(al, K_RUN, l + 1, j - 1, c, dd);
      }, wsum, nalts);
    }
  }
  emit(S, da * db, base, [&](int idx, SubAlt &a) {  // multiloop
    const int x = idx / db, y = idx % db;
    a.V = vv + (D.ml_ab + ml_term(D, i, j, s, s2, x, y));
    alt_as(a, i, s, j);
    alt_as(a, j, s2, i);
    alt_sub(a, K_QMX, i + 1, j - 1, x, y);
  }, wsum, nalts);
}

__global__ __launch_bounds__(MT) void mfe_subopt(MfeDev D, SubDev S) {
  __shared__ int wsum[MT / 64];
  __shared__ int nalts, nlv, npend, wcount, count, rc, act;  // act: 0 continue, 1 expand, 2 stop
  __shared__ int fexp[5];
  __shared__ double sbound;
  const int n = D.n, m = n / 3, tid = threadIdx.x;
  if (tid == 0) {
    nalts = 0;
    count = 0;
    rc = 0;
    SubLevel &L = S.lv[0];
    L.f[0] = -1;
    L.flen0 = 0;
    L.b0 = 0.0;
    L.a0 = 0;
    nlv = 1;
  }
  for (int p = tid; p < n; p += MT) {
    D.slot[p] = -1;
    D.pt[p] = -1;
  }
  __syncthreads();
  emit(S, D.d[n - 1], 0.0, [&](int t, SubAlt &a) {  // the root: slot of the last position
    a.V = D.Z5[(n - 1) * 6 + t];
    alt_sub(a, K_EXT, n - 1, 0, t, 0);
  }, wsum, &nalts);
  if (tid == 0) {
    S.lv[0].na = nalts;
    S.lv[0].next = 0;
  }
  __syncthreads();
  while (true) {
    if (tid == 0) {
      act = 0;
      if (nalts > S.cap_alts) {
        rc = 2;
        act = 2;
      } else if (nlv == 0) {
        act = 2;
      } else {
        SubLevel &L = S.lv[nlv - 1];
        if (L.next == L.na) {  // backtrack: put the expanded fragment back where it was taken from
          if (L.f[0] >= 0)
            for (int q = 0; q < 5; q++) S.pend[L.flen0 * 5 + q] = L.f[q];
          nalts = L.a0;
          nlv--;
        } else {
          const SubAlt &a = S.alts[L.a0 + L.next++];
          npend = L.flen0;
          for (int q = 0; q < a.nas; q++) {
            D.slot[a.as[q][0]] = a.as[q][1];
            D.pt[a.as[q][0]] = a.as[q][2];
          }
          for (int q = 0; q < a.nsub; q++) {
            for (int r = 0; r < 5; r++) S.pend[npend * 5 + r] = a.sub[q][r];
            npend++;
          }
          const double bound = L.f[0] < 0 ? a.V : (L.b0 - frag_entry(D, L.f)) + a.V;
          sbound = bound;
          if (npend == 0) {
            act = 3;  // a complete state
          } else if (nlv == S.cap_lv) {
            rc = 3;
            act = 2;
          } else {
            npend--;
            SubLevel &N = S.lv[nlv++];
            for (int q = 0; q < 5; q++) {
              N.f[q] = S.pend[npend * 5 + q];
              fexp[q] = N.f[q];
            }
            N.flen0 = npend;
            N.b0 = bound;
            N.a0 = nalts;
            act = 1;
          }
        }
      }
    }
    __syncthreads();
    const int what = act;
    if (what == 2) break;
    if (what == 3) {  // write the state out
      if (count >= S.max_states) {
        if (tid == 0) rc = 1;
        break;
      }
      const int c = count;
      for (int p = tid; p < n; p += MT) S.pairs[(size_t)c * n + p] = D.pt[p];
      for (int a = tid; a < m; a += MT) {
        const int sl = D.slot[3 * a];
        if (sl < 0 || D.slot[3 * a + 1] != sl || D.slot[3 * a + 2] != sl) atomicMax(&rc, 4);
        S.codons[(size_t)c * m + a] = (unsigned char)sl;
      }
      __syncthreads();
      if (tid == 0) {
        S.energies[c] = sbound;
        count = c + 1;
      }
      __syncthreads();
      if (rc == 4) break;
      continue;
    }
    if (what == 1) {
      int f[5];
      for (int q = 0; q < 5; q++) f[q] = fexp[q];
      const double base = sbound - frag_entry(D, f);
      const int a0 = nalts;
      sub_alternatives(D, S, f, base, wsum, &nalts, &wcount);
      if (tid == 0) {
        SubLevel &N = S.lv[nlv - 1];
        N.na = nalts - a0;
        N.next = 0;
      }
    }
    __syncthreads();
  }
  __syncthreads();
  if (tid == 0) {
    S.status[0] = count;
    S.status[1] = rc;
  }
}

struct DevBuf {
  void *p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

namespace {

// a request for the states within gap of the minimum instead of one argmin
struct SubReq {
  double gap;
  int max_states;
  double *energies;
  uint8_t *codons;
  int32_t *pairs;
  int32_t *count;
  int more;  // set when more than max_states states exist
};

cdz_status mfe_run(cdz_handle *h, const cdz_problem *prob, double *mfe, uint8_t *codons, int32_t *pairs,
                   SubReq *sub) {
  if (!h || !prob || !mfe) return cdz_fail(h, CDZ_ERR_ARG, "null argument");
  HostTables t;
  cdz_status st = build_tables(h, prob->n_aa, prob->aa, prob->theta1, prob->theta2, t);
  if (st != CDZ_OK) return st;
  const int n = t.n, m = t.m;
  const double inf = INFINITY;
  // energies: vertices, edges, hairpins by length, loop tables
  std::vector<double> v((size_t)n * 6, 0.0), e((size_t)n * 36, inf), hp(n + 1, inf);
  std::vector<signed char> nt((size_t)n * 6, 0);
  for (int p = 0; p < n; p++) {
    for (int s = 0; s < t.d[p]; s++) {
      nt[p * 6 + s] = (signed char)t.nt[p * 6 + s];
      if (p % 3 == 1 && prob->theta1) v[p * 6 + s] = -prob->theta1[(p / 3) * 6 + s];
    }
    if (p + 1 < n)
      for (int s = 0; s < t.d[p]; s++)
        for (int u = 0; u < t.d[p + 1]; u++) {
          if (p % 3 != 2) e[(size_t)p * 36 + s * 6 + u] = s == u ? 0.0 : inf;
          else e[(size_t)p * 36 + s * 6 + u] = prob->theta2 ? -prob->theta2[((p / 3 + 1) * 6 + s) * 6 + u] : 0.0;
        }
  }
  const cdz_energy &En = h->en;
  for (int L = 3; L <= n; L++) hp[L] = L <= 30 ? En.hairpin[L] : En.hairpin[30] + En.extrap * std::log((double)L / 30.0);
  // device workspace: tables, then the seven arrays
  const size_t cell = (size_t)n * n * 36;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = (off + 255) / 256 * 256;
    off = at + bytes;
    return at;
  };
  const size_t oD = take(n * sizeof(int)), oNt = take(nt.size()), oV = take(v.size() * 8), oE = take(e.size() * 8),
               oHp = take(hp.size() * 8), oSt = take(36 * 8), oBu = take(31 * 8), oIn = take(31 * 8),
               oMm = take(96 * 8), oZ5 = take((size_t)n * 6 * 8), oSl = take((size_t)n * 4), oPt = take((size_t)n * 4),
               oStk = take((size_t)(4 * n + 16) * 5 * 4), oOut = take(8), oErr = take(4);
  size_t oArr[7];
  for (int k = 0; k < 7; k++) oArr[k] = take(cell * 8);
  // suboptimal enumeration: levels, pending stack, alternatives, screened
  // windows, prefix sums of d[k-1] d[k], outputs and status
  const int cap_lv = 4 * n + 16, cap_alts = 1 << 20, nst = sub ? std::max(sub->max_states, 1) : 0;
  size_t oLv = 0, oPd = 0, oAl = 0, oWl = 0, oPk = 0, oEn = 0, oCo = 0, oPa = 0, oSs = 0;
  if (sub) {
    oLv = take((size_t)cap_lv * sizeof(SubLevel));
    oPd = take((size_t)cap_lv * 5 * 4);
    oAl = take((size_t)cap_alts * sizeof(SubAlt));
    oWl = take((size_t)31 * 31 * 36 * 4);
    oPk = take((size_t)(n + 1) * 4);
    oEn = take((size_t)nst * 8);
    oCo = take((size_t)nst * m);
    oPa = take((size_t)nst * n * 4);
    oSs = take(8);
  }
  DevBuf ws;
  if (hipMalloc(&ws.p, off) != hipSuccess) {
    (void)hipGetLastError();
    ws.p = nullptr;
    return cdz_fail(h, CDZ_ERR_NOMEM, "MFE workspace of " + std::to_string(off) + " bytes");
  }
  char *base = (char *)ws.p;
  hipStream_t sm = h->stream;
  std::vector<int> dvec(t.d.begin(), t.d.end());
  std::vector<double> tabs(36 + 31 + 31 + 96);
  memcpy(tabs.data(), En.stack, 36 * 8);
  memcpy(tabs.data() + 36, En.bulge, 31 * 8);
  memcpy(tabs.data() + 67, En.interior, 31 * 8);
  memcpy(tabs.data() + 98, En.mismatch, 96 * 8);
  HIPCHK(h, hipMemcpyAsync(base + oD, dvec.data(), n * sizeof(int), hipMemcpyHostToDevice, sm));
  HIPCHK(h, hipMemcpyAsync(base + oNt, nt.data(), nt.size(), hipMemcpyHostToDevice, sm));
  HIPCHK(h, hipMemcpyAsync(base + oV, v.data(), v.size() * 8, hipMemcpyHostToDevice, sm));
  HIPCHK(h, hipMemcpyAsync(base + oE, e.data(), e.size() * 8, hipMemcpyHostToDevice, sm));
  HIPCHK(h, hipMemcpyAsync(base + oHp, hp.data(), hp.size() * 8, hipMemcpyHostToDevice, sm));
  HIPCHK(h, hipMemcpyAsync(base + oSt, tabs.data(), 36 * 8, hipMemcpyHostToDevice, sm));
  HIPCHK(h, hipMemcpyAsync(base + oBu, tabs.data() + 36, 31 * 8, hipMemcpyHostToDevice, sm));
  HIPCHK(h, hipMemcpyAsync(base + oIn, tabs.data() + 67, 31 * 8, hipMemcpyHostToDevice, sm));
  HIPCHK(h, hipMemcpyAsync(base + oMm, tabs.data() + 98, 96 * 8, hipMemcpyHostToDevice, sm));
  MfeDev D;
  D.n = n;
  D.d = (const int *)(base + oD);
  D.nt = (const signed char *)(base + oNt);
  D.v = (const double *)(base + oV);
  D.e = (const double *)(base + oE);
  D.hp = (const double *)(base + oHp);
  D.stack = (const double *)(base + oSt);
  D.bulge = (const double *)(base + oBu);
  D.interior = (const double *)(base + oIn);
  D.mm = (const double *)(base + oMm);
  D.ml_ab = En.ml_a + En.ml_b;
  D.ml_b = En.ml_b;
  D.ml_c = En.ml_c;
  double **arr[7] = {&D.U, &D.Qb, &D.DI, &D.Qm1, &D.Qm1p, &D.QmX, &D.Qm};
  for (int k = 0; k < 7; k++) *arr[k] = (double *)(base + oArr[k]);
  D.Z5 = (double *)(base + oZ5);
  D.slot = (int *)(base + oSl);
  D.pt = (int *)(base + oPt);
  D.stk = (int *)(base + oStk);
  D.cap = 4 * n + 16;
  D.out = (double *)(base + oOut);
  D.err = (int *)(base + oErr);
  HIPCHK(h, hipEventRecord(h->ev[4], sm));
  for (int k = 0; k < 7; k++) hipLaunchKernelGGL(mfe_fill, dim3(2048), dim3(256), 0, sm, *arr[k], cell);
  hipLaunchKernelGGL(mfe_init_runs, dim3(n), dim3(64), 0, sm, D);
  HIPCHK(h, hipFuncSetAttribute((const void *)mfe_diag, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)MfeLds::bytes));
  for (int dl = 1; dl < n; dl++) hipLaunchKernelGGL(mfe_diag, dim3(n - dl), dim3(MT), MfeLds::bytes, sm, D, dl);
  hipLaunchKernelGGL(mfe_exterior, dim3(1), dim3(MT), 0, sm, D);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipEventRecord(h->ev[5], sm));
  SubDev S{};
  if (sub) {
    std::vector<int> pk(n + 1, 0);  // pk[k + 1] = pk[k] + d[k-1] d[k], k >= 1
    for (int k = 1; k < n; k++) pk[k + 1] = pk[k] + t.d[k - 1] * t.d[k];
    HIPCHK(h, hipMemcpyAsync(base + oPk, pk.data(), (n + 1) * 4, hipMemcpyHostToDevice, sm));
    S.max_states = sub->max_states;
    S.cap_alts = cap_alts;
    S.cap_lv = cap_lv;
    S.alts = (SubAlt *)(base + oAl);
    S.lv = (SubLevel *)(base + oLv);
    S.pend = (int *)(base + oPd);
    S.pk = (int *)(base + oPk);
    S.wlist = (int *)(base + oWl);
    S.energies = (double *)(base + oEn);
    S.codons = (unsigned char *)(base + oCo);
    S.pairs = (int *)(base + oPa);
    S.status = (int *)(base + oSs);
  }
  if (sub) {
    // the threshold needs the minimum: read it back first
    double mn = 0;
    HIPCHK(h, hipMemcpyAsync(&mn, D.out, 8, hipMemcpyDeviceToHost, sm));
    HIPCHK(h, hipStreamSynchronize(sm));
    if (!std::isfinite(mn)) return cdz_fail(h, CDZ_ERR_NUMERIC, "minimum free energy not finite");
    S.thr = mn + sub->gap + 1e-9 * std::max(1.0, std::fabs(mn));
    hipLaunchKernelGGL(mfe_subopt, dim3(1), dim3(MT), 0, sm, D, S);
  } else if (codons || pairs) {
    hipLaunchKernelGGL(mfe_traceback, dim3(1), dim3(MT), 0, sm, D);
  }
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipEventRecord(h->ev[6], sm));
  double res = 0;
  int err = 0;
  std::vector<int> slot(n), pt(n);
  HIPCHK(h, hipMemcpyAsync(&res, D.out, 8, hipMemcpyDeviceToHost, sm));
  if (codons || pairs) {
    HIPCHK(h, hipMemcpyAsync(&err, D.err, 4, hipMemcpyDeviceToHost, sm));
    HIPCHK(h, hipMemcpyAsync(slot.data(), D.slot, n * 4, hipMemcpyDeviceToHost, sm));
    HIPCHK(h, hipMemcpyAsync(pt.data(), D.pt, n * 4, hipMemcpyDeviceToHost, sm));
  }
  HIPCHK(h, hipStreamSynchronize(sm));
  float ms = 0;
  HIPCHK(h, hipEventElapsedTime(&ms, h->ev[4], h->ev[5]));
  h->times[0] = ms;
  if (codons || pairs || sub) {  // traceback or suboptimal search
    HIPCHK(h, hipEventElapsedTime(&ms, h->ev[5], h->ev[6]));
    h->times[2] = ms;
  }
  *mfe = res;
  if (!std::isfinite(res)) return cdz_fail(h, CDZ_ERR_NUMERIC, "minimum free energy not finite");
  if (sub) {
    int st[2] = {0, 0};
    HIPCHK(h, hipMemcpy(st, S.status, 8, hipMemcpyDeviceToHost));
    if (st[1] == 2)
      return cdz_fail(h, CDZ_ERR_BUDGET, "more than " + std::to_string(cap_alts) +
                                             " pending alternatives: lower the gap");
    if (st[1] == 3) return cdz_fail(h, CDZ_ERR_STATE, "enumeration level stack overflow");
    if (st[1] == 4) return cdz_fail(h, CDZ_ERR_STATE, "enumeration left an inconsistent codon");
    const int cnt = st[0];
    if (cnt > 0) {
      if (sub->energies) HIPCHK(h, hipMemcpy(sub->energies, S.energies, (size_t)cnt * 8, hipMemcpyDeviceToHost));
      if (sub->codons) HIPCHK(h, hipMemcpy(sub->codons, S.codons, (size_t)cnt * m, hipMemcpyDeviceToHost));
      if (sub->pairs) HIPCHK(h, hipMemcpy(sub->pairs, S.pairs, (size_t)cnt * n * 4, hipMemcpyDeviceToHost));
    }
    *sub->count = cnt;
    sub->more = st[1] == 1;
    return CDZ_OK;
  }
  if (codons || pairs) {
    if (err == 1) return cdz_fail(h, CDZ_ERR_STATE, "traceback stack overflow");
    if (err) return cdz_fail(h, CDZ_ERR_STATE, "traceback found no alternative reproducing the minimum");
    for (int a = 0; a < m; a++) {
      const int s = slot[3 * a];
      if (s < 0 || slot[3 * a + 1] != s || slot[3 * a + 2] != s)
        return cdz_fail(h, CDZ_ERR_STATE, "traceback left an inconsistent codon at residue " + std::to_string(a));
      if (codons) codons[a] = (uint8_t)s;
    }
    if (pairs)
      for (int p = 0; p < n; p++) pairs[p] = pt[p];
  }
  return CDZ_OK;
}

}  // namespace

extern "C" cdz_status cdz_mfe(cdz_handle *h, const cdz_problem *prob, double *mfe, uint8_t *codons, int32_t *pairs) {
  return mfe_run(h, prob, mfe, codons, pairs, nullptr);
}

extern "C" cdz_status cdz_subopt(cdz_handle *h, const cdz_problem *prob, double gap, int32_t max_states, double *mfe,
                                 double *energies, uint8_t *codons, int32_t *pairs, int32_t *count, int32_t *more) {
  if (!h || !prob || !mfe || !count || !(gap >= 0.0) || !std::isfinite(gap) || max_states < 0)
    return cdz_fail(h, CDZ_ERR_ARG, "null argument, negative or non-finite gap, or negative max_states");
  SubReq r{gap, max_states, energies, codons, pairs, count, 0};
  *count = 0;
  const cdz_status st = mfe_run(h, prob, mfe, nullptr, nullptr, &r);
  if (more) *more = r.more;
  return st;
}
