/*
 * mfe.c -- minimum free energy oracle (the (min, +) form of the codon-
 * constrained dynamic program) with an argmin traceback.
 *
 * TEST INFRASTRUCTURE ONLY, like oracle.c: loaded by tests/ and nothing on
 * the product path; it shares no code, table or header with the HIP library.
 *
 * What it computes (Section 4d, minimization; SI S2c, the evaluation
 * algebra in which sums become minima and products become sums of energies):
 *     MFE(psi) = min over codon assignments c and structures s of
 *                E(phi(c), s) - log W(c)          (kT)
 * with the loop model, codon slots and weights of oracle.c: W(c) =
 * exp(sum_a theta1[a][c_a] + sum_{a>=1} theta2[a][c_{a-1}][c_a]).  Every
 * DP entry of oracle.c becomes the minimum, over the same decompositions, of
 * the sum of the energies of its parts: a vertex carries -theta1 (middle base
 * of a codon) or 0, an edge inside a codon 0 (same slot) or +inf, an edge
 * across a codon boundary -theta2, and each loop its energy.  +inf marks an
 * impossible entry.
 *
 * The traceback returns one state (codon slots, pair table) of minimal
 * energy.  Each decision lists its alternatives in a fixed order, evaluates
 * each with the same additions as the forward pass, and takes the first whose
 * value is smallest:
 *   exterior at (j, t): [j unpaired, by slot of j-1], [0 pairs j, by slot of
 *       0], [k pairs j, k = 1..j-4, by (slot of k-1, slot of k)]
 *   pair (i, j): [hairpin], [stack], [windows, l1 ascending then l2
 *       ascending], [multiloop]; then the parts' slots, smallest first
 *   Qm1: [pair], [tail by slot]; Qm1p: [Qm1], [prefix by slot];
 *   Qm: [splits u ascending by slots], [Qm1p]; runs one position at a time
 *       from the right end.
 *
 * The PLANT_MFE_* switches exist only for tests/test_oracle_mfe.py, which
 * builds each into a throwaway library and checks that the pins notice it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MS 6
#define MAXL 30

static const char CODE[] =
    "KNKNTTTTRSRSIIMIQHQHPPPPRRRRLLLLEDEDAAAAGGGGVVVV*Y*YSSSS*CWCLFLF";

typedef struct {
  double stack[6][6], hairpin[31], bulge[31], interior[31], mismatch[4][4][6];
  double ml_a, ml_b, ml_c, extrap;
} MfeEnergy;

typedef struct {
  int n, m;
  int *d;                /* [n] slots of the residue of position p */
  int (*nt)[MS];         /* [n][MS] base of position p under slot s */
  double (*v)[MS];       /* [n][MS] vertex energy */
  double (*e)[MS][MS];   /* [n][MS][MS] edge energy between p and p+1 */
  const MfeEnergy *E;
  /* triangular cells [i][j], 36 energies each */
  double *U, *Qb, *DI, *Qm1, *Qm1p, *QmX, *Qm;
  double *Z5;            /* [n][MS] exterior prefix */
} Mfe;

static int bpair(int x, int y) { /* AU=0 CG=1 GC=2 UA=3 GU=4 UG=5, -1 if none */
  static const int T[4][4] = {{-1, -1, -1, 0}, {-1, -1, 1, -1}, {-1, 2, -1, 4}, {3, -1, 5, -1}};
  return T[x][y];
}

static size_t cidx(int n, int i, int j) { return ((size_t)i * (size_t)(2 * n - i + 1)) / 2 + (size_t)(j - i); }
#define C(A, i, j) ((A) + cidx(F->n, (i), (j)) * 36)

static double e_hairpin(const Mfe *F, int L) {
  if (L < 3) return INFINITY;
  if (L <= 30) return F->E->hairpin[L];
  return F->E->hairpin[30] + F->E->extrap * log((double)L / 30.0);
}

static int mfe_build(Mfe *F, int m, const char *aa, const double *t1, const double *t2, const MfeEnergy *E) {
  memset(F, 0, sizeof(*F));
  F->m = m;
  F->n = 3 * m;
  F->E = E;
  const int n = F->n;
  F->d = calloc(n, sizeof(int));
  F->nt = calloc(n, sizeof(*F->nt));
  F->v = calloc(n, sizeof(*F->v));
  F->e = calloc(n, sizeof(*F->e));
  if (!F->d || !F->nt || !F->v || !F->e) return -1;
  for (int a = 0; a < m; a++) {
    int cnt = 0, cod[MS];
    for (int c = 0; c < 64; c++)
      if (CODE[c] == aa[a] && aa[a] != '*') cod[cnt++] = c; /* lexicographic slot order */
    if (cnt == 0) return -2;
    for (int r = 0; r < 3; r++) {
      const int p = 3 * a + r;
      F->d[p] = cnt;
      for (int s = 0; s < cnt; s++) {
        const int c = cod[s];
        F->nt[p][s] = r == 0 ? c >> 4 : r == 1 ? (c >> 2) & 3 : c & 3;
        F->v[p][s] = (r == 1 && t1) ? -t1[a * MS + s] : 0.0;
      }
    }
  }
  for (int p = 0; p + 1 < n; p++)
    for (int s = 0; s < MS; s++)
      for (int t = 0; t < MS; t++) {
        if (s >= F->d[p] || t >= F->d[p + 1]) F->e[p][s][t] = INFINITY;
        else if (p % 3 != 2) F->e[p][s][t] = s == t ? 0.0 : INFINITY;
#ifdef PLANT_MFE_PAIR_SIGN
        else F->e[p][s][t] = t2 ? t2[((p / 3 + 1) * MS + s) * MS + t] : 0.0;
#else
        else F->e[p][s][t] = t2 ? -t2[((p / 3 + 1) * MS + s) * MS + t] : 0.0;
#endif
      }
  const size_t cells = (size_t)n * (n + 1) / 2 * 36;
  double **arr[] = {&F->U, &F->Qb, &F->DI, &F->Qm1, &F->Qm1p, &F->QmX, &F->Qm};
  for (int k = 0; k < 7; k++) {
    *arr[k] = malloc(cells * sizeof(double));
    if (!*arr[k]) return -1;
    for (size_t q = 0; q < cells; q++) (*arr[k])[q] = INFINITY;
  }
  F->Z5 = malloc((size_t)n * MS * sizeof(double));
  if (!F->Z5) return -1;
  return 0;
}

static void mfe_free(Mfe *F) {
  free(F->d);
  free(F->nt);
  free(F->v);
  free(F->e);
  free(F->U);
  free(F->Qb);
  free(F->DI);
  free(F->Qm1);
  free(F->Qm1p);
  free(F->QmX);
  free(F->Qm);
  free(F->Z5);
}

/* unpaired runs: U[i][j](a, b), slots a of i and b of j */
static void runs(Mfe *F) {
  const int n = F->n;
  for (int p = 0; p < n; p++)
    for (int a = 0; a < F->d[p]; a++) C(F->U, p, p)[a * 6 + a] = F->v[p][a];
  for (int dl = 1; dl < n; dl++)
    for (int i = 0; i + dl < n; i++) {
      const int j = i + dl;
      const double *ul = C(F->U, i, j - 1);
      double *u = C(F->U, i, j);
      for (int a = 0; a < F->d[i]; a++)
        for (int b = 0; b < F->d[j]; b++) {
          double best = INFINITY;
          for (int c = 0; c < F->d[j - 1]; c++) best = fmin(best, ul[a * 6 + c] + F->e[j - 1][c][b]);
          u[a * 6 + b] = best + F->v[j][b];
        }
    }
}

/* the value of each part of a pair decision, shared by the forward pass and
 * the traceback so that both add in the same order */
static double hairpin_term(const Mfe *F, int i, int j, int s, int s2, int t, int a, int b) {
  return F->e[i][s][a] + C(F->U, i + 1, j - 1)[a * 6 + b] + F->e[j - 1][b][s2] +
         F->E->mismatch[F->nt[i + 1][a]][F->nt[j - 1][b]][t];
}
static double stack_term(const Mfe *F, int i, int j, int s, int s2, int t, int x, int y) {
  const double q = C(F->Qb, i + 1, j - 1)[x * 6 + y];
  if (q == INFINITY) return INFINITY;
  const int t2 = bpair(F->nt[i + 1][x], F->nt[j - 1][y]);
#ifdef PLANT_MFE_STACK_SWAP
  return F->e[i][s][x] + q + F->e[j - 1][y][s2] + F->E->stack[t2][t];
#else
  return F->e[i][s][x] + q + F->e[j - 1][y][s2] + F->E->stack[t][t2];
#endif
}
/* left bulge l1 (k = i+1+l1, inner pair (k, j-1)): run i+1..k-1 with end slots
 * (a, b), edge (b, x), inner pair slots (x, y) */
static double lbulge_term(const Mfe *F, int i, int k, int j, int a, int b, int x, int y) {
  return C(F->U, i + 1, k - 1)[a * 6 + b] + F->e[k - 1][b][x] + C(F->Qb, k, j - 1)[x * 6 + y];
}
/* right bulge l2 (l = j-1-l2, inner pair (i+1, l)): pair slots (x, y), edge
 * (y, c), run l+1..j-1 with end slots (c, dd) */
static double rbulge_term(const Mfe *F, int i, int l, int j, int x, int y, int c, int dd) {
  return C(F->Qb, i + 1, l)[x * 6 + y] + F->e[l][y][c] + C(F->U, l + 1, j - 1)[c * 6 + dd];
}
/* interior loop: run i+1..k-1 (a, b), DI[k][l] (b, c), run l+1..j-1 (c, dd) */
static double inner_T(const Mfe *F, int i, int k, int l, int a, int c) {
  double best = INFINITY;
  for (int b = 0; b < F->d[k - 1]; b++)
    best = fmin(best, C(F->U, i + 1, k - 1)[a * 6 + b] + C(F->DI, k, l)[b * 6 + c]);
  return best;
}

/* per window (l1, l2): the minimum over the parts' inner slots for every
 * pair of outer slots (a of i+1, dd of j-1), before the outer edges and, for
 * an interior loop, the outer mismatch */
static int window_ok(int i, int j, int l1, int l2) {
  const int k = i + 1 + l1, l = j - 1 - l2;
  return !(l1 == 0 && l2 == 0) && l - k >= 4;
}
static void window_block(const Mfe *F, int i, int j, int l1, int l2, double W[6][6]) {
  const int k = i + 1 + l1, l = j - 1 - l2;
  for (int a = 0; a < 6; a++)
    for (int dd = 0; dd < 6; dd++) W[a][dd] = INFINITY;
  if (l2 == 0) { /* left bulge */
    for (int a = 0; a < F->d[i + 1]; a++)
      for (int dd = 0; dd < F->d[j - 1]; dd++) {
        double best = INFINITY;
        for (int b = 0; b < F->d[k - 1]; b++)
          for (int x = 0; x < F->d[k]; x++) best = fmin(best, lbulge_term(F, i, k, j, a, b, x, dd));
        W[a][dd] = F->E->bulge[l1] + best;
      }
  } else if (l1 == 0) { /* right bulge */
    for (int a = 0; a < F->d[i + 1]; a++)
      for (int dd = 0; dd < F->d[j - 1]; dd++) {
        double best = INFINITY;
        for (int y = 0; y < F->d[l]; y++)
          for (int c = 0; c < F->d[l + 1]; c++) best = fmin(best, rbulge_term(F, i, l, j, a, y, c, dd));
        W[a][dd] = F->E->bulge[l2] + best;
      }
  } else { /* interior loop */
    double T[6][6];
    for (int a = 0; a < F->d[i + 1]; a++)
      for (int c = 0; c < F->d[l + 1]; c++) T[a][c] = inner_T(F, i, k, l, a, c);
    for (int a = 0; a < F->d[i + 1]; a++)
      for (int dd = 0; dd < F->d[j - 1]; dd++) {
        double best = INFINITY;
        for (int c = 0; c < F->d[l + 1]; c++) best = fmin(best, T[a][c] + C(F->U, l + 1, j - 1)[c * 6 + dd]);
        W[a][dd] = F->E->interior[l1 + l2] + best;
      }
  }
}
/* outer part of a window term at outer slots (s, s2) of type t */
static double outer_term(const Mfe *F, int i, int j, int s, int s2, int a, int dd, double w) {
  return F->e[i][s][a] + F->e[j - 1][dd][s2] + w;
}
static double outer_mm(const Mfe *F, int i, int j, int t, int a, int dd) {
  return F->E->mismatch[F->nt[i + 1][a]][F->nt[j - 1][dd]][t];
}
static double ml_term(const Mfe *F, int i, int j, int s, int s2, int x, int y) {
  return F->e[i][s][x] + C(F->QmX, i + 1, j - 1)[x * 6 + y] + F->e[j - 1][y][s2];
}
static double split_term(const Mfe *F, int i, int j, int u, int s, int s2, int t, int t2) {
  return C(F->Qm, i, u - 1)[s * 6 + t] + F->e[u - 1][t][t2] + C(F->Qm1, u, j)[t2 * 6 + s2];
}
static double di_term(const Mfe *F, int i, int j, int b, int c, int x, int y) {
  const double q = C(F->Qb, i, j)[x * 6 + y];
  if (q == INFINITY) return INFINITY;
  const int t2 = bpair(F->nt[j][y], F->nt[i][x]);
  return F->e[i - 1][b][x] + q + F->e[j][y][c] + F->E->mismatch[F->nt[j + 1][c]][F->nt[i - 1][b]][t2];
}

static void cell(Mfe *F, int i, int j) {
  const int n = F->n, L = j - i - 1;
  const double bh = e_hairpin(F, L);
  double *qb = C(F->Qb, i, j);
  /* the windows' minima: left bulges GL, right bulges GR, interior loops FI */
  double GL[6][6], GR[6][6], FI[6][6], W[6][6];
  for (int a = 0; a < 6; a++)
    for (int dd = 0; dd < 6; dd++) GL[a][dd] = GR[a][dd] = FI[a][dd] = INFINITY;
  for (int l1 = 0; l1 <= MAXL; l1++)
    for (int l2 = 0; l1 + l2 <= MAXL; l2++) {
      if (!window_ok(i, j, l1, l2)) continue;
      window_block(F, i, j, l1, l2, W);
      double(*G)[6] = l2 == 0 ? GL : l1 == 0 ? GR : FI;
      for (int a = 0; a < 6; a++)
        for (int dd = 0; dd < 6; dd++) G[a][dd] = fmin(G[a][dd], W[a][dd]);
    }
  for (int s = 0; s < F->d[i]; s++)
    for (int s2 = 0; s2 < F->d[j]; s2++) {
      const int t = bpair(F->nt[i][s], F->nt[j][s2]);
      if (t < 0) continue;
      double acc = INFINITY, h = INFINITY;
      for (int a = 0; a < F->d[i + 1]; a++)
        for (int b = 0; b < F->d[j - 1]; b++) h = fmin(h, hairpin_term(F, i, j, s, s2, t, a, b));
      acc = fmin(acc, bh + h);
      if ((j - 1) - (i + 1) >= 4)
        for (int x = 0; x < F->d[i + 1]; x++)
          for (int y = 0; y < F->d[j - 1]; y++) acc = fmin(acc, stack_term(F, i, j, s, s2, t, x, y));
      for (int a = 0; a < F->d[i + 1]; a++)
        for (int dd = 0; dd < F->d[j - 1]; dd++)
          acc = fmin(acc, outer_term(F, i, j, s, s2, a, dd,
                                     fmin(fmin(GL[a][dd], GR[a][dd]), FI[a][dd] + outer_mm(F, i, j, t, a, dd))));
      double mlv = INFINITY;
      for (int x = 0; x < F->d[i + 1]; x++)
        for (int y = 0; y < F->d[j - 1]; y++) mlv = fmin(mlv, ml_term(F, i, j, s, s2, x, y));
      acc = fmin(acc, F->E->ml_a + F->E->ml_b + mlv);
      qb[s * 6 + s2] = F->v[i][s] + F->v[j][s2] + acc;
    }
  if (i >= 1 && j + 1 < n) {
    double *di = C(F->DI, i, j);
    for (int b = 0; b < F->d[i - 1]; b++)
      for (int c = 0; c < F->d[j + 1]; c++) {
        double best = INFINITY;
        for (int x = 0; x < F->d[i]; x++)
          for (int y = 0; y < F->d[j]; y++) best = fmin(best, di_term(F, i, j, b, c, x, y));
        di[b * 6 + c] = best;
      }
  }
  double *q1 = C(F->Qm1, i, j), *q1p = C(F->Qm1p, i, j), *qx = C(F->QmX, i, j), *qm = C(F->Qm, i, j);
  const double *q1l = C(F->Qm1, i, j - 1), *q1pr = C(F->Qm1p, i + 1, j);
  for (int s = 0; s < F->d[i]; s++)
    for (int s2 = 0; s2 < F->d[j]; s2++) {
      double tail = INFINITY;
      for (int t = 0; t < F->d[j - 1]; t++) tail = fmin(tail, q1l[s * 6 + t] + F->e[j - 1][t][s2]);
      q1[s * 6 + s2] = fmin(qb[s * 6 + s2] + F->E->ml_b, tail + F->v[j][s2] + F->E->ml_c);
    }
  for (int s = 0; s < F->d[i]; s++)
    for (int s2 = 0; s2 < F->d[j]; s2++) {
      double pre = INFINITY;
      for (int t = 0; t < F->d[i + 1]; t++) pre = fmin(pre, F->e[i][s][t] + q1pr[t * 6 + s2]);
      q1p[s * 6 + s2] = fmin(q1[s * 6 + s2], F->v[i][s] + F->E->ml_c + pre);
      double x = INFINITY;
#ifdef PLANT_MFE_SPLIT_RANGE
      for (int u = i + 6; u <= j - 4; u++)
#else
      for (int u = i + 5; u <= j - 4; u++)
#endif
        for (int t = 0; t < F->d[u - 1]; t++)
          for (int t2 = 0; t2 < F->d[u]; t2++) x = fmin(x, split_term(F, i, j, u, s, s2, t, t2));
      qx[s * 6 + s2] = x;
      qm[s * 6 + s2] = fmin(x, q1p[s * 6 + s2]);
    }
}

static double ext_pair_term(const Mfe *F, int k, int j, int s, int x, int t) {
  return F->Z5[(k - 1) * MS + s] + F->e[k - 1][s][x] + C(F->Qb, k, j)[x * 6 + t];
}

static double forward(Mfe *F) {
  const int n = F->n;
  runs(F);
  for (int dl = 4; dl < n; dl++) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < n - dl; i++) cell(F, i, i + dl);
  }
  for (int s = 0; s < MS; s++) F->Z5[s] = s < F->d[0] ? F->v[0][s] : INFINITY;
  for (int j = 1; j < n; j++)
    for (int t = 0; t < MS; t++) {
      double best = INFINITY;
      if (t < F->d[j]) {
        double un = INFINITY;
        for (int s = 0; s < F->d[j - 1]; s++) un = fmin(un, F->Z5[(j - 1) * MS + s] + F->e[j - 1][s][t]);
        best = un + F->v[j][t];
        if (j >= 4)
          for (int x = 0; x < F->d[0]; x++) best = fmin(best, C(F->Qb, 0, j)[x * 6 + t]);
        for (int k = 1; k <= j - 4; k++)
          for (int s = 0; s < F->d[k - 1]; s++)
            for (int x = 0; x < F->d[k]; x++) best = fmin(best, ext_pair_term(F, k, j, s, x, t));
      }
      F->Z5[j * MS + t] = best;
    }
  double mfe = INFINITY;
  for (int t = 0; t < F->d[n - 1]; t++) mfe = fmin(mfe, F->Z5[(n - 1) * MS + t]);
  return mfe;
}

/* ---- argmin traceback -------------------------------------------------- */

typedef struct {
  int kind, i, j, s, s2;
} Frag;
enum { K_EXT, K_PAIR, K_RUN, K_QM1, K_QM1P, K_QM };

typedef struct {
  const Mfe *F;
  Frag *stk;
  int top;
  int *slot;  /* [n] */
  int *pt;    /* [n] */
} Tb;

static void tpush(Tb *T, int kind, int i, int j, int s, int s2) {
  T->stk[T->top++] = (Frag){kind, i, j, s, s2};
}
static void setslot(Tb *T, int p, int s) { T->slot[p] = s; }

/* first alternative of smallest value: track (value, index) */
typedef struct {
  double v;
  int idx;
} Best;
static void consider(Best *b, double v, int idx) {
  if (v < b->v) {
    b->v = v;
    b->idx = idx;
  }
}

static void tb_ext(Tb *T, int j, int t) {
  const Mfe *F = T->F;
  setslot(T, j, t);
  if (j == 0) return;
  Best b = {INFINITY, -1};
  for (int s = 0; s < F->d[j - 1]; s++) consider(&b, (F->Z5[(j - 1) * MS + s] + F->e[j - 1][s][t]) + F->v[j][t], s);
  if (j >= 4)
    for (int x = 0; x < F->d[0]; x++) consider(&b, C(F->Qb, 0, j)[x * 6 + t], 100 + x);
  for (int k = 1; k <= j - 4; k++)
    for (int s = 0; s < F->d[k - 1]; s++)
      for (int x = 0; x < F->d[k]; x++) consider(&b, ext_pair_term(F, k, j, s, x, t), 1000 + (k * 6 + s) * 6 + x);
  if (b.idx < 100) {
    tpush(T, K_EXT, j - 1, 0, b.idx, 0);
  } else if (b.idx < 1000) {
    tpush(T, K_PAIR, 0, j, b.idx - 100, t);
  } else {
    const int r = b.idx - 1000, x = r % 6, s = (r / 6) % 6, k = r / 36;
    tpush(T, K_EXT, k - 1, 0, s, 0);
    tpush(T, K_PAIR, k, j, x, t);
  }
}

static void tb_run(Tb *T, int p, int q, int a, int b) {
  const Mfe *F = T->F;
  setslot(T, q, b);
  if (p == q) return;
  const double *ul = C(F->U, p, q - 1);
  Best bb = {INFINITY, -1};
  for (int c = 0; c < F->d[q - 1]; c++) consider(&bb, ul[a * 6 + c] + F->e[q - 1][c][b], c);
  tpush(T, K_RUN, p, q - 1, a, bb.idx);
}

static void tb_pair(Tb *T, int i, int j, int s, int s2) {
  const Mfe *F = T->F;
  setslot(T, i, s);
  setslot(T, j, s2);
  T->pt[i] = j;
  T->pt[j] = i;
  const int t = bpair(F->nt[i][s], F->nt[j][s2]);
  /* loop type first: hairpin 0, stack 1, window 2 + (l1 * 31 + l2), multiloop 2000 */
  Best b = {INFINITY, -1};
  {
    double h = INFINITY;
    for (int a = 0; a < F->d[i + 1]; a++)
      for (int bb = 0; bb < F->d[j - 1]; bb++) h = fmin(h, hairpin_term(F, i, j, s, s2, t, a, bb));
    consider(&b, e_hairpin(F, j - i - 1) + h, 0);
  }
  if ((j - 1) - (i + 1) >= 4) {
    double st = INFINITY;
    for (int x = 0; x < F->d[i + 1]; x++)
      for (int y = 0; y < F->d[j - 1]; y++) st = fmin(st, stack_term(F, i, j, s, s2, t, x, y));
    consider(&b, st, 1);
  }
  double W[6][6];
  for (int l1 = 0; l1 <= MAXL; l1++)
    for (int l2 = 0; l1 + l2 <= MAXL; l2++) {
      if (!window_ok(i, j, l1, l2)) continue;
      window_block(F, i, j, l1, l2, W);
      double w = INFINITY;
      for (int a = 0; a < F->d[i + 1]; a++)
        for (int dd = 0; dd < F->d[j - 1]; dd++)
          w = fmin(w, outer_term(F, i, j, s, s2, a, dd,
                                 l1 > 0 && l2 > 0 ? W[a][dd] + outer_mm(F, i, j, t, a, dd) : W[a][dd]));
      consider(&b, w, 2 + l1 * 31 + l2);
    }
  {
    double mlv = INFINITY;
    for (int x = 0; x < F->d[i + 1]; x++)
      for (int y = 0; y < F->d[j - 1]; y++) mlv = fmin(mlv, ml_term(F, i, j, s, s2, x, y));
    consider(&b, F->E->ml_a + F->E->ml_b + mlv, 2000);
  }
  if (b.idx == 0) {
    Best c = {INFINITY, -1};
    for (int a = 0; a < F->d[i + 1]; a++)
      for (int bb = 0; bb < F->d[j - 1]; bb++) consider(&c, hairpin_term(F, i, j, s, s2, t, a, bb), a * 6 + bb);
    tpush(T, K_RUN, i + 1, j - 1, c.idx / 6, c.idx % 6);
  } else if (b.idx == 1) {
    Best c = {INFINITY, -1};
    for (int x = 0; x < F->d[i + 1]; x++)
      for (int y = 0; y < F->d[j - 1]; y++) consider(&c, stack_term(F, i, j, s, s2, t, x, y), x * 6 + y);
    tpush(T, K_PAIR, i + 1, j - 1, c.idx / 6, c.idx % 6);
  } else if (b.idx == 2000) {
    Best c = {INFINITY, -1};
    for (int x = 0; x < F->d[i + 1]; x++)
      for (int y = 0; y < F->d[j - 1]; y++) consider(&c, ml_term(F, i, j, s, s2, x, y), x * 6 + y);
    tpush(T, K_QM, i + 1, j - 1, c.idx / 6, c.idx % 6);  /* QmX: >= 2 branches (a split of Qm) */
    T->stk[T->top - 1].kind = K_QM + 10;
  } else {
    const int w = b.idx - 2, l1 = w / 31, l2 = w % 31, k = i + 1 + l1, l = j - 1 - l2;
    window_block(F, i, j, l1, l2, W);
    Best c = {INFINITY, -1};
    for (int a = 0; a < F->d[i + 1]; a++)
      for (int dd = 0; dd < F->d[j - 1]; dd++)
        consider(&c,
                 outer_term(F, i, j, s, s2, a, dd,
                            l1 > 0 && l2 > 0 ? W[a][dd] + outer_mm(F, i, j, t, a, dd) : W[a][dd]),
                 a * 6 + dd);
    const int a = c.idx / 6, dd = c.idx % 6;
    Best g = {INFINITY, -1};
    if (l2 == 0) { /* left bulge: (b, x) */
      for (int bb = 0; bb < F->d[k - 1]; bb++)
        for (int x = 0; x < F->d[k]; x++) consider(&g, lbulge_term(F, i, k, j, a, bb, x, dd), bb * 6 + x);
      tpush(T, K_RUN, i + 1, k - 1, a, g.idx / 6);
      tpush(T, K_PAIR, k, j - 1, g.idx % 6, dd);
    } else if (l1 == 0) { /* right bulge: (y, c) */
      for (int y = 0; y < F->d[l]; y++)
        for (int cc = 0; cc < F->d[l + 1]; cc++) consider(&g, rbulge_term(F, i, l, j, a, y, cc, dd), y * 6 + cc);
      tpush(T, K_PAIR, i + 1, l, a, g.idx / 6);
      tpush(T, K_RUN, l + 1, j - 1, g.idx % 6, dd);
    } else { /* interior: c, then b, then the inner pair slots (x, y) */
      for (int cc = 0; cc < F->d[l + 1]; cc++)
        consider(&g, inner_T(F, i, k, l, a, cc) + C(F->U, l + 1, j - 1)[cc * 6 + dd], cc);
      const int cc = g.idx;
      Best h = {INFINITY, -1};
      for (int bb = 0; bb < F->d[k - 1]; bb++)
        consider(&h, C(F->U, i + 1, k - 1)[a * 6 + bb] + C(F->DI, k, l)[bb * 6 + cc], bb);
      const int bb = h.idx;
      Best q = {INFINITY, -1};
      for (int x = 0; x < F->d[k]; x++)
        for (int y = 0; y < F->d[l]; y++) consider(&q, di_term(F, k, l, bb, cc, x, y), x * 6 + y);
      tpush(T, K_RUN, i + 1, k - 1, a, bb);
      tpush(T, K_PAIR, k, l, q.idx / 6, q.idx % 6);
      tpush(T, K_RUN, l + 1, j - 1, cc, dd);
    }
  }
}

/* Qm (kind K_QM) or QmX (K_QM + 10, splits only) of (i, j) at slots (s, s2) */
static void tb_qm(Tb *T, int i, int j, int s, int s2, int splits_only) {
  const Mfe *F = T->F;
  Best b = {INFINITY, -1};
  for (int u = i + 5; u <= j - 4; u++)
    for (int t = 0; t < F->d[u - 1]; t++)
      for (int t2 = 0; t2 < F->d[u]; t2++) consider(&b, split_term(F, i, j, u, s, s2, t, t2), (u * 6 + t) * 6 + t2);
  if (!splits_only) consider(&b, C(F->Qm1p, i, j)[s * 6 + s2], -2);
  if (b.idx == -2) {
    tpush(T, K_QM1P, i, j, s, s2);
  } else {
    const int t2 = b.idx % 6, t = (b.idx / 6) % 6, u = b.idx / 36;
    tpush(T, K_QM, i, u - 1, s, t);
    tpush(T, K_QM1, u, j, t2, s2);
  }
}

static void tb_qm1(Tb *T, int i, int j, int s, int s2) {
  const Mfe *F = T->F;
  Best b = {INFINITY, -1};
  consider(&b, C(F->Qb, i, j)[s * 6 + s2] + F->E->ml_b, -2);
  for (int t = 0; t < F->d[j - 1]; t++)
    consider(&b, (C(F->Qm1, i, j - 1)[s * 6 + t] + F->e[j - 1][t][s2]) + F->v[j][s2] + F->E->ml_c, t);
  if (b.idx == -2) {
    tpush(T, K_PAIR, i, j, s, s2);
  } else {
    setslot(T, j, s2);
    tpush(T, K_QM1, i, j - 1, s, b.idx);
  }
}

static void tb_qm1p(Tb *T, int i, int j, int s, int s2) {
  const Mfe *F = T->F;
  Best b = {INFINITY, -1};
  consider(&b, C(F->Qm1, i, j)[s * 6 + s2], -2);
  for (int t = 0; t < F->d[i + 1]; t++)
    consider(&b, F->v[i][s] + F->E->ml_c + (F->e[i][s][t] + C(F->Qm1p, i + 1, j)[t * 6 + s2]), t);
  if (b.idx == -2) {
    tpush(T, K_QM1, i, j, s, s2);
  } else {
    setslot(T, i, s);
    tpush(T, K_QM1P, i + 1, j, b.idx, s2);
  }
}

static int traceback(const Mfe *F, uint8_t *codons, int32_t *pairs) {
  const int n = F->n;
  Tb T;
  T.F = F;
  T.top = 0;
  T.stk = malloc((size_t)(4 * n + 16) * sizeof(Frag));
  T.slot = malloc((size_t)n * sizeof(int));
  T.pt = malloc((size_t)n * sizeof(int));
  if (!T.stk || !T.slot || !T.pt) return -1;
  for (int p = 0; p < n; p++) {
    T.slot[p] = -1;
    T.pt[p] = -1;
  }
  Best b = {INFINITY, -1};
  for (int t = 0; t < F->d[n - 1]; t++) consider(&b, F->Z5[(n - 1) * MS + t], t);
  tpush(&T, K_EXT, n - 1, 0, b.idx, 0);
  while (T.top > 0) {
    const Frag f = T.stk[--T.top];
    switch (f.kind) {
      case K_EXT: tb_ext(&T, f.i, f.s); break;
      case K_PAIR: tb_pair(&T, f.i, f.j, f.s, f.s2); break;
      case K_RUN: tb_run(&T, f.i, f.j, f.s, f.s2); break;
      case K_QM1: tb_qm1(&T, f.i, f.j, f.s, f.s2); break;
      case K_QM1P: tb_qm1p(&T, f.i, f.j, f.s, f.s2); break;
      case K_QM: tb_qm(&T, f.i, f.j, f.s, f.s2, 0); break;
      case K_QM + 10: tb_qm(&T, f.i, f.j, f.s, f.s2, 1); break;
    }
  }
  int rc = 0;
  for (int a = 0; a < F->m; a++) {
    const int s = T.slot[3 * a];
    if (s < 0 || T.slot[3 * a + 1] != s || T.slot[3 * a + 2] != s) rc = -3;
    if (codons) codons[a] = (uint8_t)s;
  }
  if (pairs)
    for (int p = 0; p < n; p++) pairs[p] = T.pt[p];
  free(T.stk);
  free(T.slot);
  free(T.pt);
  return rc;
}

/* MFE (kT) and, if codons/pairs are given, one minimising state: codons[m]
 * slot per residue, pairs[n] partner per position (-1 unpaired).  Returns 0,
 * or < 0 for bad input / allocation failure / an inconsistent traceback. */
int orc_mfe(int m, const char *aa, const double *theta1, const double *theta2, const double *energy, double *mfe,
            uint8_t *codons, int32_t *pairs) {
  if (m < 1 || !aa || !energy || !mfe) return -1;
  Mfe F;
  int rc = mfe_build(&F, m, aa, theta1, theta2, (const MfeEnergy *)energy);
  if (rc == 0) {
    *mfe = forward(&F);
    if (codons || pairs) rc = traceback(&F, codons, pairs);
  }
  mfe_free(&F);
  return rc;
}

/* ---- suboptimal enumeration (SI S4d) ------------------------------------
 * Every state (codon assignment, structure) whose energy is at most
 * MFE + gap, by depth-first search over the same decisions as the argmin
 * traceback.  A partial state is a stack of pending fragments and a bound:
 * the energy decided so far plus the minimum (the DP value) of every pending
 * fragment.  Expanding a fragment f by an alternative a of value V(a) (its
 * own energy plus the DP values of the fragments it leaves) gives the bound
 * (bound - value(f)) + V(a); alternatives whose bound exceeds the threshold
 * MFE + gap + 1e-9 max(1, |MFE|) are dropped, the others are tried in the
 * traceback's order.  Inside a pair decision the alternatives are refined
 * level by level (loop type, window, outer slots, inner slots) and a level is
 * skipped when its minimum already exceeds the threshold.  A complete state's
 * energy is its final bound.  States come out in depth-first order. */

typedef struct {
  double V;
  int nsub;
  Frag sub[3];
  int nas;
  int as[3][3]; /* assignments: position, slot, partner (-1 unpaired) */
} Alt;

/* One level per expanded fragment.  Levels below share the pending stack and
 * may take fragments off it below flen0; each puts its own back when it is
 * left, so the stack a level sees is restored before its next alternative. */
typedef struct {
  Frag f;
  int flen0;    /* pending stack length after f was taken off */
  double b0;    /* bound before f was expanded */
  size_t a0, na, next;
} Level;

typedef struct {
  const Mfe *F;
  double thr;
  Alt *alts;
  size_t nalts, capalts;
  Level *lv;
  int nlv, caplv;
  Frag *pend;
  int npend, cappend;
  int *slot, *pt;
} Sub;

static double frag_value(const Mfe *F, const Frag *f) {
  const int n = F->n;
  switch (f->kind) {
    case K_EXT: return F->Z5[f->i * MS + f->s];
    case K_PAIR: return C(F->Qb, f->i, f->j)[f->s * 6 + f->s2];
    case K_RUN: return C(F->U, f->i, f->j)[f->s * 6 + f->s2];
    case K_QM1: return C(F->Qm1, f->i, f->j)[f->s * 6 + f->s2];
    case K_QM1P: return C(F->Qm1p, f->i, f->j)[f->s * 6 + f->s2];
    case K_QM: return C(F->Qm, f->i, f->j)[f->s * 6 + f->s2];
    default: return C(F->QmX, f->i, f->j)[f->s * 6 + f->s2]; /* K_QM + 10 */
  }
}

static int alt_push(Sub *S, double V, double base) {
  if (!(base + V <= S->thr)) return 0;
  if (S->nalts == S->capalts) {
    S->capalts = S->capalts ? 2 * S->capalts : 1024;
    S->alts = realloc(S->alts, S->capalts * sizeof(Alt));
    if (!S->alts) return -1;
  }
  Alt *a = &S->alts[S->nalts++];
  a->V = V;
  a->nsub = 0;
  a->nas = 0;
  return 1;
}
static Alt *alt_last(Sub *S) { return &S->alts[S->nalts - 1]; }
static void alt_sub(Alt *a, int kind, int i, int j, int s, int s2) { a->sub[a->nsub++] = (Frag){kind, i, j, s, s2}; }
static void alt_as(Alt *a, int p, int s, int partner) {
  a->as[a->nas][0] = p;
  a->as[a->nas][1] = s;
  a->as[a->nas][2] = partner;
  a->nas++;
}

/* alternatives of fragment f, given base = bound - value(f) */
static int sub_alternatives(Sub *S, const Frag *f, double base) {
  const Mfe *F = S->F;
  const int i = f->i, j = f->j, s = f->s, s2 = f->s2;
  int r;
  if (f->kind == K_EXT) {
    const int jj = i, t = s;
    if (jj == 0) {
      if ((r = alt_push(S, F->Z5[t], base)) < 0) return r;
      if (r) alt_as(alt_last(S), 0, t, -1);
      return 0;
    }
    for (int sp = 0; sp < F->d[jj - 1]; sp++) {
      if ((r = alt_push(S, (F->Z5[(jj - 1) * MS + sp] + F->e[jj - 1][sp][t]) + F->v[jj][t], base)) < 0) return r;
      if (r) {
        alt_as(alt_last(S), jj, t, -1);
        alt_sub(alt_last(S), K_EXT, jj - 1, 0, sp, 0);
      }
    }
    if (jj >= 4)
      for (int x = 0; x < F->d[0]; x++) {
        if ((r = alt_push(S, C(F->Qb, 0, jj)[x * 6 + t], base)) < 0) return r;
        if (r) alt_sub(alt_last(S), K_PAIR, 0, jj, x, t);
      }
    for (int k = 1; k <= jj - 4; k++)
      for (int sp = 0; sp < F->d[k - 1]; sp++)
        for (int x = 0; x < F->d[k]; x++) {
          if ((r = alt_push(S, ext_pair_term(F, k, jj, sp, x, t), base)) < 0) return r;
          if (r) {
            alt_sub(alt_last(S), K_EXT, k - 1, 0, sp, 0);
            alt_sub(alt_last(S), K_PAIR, k, jj, x, t);
          }
        }
    return 0;
  }
  if (f->kind == K_RUN) {
    if (i == j) {
      if ((r = alt_push(S, C(F->U, i, i)[s * 6 + s2], base)) < 0) return r;
      if (r) alt_as(alt_last(S), i, s2, -1);
      return 0;
    }
    for (int c = 0; c < F->d[j - 1]; c++) {
      if ((r = alt_push(S, (C(F->U, i, j - 1)[s * 6 + c] + F->e[j - 1][c][s2]) + F->v[j][s2], base)) < 0) return r;
      if (r) {
        alt_as(alt_last(S), j, s2, -1);
        alt_sub(alt_last(S), K_RUN, i, j - 1, s, c);
      }
    }
    return 0;
  }
  if (f->kind == K_QM1) {
    if ((r = alt_push(S, C(F->Qb, i, j)[s * 6 + s2] + F->E->ml_b, base)) < 0) return r;
    if (r) alt_sub(alt_last(S), K_PAIR, i, j, s, s2);
    for (int t = 0; t < F->d[j - 1]; t++) {
      if ((r = alt_push(S, (C(F->Qm1, i, j - 1)[s * 6 + t] + F->e[j - 1][t][s2]) + F->v[j][s2] + F->E->ml_c,
                        base)) < 0)
        return r;
      if (r) {
        alt_as(alt_last(S), j, s2, -1);
        alt_sub(alt_last(S), K_QM1, i, j - 1, s, t);
      }
    }
    return 0;
  }
  if (f->kind == K_QM1P) {
    if ((r = alt_push(S, C(F->Qm1, i, j)[s * 6 + s2], base)) < 0) return r;
    if (r) alt_sub(alt_last(S), K_QM1, i, j, s, s2);
    for (int t = 0; t < F->d[i + 1]; t++) {
      if ((r = alt_push(S, F->v[i][s] + F->E->ml_c + (F->e[i][s][t] + C(F->Qm1p, i + 1, j)[t * 6 + s2]), base)) < 0)
        return r;
      if (r) {
        alt_as(alt_last(S), i, s, -1);
        alt_sub(alt_last(S), K_QM1P, i + 1, j, t, s2);
      }
    }
    return 0;
  }
  if (f->kind == K_QM || f->kind == K_QM + 10) {
    for (int u = i + 5; u <= j - 4; u++)
      for (int t = 0; t < F->d[u - 1]; t++)
        for (int t2 = 0; t2 < F->d[u]; t2++) {
          if ((r = alt_push(S, split_term(F, i, j, u, s, s2, t, t2), base)) < 0) return r;
          if (r) {
            alt_sub(alt_last(S), K_QM, i, u - 1, s, t);
            alt_sub(alt_last(S), K_QM1, u, j, t2, s2);
          }
        }
    if (f->kind == K_QM) {
      if ((r = alt_push(S, C(F->Qm1p, i, j)[s * 6 + s2], base)) < 0) return r;
      if (r) alt_sub(alt_last(S), K_QM1P, i, j, s, s2);
    }
    return 0;
  }
  /* K_PAIR: value(f) = Qb = (v_i + v_j) + acc; each alternative's value is
   * (v_i + v_j) + its term of acc */
  const double vv = F->v[i][s] + F->v[j][s2];
  const int t = bpair(F->nt[i][s], F->nt[j][s2]);
#define PAIR_AS(a)               \
  do {                           \
    alt_as((a), i, s, j);        \
    alt_as((a), j, s2, i);       \
  } while (0)
  {
    const double bh = e_hairpin(F, j - i - 1);
    for (int a = 0; a < F->d[i + 1]; a++)
      for (int b = 0; b < F->d[j - 1]; b++) {
        if ((r = alt_push(S, vv + (bh + hairpin_term(F, i, j, s, s2, t, a, b)), base)) < 0) return r;
        if (r) {
          PAIR_AS(alt_last(S));
          alt_sub(alt_last(S), K_RUN, i + 1, j - 1, a, b);
        }
      }
  }
  if ((j - 1) - (i + 1) >= 4)
    for (int x = 0; x < F->d[i + 1]; x++)
      for (int y = 0; y < F->d[j - 1]; y++) {
        if ((r = alt_push(S, vv + stack_term(F, i, j, s, s2, t, x, y), base)) < 0) return r;
        if (r) {
          PAIR_AS(alt_last(S));
          alt_sub(alt_last(S), K_PAIR, i + 1, j - 1, x, y);
        }
      }
  double W[6][6];
  for (int l1 = 0; l1 <= MAXL; l1++)
    for (int l2 = 0; l1 + l2 <= MAXL; l2++) {
      if (!window_ok(i, j, l1, l2)) continue;
      const int k = i + 1 + l1, l = j - 1 - l2;
      window_block(F, i, j, l1, l2, W);
      for (int a = 0; a < F->d[i + 1]; a++)
        for (int dd = 0; dd < F->d[j - 1]; dd++) {
          const int inter = l1 > 0 && l2 > 0;
          const double mm = inter ? outer_mm(F, i, j, t, a, dd) : 0.0;
          const double wv = inter ? W[a][dd] + mm : W[a][dd];
          if (!(base + (vv + outer_term(F, i, j, s, s2, a, dd, wv)) <= S->thr)) continue;
          if (l2 == 0) {
            for (int b = 0; b < F->d[k - 1]; b++)
              for (int x = 0; x < F->d[k]; x++) {
                const double w = F->E->bulge[l1] + lbulge_term(F, i, k, j, a, b, x, dd);
                if ((r = alt_push(S, vv + outer_term(F, i, j, s, s2, a, dd, w), base)) < 0) return r;
                if (r) {
                  PAIR_AS(alt_last(S));
                  alt_sub(alt_last(S), K_RUN, i + 1, k - 1, a, b);
                  alt_sub(alt_last(S), K_PAIR, k, j - 1, x, dd);
                }
              }
          } else if (l1 == 0) {
            for (int y = 0; y < F->d[l]; y++)
              for (int c = 0; c < F->d[l + 1]; c++) {
                const double w = F->E->bulge[l2] + rbulge_term(F, i, l, j, a, y, c, dd);
                if ((r = alt_push(S, vv + outer_term(F, i, j, s, s2, a, dd, w), base)) < 0) return r;
                if (r) {
                  PAIR_AS(alt_last(S));
                  alt_sub(alt_last(S), K_PAIR, i + 1, l, a, y);
                  alt_sub(alt_last(S), K_RUN, l + 1, j - 1, c, dd);
                }
              }
          } else {
            for (int c = 0; c < F->d[l + 1]; c++)
              for (int b = 0; b < F->d[k - 1]; b++) {
                const double di = C(F->DI, k, l)[b * 6 + c];
                const double wbc = F->E->interior[l1 + l2] +
                                   ((C(F->U, i + 1, k - 1)[a * 6 + b] + di) + C(F->U, l + 1, j - 1)[c * 6 + dd]);
                if (!(base + (vv + outer_term(F, i, j, s, s2, a, dd, wbc + mm)) <= S->thr)) continue;
                for (int x = 0; x < F->d[k]; x++)
                  for (int y = 0; y < F->d[l]; y++) {
                    const double dt = di_term(F, k, l, b, c, x, y);
                    const double w = F->E->interior[l1 + l2] +
                                     ((C(F->U, i + 1, k - 1)[a * 6 + b] + dt) + C(F->U, l + 1, j - 1)[c * 6 + dd]);
                    if ((r = alt_push(S, vv + outer_term(F, i, j, s, s2, a, dd, w + mm), base)) < 0) return r;
                    if (r) {
                      PAIR_AS(alt_last(S));
                      alt_sub(alt_last(S), K_RUN, i + 1, k - 1, a, b);
                      alt_sub(alt_last(S), K_PAIR, k, l, x, y);
                      alt_sub(alt_last(S), K_RUN, l + 1, j - 1, c, dd);
                    }
                  }
              }
          }
        }
    }
  for (int x = 0; x < F->d[i + 1]; x++)
    for (int y = 0; y < F->d[j - 1]; y++) {
      if ((r = alt_push(S, vv + (F->E->ml_a + F->E->ml_b + ml_term(F, i, j, s, s2, x, y)), base)) < 0) return r;
      if (r) {
        PAIR_AS(alt_last(S));
        alt_sub(alt_last(S), K_QM + 10, i + 1, j - 1, x, y);
      }
    }
#undef PAIR_AS
  return 0;
}

/* All states within gap >= 0 of the MFE (at most max_states): energies[k],
 * codons[k][m], pairs[k][n] in depth-first order; *count states.  Returns 0,
 * 1 if more than max_states states exist (the first max_states are given),
 * < 0 on bad input (a negative or NaN gap among them: the single argmin is
 * orc_mfe's), allocation failure or an inconsistent state. */
int orc_subopt(int m, const char *aa, const double *theta1, const double *theta2, const double *energy, double gap,
               int max_states, double *mfe, double *energies, uint8_t *codons, int32_t *pairs, int *count) {
  if (m < 1 || !aa || !energy || !mfe || !count || max_states < 0 || !(gap >= 0)) return -1;
  Mfe F;
  int rc = mfe_build(&F, m, aa, theta1, theta2, (const MfeEnergy *)energy);
  *count = 0;
  if (rc != 0) {
    mfe_free(&F);
    return rc;
  }
  *mfe = forward(&F);
  const int n = F.n;
  Sub S;
  memset(&S, 0, sizeof(S));
  S.F = &F;
  S.thr = *mfe + gap + 1e-9 * fmax(1.0, fabs(*mfe));
  S.caplv = 4 * n + 16;
  S.cappend = 4 * n + 16;
  S.lv = malloc(S.caplv * sizeof(Level));
  S.pend = malloc(S.cappend * sizeof(Frag));
  S.slot = malloc(n * sizeof(int));
  S.pt = malloc(n * sizeof(int));
  if (!S.lv || !S.pend || !S.slot || !S.pt) rc = -1;
  /* root level: the slot of the last position */
  if (rc == 0) {
    S.lv[0].f = (Frag){-1, 0, 0, 0, 0};
    S.lv[0].flen0 = 0;
    S.lv[0].b0 = 0.0;
    S.lv[0].a0 = 0;
    for (int t = 0; t < F.d[n - 1]; t++) {
      const int r = alt_push(&S, F.Z5[(n - 1) * MS + t], 0.0);
      if (r < 0) {
        rc = -1;
        break;
      }
      if (r) alt_sub(alt_last(&S), K_EXT, n - 1, 0, t, 0);
    }
    S.lv[0].na = S.nalts;
    S.lv[0].next = 0;
    S.nlv = 1;
  }
  while (rc == 0 && S.nlv > 0) {
    Level *L = &S.lv[S.nlv - 1];
    if (L->next == L->na) { /* backtrack: put the expanded fragment back where it was taken from */
#ifndef PLANT_SUBOPT_NO_RESTORE
      if (L->f.kind >= 0) S.pend[L->flen0] = L->f;
#endif
      S.nalts = L->a0;
      S.nlv--;
      continue;
    }
    const Alt *a = &S.alts[L->a0 + L->next++];
    S.npend = L->flen0;
    for (int q = 0; q < a->nas; q++) {
      S.slot[a->as[q][0]] = a->as[q][1];
      S.pt[a->as[q][0]] = a->as[q][2];
    }
    for (int q = 0; q < a->nsub; q++) S.pend[S.npend++] = a->sub[q];
    const double bound = L->f.kind < 0 ? a->V : (L->b0 - frag_value(&F, &L->f)) + a->V;
    if (S.npend == 0) { /* complete */
      if (*count >= max_states) {
        rc = 1;
        break;
      }
      if (energies) energies[*count] = bound;
      int ok = 1;
      for (int aa2 = 0; aa2 < m; aa2++) {
        const int sl = S.slot[3 * aa2];
        if (sl < 0 || S.slot[3 * aa2 + 1] != sl || S.slot[3 * aa2 + 2] != sl) ok = 0;
        if (codons) codons[(size_t)*count * m + aa2] = (uint8_t)sl;
      }
      if (pairs)
        for (int p = 0; p < n; p++) pairs[(size_t)*count * n + p] = S.pt[p];
      if (!ok) {
        rc = -3;
        break;
      }
      (*count)++;
      continue;
    }
    if (S.nlv == S.caplv) {
      rc = -1;
      break;
    }
    const Frag f = S.pend[--S.npend];
    Level *N = &S.lv[S.nlv++];
    N->f = f;
    N->flen0 = S.npend;
    N->b0 = bound;
    N->a0 = S.nalts;
    if (sub_alternatives(&S, &f, bound - frag_value(&F, &f)) < 0) {
      rc = -1;
      break;
    }
    N->na = S.nalts - N->a0;
    N->next = 0;
  }
  free(S.alts);
  free(S.lv);
  free(S.pend);
  free(S.slot);
  free(S.pt);
  mfe_free(&F);
  return rc;
}
