/*
 * oracle.c -- plain FP64 CPU oracle for the codon-constrained McCaskill
 * partition function.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU
 * baseline leg of bench.py may load this library.  It shares no code, table
 * or header with the HIP library it checks.
 *
 * What it computes (paper, Section 2b equations structure-q/sequence-q/
 * amino-q and Section 2c): for an amino-acid sequence psi with m residues and
 * n = 3m bases, the sum over every codon assignment c (each codon from the
 * standard genetic code for its residue, start/stop removed as in SI S3c) and
 * every non-crossing secondary structure s of the spelled RNA phi(c) of
 *      W(c) * exp(-E(phi(c), s)),
 * where W(c) = exp(sum_a theta1[a][c_a] + sum_{a>=1} theta2[a][c_{a-1}][c_a])
 * is the soft-constraint bias of Section 3a (codon weight on the middle base
 * of a codon, codon-pair weight on the codon boundary) and E is a
 * nearest-neighbour loop energy in kT.  The outputs are log Z, the pair
 * matrix P (eq. pair-probability, diagonal = unpaired), base marginals
 * (eq. marginal-base), codon marginals (eq. marginal-codon), codon-pair
 * marginals, and exact joint samples (Section 4a).
 *
 * How: the sequence tensor train of Section 3a with one codon slot per bond
 * is pre-contracted into a McCaskill dynamic program (the substitution of the
 * sequence-summed fold for the fixed-sequence fold in Section 3c): every DP
 * entry for a range [i..j] becomes a small tensor over the codon slots of its
 * two end positions.  The loop model is the reading written down in the
 * design notes (the paper fixes none for this path):
 *   hairpin   L = j-i-1 >= 3 : hairpin[L] (L<=30) or hairpin[30]+extrap*ln(L/30),
 *                              plus mismatch[phi_{i+1}][phi_{j-1}][t(i,j)]
 *   stack     (i+1, j-1)     : stack[t(i,j)][t(i+1,j-1)]
 *   bulge     one side empty : bulge[L], 1 <= L <= 30
 *   interior  l1,l2 >= 1, l1+l2 <= 30 :
 *             interior[l1+l2] + mismatch[phi_{i+1}][phi_{j-1}][t(i,j)]
 *                             + mismatch[phi_{l+1}][phi_{k-1}][t(l,k)]
 *   multiloop ml_a + ml_b*(branches+1) + ml_c*(unpaired)
 *   exterior  0
 * Pairs AU CG GC UA GU UG; hairpins have >= 3 unpaired bases (SI S2c).
 *
 * Scaling: every vertex factor is multiplied by exp(-g).  Each position
 * contributes exactly one vertex factor to every term, so all entries of a
 * range of length L carry exp(-g L) and the result is exact in real
 * arithmetic: log Z = log Z~ + g n.
 *
 * The PLANT_* switches exist only for tests/test_oracle_mutations.py, which
 * builds each one into a throwaway library and checks that the pins notice
 * the planted mistake; the default build defines none of them.
 *
 * Marginals come from a literal reverse-mode (push/scatter) pass over the
 * same statements.  Because each derivation uses every vertex factor v_p and
 * every backbone edge factor e_p exactly once,
 *     Pr[slot of position p = s]       = v_p(s) * dZ/dv_p(s) / Z
 *     Pr[slots across edge p = (s,t)]  = e_p(s,t) * dZ/de_p(s,t) / Z
 *     Pr[i pairs with j]               = sum Qb[i][j] * dZ/dQb[i][j] / Z.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NS 6          /* max codon slots per residue */
#define MAXLOOP 30    /* bulge / interior loop size bound */
#define CELLSZ 36

/* Standard genetic code; codon index 16*b1 + 4*b2 + b3 with A=0 C=1 G=2 U=3.
 * '*' marks the stop codons, which are never used (SI S3c). */
static const char CODE64[] =
    "KNKNTTTTRSRSIIMIQHQHPPPPRRRRLLLLEDEDAAAAGGGGVVVV*Y*YSSSS*CWCLFLF";
static const char AAS[] = "ARNDCQEGHILKMFPSTWYV";

typedef struct {
  double stack[6][6];
  double hairpin[31];
  double bulge[31];
  double interior[31];
  double mismatch[4][4][6];
  double ml_a, ml_b, ml_c, extrap;
} orc_energy;

typedef struct {
  int n, m;
  int *d;                 /* [n] slot count of the residue of position p */
  int (*nt)[NS];          /* [n][NS] base of position p under slot s */
  double (*v)[NS];        /* [n][NS] vertex factor (scaled by exp(-g)) */
  double (*e)[NS][NS];    /* [n][NS][NS] edge factor between p and p+1 */
  double g;
  double Bst[6][6], Bbu[31], Bin[31], Bmm[4][4][6];
  double hp[31], hp30, extrap;
  double Bmla_b, Bmlb, Bmlc;
} Model;

typedef struct {
  size_t ncell;
  double *U, *Qb, *DI, *Qm1, *Qm1p, *QmX, *Qm; /* forward */
  double *Z5;                                  /* [n][NS] */
  double *Ub, *Qbb, *DIb, *Qm1b, *Qm1pb, *QmXb, *Qmb, *Z5b;
  double *vb, *eb;                             /* [n][NS], [n][NS][NS] */
} Arrays;

/* pair type of bases (x, y): AU=0 CG=1 GC=2 UA=3 GU=4 UG=5, -1 if none */
static int ptype(int x, int y) {
  static const int T[4][4] = {{-1, -1, -1, 0}, {-1, -1, 1, -1},
                              {-1, 2, -1, 4}, {3, -1, 5, -1}};
  return T[x][y];
}

static size_t cell_index(int n, int i, int j) {
  return ((size_t)i * (size_t)(2 * n - i + 1)) / 2 + (size_t)(j - i);
}
#define CELL(A, i, j) ((A) + cell_index(M->n, (i), (j)) * CELLSZ)

static int aa_index(char c) {
  for (int k = 0; k < 20; k++)
    if (AAS[k] == c) return k;
  return -1;
}

/* Build per-position slot tables and Boltzmann factors.  Returns 0 on success. */
static int model_build(Model *M, int m, const char *aa, const double *theta1,
                       const double *theta2, const orc_energy *E, double g) {
  memset(M, 0, sizeof(*M));
  M->m = m;
  M->n = 3 * m;
  int n = M->n;
  M->d = calloc(n, sizeof(int));
  M->nt = calloc(n, sizeof(*M->nt));
  M->v = calloc(n, sizeof(*M->v));
  M->e = calloc(n, sizeof(*M->e));
  if (!M->d || !M->nt || !M->v || !M->e) return -1;
  M->g = g;
  double eg = exp(-g);
  for (int a = 0; a < m; a++) {
    if (aa_index(aa[a]) < 0) return -2;
    int cnt = 0;
    int codons[NS];
    for (int c = 0; c < 64; c++)
      if (CODE64[c] == aa[a]) codons[cnt++] = c; /* lexicographic slot order */
    for (int r = 0; r < 3; r++) {
      int p = 3 * a + r;
      M->d[p] = cnt;
      for (int s = 0; s < cnt; s++) {
        int c = codons[s];
        M->nt[p][s] = (r == 0) ? (c >> 4) : (r == 1) ? ((c >> 2) & 3) : (c & 3);
        double w = 1.0;
        if (r == 1 && theta1) w = exp(theta1[a * NS + s]);
        M->v[p][s] = w * eg;
      }
    }
  }
  for (int p = 0; p + 1 < n; p++) {
    for (int s = 0; s < M->d[p]; s++)
      for (int t = 0; t < M->d[p + 1]; t++) {
        if (p % 3 != 2) {
          M->e[p][s][t] = (s == t) ? 1.0 : 0.0;
        } else {
          int a = p / 3 + 1; /* codon-pair weight of codons a-1, a */
#ifdef PLANT_PAIR_TRANSPOSE
          M->e[p][s][t] = theta2 ? exp(theta2[(a * NS + t) * NS + s]) : 1.0;
#else
          M->e[p][s][t] = theta2 ? exp(theta2[(a * NS + s) * NS + t]) : 1.0;
#endif
        }
      }
  }
  for (int x = 0; x < 6; x++)
    for (int y = 0; y < 6; y++) M->Bst[x][y] = exp(-E->stack[x][y]);
  for (int L = 0; L <= 30; L++) {
    M->Bbu[L] = exp(-E->bulge[L]);
    M->Bin[L] = exp(-E->interior[L]);
    M->hp[L] = E->hairpin[L];
  }
  for (int x = 0; x < 4; x++)
    for (int y = 0; y < 4; y++)
      for (int t = 0; t < 6; t++) M->Bmm[x][y][t] = exp(-E->mismatch[x][y][t]);
  M->hp30 = E->hairpin[30];
  M->extrap = E->extrap;
#ifdef PLANT_ML_CLOSING
  M->Bmla_b = exp(-E->ml_a);
#else
  M->Bmla_b = exp(-(E->ml_a + E->ml_b));
#endif
  M->Bmlb = exp(-E->ml_b);
  M->Bmlc = exp(-E->ml_c);
  return 0;
}

static void model_free(Model *M) {
  free(M->d);
  free(M->nt);
  free(M->v);
  free(M->e);
}

/* Boltzmann factor of a hairpin with L unpaired bases (mismatch excluded). */
static double hairpin_B(const Model *M, int L) {
  if (L < 3) return 0.0;
  if (L <= 30) return exp(-M->hp[L]);
#ifdef PLANT_HAIRPIN_EXTRAP
  return exp(-M->hp30);
#else
  return exp(-(M->hp30 + M->extrap * log((double)L / 30.0)));
#endif
}

static int arrays_alloc(Arrays *A, int n, int with_adjoint) {
  memset(A, 0, sizeof(*A));
  A->ncell = (size_t)n * (n + 1) / 2;
  size_t sz = A->ncell * CELLSZ;
  double **fw[] = {&A->U, &A->Qb, &A->DI, &A->Qm1, &A->Qm1p, &A->QmX, &A->Qm};
  for (int k = 0; k < 7; k++)
    if (!(*fw[k] = calloc(sz, sizeof(double)))) return -1;
  if (!(A->Z5 = calloc((size_t)n * NS, sizeof(double)))) return -1;
  if (with_adjoint) {
    double **bw[] = {&A->Ub, &A->Qbb, &A->DIb, &A->Qm1b, &A->Qm1pb, &A->QmXb, &A->Qmb};
    for (int k = 0; k < 7; k++)
      if (!(*bw[k] = calloc(sz, sizeof(double)))) return -1;
    if (!(A->Z5b = calloc((size_t)n * NS, sizeof(double)))) return -1;
    if (!(A->vb = calloc((size_t)n * NS, sizeof(double)))) return -1;
    if (!(A->eb = calloc((size_t)n * NS * NS, sizeof(double)))) return -1;
  }
  return 0;
}

static void arrays_free(Arrays *A) {
  double *p[] = {A->U, A->Qb, A->DI, A->Qm1, A->Qm1p, A->QmX, A->Qm, A->Z5,
                 A->Ub, A->Qbb, A->DIb, A->Qm1b, A->Qm1pb, A->QmXb, A->Qmb,
                 A->Z5b, A->vb, A->eb};
  for (unsigned k = 0; k < sizeof(p) / sizeof(p[0]); k++) free(p[k]);
}

/* ------------------------------------------------------------------------ */
/* Forward                                                                   */
/* ------------------------------------------------------------------------ */

/* Unpaired run U[i][j](a,b): sum over slots of positions strictly inside of
 * the product of their vertex factors and the edges between them; a, b are
 * the slots of positions i and j, whose vertex factors are included. */
static void forward_runs(const Model *M, Arrays *A) {
  int n = M->n;
  for (int p = 0; p < n; p++) {
    double *u = CELL(A->U, p, p);
    for (int a = 0; a < M->d[p]; a++) u[a * 6 + a] = M->v[p][a];
  }
  for (int dl = 1; dl < n; dl++)
    for (int i = 0; i + dl < n; i++) {
      int j = i + dl;
      const double *ul = CELL(A->U, i, j - 1);
      double *u = CELL(A->U, i, j);
      for (int a = 0; a < M->d[i]; a++)
        for (int b = 0; b < M->d[j]; b++) {
          double s = 0;
          for (int c = 0; c < M->d[j - 1]; c++) s += ul[a * 6 + c] * M->e[j - 1][c][b];
          u[a * 6 + b] = s * M->v[j][b];
        }
    }
}

/* All DP entries of the range [i..j] (j - i >= 4), in dependency order:
 * Qb (pair i.j closes a hairpin, stack/bulge/interior or multiloop), DI (Qb
 * dressed as the inner pair of an interior loop), Qm1 (one branch starting
 * at i, unpaired tail), Qm1p (unpaired prefix + one branch), QmX (>= 2
 * branches), Qm (>= 1 branch). */
static void cell_forward(const Model *M, Arrays *A, int i, int j) {
  int n = M->n;
  int di = M->d[i], dj = M->d[j];
  int L = j - i - 1;
  double acc[6][6];
  memset(acc, 0, sizeof(acc));
  int pt[6][6];
  for (int s = 0; s < di; s++)
    for (int s2 = 0; s2 < dj; s2++) pt[s][s2] = ptype(M->nt[i][s], M->nt[j][s2]);

  /* hairpin */
  {
    double bh = hairpin_B(M, L);
    const double *u = CELL(A->U, i + 1, j - 1);
    for (int s = 0; s < di; s++)
      for (int s2 = 0; s2 < dj; s2++) {
        int t = pt[s][s2];
        if (t < 0) continue;
        double sum = 0;
        for (int a = 0; a < M->d[i + 1]; a++)
          for (int b = 0; b < M->d[j - 1]; b++)
            sum += M->e[i][s][a] * u[a * 6 + b] * M->e[j - 1][b][s2] *
                   M->Bmm[M->nt[i + 1][a]][M->nt[j - 1][b]][t];
        acc[s][s2] += bh * sum;
      }
  }
  /* stack: inner pair (i+1, j-1) */
  if ((j - 1) - (i + 1) >= 4) {
    const double *q = CELL(A->Qb, i + 1, j - 1);
    for (int s = 0; s < di; s++)
      for (int s2 = 0; s2 < dj; s2++) {
        int t = pt[s][s2];
        if (t < 0) continue;
        double sum = 0;
        for (int x = 0; x < M->d[i + 1]; x++)
          for (int y = 0; y < M->d[j - 1]; y++) {
            double qq = q[x * 6 + y];
            if (qq == 0.0) continue;
            int t2 = ptype(M->nt[i + 1][x], M->nt[j - 1][y]);
#ifdef PLANT_STACK_SWAP
            sum += M->e[i][s][x] * qq * M->e[j - 1][y][s2] * M->Bst[t2][t];
#else
            sum += M->e[i][s][x] * qq * M->e[j - 1][y][s2] * M->Bst[t][t2];
#endif
          }
        acc[s][s2] += sum;
      }
  }
  /* bulges and interior loops; GL/GR/F are the loop sums with the outer
   * edges (and, for interior loops, the outer mismatch) not yet applied */
  double GL[6][6], GR[6][6], F[6][6];
  memset(GL, 0, sizeof(GL));
  memset(GR, 0, sizeof(GR));
  memset(F, 0, sizeof(F));
  int d1 = M->d[i + 1], dm = M->d[j - 1];
  for (int l1 = 0; l1 <= MAXLOOP; l1++)
    for (int l2 = 0; l1 + l2 <= MAXLOOP; l2++) {
      if (l1 == 0 && l2 == 0) continue;
      int k = i + 1 + l1, l = j - 1 - l2;
      if (l - k < 4) continue;
      const double *q = CELL(A->Qb, k, l);
      if (l2 == 0) { /* left bulge: run i+1..k-1, pair (k, j-1) */
        const double *ul = CELL(A->U, i + 1, k - 1);
        double w = M->Bbu[l1];
        for (int a = 0; a < d1; a++)
          for (int y = 0; y < M->d[l]; y++) {
            double s = 0;
            for (int b = 0; b < M->d[k - 1]; b++)
              for (int x = 0; x < M->d[k]; x++)
                s += ul[a * 6 + b] * M->e[k - 1][b][x] * q[x * 6 + y];
            GL[a][y] += w * s;
          }
      } else if (l1 == 0) { /* right bulge: pair (i+1, l), run l+1..j-1 */
        const double *ur = CELL(A->U, l + 1, j - 1);
        double w = M->Bbu[l2];
        for (int x = 0; x < M->d[k]; x++)
          for (int dd = 0; dd < dm; dd++) {
            double s = 0;
            for (int y = 0; y < M->d[l]; y++)
              for (int c = 0; c < M->d[l + 1]; c++)
                s += q[x * 6 + y] * M->e[l][y][c] * ur[c * 6 + dd];
            GR[x][dd] += w * s;
          }
      } else { /* interior loop */
        const double *ul = CELL(A->U, i + 1, k - 1);
        const double *ur = CELL(A->U, l + 1, j - 1);
        const double *di_kl = CELL(A->DI, k, l);
        double w = M->Bin[l1 + l2];
        double T[6][6];
        for (int a = 0; a < d1; a++)
          for (int c = 0; c < M->d[l + 1]; c++) {
            double s = 0;
            for (int b = 0; b < M->d[k - 1]; b++) s += ul[a * 6 + b] * di_kl[b * 6 + c];
            T[a][c] = s;
          }
        for (int a = 0; a < d1; a++)
          for (int dd = 0; dd < dm; dd++) {
            double s = 0;
            for (int c = 0; c < M->d[l + 1]; c++) s += T[a][c] * ur[c * 6 + dd];
            F[a][dd] += w * s;
          }
      }
    }
  for (int s = 0; s < di; s++)
    for (int s2 = 0; s2 < dj; s2++) {
      int t = pt[s][s2];
      if (t < 0) continue;
      double sum = 0;
      for (int a = 0; a < d1; a++)
        for (int dd = 0; dd < dm; dd++)
          sum += M->e[i][s][a] * M->e[j - 1][dd][s2] *
                 (GL[a][dd] + GR[a][dd] +
                  F[a][dd] * M->Bmm[M->nt[i + 1][a]][M->nt[j - 1][dd]][t]);
      acc[s][s2] += sum;
    }
  /* multiloop closed by (i, j): >= 2 branches inside */
  {
    const double *qx = CELL(A->QmX, i + 1, j - 1);
    for (int s = 0; s < di; s++)
      for (int s2 = 0; s2 < dj; s2++) {
        if (pt[s][s2] < 0) continue;
        double sum = 0;
        for (int x = 0; x < d1; x++)
          for (int y = 0; y < dm; y++)
            sum += M->e[i][s][x] * qx[x * 6 + y] * M->e[j - 1][y][s2];
        acc[s][s2] += M->Bmla_b * sum;
      }
  }
  double *qb = CELL(A->Qb, i, j);
  for (int s = 0; s < di; s++)
    for (int s2 = 0; s2 < dj; s2++)
      if (pt[s][s2] >= 0) qb[s * 6 + s2] = M->v[i][s] * M->v[j][s2] * acc[s][s2];

  /* DI[i][j](b, c): Qb[i][j] seen as the inner pair of an interior loop,
   * with the edges to i-1 and j+1 and the inner mismatch applied */
  if (i >= 1 && j + 1 < n) {
    double *dI = CELL(A->DI, i, j);
    for (int b = 0; b < M->d[i - 1]; b++)
      for (int c = 0; c < M->d[j + 1]; c++) {
        double s = 0;
        for (int x = 0; x < di; x++)
          for (int y = 0; y < dj; y++) {
            double qq = qb[x * 6 + y];
            if (qq == 0.0) continue;
            int t2 = ptype(M->nt[j][y], M->nt[i][x]);
#ifdef PLANT_INNER_MISMATCH
            s += M->e[i - 1][b][x] * qq * M->e[j][y][c] *
                 M->Bmm[M->nt[i - 1][b]][M->nt[j + 1][c]][t2];
#else
            s += M->e[i - 1][b][x] * qq * M->e[j][y][c] *
                 M->Bmm[M->nt[j + 1][c]][M->nt[i - 1][b]][t2];
#endif
          }
        dI[b * 6 + c] = s;
      }
  }
  /* Qm1: branch starting at i, unpaired tail */
  double *q1 = CELL(A->Qm1, i, j);
  {
    const double *q1l = CELL(A->Qm1, i, j - 1);
    for (int s = 0; s < di; s++)
      for (int s2 = 0; s2 < dj; s2++) {
        double sum = 0;
        for (int t = 0; t < M->d[j - 1]; t++) sum += q1l[s * 6 + t] * M->e[j - 1][t][s2];
        q1[s * 6 + s2] = sum * M->v[j][s2] * M->Bmlc + qb[s * 6 + s2] * M->Bmlb;
      }
  }
  /* Qm1p: unpaired prefix then one branch */
  double *q1p = CELL(A->Qm1p, i, j);
  {
    const double *q1pr = CELL(A->Qm1p, i + 1, j);
    for (int s = 0; s < di; s++)
      for (int s2 = 0; s2 < dj; s2++) {
        double sum = 0;
        for (int t = 0; t < d1; t++) sum += M->e[i][s][t] * q1pr[t * 6 + s2];
        q1p[s * 6 + s2] = q1[s * 6 + s2] + M->v[i][s] * M->Bmlc * sum;
      }
  }
  /* QmX: >= 1 branch in [i..u-1] followed by the last branch starting at u.
   * Qm[i][u-1] vanishes for u-1-i < 4 and Qm1[u][j] for j-u < 4. */
  double *qx = CELL(A->QmX, i, j);
#ifdef PLANT_SPLIT_RANGE
  for (int u = i + 6; u <= j - 4; u++) {
#else
  for (int u = i + 5; u <= j - 4; u++) {
#endif
    const double *qm = CELL(A->Qm, i, u - 1);
    const double *q1u = CELL(A->Qm1, u, j);
    int du1 = M->d[u - 1], du = M->d[u];
    for (int s = 0; s < di; s++)
      for (int s2 = 0; s2 < dj; s2++) {
        double sum = 0;
        for (int t = 0; t < du1; t++)
          for (int t2 = 0; t2 < du; t2++)
            sum += qm[s * 6 + t] * M->e[u - 1][t][t2] * q1u[t2 * 6 + s2];
        qx[s * 6 + s2] += sum;
      }
  }
  double *qm = CELL(A->Qm, i, j);
  for (int k = 0; k < 36; k++) qm[k] = qx[k] + q1p[k];
}

/* Exterior loop: Z5[j](t) sums over structures of [0..j] with slot t at j. */
static double forward_exterior(const Model *M, Arrays *A) {
  int n = M->n;
  double *Z5 = A->Z5;
  for (int s = 0; s < M->d[0]; s++) Z5[s] = M->v[0][s];
  for (int j = 1; j < n; j++) {
    for (int t = 0; t < M->d[j]; t++) {
      double sum = 0;
      for (int s = 0; s < M->d[j - 1]; s++)
        sum += Z5[(j - 1) * NS + s] * M->e[j - 1][s][t];
      sum *= M->v[j][t];
      for (int k = 1; k <= j - 4; k++) {
        const double *q = CELL(A->Qb, k, j);
        for (int s = 0; s < M->d[k - 1]; s++)
          for (int x = 0; x < M->d[k]; x++)
            sum += Z5[(k - 1) * NS + s] * M->e[k - 1][s][x] * q[x * 6 + t];
      }
      if (j >= 4) {
        const double *q = CELL(A->Qb, 0, j);
        for (int x = 0; x < M->d[0]; x++) sum += q[x * 6 + t];
      }
      Z5[j * NS + t] = sum;
    }
  }
  double Z = 0;
  for (int t = 0; t < M->d[n - 1]; t++) Z += Z5[(n - 1) * NS + t];
  return Z;
}

static double forward_all(const Model *M, Arrays *A) {
  int n = M->n;
  forward_runs(M, A);
  for (int dl = 4; dl < n; dl++) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < n - dl; i++) cell_forward(M, A, i, i + dl);
  }
  return forward_exterior(M, A);
}

/* ------------------------------------------------------------------------ */
/* Reverse mode (push form): adjoint of every statement above, in reverse.   */
/* ------------------------------------------------------------------------ */

#define EB(p, s, t) (A->eb[((size_t)(p) * NS + (s)) * NS + (t)])
#define VB(p, s) (A->vb[(size_t)(p) * NS + (s)])

static void reverse_exterior(const Model *M, Arrays *A) {
  int n = M->n;
  double *Z5 = A->Z5, *Z5b = A->Z5b;
  for (int t = 0; t < M->d[n - 1]; t++) Z5b[(n - 1) * NS + t] = 1.0;
  for (int j = n - 1; j >= 1; j--) {
    for (int t = 0; t < M->d[j]; t++) {
      double gt = Z5b[j * NS + t];
      if (gt == 0.0) continue;
      for (int s = 0; s < M->d[j - 1]; s++) {
        double z = Z5[(j - 1) * NS + s], e = M->e[j - 1][s][t], v = M->v[j][t];
        Z5b[(j - 1) * NS + s] += gt * e * v;
        EB(j - 1, s, t) += gt * z * v;
        VB(j, t) += gt * z * e;
      }
      for (int k = 1; k <= j - 4; k++) {
        const double *q = CELL(A->Qb, k, j);
        double *qbb = CELL(A->Qbb, k, j);
        for (int s = 0; s < M->d[k - 1]; s++)
          for (int x = 0; x < M->d[k]; x++) {
            double z = Z5[(k - 1) * NS + s], e = M->e[k - 1][s][x], qq = q[x * 6 + t];
            Z5b[(k - 1) * NS + s] += gt * e * qq;
            EB(k - 1, s, x) += gt * z * qq;
            qbb[x * 6 + t] += gt * z * e;
          }
      }
      if (j >= 4) {
        double *qbb = CELL(A->Qbb, 0, j);
        for (int x = 0; x < M->d[0]; x++) qbb[x * 6 + t] += gt;
      }
    }
  }
  for (int s = 0; s < M->d[0]; s++) VB(0, s) += Z5b[s];
}

static void cell_reverse(const Model *M, Arrays *A, int i, int j) {
  int n = M->n;
  int di = M->d[i], dj = M->d[j];
  int L = j - i - 1;
  int d1 = M->d[i + 1], dm = M->d[j - 1];
  const double *qb = CELL(A->Qb, i, j);
  double *qbb = CELL(A->Qbb, i, j);
  double *q1b = CELL(A->Qm1b, i, j), *q1pb = CELL(A->Qm1pb, i, j);
  double *qxb = CELL(A->QmXb, i, j), *qmb = CELL(A->Qmb, i, j);

  /* Qm = QmX + Qm1p */
  for (int k = 0; k < 36; k++) {
    qxb[k] += qmb[k];
    q1pb[k] += qmb[k];
  }
  /* QmX splits */
  for (int u = i + 5; u <= j - 4; u++) {
    const double *qm = CELL(A->Qm, i, u - 1);
    const double *q1u = CELL(A->Qm1, u, j);
    double *qmbu = CELL(A->Qmb, i, u - 1);
    double *q1bu = CELL(A->Qm1b, u, j);
    int du1 = M->d[u - 1], du = M->d[u];
    for (int s = 0; s < di; s++)
      for (int s2 = 0; s2 < dj; s2++) {
        double g = qxb[s * 6 + s2];
        if (g == 0.0) continue;
        for (int t = 0; t < du1; t++)
          for (int t2 = 0; t2 < du; t2++) {
            double a = qm[s * 6 + t], e = M->e[u - 1][t][t2], b = q1u[t2 * 6 + s2];
            qmbu[s * 6 + t] += g * e * b;
            EB(u - 1, t, t2) += g * a * b;
            q1bu[t2 * 6 + s2] += g * a * e;
          }
      }
  }
  /* Qm1p = Qm1 + v_i c e_i Qm1p[i+1][j] */
  {
    const double *q1pr = CELL(A->Qm1p, i + 1, j);
    double *q1prb = CELL(A->Qm1pb, i + 1, j);
    for (int s = 0; s < di; s++)
      for (int s2 = 0; s2 < dj; s2++) {
        double g = q1pb[s * 6 + s2];
        if (g == 0.0) continue;
        q1b[s * 6 + s2] += g;
        for (int t = 0; t < d1; t++) {
          double e = M->e[i][s][t], q = q1pr[t * 6 + s2];
          VB(i, s) += g * M->Bmlc * e * q;
          EB(i, s, t) += g * M->v[i][s] * M->Bmlc * q;
          q1prb[t * 6 + s2] += g * M->v[i][s] * M->Bmlc * e;
        }
      }
  }
  /* Qm1 = Qm1[i][j-1] e_{j-1} v_j c + Qb b */
  {
    const double *q1l = CELL(A->Qm1, i, j - 1);
    double *q1lb = CELL(A->Qm1b, i, j - 1);
    for (int s = 0; s < di; s++)
      for (int s2 = 0; s2 < dj; s2++) {
        double g = q1b[s * 6 + s2];
        if (g == 0.0) continue;
        qbb[s * 6 + s2] += g * M->Bmlb;
        for (int t = 0; t < dm; t++) {
          double a = q1l[s * 6 + t], e = M->e[j - 1][t][s2], v = M->v[j][s2];
          q1lb[s * 6 + t] += g * e * v * M->Bmlc;
#ifndef PLANT_REVERSE_EDGE
          EB(j - 1, t, s2) += g * a * v * M->Bmlc;
#endif
          VB(j, s2) += g * a * e * M->Bmlc;
        }
      }
  }
  /* DI */
  if (i >= 1 && j + 1 < n) {
    const double *dIb = CELL(A->DIb, i, j);
    for (int b = 0; b < M->d[i - 1]; b++)
      for (int c = 0; c < M->d[j + 1]; c++) {
        double g = dIb[b * 6 + c];
        if (g == 0.0) continue;
        for (int x = 0; x < di; x++)
          for (int y = 0; y < dj; y++) {
            double qq = qb[x * 6 + y];
            if (qq == 0.0) continue;
            int t2 = ptype(M->nt[j][y], M->nt[i][x]);
            double mm = M->Bmm[M->nt[j + 1][c]][M->nt[i - 1][b]][t2];
            double e1 = M->e[i - 1][b][x], e2 = M->e[j][y][c];
            qbb[x * 6 + y] += g * e1 * e2 * mm;
            EB(i - 1, b, x) += g * qq * e2 * mm;
            EB(j, y, c) += g * e1 * qq * mm;
          }
      }
  }
  /* Qb = [allowed] v_i v_j acc  ->  accb */
  double accb[6][6];
  memset(accb, 0, sizeof(accb));
  int pt[6][6];
  for (int s = 0; s < di; s++)
    for (int s2 = 0; s2 < dj; s2++) pt[s][s2] = ptype(M->nt[i][s], M->nt[j][s2]);
  for (int s = 0; s < di; s++)
    for (int s2 = 0; s2 < dj; s2++) {
      if (pt[s][s2] < 0) continue;
      double g = qbb[s * 6 + s2];
      if (g == 0.0) continue;
      double vi = M->v[i][s], vj = M->v[j][s2];
      accb[s][s2] = g * vi * vj;
      /* acc = Qb / (v_i v_j); recompute it rather than divide */
    }
  /* the vertex adjoints need acc itself: recompute the forward acc terms
   * while pushing; first the vertex part via Qb = v_i v_j acc */
  for (int s = 0; s < di; s++)
    for (int s2 = 0; s2 < dj; s2++) {
      if (pt[s][s2] < 0) continue;
      double g = qbb[s * 6 + s2];
      if (g == 0.0) continue;
      double vi = M->v[i][s], vj = M->v[j][s2];
      /* Qb(s,s2) = vi * vj * acc  =>  d/dvi = vj*acc = Qb/vi (vi > 0 here
       * unless the slot is clamped away, in which case Qb = 0 and the
       * product v*vb used for marginals is 0 either way) */
      if (vi != 0.0) VB(i, s) += g * qb[s * 6 + s2] / vi;
      if (vj != 0.0) VB(j, s2) += g * qb[s * 6 + s2] / vj;
    }
  /* hairpin */
  {
    double bh = hairpin_B(M, L);
    const double *u = CELL(A->U, i + 1, j - 1);
    double *ub = CELL(A->Ub, i + 1, j - 1);
    for (int s = 0; s < di; s++)
      for (int s2 = 0; s2 < dj; s2++) {
        int t = pt[s][s2];
        double g = accb[s][s2];
        if (t < 0 || g == 0.0) continue;
        for (int a = 0; a < d1; a++)
          for (int b = 0; b < dm; b++) {
            double mm = M->Bmm[M->nt[i + 1][a]][M->nt[j - 1][b]][t];
            double e1 = M->e[i][s][a], uu = u[a * 6 + b], e2 = M->e[j - 1][b][s2];
            EB(i, s, a) += g * bh * uu * e2 * mm;
            ub[a * 6 + b] += g * bh * e1 * e2 * mm;
            EB(j - 1, b, s2) += g * bh * e1 * uu * mm;
          }
      }
  }
  /* stack */
  if ((j - 1) - (i + 1) >= 4) {
    const double *q = CELL(A->Qb, i + 1, j - 1);
    double *qb_in = CELL(A->Qbb, i + 1, j - 1);
    for (int s = 0; s < di; s++)
      for (int s2 = 0; s2 < dj; s2++) {
        int t = pt[s][s2];
        double g = accb[s][s2];
        if (t < 0 || g == 0.0) continue;
        for (int x = 0; x < d1; x++)
          for (int y = 0; y < dm; y++) {
            int t2 = ptype(M->nt[i + 1][x], M->nt[j - 1][y]);
            if (t2 < 0) continue;
            double w = M->Bst[t][t2];
            double e1 = M->e[i][s][x], qq = q[x * 6 + y], e2 = M->e[j - 1][y][s2];
            EB(i, s, x) += g * w * qq * e2;
            qb_in[x * 6 + y] += g * w * e1 * e2;
            EB(j - 1, y, s2) += g * w * e1 * qq;
          }
      }
  }
  /* bulges and interior: adjoints of GL, GR, F, then of their terms */
  double GLb[6][6], GRb[6][6], Fb[6][6];
  memset(GLb, 0, sizeof(GLb));
  memset(GRb, 0, sizeof(GRb));
  memset(Fb, 0, sizeof(Fb));
  {
    /* recompute GL, GR, F (needed for the outer edge adjoints) */
    double GL[6][6], GR[6][6], F[6][6];
    memset(GL, 0, sizeof(GL));
    memset(GR, 0, sizeof(GR));
    memset(F, 0, sizeof(F));
    for (int l1 = 0; l1 <= MAXLOOP; l1++)
      for (int l2 = 0; l1 + l2 <= MAXLOOP; l2++) {
        if (l1 == 0 && l2 == 0) continue;
        int k = i + 1 + l1, l = j - 1 - l2;
        if (l - k < 4) continue;
        const double *q = CELL(A->Qb, k, l);
        if (l2 == 0) {
          const double *ul = CELL(A->U, i + 1, k - 1);
          for (int a = 0; a < d1; a++)
            for (int y = 0; y < M->d[l]; y++) {
              double s = 0;
              for (int b = 0; b < M->d[k - 1]; b++)
                for (int x = 0; x < M->d[k]; x++)
                  s += ul[a * 6 + b] * M->e[k - 1][b][x] * q[x * 6 + y];
              GL[a][y] += M->Bbu[l1] * s;
            }
        } else if (l1 == 0) {
          const double *ur = CELL(A->U, l + 1, j - 1);
          for (int x = 0; x < M->d[k]; x++)
            for (int dd = 0; dd < dm; dd++) {
              double s = 0;
              for (int y = 0; y < M->d[l]; y++)
                for (int c = 0; c < M->d[l + 1]; c++)
                  s += q[x * 6 + y] * M->e[l][y][c] * ur[c * 6 + dd];
              GR[x][dd] += M->Bbu[l2] * s;
            }
        } else {
          const double *ul = CELL(A->U, i + 1, k - 1);
          const double *ur = CELL(A->U, l + 1, j - 1);
          const double *dI = CELL(A->DI, k, l);
          for (int a = 0; a < d1; a++)
            for (int dd = 0; dd < dm; dd++) {
              double s = 0;
              for (int b = 0; b < M->d[k - 1]; b++)
                for (int c = 0; c < M->d[l + 1]; c++)
                  s += ul[a * 6 + b] * dI[b * 6 + c] * ur[c * 6 + dd];
              F[a][dd] += M->Bin[l1 + l2] * s;
            }
        }
      }
    for (int s = 0; s < di; s++)
      for (int s2 = 0; s2 < dj; s2++) {
        int t = pt[s][s2];
        double g = accb[s][s2];
        if (t < 0 || g == 0.0) continue;
        for (int a = 0; a < d1; a++)
          for (int dd = 0; dd < dm; dd++) {
            double mm = M->Bmm[M->nt[i + 1][a]][M->nt[j - 1][dd]][t];
            double e1 = M->e[i][s][a], e2 = M->e[j - 1][dd][s2];
            double inner = GL[a][dd] + GR[a][dd] + F[a][dd] * mm;
            EB(i, s, a) += g * e2 * inner;
            EB(j - 1, dd, s2) += g * e1 * inner;
            GLb[a][dd] += g * e1 * e2;
            GRb[a][dd] += g * e1 * e2;
            Fb[a][dd] += g * e1 * e2 * mm;
          }
      }
  }
  for (int l1 = 0; l1 <= MAXLOOP; l1++)
    for (int l2 = 0; l1 + l2 <= MAXLOOP; l2++) {
      if (l1 == 0 && l2 == 0) continue;
      int k = i + 1 + l1, l = j - 1 - l2;
      if (l - k < 4) continue;
      const double *q = CELL(A->Qb, k, l);
      double *qbk = CELL(A->Qbb, k, l);
      if (l2 == 0) {
        const double *ul = CELL(A->U, i + 1, k - 1);
        double *ulb = CELL(A->Ub, i + 1, k - 1);
        double w = M->Bbu[l1];
        for (int a = 0; a < d1; a++)
          for (int y = 0; y < M->d[l]; y++) {
            double g = GLb[a][y] * w;
            if (g == 0.0) continue;
            for (int b = 0; b < M->d[k - 1]; b++)
              for (int x = 0; x < M->d[k]; x++) {
                double uu = ul[a * 6 + b], e = M->e[k - 1][b][x], qq = q[x * 6 + y];
                ulb[a * 6 + b] += g * e * qq;
                EB(k - 1, b, x) += g * uu * qq;
                qbk[x * 6 + y] += g * uu * e;
              }
          }
      } else if (l1 == 0) {
        const double *ur = CELL(A->U, l + 1, j - 1);
        double *urb = CELL(A->Ub, l + 1, j - 1);
        double w = M->Bbu[l2];
        for (int x = 0; x < M->d[k]; x++)
          for (int dd = 0; dd < dm; dd++) {
            double g = GRb[x][dd] * w;
            if (g == 0.0) continue;
            for (int y = 0; y < M->d[l]; y++)
              for (int c = 0; c < M->d[l + 1]; c++) {
                double qq = q[x * 6 + y], e = M->e[l][y][c], uu = ur[c * 6 + dd];
                qbk[x * 6 + y] += g * e * uu;
                EB(l, y, c) += g * qq * uu;
                urb[c * 6 + dd] += g * qq * e;
              }
          }
      } else {
        const double *ul = CELL(A->U, i + 1, k - 1);
        const double *ur = CELL(A->U, l + 1, j - 1);
        const double *dI = CELL(A->DI, k, l);
        double *ulb = CELL(A->Ub, i + 1, k - 1);
        double *urb = CELL(A->Ub, l + 1, j - 1);
        double *dIb = CELL(A->DIb, k, l);
        double w = M->Bin[l1 + l2];
        for (int a = 0; a < d1; a++)
          for (int dd = 0; dd < dm; dd++) {
            double g = Fb[a][dd] * w;
            if (g == 0.0) continue;
            for (int b = 0; b < M->d[k - 1]; b++)
              for (int c = 0; c < M->d[l + 1]; c++) {
                double uu = ul[a * 6 + b], dd_ = dI[b * 6 + c], vv = ur[c * 6 + dd];
                ulb[a * 6 + b] += g * dd_ * vv;
                dIb[b * 6 + c] += g * uu * vv;
                urb[c * 6 + dd] += g * uu * dd_;
              }
          }
      }
    }
  /* multiloop closing */
  {
    const double *qx = CELL(A->QmX, i + 1, j - 1);
    double *qxb2 = CELL(A->QmXb, i + 1, j - 1);
    for (int s = 0; s < di; s++)
      for (int s2 = 0; s2 < dj; s2++) {
        double g = accb[s][s2];
        if (pt[s][s2] < 0 || g == 0.0) continue;
        g *= M->Bmla_b;
        for (int x = 0; x < d1; x++)
          for (int y = 0; y < dm; y++) {
            double e1 = M->e[i][s][x], q = qx[x * 6 + y], e2 = M->e[j - 1][y][s2];
            EB(i, s, x) += g * q * e2;
            qxb2[x * 6 + y] += g * e1 * e2;
            EB(j - 1, y, s2) += g * e1 * q;
          }
      }
  }
}

static void reverse_runs(const Model *M, Arrays *A) {
  int n = M->n;
  for (int dl = n - 1; dl >= 1; dl--)
    for (int i = 0; i + dl < n; i++) {
      int j = i + dl;
      const double *ul = CELL(A->U, i, j - 1);
      double *ulb = CELL(A->Ub, i, j - 1);
      const double *ub = CELL(A->Ub, i, j);
      for (int a = 0; a < M->d[i]; a++)
        for (int b = 0; b < M->d[j]; b++) {
          double g = ub[a * 6 + b];
          if (g == 0.0) continue;
          double s = 0;
          for (int c = 0; c < M->d[j - 1]; c++) {
            s += ul[a * 6 + c] * M->e[j - 1][c][b];
            ulb[a * 6 + c] += g * M->e[j - 1][c][b] * M->v[j][b];
            EB(j - 1, c, b) += g * ul[a * 6 + c] * M->v[j][b];
          }
          VB(j, b) += g * s;
        }
    }
  for (int p = 0; p < n; p++) {
    const double *ub = CELL(A->Ub, p, p);
    for (int a = 0; a < M->d[p]; a++) VB(p, a) += ub[a * 6 + a];
  }
}

static void reverse_all(const Model *M, Arrays *A) {
  int n = M->n;
  reverse_exterior(M, A);
  for (int dl = n - 1; dl >= 4; dl--)
    for (int i = 0; i < n - dl; i++) cell_reverse(M, A, i, i + dl);
  reverse_runs(M, A);
}

/* ------------------------------------------------------------------------ */
/* Driver: choose the scale g so that no entry leaves the double range.      */
/* ------------------------------------------------------------------------ */

static int finite_and_bounded(const Arrays *A, double bound) {
  size_t sz = A->ncell * CELLSZ;
  const double *p[] = {A->Qb, A->Qm, A->Qm1p, A->U};
  for (int k = 0; k < 4; k++)
    for (size_t x = 0; x < sz; x++) {
      double v = p[k][x];
      if (!(fabs(v) <= bound)) return 0;
    }
  return 1;
}

static int setup_forward(int m, const char *aa, const double *theta1, const double *theta2,
                         const orc_energy *E, int with_adjoint, Model *M, Arrays *A,
                         double *Zs) {
  /* first guess of the log growth per base from a prefix of at most 30
   * residues run unscaled (its Z stays far inside the double range) */
  double g = 0.0;
  if (m > 30) {
    Model Mp;
    Arrays Ap;
    int rc = model_build(&Mp, 30, aa, theta1, theta2, E, 0.0);
    if (rc) { model_free(&Mp); return rc; }
    if (arrays_alloc(&Ap, Mp.n, 0)) { model_free(&Mp); arrays_free(&Ap); return -1; }
    double Zp = forward_all(&Mp, &Ap);
    model_free(&Mp);
    arrays_free(&Ap);
    if (!(Zp > 0) || !isfinite(Zp)) return -3;
    g = log(Zp) / 90.0;
  }
  for (int attempt = 0; attempt < 6; attempt++) {
    int rc = model_build(M, m, aa, theta1, theta2, E, g);
    if (rc) { model_free(M); return rc; }
    if (arrays_alloc(A, M->n, with_adjoint)) { model_free(M); arrays_free(A); return -1; }
    double Z = forward_all(M, A);
    if (Z > 1e-250 && Z < 1e250 && isfinite(Z) && finite_and_bounded(A, 1e280)) {
      *Zs = Z;
      return 0;
    }
    double lz = (Z > 0 && isfinite(Z)) ? log(Z) : (Z > 0 ? 700.0 : -700.0);
    g += lz / M->n + ((Z > 0 && isfinite(Z)) ? 0.0 : 0.5);
    model_free(M);
    arrays_free(A);
  }
  return -3;
}

/* ------------------------------------------------------------------------ */
/* Exported entry points                                                     */
/* ------------------------------------------------------------------------ */

int orc_logz(int m, const char *aa, const double *theta1, const double *theta2,
             const double *energy, double *logz) {
  if (m < 1 || !aa || !energy || !logz) return -1;
  Model M;
  Arrays A;
  double Z;
  int rc = setup_forward(m, aa, theta1, theta2, (const orc_energy *)energy, 0, &M, &A, &Z);
  if (rc) return rc;
  *logz = log(Z) + M.g * M.n;
  model_free(&M);
  arrays_free(&A);
  return 0;
}

/* log Z plus marginals.  pair [n*n], base [n*4], codon [m*6],
 * codon_pair [m*36] (row a: codon a-1 by codon a; row 0 zero),
 * vcheck [n] = sum_s v_p(s) dZ/dv_p(s) / Z (1 for every p if the reverse pass
 * is consistent), echeck [n-1] likewise for edges.  Any output may be NULL. */
int orc_marginals(int m, const char *aa, const double *theta1, const double *theta2,
                  const double *energy, double *logz, double *pair, double *base,
                  double *codon, double *codon_pair, double *vcheck, double *echeck) {
  if (m < 1 || !aa || !energy) return -1;
  Model M;
  Arrays A;
  double Z;
  int rc = setup_forward(m, aa, theta1, theta2, (const orc_energy *)energy, 1, &M, &A, &Z);
  if (rc) return rc;
  int n = M.n;
  const Model *Mp = &M;
  reverse_all(&M, &A);
  if (logz) *logz = log(Z) + M.g * n;
  if (pair) {
    for (size_t x = 0; x < (size_t)n * n; x++) pair[x] = 0.0;
    for (int i = 0; i < n; i++)
      for (int j = i + 4; j < n; j++) {
        const double *q = A.Qb + cell_index(n, i, j) * CELLSZ;
        const double *g = A.Qbb + cell_index(n, i, j) * CELLSZ;
        double s = 0;
        for (int k = 0; k < 36; k++) s += q[k] * g[k];
        pair[(size_t)i * n + j] = pair[(size_t)j * n + i] = s / Z;
      }
    for (int i = 0; i < n; i++) {
      double s = 0;
      for (int j = 0; j < n; j++)
        if (j != i) s += pair[(size_t)i * n + j];
      pair[(size_t)i * n + i] = 1.0 - s;
    }
  }
  double *cod = calloc((size_t)m * NS, sizeof(double));
  for (int a = 0; a < m; a++) {
    int p = 3 * a + 1;
    for (int s = 0; s < Mp->d[p]; s++) cod[a * NS + s] = Mp->v[p][s] * A.vb[p * NS + s] / Z;
  }
  if (codon) memcpy(codon, cod, sizeof(double) * m * NS);
  if (base) {
    for (int p = 0; p < n; p++) {
      for (int b = 0; b < 4; b++) base[p * 4 + b] = 0.0;
      for (int s = 0; s < Mp->d[p]; s++) base[p * 4 + Mp->nt[p][s]] += cod[(p / 3) * NS + s];
    }
  }
  if (codon_pair) {
    for (int k = 0; k < m * 36; k++) codon_pair[k] = 0.0;
    for (int a = 1; a < m; a++) {
      int p = 3 * a - 1;
      for (int s = 0; s < Mp->d[p]; s++)
        for (int t = 0; t < Mp->d[p + 1]; t++)
          codon_pair[a * 36 + s * 6 + t] =
              Mp->e[p][s][t] * A.eb[((size_t)p * NS + s) * NS + t] / Z;
    }
  }
  if (vcheck)
    for (int p = 0; p < n; p++) {
      double s = 0;
      for (int t = 0; t < Mp->d[p]; t++) s += Mp->v[p][t] * A.vb[p * NS + t];
      vcheck[p] = s / Z;
    }
  if (echeck)
    for (int p = 0; p + 1 < n; p++) {
      double s = 0;
      for (int x = 0; x < Mp->d[p]; x++)
        for (int y = 0; y < Mp->d[p + 1]; y++)
          s += Mp->e[p][x][y] * A.eb[((size_t)p * NS + x) * NS + y];
      echeck[p] = s / Z;
    }
  free(cod);
  model_free(&M);
  arrays_free(&A);
  return 0;
}

/* Slot spelling used by this oracle: base of residue letter `aa` in slot s at
 * codon position r (or -1).  Lets tests compare slot orders across sides. */
int orc_slot_base(char aa, int s, int r) {
  int cnt = 0;
  for (int c = 0; c < 64; c++)
    if (CODE64[c] == aa) {
      if (cnt == s) return (r == 0) ? (c >> 4) : (r == 1) ? ((c >> 2) & 3) : (c & 3);
      cnt++;
    }
  return -1;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}


/* ------------------------------------------------------------------------ */
/* Exact joint sampler: stochastic backtracking of the same DP (Section 4a). */
/*                                                                          */
/* Protocol (shared with the GPU sampler by specification only):            */
/*  - one uniform u in [0,1) per decision, u = (x >> 11) * 2^-53 with x the  */
/*    low 64 bits (word1:word0) of Philox4x32-10 under key (seed lo, seed   */
/*    hi) and counter (draw index, sample index, 0, 0);                     */
/*  - a decision lists its alternatives in a fixed order, sums them left to */
/*    right and takes the first whose running sum exceeds u * total;        */
/*  - fragments are processed depth first from an explicit stack, the left  */
/*    (5') fragment before the right one.                                   */
/* ------------------------------------------------------------------------ */

static void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; r++) {
    uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c[0] = n0;
    c[1] = n1;
    c[2] = n2;
    c[3] = n3;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

/* raw Philox4x32-10 block, for known-answer tests */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  philox4x32_10(c, key[0], key[1]);
  for (int k = 0; k < 4; k++) out[k] = c[k];
}

double orc_philox_u01(uint64_t seed, uint32_t sample_id, uint32_t draw) {
  uint32_t c[4] = {draw, sample_id, 0u, 0u};
  philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  uint64_t x = ((uint64_t)c[1] << 32) | c[0];
  return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

enum { F_EXT, F_B, F_M1, F_M1P, F_MX, F_M, F_RUN };
typedef struct {
  int kind, i, j, s, t;
} Frag;

typedef struct {
  const Model *M;
  const Arrays *A;
  uint64_t seed;
  uint32_t sid, draw;
  int *state;
  int32_t *pairs;
  Frag *stk;
  int top, cap;
  double *buf;
  long bufcap;
  int err;
} Samp;

static void push(Samp *S, int kind, int i, int j, int s, int t) {
  if (S->top == S->cap) {
    S->cap = S->cap ? 2 * S->cap : 64;
    S->stk = realloc(S->stk, sizeof(Frag) * S->cap);
  }
  Frag f = {kind, i, j, s, t};
  S->stk[S->top++] = f;
}

static void put(Samp *S, long idx, double w) {
  if (idx >= S->bufcap) {
    S->bufcap = 2 * (idx + 1);
    S->buf = realloc(S->buf, sizeof(double) * S->bufcap);
  }
  S->buf[idx] = w;
}

static long choose(Samp *S, long nalt) {
  double u = orc_philox_u01(S->seed, S->sid, S->draw++);
  double tot = 0;
  for (long k = 0; k < nalt; k++) tot += S->buf[k];
  if (!(tot > 0)) {
    S->err = 1;
    return -1;
  }
  double target = u * tot, cum = 0;
  long last = -1;
  for (long k = 0; k < nalt; k++) {
    cum += S->buf[k];
    if (S->buf[k] > 0) last = k;
    if (cum > target) return k;
  }
  return last;
}

static void set_state(Samp *S, int p, int s) {
  if (S->state[p] >= 0 && S->state[p] != s) S->err = 2;
  S->state[p] = s;
}

/* alternative bookkeeping for the two passes of a decision: pass 0 lists
 * the weights, pass 1 replays the same loops and acts on the chosen one */
#define ALT(w, action)                   \
  do {                                   \
    if (pass == 0) {                     \
      put(S, idx, (w));                  \
    } else if (idx == pick) {            \
      action;                            \
      return;                            \
    }                                    \
    idx++;                               \
  } while (0)
#define DECIDE                           \
  if (pass == 0) {                       \
    pick = choose(S, idx);               \
    if (pick < 0) return;                \
  }

#define Z5v(k, s) (A->Z5[(size_t)(k) * NS + (s)])

static void s_ext(Samp *S, int j, int t) {
  const Model *M = S->M;
  const Arrays *A = S->A;
  set_state(S, j, t);
  if (j == 0) return;
  long pick = -1;
  for (int pass = 0; pass < 2; pass++) {
    long idx = 0;
    for (int s = 0; s < M->d[j - 1]; s++)
      ALT(Z5v(j - 1, s) * M->e[j - 1][s][t] * M->v[j][t], push(S, F_EXT, j - 1, 0, s, 0));
    if (j >= 4) {
      const double *q = CELL(A->Qb, 0, j);
      for (int x = 0; x < M->d[0]; x++)
        ALT(q[x * 6 + t], push(S, F_B, 0, j, x, t));
    }
    for (int k = 1; k <= j - 4; k++) {
      const double *q = CELL(A->Qb, k, j);
      for (int s = 0; s < M->d[k - 1]; s++)
        for (int x = 0; x < M->d[k]; x++)
          ALT(Z5v(k - 1, s) * M->e[k - 1][s][x] * q[x * 6 + t],
              { push(S, F_B, k, j, x, t); push(S, F_EXT, k - 1, 0, s, 0); });
    }
    DECIDE
  }
}

static void s_run(Samp *S, int p, int q, int a, int b) {
  const Model *M = S->M;
  const Arrays *A = S->A;
  int cp = p / 3, cq = q / 3;
  for (int x = p; x <= q && x / 3 == cp; x++) set_state(S, x, a);
  for (int x = q; x >= p && x / 3 == cq; x--) set_state(S, x, b);
  int prev = a;
  for (int c = cp + 1; c < cq; c++) {
    int f = 3 * c;
    long pick = -1;
    int chosen = -1;
    for (int pass = 0; pass < 2 && chosen < 0; pass++) {
      long idx = 0;
      for (int x = 0; x < M->d[f]; x++) {
        double w = M->e[f - 1][prev][x] * CELL(A->U, f, q)[x * 6 + b];
        if (pass == 0) put(S, idx, w);
        else if (idx == pick) { chosen = x; break; }
        idx++;
      }
      if (pass == 0) {
        pick = choose(S, idx);
        if (pick < 0) return;
      }
    }
    for (int x = f; x < f + 3; x++) set_state(S, x, chosen);
    prev = chosen;
  }
}

static void s_pair(Samp *S, int i, int j, int s, int s2) {
  const Model *M = S->M;
  const Arrays *A = S->A;
  set_state(S, i, s);
  set_state(S, j, s2);
  S->pairs[i] = j;
  S->pairs[j] = i;
  int t = ptype(M->nt[i][s], M->nt[j][s2]);
  int L = j - i - 1, d1 = M->d[i + 1], dm = M->d[j - 1];
  /* decision 1: which loop (k ascending, then l descending) */
  int kind = -1, ck = 0, cl = 0;
  {
    long pick = -1;
    for (int pass = 0; pass < 2 && kind < 0; pass++) {
      long idx = 0;
      /* hairpin */
      {
        double bh = hairpin_B(M, L), w = 0;
        const double *u = CELL(A->U, i + 1, j - 1);
        for (int a = 0; a < d1; a++)
          for (int b = 0; b < dm; b++)
            w += M->e[i][s][a] * u[a * 6 + b] * M->e[j - 1][b][s2] *
                 M->Bmm[M->nt[i + 1][a]][M->nt[j - 1][b]][t];
        if (pass == 0) put(S, idx, bh * w);
        else if (idx == pick) kind = 0;
        idx++;
      }
      for (int l1 = 0; l1 <= MAXLOOP && kind < 0; l1++)
        for (int l2 = 0; l1 + l2 <= MAXLOOP && kind < 0; l2++) {
          int k = i + 1 + l1, l = j - 1 - l2;
          if (l - k < 4) continue;
          const double *q = CELL(A->Qb, k, l);
          double w = 0;
          if (l1 == 0 && l2 == 0) {
            for (int x = 0; x < d1; x++)
              for (int y = 0; y < dm; y++) {
                int t2 = ptype(M->nt[k][x], M->nt[l][y]);
                if (t2 < 0) continue;
                w += M->e[i][s][x] * q[x * 6 + y] * M->e[j - 1][y][s2] * M->Bst[t][t2];
              }
          } else if (l2 == 0) {
            const double *ul = CELL(A->U, i + 1, k - 1);
            for (int a = 0; a < d1; a++)
              for (int b = 0; b < M->d[k - 1]; b++)
                for (int x = 0; x < M->d[k]; x++)
                  for (int y = 0; y < M->d[l]; y++)
                    w += M->e[i][s][a] * ul[a * 6 + b] * M->e[k - 1][b][x] * q[x * 6 + y] *
                         M->e[j - 1][y][s2];
            w *= M->Bbu[l1];
          } else if (l1 == 0) {
            const double *ur = CELL(A->U, l + 1, j - 1);
            for (int x = 0; x < M->d[k]; x++)
              for (int y = 0; y < M->d[l]; y++)
                for (int c = 0; c < M->d[l + 1]; c++)
                  for (int dd = 0; dd < dm; dd++)
                    w += M->e[i][s][x] * q[x * 6 + y] * M->e[l][y][c] * ur[c * 6 + dd] *
                         M->e[j - 1][dd][s2];
            w *= M->Bbu[l2];
          } else {
            const double *ul = CELL(A->U, i + 1, k - 1), *ur = CELL(A->U, l + 1, j - 1);
            const double *dI = CELL(A->DI, k, l);
            for (int a = 0; a < d1; a++)
              for (int b = 0; b < M->d[k - 1]; b++)
                for (int c = 0; c < M->d[l + 1]; c++)
                  for (int dd = 0; dd < dm; dd++)
                    w += M->e[i][s][a] * ul[a * 6 + b] * dI[b * 6 + c] * ur[c * 6 + dd] *
                         M->e[j - 1][dd][s2] * M->Bmm[M->nt[i + 1][a]][M->nt[j - 1][dd]][t];
            w *= M->Bin[l1 + l2];
          }
          if (pass == 0) put(S, idx, w);
          else if (idx == pick) { kind = 1; ck = k; cl = l; }
          idx++;
        }
      if (kind < 0) {
        const double *qx = CELL(A->QmX, i + 1, j - 1);
        double w = 0;
        for (int x = 0; x < d1; x++)
          for (int y = 0; y < dm; y++) w += M->e[i][s][x] * qx[x * 6 + y] * M->e[j - 1][y][s2];
        if (pass == 0) put(S, idx, M->Bmla_b * w);
        else if (idx == pick) kind = 2;
        idx++;
      }
      if (pass == 0) {
        pick = choose(S, idx);
        if (pick < 0) return;
      }
    }
  }
  /* decision 2: slots of the loop's inner boundary positions */
  long pick = -1;
  if (kind == 0) {
    const double *u = CELL(A->U, i + 1, j - 1);
    for (int pass = 0; pass < 2; pass++) {
      long idx = 0;
      for (int a = 0; a < d1; a++)
        for (int b = 0; b < dm; b++)
          ALT(M->e[i][s][a] * u[a * 6 + b] * M->e[j - 1][b][s2] *
                  M->Bmm[M->nt[i + 1][a]][M->nt[j - 1][b]][t],
              push(S, F_RUN, i + 1, j - 1, a, b));
      DECIDE
    }
  } else if (kind == 2) {
    const double *qx = CELL(A->QmX, i + 1, j - 1);
    for (int pass = 0; pass < 2; pass++) {
      long idx = 0;
      for (int x = 0; x < d1; x++)
        for (int y = 0; y < dm; y++)
          ALT(M->e[i][s][x] * qx[x * 6 + y] * M->e[j - 1][y][s2],
              push(S, F_MX, i + 1, j - 1, x, y));
      DECIDE
    }
  } else {
    int k = ck, l = cl, l1 = k - i - 1, l2 = j - l - 1;
    const double *q = CELL(A->Qb, k, l);
    if (l1 == 0 && l2 == 0) {
      for (int pass = 0; pass < 2; pass++) {
        long idx = 0;
        for (int x = 0; x < d1; x++)
          for (int y = 0; y < dm; y++) {
            int t2 = ptype(M->nt[k][x], M->nt[l][y]);
            double w = t2 < 0 ? 0.0
                              : M->e[i][s][x] * q[x * 6 + y] * M->e[j - 1][y][s2] * M->Bst[t][t2];
            ALT(w, push(S, F_B, k, l, x, y));
          }
        DECIDE
      }
    } else if (l2 == 0) {
      const double *ul = CELL(A->U, i + 1, k - 1);
      for (int pass = 0; pass < 2; pass++) {
        long idx = 0;
        for (int a = 0; a < d1; a++)
          for (int b = 0; b < M->d[k - 1]; b++)
            for (int x = 0; x < M->d[k]; x++)
              for (int y = 0; y < M->d[l]; y++)
                ALT(M->e[i][s][a] * ul[a * 6 + b] * M->e[k - 1][b][x] * q[x * 6 + y] *
                        M->e[j - 1][y][s2],
                    { push(S, F_B, k, l, x, y); push(S, F_RUN, i + 1, k - 1, a, b); });
        DECIDE
      }
    } else if (l1 == 0) {
      const double *ur = CELL(A->U, l + 1, j - 1);
      for (int pass = 0; pass < 2; pass++) {
        long idx = 0;
        for (int x = 0; x < M->d[k]; x++)
          for (int y = 0; y < M->d[l]; y++)
            for (int c = 0; c < M->d[l + 1]; c++)
              for (int dd = 0; dd < dm; dd++)
                ALT(M->e[i][s][x] * q[x * 6 + y] * M->e[l][y][c] * ur[c * 6 + dd] *
                        M->e[j - 1][dd][s2],
                    { push(S, F_RUN, l + 1, j - 1, c, dd); push(S, F_B, k, l, x, y); });
        DECIDE
      }
    } else {
      /* interior loop: first the four run-end slots, then the inner pair */
      const double *ul = CELL(A->U, i + 1, k - 1), *ur = CELL(A->U, l + 1, j - 1);
      const double *dI = CELL(A->DI, k, l);
      int ca = -1, cb = -1, cc = -1, cd = -1;
      for (int pass = 0; pass < 2 && ca < 0; pass++) {
        long idx = 0;
        for (int a = 0; a < d1 && ca < 0; a++)
          for (int b = 0; b < M->d[k - 1] && ca < 0; b++)
            for (int c = 0; c < M->d[l + 1] && ca < 0; c++)
              for (int dd = 0; dd < dm; dd++) {
                double w = M->e[i][s][a] * ul[a * 6 + b] * dI[b * 6 + c] * ur[c * 6 + dd] *
                           M->e[j - 1][dd][s2] * M->Bmm[M->nt[i + 1][a]][M->nt[j - 1][dd]][t];
                if (pass == 0) put(S, idx, w);
                else if (idx == pick) { ca = a; cb = b; cc = c; cd = dd; break; }
                idx++;
              }
        DECIDE
      }
      pick = -1;
      for (int pass = 0; pass < 2; pass++) {
        long idx = 0;
        for (int x = 0; x < M->d[k]; x++)
          for (int y = 0; y < M->d[l]; y++) {
            int t2 = ptype(M->nt[l][y], M->nt[k][x]);
#ifdef PLANT_SAMPLER_BULGE
            double w = t2 < 0 ? 0.0 : M->e[k - 1][cb][x] * q[x * 6 + y] * M->e[l][y][cc];
#else
            double w = t2 < 0 ? 0.0
                              : M->e[k - 1][cb][x] * q[x * 6 + y] * M->e[l][y][cc] *
                                    M->Bmm[M->nt[l + 1][cc]][M->nt[k - 1][cb]][t2];
#endif
            ALT(w, {
              push(S, F_RUN, l + 1, j - 1, cc, cd);
              push(S, F_B, k, l, x, y);
              push(S, F_RUN, i + 1, k - 1, ca, cb);
            });
          }
        DECIDE
      }
    }
  }
}

/* QmX splits; with_m1p also lists the Qm1p alternative (the Qm fragment) */
static void s_split(Samp *S, int i, int j, int s, int s2, int with_m1p) {
  const Model *M = S->M;
  const Arrays *A = S->A;
  long pick = -1;
  for (int pass = 0; pass < 2; pass++) {
    long idx = 0;
    for (int u = i + 5; u <= j - 4; u++) {
      const double *qm = CELL(A->Qm, i, u - 1), *q1 = CELL(A->Qm1, u, j);
      for (int t = 0; t < M->d[u - 1]; t++)
        for (int t2 = 0; t2 < M->d[u]; t2++)
          ALT(qm[s * 6 + t] * M->e[u - 1][t][t2] * q1[t2 * 6 + s2],
              { push(S, F_M1, u, j, t2, s2); push(S, F_M, i, u - 1, s, t); });
    }
    if (with_m1p) ALT(CELL(A->Qm1p, i, j)[s * 6 + s2], push(S, F_M1P, i, j, s, s2));
    DECIDE
  }
}

static void s_m1(Samp *S, int i, int j, int s, int s2) {
  const Model *M = S->M;
  const Arrays *A = S->A;
  set_state(S, i, s);
  set_state(S, j, s2);
  long pick = -1;
  for (int pass = 0; pass < 2; pass++) {
    long idx = 0;
    ALT(CELL(A->Qb, i, j)[s * 6 + s2] * M->Bmlb, push(S, F_B, i, j, s, s2));
    const double *q1 = CELL(A->Qm1, i, j - 1);
    for (int t = 0; t < M->d[j - 1]; t++)
      ALT(q1[s * 6 + t] * M->e[j - 1][t][s2] * M->v[j][s2] * M->Bmlc,
          push(S, F_M1, i, j - 1, s, t));
    DECIDE
  }
}

static void s_m1p(Samp *S, int i, int j, int s, int s2) {
  const Model *M = S->M;
  const Arrays *A = S->A;
  set_state(S, i, s);
  set_state(S, j, s2);
  long pick = -1;
  for (int pass = 0; pass < 2; pass++) {
    long idx = 0;
    ALT(CELL(A->Qm1, i, j)[s * 6 + s2], push(S, F_M1, i, j, s, s2));
    const double *qp = CELL(A->Qm1p, i + 1, j);
    for (int t = 0; t < M->d[i + 1]; t++)
      ALT(M->v[i][s] * M->Bmlc * M->e[i][s][t] * qp[t * 6 + s2],
          push(S, F_M1P, i + 1, j, t, s2));
    DECIDE
  }
}

/* codons [nsamp][m] (slot indices), pairs [nsamp][n] (partner or -1) */
int orc_sample(int m, const char *aa, const double *theta1, const double *theta2,
               const double *energy, uint64_t seed, int nsamp, uint8_t *codons,
               int32_t *pairs) {
  if (m < 1 || !aa || !energy || nsamp < 0 || (nsamp > 0 && (!codons || !pairs))) return -1;
  Model Mo;
  Arrays A;
  double Z;
  int rc = setup_forward(m, aa, theta1, theta2, (const orc_energy *)energy, 0, &Mo, &A, &Z);
  if (rc) return rc;
  const Model *M = &Mo;
  int n = M->n;
  Samp S;
  memset(&S, 0, sizeof(S));
  S.M = M;
  S.A = &A;
  S.seed = seed;
  S.state = malloc(sizeof(int) * n);
  for (int k = 0; k < nsamp && !rc; k++) {
    S.sid = (uint32_t)k;
    S.draw = 0;
    S.top = 0;
    S.err = 0;
    S.pairs = pairs + (size_t)k * n;
    for (int p = 0; p < n; p++) {
      S.state[p] = -1;
      S.pairs[p] = -1;
    }
    /* slot of the last position */
    {
      Samp *Sp = &S;
      long idx = 0;
      for (int t = 0; t < M->d[n - 1]; t++) put(Sp, idx++, A.Z5[(size_t)(n - 1) * NS + t]);
      long pick = choose(Sp, idx);
      if (pick < 0) { rc = -4; break; }
      push(Sp, F_EXT, n - 1, 0, (int)pick, 0);
    }
    while (S.top > 0 && !S.err) {
      Frag f = S.stk[--S.top];
      switch (f.kind) {
        case F_EXT: s_ext(&S, f.i, f.s); break;
        case F_B: s_pair(&S, f.i, f.j, f.s, f.t); break;
        case F_M1: s_m1(&S, f.i, f.j, f.s, f.t); break;
        case F_M1P: s_m1p(&S, f.i, f.j, f.s, f.t); break;
        case F_MX: s_split(&S, f.i, f.j, f.s, f.t, 0); break;
        case F_M: s_split(&S, f.i, f.j, f.s, f.t, 1); break;
        case F_RUN: s_run(&S, f.i, f.j, f.s, f.t); break;
      }
    }
    if (S.err) { rc = -5; break; }
    for (int a = 0; a < m; a++) {
      int s0 = S.state[3 * a];
      if (s0 < 0 || S.state[3 * a + 1] != s0 || S.state[3 * a + 2] != s0) { rc = -6; break; }
      codons[(size_t)k * m + a] = (uint8_t)s0;
    }
  }
  free(S.state);
  free(S.stk);
  free(S.buf);
  model_free(&Mo);
  arrays_free(&A);
  return rc;
}
