/*
 * seqmcc.c -- single-sequence McCaskill partition function, FP64.
 *
 * TEST INFRASTRUCTURE ONLY (a pin for the codon-constrained oracle).  It
 * evaluates the same nearest-neighbour loop model as oracle.c for ONE fixed
 * RNA sequence, written independently and in a different decomposition:
 * multiloop segments carry explicit powers of the unpaired-base factor
 * instead of a recursive unpaired prefix, and there are no codon slots.
 * Summing W(c) * Z(phi(c)) over every codon assignment c reproduces the
 * amino-acid partition function of eq. amino-q (paper Section 2b) by its
 * definition, and a protein whose every residue has one codon reduces design
 * to analysis of one sequence (Sections 3b vs 3c).
 *
 * Bases A=0 C=1 G=2 U=3; pairs AU CG GC UA GU UG (types 0..5).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  double stack[6][6];
  double hairpin[31];
  double bulge[31];
  double interior[31];
  double mismatch[4][4][6];
  double ml_a, ml_b, ml_c, extrap;
} seq_energy;

static int seq_pair(int x, int y) {
  if (x == 0 && y == 3) return 0;
  if (x == 1 && y == 2) return 1;
  if (x == 2 && y == 1) return 2;
  if (x == 3 && y == 0) return 3;
  if (x == 2 && y == 3) return 4;
  if (x == 3 && y == 2) return 5;
  return -1;
}

/* free energy (kT) of the loop closed by (i,j) with inner pair (k,l) */
static double e_two_loop(const seq_energy *E, const int *s, int i, int j, int k, int l) {
  int l1 = k - i - 1, l2 = j - l - 1;
  int t = seq_pair(s[i], s[j]);
  if (l1 == 0 && l2 == 0) return E->stack[t][seq_pair(s[k], s[l])];
  if (l1 == 0 || l2 == 0) return E->bulge[l1 + l2];
  return E->interior[l1 + l2] + E->mismatch[s[i + 1]][s[j - 1]][t] +
         E->mismatch[s[l + 1]][s[k - 1]][seq_pair(s[l], s[k])];
}

static double e_hairpin(const seq_energy *E, const int *s, int i, int j) {
  int L = j - i - 1;
  double h = (L <= 30) ? E->hairpin[L] : E->hairpin[30] + E->extrap * log(L / 30.0);
  return h + E->mismatch[s[i + 1]][s[j - 1]][seq_pair(s[i], s[j])];
}

/* log Z of sequence s[0..n); if fi >= 0 the pair (fi, fj) is forbidden. */
double seq_logz(int n, const int *s, const double *energy, int fi, int fj) {
  const seq_energy *E = (const seq_energy *)energy;
  if (n <= 0 || n > 400) return NAN;
  size_t N = (size_t)n;
  double *QB = calloc(N * N, sizeof(double));
  double *QM1 = calloc(N * N, sizeof(double));
  double *QM = calloc(N * N, sizeof(double));
  double *Z5 = calloc(N + 1, sizeof(double)); /* Z5[j+1]: prefix [0..j] */
  double c = exp(-E->ml_c), b = exp(-E->ml_b), ab = exp(-(E->ml_a + E->ml_b));
#define at(X, i, j) X[(size_t)(i) * N + (j)]
  for (int d = 4; d < n; d++)
    for (int i = 0; i + d < n; i++) {
      int j = i + d;
      double qb = 0;
      if (seq_pair(s[i], s[j]) >= 0 && !(i == fi && j == fj)) {
        qb = exp(-e_hairpin(E, s, i, j));
        for (int k = i + 1; k <= i + 31 && k < j; k++)
          for (int l = j - 1; l > k + 3; l--) {
            int sz = (k - i - 1) + (j - l - 1);
            if (sz > 30) break;
            if (at(QB, k, l) == 0.0) continue;
            qb += exp(-e_two_loop(E, s, i, j, k, l)) * at(QB, k, l);
          }
        double ml = 0;
        for (int u = i + 6; u <= j - 5; u++) ml += at(QM, i + 1, u - 1) * at(QM1, u, j - 1);
        qb += ab * ml;
      }
      at(QB, i, j) = qb;
      /* QM1[i][j]: pair (i, l) with l <= j, then j-l unpaired bases */
      double q1 = 0;
      for (int l = i + 4; l <= j; l++) q1 += at(QB, i, l) * b * pow(c, j - l);
      at(QM1, i, j) = q1;
      /* QM[i][j]: >= 1 branch; last branch starts at u */
      double qm = 0;
      for (int u = i; u <= j - 4; u++) {
        double left = pow(c, u - i) + (u - 1 >= i ? at(QM, i, u - 1) : 0.0);
        qm += left * at(QM1, u, j);
      }
      at(QM, i, j) = qm;
    }
  Z5[0] = 1.0;
  for (int j = 0; j < n; j++) {
    double z = Z5[j];
    for (int k = 0; k + 4 <= j; k++) z += Z5[k] * at(QB, k, j);
    Z5[j + 1] = z;
  }
  double r = log(Z5[n]);
#undef at
  free(QB);
  free(QM1);
  free(QM);
  free(Z5);
  return r;
}

/* Energy (kT) of one structure by loop decomposition; pt[i] = partner or -1.
 * Returns +inf for a structure the model forbids. */
double seq_energy_eval(int n, const int *s, const int *pt, const double *energy) {
  const seq_energy *E = (const seq_energy *)energy;
  double tot = 0;
  for (int i = 0; i < n; i++) {
    int j = pt[i];
    if (j <= i) continue;
    if (seq_pair(s[i], s[j]) < 0) return INFINITY;
    /* children of (i, j) and unpaired count */
    int nb = 0, unp = 0, ck = -1, cl = -1;
    for (int k = i + 1; k < j; k++) {
      if (pt[k] > k) {
        nb++;
        ck = k;
        cl = pt[k];
        k = pt[k];
      } else {
        unp++;
      }
    }
    if (nb == 0) {
      if (j - i - 1 < 3) return INFINITY;
      tot += e_hairpin(E, s, i, j);
    } else if (nb == 1) {
      int sz = (ck - i - 1) + (j - cl - 1);
      if (sz > 30) return INFINITY;
      tot += e_two_loop(E, s, i, j, ck, cl);
    } else {
      tot += E->ml_a + E->ml_b * (nb + 1) + E->ml_c * unp;
    }
  }
  return tot;
}
