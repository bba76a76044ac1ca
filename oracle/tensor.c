/*
 * tensor.c -- oracle of the sequence-summed free energy under a tensor-based
 * secondary-structure model (the paper's own workload: Sections 3b-3c and
 * SI S2b-S2c, S4a).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/, the stored-value script under
 * tests/golden/ and the benchmark's CPU baseline; nothing on the product path
 * calls it, and it shares no code, table or header with the HIP library.
 *
 * The model (SI S2b): per base b a matrix V_b (gamma x gamma), per ordered
 * base pair (x, y) and rank index rho < xi a matrix B^rho_{x,y}, and a matrix
 * S giving the weighted trace Tr_S[X] = Tr[S X].  For one sequence phi and
 * structure s, every loop contributes Tr_S of the product of the matrices met
 * along its backbone (V for an unpaired base, B_{k,l} for base k paired to
 * the next base l of the loop), summed over one rho per pair shared by both of
 * its sides (eq. general-model).
 *
 * The codon constraint is the single-codon tensor train of Section 3a
 * (eq. single-tt) with a per-codon bonus exp(theta1) on the middle core (the
 * CAI-style soft constraint of Section 3a): dimensions Sigma_p = 1 at codon
 * starts, the number of distinct first bases after a codon start, the number
 * of distinct third bases before a codon end.
 *
 * What is computed: Alg. complex-pf on the flattened block matrix Q (rows and
 * columns grouped (sigma, zeta), sigma-major), with the folding function of
 * eq. design-fold:
 *     upper blocks  Q_{i,j} = sum_{k in [i, j)} Q_{i,k} E_{k,j}        (i < j)
 *     lower blocks  Q_{j,k} = E_{k,j}^T, the fold of the element on [k, j):
 *       k = j-1:  sum_phi T_{j-1}^phi (x) V_phi                 (unpaired base)
 *       j-1-k >= 4:  sum over phi_k, phi_l, rho, sigma_b, sigma_e of
 *           T_k^{phi_k}[., sigma_b] t[sigma_b, sigma_e] T_l^{phi_l}[sigma_e, .]
 *           (x) B^rho_{phi_k, phi_l},
 *         t[sigma_b, sigma_e] = Tr[S B^rho_{phi_l, phi_k} X^{sigma_b, sigma_e}],
 *         X = Q_{k+1, l}, l = j-1                                (pair k.l)
 *       otherwise 0 (no hairpin of fewer than three bases),
 *     diagonal blocks Q_{i,i} = identity,
 *     Z = Tr_{I (x) S}[Q_{0,n}]  (eq. complex-logq; Sigma_0 = Sigma_n = 1).
 * Alg. complex-pf's fold argument reads Q_{j+1,i-1}; Alg. fast-pf and the
 * recursion of SI S2c read the inner interval Q_{i+1,j-1}, which is the one
 * taken here.
 *
 * Renormalization (Alg. fast-pf): each new column j is divided by a positive
 * factor h_{j-1}, here the largest entry of its row-0 block, so that the
 * prefix block keeps unit scale; the folds then divide by the factor of their
 * first position, and log Z adds sum log h.  Any positive choice leaves Z
 * unchanged.
 *
 * Prefix values: at every codon boundary j = 3a (Sigma_j = 1), Tr_S[Q_{0,j}]
 * is the partition function of the first a residues, returned as prefix[a-1].
 *
 * The PLANT_TENSOR_* switches exist only for tests/test_oracle_tensor.py,
 * which builds each into a throwaway library and checks that a pin breaks.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static const char TCODE[] =
    "KNKNTTTTRSRSIIMIQHQHPPPPRRRRLLLLEDEDAAAAGGGGVVVV*Y*YSSSS*CWCLFLF";

typedef struct {
  int n, g, xi;
  int *sig;      /* [n+1] tensor-train bond dimensions */
  size_t *off;   /* [n+1] first flattened row/column of each position */
  size_t N;      /* flattened size */
  double *T;     /* [n][4][4][4]: core p, base, sigma_a, sigma_b */
} TtModel;

#define TT(M, p, phi, a, b) ((M)->T[(((size_t)(p) * 4 + (phi)) * 4 + (a)) * 4 + (b)])

static int tt_build(TtModel *M, int m, const char *aa, const double *theta1, int g, int xi) {
  memset(M, 0, sizeof(*M));
  M->n = 3 * m;
  M->g = g;
  M->xi = xi;
  const int n = M->n;
  M->sig = calloc(n + 1, sizeof(int));
  M->off = calloc(n + 1, sizeof(size_t));
  M->T = calloc((size_t)n * 64, sizeof(double));
  if (!M->sig || !M->off || !M->T) return -1;
  for (int a = 0; a < m; a++) {
    int cod[6], cnt = 0;
    for (int c = 0; c < 64; c++)
      if (TCODE[c] == aa[a] && aa[a] != '*') cod[cnt++] = c;
    if (cnt == 0) return -2;
    int fb[4], nf = 0, tb[4], nt = 0;
    for (int b = 0; b < 4; b++) {
      int hf = 0, ht = 0;
      for (int s = 0; s < cnt; s++) {
        hf |= (cod[s] >> 4) == b;
        ht |= (cod[s] & 3) == b;
      }
      if (hf) fb[nf++] = b;
      if (ht) tb[nt++] = b;
    }
    const int p = 3 * a;
    M->sig[p] = 1;
    M->sig[p + 1] = nf;
    M->sig[p + 2] = nt;
    for (int x = 0; x < nf; x++) TT(M, p, fb[x], 0, x) = 1.0;
    for (int s = 0; s < cnt; s++) {
      const int c = cod[s], x0 = c >> 4, mid = (c >> 2) & 3, x2 = c & 3;
      int x = 0, y = 0;
      while (fb[x] != x0) x++;
      while (tb[y] != x2) y++;
      TT(M, p + 1, mid, x, y) += theta1 ? exp(theta1[a * 6 + s]) : 1.0;
    }
    for (int y = 0; y < nt; y++) TT(M, p + 2, tb[y], y, 0) = 1.0;
  }
  M->sig[n] = 1;
  size_t o = 0;
  for (int p = 0; p <= n; p++) {
    M->off[p] = o;
    o += (size_t)g * M->sig[p];
  }
  M->N = o;
  return 0;
}

static void tt_free(TtModel *M) {
  free(M->sig);
  free(M->off);
  free(M->T);
}

/* element (r, c) of the fold block E_{k,j} is stored at Q[off[j] + c][off[k] + r] */
static void fold_column(const TtModel *M, double *Q, int j, const double *V, const double *B, const double *S,
                        const double *h) {
  const int g = M->g, xi = M->xi;
  const size_t N = M->N;
#pragma omp parallel for schedule(dynamic, 8)
  for (int k = 0; k < j; k++) {
    const int sk = M->sig[k], sj = M->sig[j];
    const int R = g * sk, Cc = g * sj;
    double *E = calloc((size_t)R * Cc, sizeof(double));
    if (k == j - 1) {
      for (int phi = 0; phi < 4; phi++)
        for (int a = 0; a < sk; a++)
          for (int b = 0; b < sj; b++) {
            const double t = TT(M, k, phi, a, b);
            if (t == 0.0) continue;
            for (int za = 0; za < g; za++)
              for (int zb = 0; zb < g; zb++)
                E[(size_t)(a * g + za) * Cc + b * g + zb] += t * V[(phi * g + za) * g + zb];
          }
#ifdef PLANT_TENSOR_HAIRPIN
    } else if (j - 1 - k >= 3) {
#else
    } else if (j - 1 - k >= 4) {
#endif
      const int l = j - 1, sb = M->sig[k + 1], se = M->sig[l];
      const size_t r0 = M->off[k + 1], c0 = M->off[l];
      double *t = malloc((size_t)sb * se * sizeof(double));
      double *SB = malloc((size_t)g * g * sizeof(double));
      for (int rho = 0; rho < xi; rho++)
        for (int pk = 0; pk < 4; pk++)
          for (int pl = 0; pl < 4; pl++) {
#ifdef PLANT_TENSOR_INNER_ORDER
            const double *Bin = B + ((((size_t)rho * 4 + pk) * 4 + pl) * g) * g;
#else
            const double *Bin = B + ((((size_t)rho * 4 + pl) * 4 + pk) * g) * g;  /* B^rho_{phi_l, phi_k} */
#endif
            const double *Bout = B + ((((size_t)rho * 4 + pk) * 4 + pl) * g) * g; /* B^rho_{phi_k, phi_l} */
            /* S B_in */
            for (int x = 0; x < g; x++)
              for (int y = 0; y < g; y++) {
                double acc = 0.0;
                for (int z = 0; z < g; z++) acc += S[x * g + z] * Bin[z * g + y];
                SB[x * g + y] = acc;
              }
            /* t[sigma_b][sigma_e] = Tr[S B_in X^{sigma_b, sigma_e}] */
            for (int b = 0; b < sb; b++)
              for (int e = 0; e < se; e++) {
                double acc = 0.0;
                for (int x = 0; x < g; x++)
                  for (int y = 0; y < g; y++) acc += SB[x * g + y] * Q[(r0 + b * g + y) * N + c0 + e * g + x];
                t[b * se + e] = acc;
              }
            /* (T_k t T_l)[sigma_k][sigma_j] (x) B_out */
            for (int a = 0; a < sk; a++)
              for (int c = 0; c < sj; c++) {
                double u = 0.0;
                for (int b = 0; b < sb; b++)
                  for (int e = 0; e < se; e++)
                    u += TT(M, k, pk, a, b) * t[b * se + e] * TT(M, l, pl, e, c);
                if (u == 0.0) continue;
                for (int za = 0; za < g; za++)
                  for (int zb = 0; zb < g; zb++)
                    E[(size_t)(a * g + za) * Cc + c * g + zb] += u * Bout[za * g + zb];
              }
          }
      /* the inner block carries the scale of positions k+1..l-1 (the column
       * factors already applied), the element spans k..l: divide by h_k */
#ifndef PLANT_TENSOR_SCALE
      for (size_t q = 0; q < (size_t)R * Cc; q++) E[q] /= h[k];
#endif
      free(t);
      free(SB);
    }
    for (int r = 0; r < R; r++)
      for (int c = 0; c < Cc; c++) Q[(M->off[j] + c) * N + M->off[k] + r] = E[(size_t)r * Cc + c];
    free(E);
  }
}

int orc_tensor_logz(int m, const char *aa, const double *theta1, int g, int xi, const double *V, const double *B,
                    const double *S, double *logz, double *prefix) {
  if (m < 1 || !aa || g < 1 || xi < 1 || !V || !B || !S || !logz) return -1;
  TtModel M;
  int rc = tt_build(&M, m, aa, theta1, g, xi);
  if (rc != 0) {
    tt_free(&M);
    return rc;
  }
  const int n = M.n;
  const size_t N = M.N;
  double *Q = calloc(N * N, sizeof(double));
  double *h = calloc(n, sizeof(double));
  if (!Q || !h) {
    free(Q);
    free(h);
    tt_free(&M);
    return -1;
  }
  for (size_t r = 0; r < N; r++) Q[r * N + r] = 1.0; /* diagonal blocks: identity */
  double logscale = 0.0;
  for (int j = 1; j <= n; j++) {
    fold_column(&M, Q, j, V, B, S, h);
    /* propagation: Q_{i,j} = sum_{k in [i, j)} Q_{i,k} E_{k,j} for every row of blocks i < j */
    const size_t cj = M.off[j], w = (size_t)g * M.sig[j];
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < j; i++)
      for (size_t r = M.off[i]; r < M.off[i + 1]; r++)
        for (size_t c = 0; c < w; c++) {
          double acc = 0.0;
          for (size_t kk = M.off[i]; kk < cj; kk++) acc += Q[r * N + kk] * Q[(cj + c) * N + kk];
          Q[r * N + cj + c] = acc;
        }
    /* renormalization of the new column by its row-0 block's largest entry */
    double hm = 0.0;
    for (size_t r = 0; r < (size_t)g; r++)
      for (size_t c = 0; c < w; c++) hm = fmax(hm, Q[r * N + cj + c]);
    if (!(hm > 0.0) || !isfinite(hm)) {
      rc = -4;
      break;
    }
    h[j - 1] = hm;
    logscale += log(hm);
    for (size_t r = 0; r < cj; r++)
      for (size_t c = 0; c < w; c++) Q[r * N + cj + c] /= hm;
    if (j % 3 == 0) {
      double tr = 0.0;
      for (int x = 0; x < g; x++)
        for (int y = 0; y < g; y++) tr += S[x * g + y] * Q[(size_t)y * N + cj + x];
      const double lz = log(tr) + logscale;
      if (prefix) prefix[j / 3 - 1] = lz;
      if (j == n) *logz = lz;
    }
  }
  free(Q);
  free(h);
  tt_free(&M);
  return rc;
}

/* bond dimensions Sigma_p (p = 0..n) of the single-codon tensor train */
int orc_tensor_dims(int m, const char *aa, int *sig) {
  TtModel M;
  int rc = tt_build(&M, m, aa, NULL, 1, 1);
  if (rc == 0)
    for (int p = 0; p <= M.n; p++) sig[p] = M.sig[p];
  tt_free(&M);
  return rc;
}
