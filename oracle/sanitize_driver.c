/*
 * sanitize_driver.c -- runs the oracle's entry points once on a problem read
 * from a file, for a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * (tests/test_oracle_sanitized.py).  TEST INFRASTRUCTURE ONLY.
 *
 * Input file (native doubles): 229 energy values, then theta1 [m][6], then
 * theta2 [m][6][6].  Arguments: <file> <protein letters> <samples>.
 * Prints log Z from the forward call and from the marginal call.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int orc_logz(int m, const char *aa, const double *theta1, const double *theta2, const double *energy,
             double *logz);
int orc_marginals(int m, const char *aa, const double *theta1, const double *theta2, const double *energy,
                  double *logz, double *pair, double *base, double *codon, double *codon_pair, double *vcheck,
                  double *echeck);
int orc_sample(int m, const char *aa, const double *theta1, const double *theta2, const double *energy,
               uint64_t seed, int nsamp, uint8_t *codons, int32_t *pairs);

int main(int argc, char **argv) {
  if (argc != 4) return 2;
  const char *aa = argv[2];
  const int m = (int)strlen(aa), n = 3 * m, ns = atoi(argv[3]);
  const size_t count = 229 + (size_t)m * 6 + (size_t)m * 36;
  double *buf = malloc(count * sizeof(double));
  FILE *f = fopen(argv[1], "rb");
  if (!f || !buf || fread(buf, sizeof(double), count, f) != count) return 3;
  fclose(f);
  const double *en = buf, *t1 = buf + 229, *t2 = buf + 229 + m * 6;
  double lz1 = 0, lz2 = 0;
  double *pair = calloc((size_t)n * n, sizeof(double)), *base = calloc((size_t)n * 4, sizeof(double));
  double *cod = calloc((size_t)m * 6, sizeof(double)), *cp = calloc((size_t)m * 36, sizeof(double));
  double *vchk = calloc((size_t)n, sizeof(double)), *echk = calloc((size_t)n, sizeof(double));
  uint8_t *sc = calloc((size_t)(ns > 0 ? ns : 1) * m, 1);
  int32_t *sp = calloc((size_t)(ns > 0 ? ns : 1) * n, sizeof(int32_t));
  int rc = orc_logz(m, aa, t1, t2, en, &lz1);
  if (rc == 0) rc = orc_marginals(m, aa, t1, t2, en, &lz2, pair, base, cod, cp, vchk, echk);
  if (rc == 0) rc = orc_sample(m, aa, t1, t2, en, 12345u, ns, sc, sp);
  printf("%.17g %.17g %d\n", lz1, lz2, rc);
  free(buf);
  free(pair);
  free(base);
  free(cod);
  free(cp);
  free(vchk);
  free(echk);
  free(sc);
  free(sp);
  return rc == 0 ? 0 : 1;
}
