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

// FP64 exterior loop, one step each way (see the host-side description):
//   Z5[j](t) = prefix [0..j] with slot t at j
//   Z3[p](s) = suffix [p+1..n-1] given slot s at p, edge e_p included
template <typename T>
__device__ void exterior_step(const DevProb<T> &D, int dl, const int *sE, double *red) {
  const int n = D.n, tid = threadIdx.x;
  const long long ld = D.ld;
  // ---- prefix Z5[j], j = dl - 1
  int j = dl - 1;
  if (j == 0) {
    if (tid < 6) D.Z5[tid] = tid < D.d[0] ? D.vd[tid] : 0.0;
    if (tid == 0) D.G5[0] = 0;
  } else if (j > 0 && j < n) {
    const int R = D.G5[j - 1], dj = D.d[j], Pj = D.P[j];
    double part[6] = {0, 0, 0, 0, 0, 0};
    for (int k = 1 + tid; k <= j - 4; k += CDZ_NT) {
      const int dk = D.d[k], dk1 = D.d[k - 1], Pk = D.P[k];
      const double sc = ldexp(1.0, D.G5[k - 1] + sE[j - k] - R);
      double zl[6];
#pragma unroll
      for (int x = 0; x < 6; x++) {
        double a = 0;
        if (x < dk)
          for (int s = 0; s < dk1; s++) a += D.Z5[(k - 1) * 6 + s] * D.ed[(k - 1) * 36 + s * 6 + x];
        zl[x] = a * sc;
      }
#pragma unroll
      for (int t = 0; t < 6; t++) {
        if (t < dj) {
          double a = 0;
#pragma unroll
          for (int x = 0; x < 6; x++)
            if (x < dk) a += zl[x] * (double)D.Qb[(Pk + x) * ld + Pj + t];
          part[t] += a;
        }
      }
    }
    if (tid == 0) {
      const int dp = D.d[j - 1];
      for (int t = 0; t < dj; t++) {
        double a = 0;
        for (int s = 0; s < dp; s++) a += D.Z5[(j - 1) * 6 + s] * D.ed[(j - 1) * 36 + s * 6 + t];
        part[t] += a * D.vd[j * 6 + t];
      }
      if (j >= 4) {
        const double sc = ldexp(1.0, sE[j] - R);
        for (int t = 0; t < dj; t++) {
          double a = 0;
          for (int x = 0; x < D.d[0]; x++) a += (double)D.Qb[x * ld + Pj + t];
          part[t] += a * sc;
        }
      }
    }
    double *tot = red + 4 * 6;  // LDS, after the reduction scratch
    cdz_block_sum<double, 6>(part, red, tot);
    if (tid == 0) {
      double mx = 0;
      for (int t = 0; t < dj; t++) mx = fmax(mx, fabs(tot[t]));
      int e = (mx > 0 && isfinite(mx)) ? ilogb(mx) : 0;
      for (int t = 0; t < 6; t++) D.Z5[j * 6 + t] = t < dj ? ldexp(tot[t], -e) : 0.0;
      D.G5[j] = R + e;
    }
    __syncthreads();
  }
  // ---- suffix Z3[p], p = n - 1 - dl
  int p = n - 1 - dl;
  if (p == n - 1) {
    if (tid < 6) D.Z3[p * 6 + tid] = tid < D.d[p] ? 1.0 : 0.0;
    if (tid == 0) D.H3[p] = 0;
  } else if (p >= 0) {
    const int R = D.H3[p + 1], dp = D.d[p], d1 = D.d[p + 1], P1 = D.P[p + 1];
    double part[6] = {0, 0, 0, 0, 0, 0};
    for (int jj = p + 5 + tid; jj <= n - 1; jj += CDZ_NT) {
      const int dq = D.d[jj], Pq = D.P[jj];
      const double sc = ldexp(1.0, sE[jj - p - 1] + D.H3[jj] - R);
      double w[6];
#pragma unroll
      for (int x = 0; x < 6; x++) {
        double a = 0;
        if (x < d1)
          for (int t = 0; t < dq; t++) a += (double)D.Qb[(P1 + x) * ld + Pq + t] * D.Z3[jj * 6 + t];
        w[x] = a * sc;
      }
#pragma unroll
      for (int s = 0; s < 6; s++)
        if (s < dp) {
          double a = 0;
#pragma unroll
          for (int x = 0; x < 6; x++)
            if (x < d1) a += D.ed[p * 36 + s * 6 + x] * w[x];
          part[s] += a;
        }
    }
    if (tid == 0) {
      for (int s = 0; s < dp; s++) {
        double a = 0;
        for (int t = 0; t < d1; t++)
          a += D.ed[p * 36 + s * 6 + t] * D.vd[(p + 1) * 6 + t] * D.Z3[(p + 1) * 6 + t];
        part[s] += a;
      }
    }
    double *tot = red + 4 * 6;
    cdz_block_sum<double, 6>(part, red, tot);
    if (tid == 0) {
      double mx = 0;
      for (int s = 0; s < dp; s++) mx = fmax(mx, fabs(tot[s]));
      int e = (mx > 0 && isfinite(mx)) ? ilogb(mx) : 0;
      for (int s = 0; s < 6; s++) D.Z3[p * 6 + s] = s < dp ? ldexp(tot[s], -e) : 0.0;
      D.H3[p] = R + e;
    }
    __syncthreads();
  }
  // ---- totals after the last diagonal
  if (dl == n) {
    double part[2] = {0, 0};
    for (int jj = 4 + tid; jj < n; jj += CDZ_NT) {
      // position 0 pairs with jj, suffix after jj
      const int dq = D.d[jj], Pq = D.P[jj];
      double a = 0;
      for (int x = 0; x < D.d[0]; x++)
        for (int t = 0; t < dq; t++) a += (double)D.Qb[x * ld + Pq + t] * D.Z3[jj * 6 + t];
      part[0] += a * ldexp(1.0, sE[jj] + D.H3[jj] - D.H3[0]);
    }
    if (tid == 0)
      for (int s = 0; s < D.d[0]; s++) part[0] += D.vd[s] * D.Z3[s];
    double *tot = red + 4 * 2;
    cdz_block_sum<double, 2>(part, red, tot);
    if (tid == 0) {
      double z5 = 0;
      for (int t = 0; t < D.d[n - 1]; t++) z5 += D.Z5[(n - 1) * 6 + t];
      const double L2 = 0.6931471805599453094;
      double lz5 = log(z5) + D.G5[n - 1] * L2;
      double lz3 = log(tot[0]) + D.H3[0] * L2;
      D.res[0] = lz5;
      D.res[1] = lz3;
      D.res[2] = rint(lz5 / L2);  // EZ, the adjoint scale exponent
    }
  }
}

}  // namespace

template <typename T>
__global__ __launch_bounds__(CDZ_NT) void cdz_fwd_diag(DevProb<T> D, int dl) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  int *sE = reinterpret_cast<int *>(smem_raw);  // [n + 1]
  T *sbuf = reinterpret_cast<T *>(smem_raw + ((size_t)(D.n + 1) * 4 + 15) / 16 * 16);
  T *red = sbuf;                        // (NT/64) * 72
  T *sSplit = red + (CDZ_NT / 64) * 72; // 36
  T *sGF = sSplit + 36;                 // 72 (G then F)
  T *sQb = sGF + 72;                    // 36
  T *sQm1 = sQb + 36;                   // 36
  const int n = D.n, tid = threadIdx.x;
  const long long ld = D.ld;
  for (int k = tid; k < dl && k <= n; k += CDZ_NT) sE[k] = D.E[k];
  __syncthreads();
  const int Ed = choose_exponent(D, dl, sE);
  if (tid == 0) sE[dl] = Ed;
  if (blockIdx.x == 0 && tid == 0) D.E[dl] = Ed;
  __syncthreads();
  const int ncell = n - dl > 0 ? n - dl : 0;
  if ((int)blockIdx.x == ncell) {
    exterior_step<T>(D, dl, sE, reinterpret_cast<double *>(red));
    return;
  }
  const int i = blockIdx.x, j = i + dl;
  const int di = D.d[i], dj = D.d[j], Pi = D.P[i], Pj = D.P[j];
  float vmax = 0.f;

  // ---- unpaired run U[i][j]
  if (tid < 36) {
    const int s = tid / 6, t = tid % 6;
    if (s < di && t < dj) {
      T u = 0;
      if (dl == 0) {
        u = (s == t) ? D.v[i * 6 + s] : T(0);
      } else {
        const int dp = D.d[j - 1], Pp = D.P[j - 1];
        T a = 0;
        for (int c = 0; c < dp; c++) a += D.U[(Pi + s) * ld + Pp + c] * D.e[(j - 1) * 36 + c * 6 + t];
        u = a * D.v[j * 6 + t] * cdz_p2<T>(sE[dl - 1] - Ed);
      }
      D.U[(Pi + s) * ld + Pj + t] = u;
      vmax = fmaxf(vmax, (float)fabs(u));
      if (dl < 4) {
        const long long o = (Pi + s) * ld + Pj + t;
        D.Qb[o] = 0;
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
    //      states of positions i+4 .. j-5 (u - 1 = pos(k))
    {
      T acc[36];
#pragma unroll
      for (int r = 0; r < 36; r++) acc[r] = 0;
      const int K0 = D.P[i + 4], K1 = D.P[j - 4];
      for (int k = K0 + tid; k < K1; k += CDZ_NT) {
        const int p = D.posOf[k];
        const T f = cdz_p2<T>(sE[p - i] + sE[j - p - 1] - Ed);
        T a[6], b[6];
#pragma unroll
        for (int s = 0; s < 6; s++) a[s] = s < di ? D.Qm[(Pi + s) * ld + k] * f : T(0);
#pragma unroll
        for (int t = 0; t < 6; t++) b[t] = t < dj ? D.Qm1Lt[(Pj + t) * ld + k] : T(0);
#pragma unroll
        for (int s = 0; s < 6; s++)
#pragma unroll
          for (int t = 0; t < 6; t++) acc[s * 6 + t] = fma(a[s], b[t], acc[s * 6 + t]);
      }
      cdz_block_sum<T, 36>(acc, red, sSplit);
    }
    // ---- bulge and interior window: G (bulges, outer edges not applied),
    //      F (interior loops, outer edges and outer mismatch not applied);
    //      indices (a, dd) = slots of positions i+1 and j-1
    {
      T gf[72];
#pragma unroll
      for (int r = 0; r < 72; r++) gf[r] = 0;
      const int d1 = D.d[i + 1], dm = D.d[j - 1], Pa = D.P[i + 1], Pm = D.P[j - 1];
      for (int w = 1 + tid; w < CDZ_NWIN; w += CDZ_NT) {
        int l1, l2;
        cdz_win(w, l1, l2);
        const int k = i + 1 + l1, l = j - 1 - l2;
        if (l - k < 4) continue;
        const int din = l - k, dk = D.d[k], dlp = D.d[l], Pk = D.P[k], Pl = D.P[l];
        if (l2 == 0) {
          // left bulge: run i+1..k-1, inner pair (k, j-1)
          const T f = D.tab[TB_BU + l1] * cdz_p2<T>(sE[l1 - 1] + sE[din] - Ed);
          const int db = D.d[k - 1], Pb = D.P[k - 1];
          T m[36];  // m(b, y) = sum_x e_{k-1}(b,x) Qb[k][l](x,y)
#pragma unroll
          for (int b = 0; b < 6; b++)
#pragma unroll
            for (int y = 0; y < 6; y++) {
              T a = 0;
              if (b < db && y < dlp)
#pragma unroll
                for (int x = 0; x < 6; x++)
                  if (x < dk) a += D.e[(k - 1) * 36 + b * 6 + x] * D.Qb[(Pk + x) * ld + Pl + y];
              m[b * 6 + y] = a;
            }
#pragma unroll
          for (int a = 0; a < 6; a++) {
            if (a >= d1) continue;
            T ur[6];
#pragma unroll
            for (int b = 0; b < 6; b++) ur[b] = b < db ? D.U[(Pa + a) * ld + Pb + b] : T(0);
#pragma unroll
            for (int y = 0; y < 6; y++) {
              T s = 0;
#pragma unroll
              for (int b = 0; b < 6; b++) s += ur[b] * m[b * 6 + y];
              gf[a * 6 + y] += f * s;
            }
          }
        } else if (l1 == 0) {
          // right bulge: inner pair (i+1, l), run l+1..j-1
          const T f = D.tab[TB_BU + l2] * cdz_p2<T>(sE[l2 - 1] + sE[din] - Ed);
          const int dc = D.d[l + 1], Pc = D.P[l + 1];
          T m[36];  // m(y, dd) = sum_c e_l(y,c) U[l+1][j-1](c,dd)
#pragma unroll
          for (int y = 0; y < 6; y++)
#pragma unroll
            for (int dd = 0; dd < 6; dd++) {
              T a = 0;
              if (y < dlp && dd < dm)
#pragma unroll
                for (int c = 0; c < 6; c++)
                  if (c < dc) a += D.e[l * 36 + y * 6 + c] * D.U[(Pc + c) * ld + Pm + dd];
              m[y * 6 + dd] = a;
            }
#pragma unroll
          for (int x = 0; x < 6; x++) {
            if (x >= dk) continue;
            T q[6];
#pragma unroll
            for (int y = 0; y < 6; y++) q[y] = y < dlp ? D.Qb[(Pk + x) * ld + Pl + y] : T(0);
#pragma unroll
            for (int dd = 0; dd < 6; dd++) {
              T s = 0;
#pragma unroll
              for (int y = 0; y < 6; y++) s += q[y] * m[y * 6 + dd];
              gf[x * 6 + dd] += f * s;
            }
          }
        } else {
          // interior loop: U[i+1][k-1] . DI[k][l] . U[l+1][j-1]
          const T f = D.tab[TB_IN + l1 + l2] *
                      cdz_p2<T>(sE[l1 - 1] + sE[din] + sE[l2 - 1] - Ed);
          const int db = D.d[k - 1], Pb = D.P[k - 1], dc = D.d[l + 1], Pc = D.P[l + 1];
          T m[36];  // m(b, dd) = sum_c DI[k][l](b,c) U[l+1][j-1](c,dd)
#pragma unroll
          for (int b = 0; b < 6; b++)
#pragma unroll
            for (int dd = 0; dd < 6; dd++) {
              T a = 0;
              if (b < db && dd < dm)
#pragma unroll
                for (int c = 0; c < 6; c++)
                  if (c < dc) a += D.DI[(Pb + b) * ld + Pc + c] * D.U[(Pc + c) * ld + Pm + dd];
              m[b * 6 + dd] = a;
            }
#pragma unroll
          for (int a = 0; a < 6; a++) {
            if (a >= d1) continue;
            T ul[6];
#pragma unroll
            for (int b = 0; b < 6; b++) ul[b] = b < db ? D.U[(Pa + a) * ld + Pb + b] : T(0);
#pragma unroll
            for (int dd = 0; dd < 6; dd++) {
              T s = 0;
#pragma unroll
              for (int b = 0; b < 6; b++) s += ul[b] * m[b * 6 + dd];
              gf[36 + a * 6 + dd] += f * s;
            }
          }
        }
      }
      cdz_block_sum<T, 72>(gf, red, sGF);
    }
    // ---- Qb (one thread per slot pair)
    const int d1 = D.d[i + 1], dm = D.d[j - 1], Pa = D.P[i + 1], Pm = D.P[j - 1];
    if (tid < 36) {
      const int s = tid / 6, s2 = tid % 6;
      T qb = 0;
      if (s < di && s2 < dj) {
        const int t = cdz_ptype(D.nt[i * 6 + s], D.nt[j * 6 + s2]);
        if (t >= 0) {
          const T *ei = D.e + i * 36 + s * 6;     // e_i(s, .)
          const T *ej = D.e + (j - 1) * 36 + s2;  // e_{j-1}(., s2), stride 6
          const T f2 = cdz_p2<T>(sE[dl - 2] - Ed);
          T acc = 0, hp = 0, st = 0, ml = 0;
          for (int a = 0; a < d1; a++) {
            const int na = D.nt[(i + 1) * 6 + a];
            for (int b = 0; b < dm; b++) {
              const int nb = D.nt[(j - 1) * 6 + b];
              const T w = ei[a] * ej[b * 6];
              if (w == T(0)) continue;
              const T mmo = D.tab[TB_MM + na * 24 + nb * 6 + t];
              hp += w * D.U[(Pa + a) * ld + Pm + b] * mmo;
              acc += w * (sGF[a * 6 + b] + sGF[36 + a * 6 + b] * mmo);
              ml += w * D.QmX[(Pa + a) * ld + Pm + b];
              if (dl - 2 >= 4) {
                const int t2 = cdz_ptype(na, nb);
                if (t2 >= 0) st += w * D.Qb[(Pa + a) * ld + Pm + b] * D.tab[TB_ST + t * 6 + t2];
              }
            }
          }
          acc += (hp * D.Bhp[dl - 1] + st + ml * D.tab[TB_MLAB]) * f2;
          qb = D.v[i * 6 + s] * D.v[j * 6 + s2] * acc;
        }
        D.Qb[(Pi + s) * ld + Pj + s2] = qb;
        vmax = fmaxf(vmax, (float)fabs(qb));
      }
      sQb[tid] = qb;
      // keep the window sums of this cell for the adjoint (block (i+1, j-1))
      if (s < d1 && s2 < dm) {
        D.G[(Pa + s) * ld + Pm + s2] = sGF[tid];
        D.F[(Pa + s) * ld + Pm + s2] = sGF[36 + tid];
      }
    }
    __syncthreads();
    // ---- Qm1 and DI (Qb dressed as an interior loop's inner pair)
    if (tid < 36) {
      const int s = tid / 6, s2 = tid % 6;
      T q1 = 0;
      if (s < di && s2 < dj) {
        const int dp = D.d[j - 1], Pp = D.P[j - 1];
        T a = 0;
        for (int t = 0; t < dp; t++) a += D.Qm1[(Pi + s) * ld + Pp + t] * D.e[(j - 1) * 36 + t * 6 + s2];
        q1 = a * D.v[j * 6 + s2] * D.tab[TB_MLC] * cdz_p2<T>(sE[dl - 1] - Ed) + sQb[tid] * D.tab[TB_MLB];
        D.Qm1[(Pi + s) * ld + Pj + s2] = q1;
        vmax = fmaxf(vmax, (float)fabs(q1));
      }
      sQm1[tid] = q1;
      if (i >= 1 && j + 1 < n) {
        const int b = tid / 6, c = tid % 6;
        if (b < D.d[i - 1] && c < D.d[j + 1]) {
          const int nb = D.nt[(i - 1) * 6 + b], nc = D.nt[(j + 1) * 6 + c];
          T a = 0;
          for (int x = 0; x < di; x++) {
            const T ex = D.e[(i - 1) * 36 + b * 6 + x];
            if (ex == T(0)) continue;
            for (int y = 0; y < dj; y++) {
              const T q = sQb[x * 6 + y];
              if (q == T(0)) continue;
              const int t2 = cdz_ptype(D.nt[j * 6 + y], D.nt[i * 6 + x]);
              a += ex * q * D.e[j * 36 + y * 6 + c] * D.tab[TB_MM + nc * 24 + nb * 6 + t2];
            }
          }
          D.DI[(D.P[i - 1] + b) * ld + D.P[j + 1] + c] = a;
        }
      }
    }
    __syncthreads();
    // ---- Qm1L, Qm1p, QmX, Qm
    if (tid < 36) {
      const int s = tid / 6, s2 = tid % 6;
      if (i >= 1 && s < D.d[i - 1] && s2 < dj) {
        T a = 0;
        for (int t = 0; t < di; t++) a += D.e[(i - 1) * 36 + s * 6 + t] * sQm1[t * 6 + s2];
        D.Qm1Lr[(D.P[i - 1] + s) * ld + Pj + s2] = a;
        D.Qm1Lt[(Pj + s2) * ld + D.P[i - 1] + s] = a;
      }
      if (s < di && s2 < dj) {
        T a = 0;
        for (int t = 0; t < d1; t++) a += D.e[i * 36 + s * 6 + t] * D.Qm1p[(Pa + t) * ld + Pj + s2];
        const T qp = sQm1[tid] + D.tab[TB_MLC] * D.v[i * 6 + s] * cdz_p2<T>(sE[dl - 1] - Ed) * a;
        const T qx = sSplit[tid];
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

// Per-position scale from a finished forward pass: C[p] = log2 of the prefix
// exterior partition function Z5[p] (FP64).  Every vertex factor v_p is
// multiplied by 2^-g_p with g_p = round(C[p]) - round(C[p-1]); each range
// [i..j] then carries the exact factor 2^-(round C[j] - round C[i-1]), which
// follows the free-energy landscape of the sequence, so inside and outside
// values of every cell stay near 1 in the next pass.  res[3] accumulates the
// total shift sum_p g_p (log Z = log Z~ + res[3] ln 2).
template <typename T>
__global__ void cdz_rescale(DevProb<T> D) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= D.n) return;
  auto C = [&](int q) -> long long {
    if (q < 0) return 0;
    double z = 0;
    for (int t = 0; t < 6; t++) z += D.Z5[q * 6 + t];
    return (z > 0 && isfinite(z)) ? llrint(D.G5[q] + log2(z)) : 0;
  };
  const long long g = C(p) - C(p - 1);
  const double f = ldexp(1.0, (int)(-g));
  double *vd = const_cast<double *>(D.vd);
  T *v = const_cast<T *>(D.v);
  for (int s = 0; s < 6; s++) {
    vd[p * 6 + s] *= f;
    v[p * 6 + s] = (T)((double)v[p * 6 + s] * f);
  }
  if (p == D.n - 1) D.res[3] += (double)C(p);
}

template __global__ void cdz_rescale<float>(DevProb<float>);
template __global__ void cdz_rescale<double>(DevProb<double>);
template __global__ void cdz_fwd_diag<float>(DevProb<float>, int);
template __global__ void cdz_fwd_diag<double>(DevProb<double>, int);
