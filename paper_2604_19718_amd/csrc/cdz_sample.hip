// cdz_sample.hip -- exact joint samples of (codon sequence, structure) by
// stochastic traceback of the forward pass (the backtracking sampler of the
// paper's Section 4a), one wavefront per sample.
//
// Protocol (fixed so that the FP64 mode reproduces the CPU oracle's samples
// draw for draw):
//   * one uniform per decision, u = (x >> 11) * 2^-53, x = words 1:0 of
//     Philox4x32-10 with key (seed lo, seed hi) and counter
//     (draw index, sample index, 0, 0);
//   * a decision lists its alternatives in a fixed order and takes the first
//     one whose running sum exceeds u * total;
//   * fragments are processed depth first from an explicit stack, the 5'
//     fragment first;
//   * orders: exterior (j unpaired by slot of j-1, then 0 pairs j, then k = 1..
//     j-4 pairs j by slots (k-1, k)); pair (hairpin, then inner pairs with
//     l1 ascending and l2 ascending, then multiloop), then the slots of the
//     chosen loop; Qm1 (pair, then unpaired tail by slot); Qm1p (Qm1, then
//     unpaired prefix by slot); QmX/Qm (splits u ascending by slots, then
//     Qm1p); unpaired runs codon by codon.
// The lanes of a wave evaluate groups of alternatives in parallel, a wave
// prefix sum finds the group holding the target, and the group is scanned in
// order.
#include <cmath>
#include <cstring>

#include <map>
#include <mutex>

#include "cdz_internal.h"

namespace {

enum { F_EXT = 0, F_B, F_M1, F_M1P, F_MX, F_M, F_RUN };

__device__ __forceinline__ void philox10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; r++) {
    const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
    const uint32_t hi0 = __umulhi(m0, c[0]), lo0 = m0 * c[0];
    const uint32_t hi1 = __umulhi(m1, c[2]), lo1 = m1 * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
}

__device__ __forceinline__ double uniform01(uint64_t seed, uint32_t sid, uint32_t draw) {
  uint32_t c[4] = {draw, sid, 0u, 0u};
  philox10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  const uint64_t x = ((uint64_t)c[1] << 32) | c[0];
  return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ double wsum(double x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

__device__ __forceinline__ double wscan(double x, int lane) {  // inclusive
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

template <typename T>
struct Smp {
  DevProb<T> D;
  uint64_t seed;
  int nsamp, cap, gcap;
  uint8_t *codons;
  int32_t *pairs;
  int *stack;
  double *gbuf;
  signed char *state;
  int *err;
};

template <typename T>
struct W {  // per-wave state
  const Smp<T> *S;
  int sid, lane, top;
  int hk, hi, hj, hs, ht;  // top entry of the stack, held in registers (hk < 0: none)
  uint32_t draw;
  int *stk;
  double *gb;
  signed char *st;
  int32_t *pt;
  bool bad;
};

template <typename T>
__device__ __forceinline__ double Qv(const T *A, long long ld, int r, int c) {
  return (double)A[(long long)r * ld + c];
}

// The top entry of the stack is held in registers (depth first, the fragment
// pushed last is taken next, so most pushes never reach memory); a push moves
// the entry held before it to the stack in memory.  Stack entries, slots and
// partners are written by every lane with the same (wave-uniform) value, so
// each lane later reads back its own store.
template <typename T>
__device__ __forceinline__ void push(W<T> &w, int kind, int i, int j, int s, int t) {
  if (w.hk >= 0) {
    if (w.top >= w.S->cap) {
      w.bad = true;
      return;
    }
    int *e = w.stk + 5 * w.top;
    e[0] = w.hk;
    e[1] = w.hi;
    e[2] = w.hj;
    e[3] = w.hs;
    e[4] = w.ht;
    w.top++;
  }
  w.hk = kind, w.hi = i, w.hj = j, w.hs = s, w.ht = t;
}

template <typename T>
__device__ __forceinline__ void set_state(W<T> &w, int p, int s) {
  if (w.st[p] >= 0 && w.st[p] != s) w.bad = true;
  w.st[p] = (signed char)s;
}

// One decision over G groups.  gsum(g) gives a group's total (computed by the
// lane that owns g); scan(g, running, target) walks group g in order and
// returns the index of the chosen alternative (wave-uniform).  Returns false
// if every weight vanished.
template <typename T, typename GS, typename SC>
__device__ __forceinline__ bool decide(W<T> &w, int G, GS gsum, SC scan, int &gsel, int &asel) {
  const double u = uniform01(w.S->seed, (uint32_t)w.sid, w.draw++);
  double tot = 0;
  for (int base = 0; base < G; base += 64) {
    const int g = base + w.lane;
    double s = 0;
    if (g < G) {
      s = gsum(g);
      if (g < w.S->gcap) w.gb[g] = s;
    }
    tot += wsum(s);
  }
  if (!(tot > 0)) return false;
  const double target = u * tot;
  double cum = 0, before = 0;
  int last_nz = -1;
  gsel = -1;
  for (int base = 0; base < G && gsel < 0; base += 64) {
    const int g = base + w.lane;
    const double s = g < G ? w.gb[g] : 0.0;
    const double incl = wscan(s, w.lane) + cum;
    const unsigned long long hit = __ballot(g < G && incl > target);
    const unsigned long long nz = __ballot(g < G && s > 0);
    if (nz) last_nz = base + 63 - __clzll(nz);
    if (hit) {
      const int l = __ffsll((long long)hit) - 1;
      gsel = base + l;
      before = __shfl(incl - s, l, 64);
    } else {
      cum = __shfl(incl, 63, 64);
    }
  }
  if (gsel < 0) {
    gsel = last_nz;
    if (gsel < 0) return false;
    before = -1.0;  // take the group's last nonzero alternative
  }
  asel = scan(gsel, before, target);
  return asel >= 0;
}

// The same decision when the total is already known (the forward pass stored
// it): the groups are evaluated in order, the first chunk FIRST wide and then
// 64 at a time, and the walk stops at the chunk where the running sum passes
// u * total.  Most decisions end in the first few groups.  If rounding leaves
// the target beyond the last group, the last nonzero group is taken.
template <typename T, typename GS, typename SC>
__device__ __forceinline__ bool decide_total(W<T> &w, int G, double tot, int first, GS gsum, SC scan, int &gsel, int &asel) {
  const double u = uniform01(w.S->seed, (uint32_t)w.sid, w.draw++);
  if (!(tot > 0)) return false;
  const double target = u * tot;
  double cum = 0, before = 0;
  int last_nz = -1;
  gsel = -1;
  for (int base = 0; base < G && gsel < 0;) {
    const int width = base == 0 ? first : 64;
    const int g = base + w.lane;
    const bool in = w.lane < width && g < G;
    const double s = in ? gsum(g) : 0.0;
    const double incl = wscan(s, w.lane) + cum;
    const unsigned long long hit = __ballot(in && incl > target);
    const unsigned long long nz = __ballot(in && s > 0);
    if (nz) last_nz = base + 63 - __clzll(nz);
    if (hit) {
      const int l = __ffsll((long long)hit) - 1;
      gsel = base + l;
      before = __shfl(incl - s, l, 64);
    } else {
      cum = __shfl(incl, 63, 64);
    }
    base += width;
  }
  if (gsel < 0) {
    gsel = last_nz;
    if (gsel < 0) return false;
    before = -1.0;
  }
  asel = scan(gsel, before, target);
  return asel >= 0;
}

// ---- fragment handlers ----------------------------------------------------

template <typename T>
__device__ __forceinline__ void f_ext(W<T> &w, int j, int t) {
  const DevProb<T> &D = w.S->D;
  const long long ld = D.ld;
  set_state(w, j, t);
  if (j == 0) return;
  const int G = 2 + (j - 4 > 0 ? j - 4 : 0);
  const int Gj = D.G5[j], Pj = D.P[j];
  auto alt = [&](int g, int a) -> double {  // weight of alternative a of group g
    if (g == 0) {
      return D.Z5[(j - 1) * 6 + a] * D.ed[(j - 1) * 36 + a * 6 + t] * D.vd[j * 6 + t] *
             ldexp(1.0, D.G5[j - 1] - Gj);
    }
    if (g == 1) return j >= 4 ? Qv(D.Qb, ld, a, Pj + t) * ldexp(1.0, D.E[j] - Gj) : 0.0;
    const int k = g - 1, dk = D.d[k], s = a / dk, x = a % dk;
    return D.Z5[(k - 1) * 6 + s] * D.ed[(k - 1) * 36 + s * 6 + x] * Qv(D.Qb, ld, D.P[k] + x, Pj + t) *
           ldexp(1.0, D.G5[k - 1] + D.E[j - k] - Gj);
  };
  auto cnt = [&](int g) -> int {
    if (g == 0) return D.d[j - 1];
    if (g == 1) return D.d[0];
    return D.d[g - 2] * D.d[g - 1];
  };
  // group totals with every load of a group issued at once
  auto gsum = [&](int g) -> double {
    if (g == 0) {
      double z = 0;
#pragma unroll
      for (int s = 0; s < 6; s++) z += D.Z5[(j - 1) * 6 + s] * D.ed[(j - 1) * 36 + s * 6 + t];
      return z * D.vd[j * 6 + t] * ldexp(1.0, D.G5[j - 1] - Gj);
    }
    if (g == 1) {
      if (j < 4) return 0.0;
      const int d0 = D.d[0];
      double z = 0;
#pragma unroll
      for (int x = 0; x < 6; x++) z += x < d0 ? Qv(D.Qb, ld, x, Pj + t) : 0.0;
      return z * ldexp(1.0, D.E[j] - Gj);
    }
    const int k = g - 1, dk = D.d[k], Pk = D.P[k];
    double zl[6], q[6];
#pragma unroll
    for (int x = 0; x < 6; x++) {
      double a = 0;
#pragma unroll
      for (int s = 0; s < 6; s++) a += D.Z5[(k - 1) * 6 + s] * D.ed[(k - 1) * 36 + s * 6 + x];
      zl[x] = a;
      q[x] = x < dk ? Qv(D.Qb, ld, Pk + x, Pj + t) : 0.0;
    }
    double z = 0;
#pragma unroll
    for (int x = 0; x < 6; x++) z += zl[x] * q[x];
    return z * ldexp(1.0, D.G5[k - 1] + D.E[j - k] - Gj);
  };
  auto scan = [&](int g, double run, double target) {
    const int c = cnt(g);
    int last = -1;
    for (int a = 0; a < c; a++) {
      const double x = alt(g, a);
      if (x > 0) last = a;
      if (run >= 0) {
        run += x;
        if (run > target) return a;
      }
    }
    return last;
  };
  int g, a;
  if (!decide(w, G, gsum, scan, g, a)) {
    w.bad = true;
    return;
  }
  if (g == 0) {
    push(w, F_EXT, j - 1, 0, a, 0);
  } else if (g == 1) {
    push(w, F_B, 0, j, a, t);
  } else {
    const int k = g - 1, dk = D.d[k];
    push(w, F_B, k, j, a % dk, t);
    push(w, F_EXT, k - 1, 0, a / dk, 0);
  }
}

template <typename T>
__device__ __forceinline__ void f_run(W<T> &w, int p, int q, int a, int b) {
  const DevProb<T> &D = w.S->D;
  const long long ld = D.ld;
  const int cp = p / 3, cq = q / 3;
  for (int x = p; x <= q && x / 3 == cp; x++) set_state(w, x, a);
  for (int x = q; x >= p && x / 3 == cq; x--) set_state(w, x, b);
  int prev = a;
  const int Pq = D.P[q];
  for (int c = cp + 1; c < cq && !w.bad; c++) {
    const int f = 3 * c, df = D.d[f], Pf = D.P[f];
    auto alt = [&](int x) { return (double)D.e[(f - 1) * 36 + prev * 6 + x] * Qv(D.U, ld, Pf + x, Pq + b); };
    auto gsum = [&](int) {
      double s = 0;
      for (int x = 0; x < df; x++) s += alt(x);
      return s;
    };
    auto scan = [&](int, double run, double target) {
      int last = -1;
      for (int x = 0; x < df; x++) {
        const double v = alt(x);
        if (v > 0) last = x;
        if (run >= 0) {
          run += v;
          if (run > target) return x;
        }
      }
      return last;
    };
    int g, x;
    if (!decide(w, 1, gsum, scan, g, x)) {
      w.bad = true;
      return;
    }
    for (int y = f; y < f + 3; y++) set_state(w, y, x);
    prev = x;
  }
}

// generic small decision: alternatives a = 0..count-1 (a single group)
template <typename T, typename F>
__device__ __forceinline__ int small_decide(W<T> &w, int count, F alt) {
  auto gsum = [&](int) {
    double s = 0;
    for (int a = 0; a < count; a++) s += alt(a);
    return s;
  };
  auto scan = [&](int, double run, double target) {
    int last = -1;
    for (int a = 0; a < count; a++) {
      const double v = alt(a);
      if (v > 0) last = a;
      if (run >= 0) {
        run += v;
        if (run > target) return a;
      }
    }
    return last;
  };
  int g, a;
  if (!decide(w, 1, gsum, scan, g, a)) {
    w.bad = true;
    return -1;
  }
  return a;
}

// grouped decision: groups g = 0..G-1, alternatives a = 0..A-1 in each
template <typename T, typename F>
__device__ __forceinline__ bool grid_decide(W<T> &w, int G, int A, F alt, int &g, int &a) {
  auto gsum = [&](int gg) {
    double s = 0;
    for (int x = 0; x < A; x++) s += alt(gg, x);
    return s;
  };
  auto scan = [&](int gg, double run, double target) {
    int last = -1;
    for (int x = 0; x < A; x++) {
      const double v = alt(gg, x);
      if (v > 0) last = x;
      if (run >= 0) {
        run += v;
        if (run > target) return x;
      }
    }
    return last;
  };
  if (!decide(w, G, gsum, scan, g, a)) {
    w.bad = true;
    return false;
  }
  return true;
}

template <typename T>
__device__ __forceinline__ void f_pair(W<T> &w, int i, int j, int s, int s2) {
  const DevProb<T> &D = w.S->D;
  const long long ld = D.ld;
  const T *tab = D.tab;
  set_state(w, i, s);
  set_state(w, j, s2);
  w.pt[i] = j;
  w.pt[j] = i;
  const int dl = j - i, t = cdz_ptype(D.nt[i * 6 + s], D.nt[j * 6 + s2]);
  const int d1 = D.d[i + 1], dm = D.d[j - 1], P1 = D.P[i + 1], Pm = D.P[j - 1];
  const int E0 = D.E[dl];
  const double f2 = ldexp(1.0, D.E[dl - 2] - E0);
  auto ei = [&](int a) { return (double)D.e[i * 36 + s * 6 + a]; };
  auto ej = [&](int b) { return (double)D.e[(j - 1) * 36 + b * 6 + s2]; };
  auto mmo = [&](int a, int b) {
    return (double)tab[TB_MM + D.nt[(i + 1) * 6 + a] * 24 + D.nt[(j - 1) * 6 + b] * 6 + t];
  };
  // weight of inner-pair group w (window index, (l1,l2)) for the fixed outer
  // slots; each block is loaded whole (predicated) so the loads overlap
  auto blk = [&](const T *A, int r0, int c0, int dr, int dc, double (&o)[36]) {
#pragma unroll
    for (int r = 0; r < 36; r++) o[r] = (r / 6 < dr && r % 6 < dc) ? Qv(A, ld, r0 + r / 6, c0 + r % 6) : 0.0;
  };
  double eiv[6], ejv[6];
#pragma unroll
  for (int a = 0; a < 6; a++) {
    eiv[a] = ei(a);
    ejv[a] = ej(a);
  }
  auto win_weight = [&](int wi) -> double {
    int l1, l2;
    cdz_win(wi, l1, l2);
    const int k = i + 1 + l1, l = j - 1 - l2;
    if (l - k < 4) return 0.0;
    const int din = l - k, dk = D.d[k], dL = D.d[l], Pk = D.P[k], Pl = D.P[l];
    double wsum_ = 0;
    if (l1 == 0 && l2 == 0) {
      double q[36];
      blk(D.Qb, Pk, Pl, dk, dL, q);
#pragma unroll
      for (int x = 0; x < 6; x++)
#pragma unroll
        for (int y = 0; y < 6; y++) {
          const int t2 = cdz_ptype(D.nt[k * 6 + x], D.nt[l * 6 + y]);
          if (t2 >= 0) wsum_ += eiv[x] * q[x * 6 + y] * ejv[y] * (double)tab[TB_ST + t * 6 + t2];
        }
      return wsum_ * f2;
    }
    if (l2 == 0) {
      const int db = D.d[k - 1], Pb = D.P[k - 1];
      double ul[36], q[36];
      blk(D.U, P1, Pb, d1, db, ul);
      blk(D.Qb, Pk, Pl, dk, dL, q);
      double lft[6], rgt[6];  // sum_a e_i ul, sum_y q e_{j-1}
#pragma unroll
      for (int b = 0; b < 6; b++) {
        double a_ = 0;
#pragma unroll
        for (int a = 0; a < 6; a++) a_ += eiv[a] * ul[a * 6 + b];
        lft[b] = a_;
      }
#pragma unroll
      for (int x = 0; x < 6; x++) {
        double a_ = 0;
#pragma unroll
        for (int y = 0; y < 6; y++) a_ += q[x * 6 + y] * ejv[y];
        rgt[x] = a_;
      }
#pragma unroll
      for (int b = 0; b < 6; b++)
#pragma unroll
        for (int x = 0; x < 6; x++) wsum_ += lft[b] * (double)D.e[(k - 1) * 36 + b * 6 + x] * rgt[x];
      return wsum_ * (double)tab[TB_BU + l1] * ldexp(1.0, D.E[l1 - 1] + D.E[din] - E0);
    }
    if (l1 == 0) {
      const int dc = D.d[l + 1], Pc = D.P[l + 1];
      double q[36], ur[36];
      blk(D.Qb, Pk, Pl, dk, dL, q);
      blk(D.U, Pc, Pm, dc, dm, ur);
      double lft[6], rgt[6];  // sum_x e_i q, sum_dd ur e_{j-1}
#pragma unroll
      for (int y = 0; y < 6; y++) {
        double a_ = 0;
#pragma unroll
        for (int x = 0; x < 6; x++) a_ += eiv[x] * q[x * 6 + y];
        lft[y] = a_;
      }
#pragma unroll
      for (int c = 0; c < 6; c++) {
        double a_ = 0;
#pragma unroll
        for (int dd = 0; dd < 6; dd++) a_ += ur[c * 6 + dd] * ejv[dd];
        rgt[c] = a_;
      }
#pragma unroll
      for (int y = 0; y < 6; y++)
#pragma unroll
        for (int c = 0; c < 6; c++) wsum_ += lft[y] * (double)D.e[l * 36 + y * 6 + c] * rgt[c];
      return wsum_ * (double)tab[TB_BU + l2] * ldexp(1.0, D.E[din] + D.E[l2 - 1] - E0);
    }
    const int db = D.d[k - 1], Pb = D.P[k - 1], dc = D.d[l + 1], Pc = D.P[l + 1];
    double ul[36], dI[36], ur[36];
    blk(D.U, P1, Pb, d1, db, ul);
    blk(D.DI, Pb, Pc, db, dc, dI);
    blk(D.U, Pc, Pm, dc, dm, ur);
    double m[36];  // m(b, dd) = sum_c DI(b,c) ur(c,dd)
#pragma unroll
    for (int b = 0; b < 6; b++)
#pragma unroll
      for (int dd = 0; dd < 6; dd++) {
        double a_ = 0;
#pragma unroll
        for (int c = 0; c < 6; c++) a_ += dI[b * 6 + c] * ur[c * 6 + dd];
        m[b * 6 + dd] = a_;
      }
#pragma unroll
    for (int a = 0; a < 6; a++)
#pragma unroll
      for (int dd = 0; dd < 6; dd++) {
        const double o = eiv[a] * ejv[dd] * (a < d1 && dd < dm ? mmo(a, dd) : 0.0);
        double in = 0;
#pragma unroll
        for (int b = 0; b < 6; b++) in += ul[a * 6 + b] * m[b * 6 + dd];
        wsum_ += o * in;
      }
    return wsum_ * (double)tab[TB_IN + l1 + l2] * ldexp(1.0, D.E[l1 - 1] + D.E[din] + D.E[l2 - 1] - E0);
  };
  // decision 1: which loop (group 0 hairpin, 1 + w window, CDZ_NWIN + 1 multiloop)
  auto gsum1 = [&](int g) -> double {
    if (g == 0) {
      double u[36], h = 0;
      blk(D.U, P1, Pm, d1, dm, u);
#pragma unroll
      for (int a = 0; a < 6; a++)
#pragma unroll
        for (int b = 0; b < 6; b++)
          if (a < d1 && b < dm) h += eiv[a] * u[a * 6 + b] * ejv[b] * mmo(a, b);
      return h * (double)D.Bhp[dl - 1] * f2;
    }
    if (g <= CDZ_NWIN) return win_weight(g - 1);
    double x_[36], m = 0;
    blk(D.QmX, P1, Pm, d1, dm, x_);
#pragma unroll
    for (int x = 0; x < 6; x++)
#pragma unroll
      for (int y = 0; y < 6; y++) m += eiv[x] * x_[x * 6 + y] * ejv[y];
    return m * (double)tab[TB_MLAB] * f2;
  };
  auto scan1 = [&](int g, double, double) { return 0; };
  // the total over all loops closed by (i, j) is the stored Qb entry without
  // its two vertex factors; hairpin and stack come first in the order
  const double tot1 = Qv(D.Qb, ld, D.P[i] + s, D.P[j] + s2) / ((double)D.v[i * 6 + s] * (double)D.v[j * 6 + s2]);
  int g1, a1;
  if (!decide_total(w, CDZ_NWIN + 2, tot1, 2, gsum1, scan1, g1, a1)) {
    w.bad = true;
    return;
  }
  int ga, aa;
  if (g1 == 0) {  // hairpin: slots of i+1 and j-1, then the run
    if (!grid_decide(w, d1, dm, [&](int a, int b) {
          return b < dm ? ei(a) * Qv(D.U, ld, P1 + a, Pm + b) * ej(b) * mmo(a, b) : 0.0;
        }, ga, aa))
      return;
    push(w, F_RUN, i + 1, j - 1, ga, aa);
    return;
  }
  if (g1 == CDZ_NWIN + 1) {  // multiloop
    if (!grid_decide(w, d1, dm, [&](int x, int y) {
          return ei(x) * Qv(D.QmX, ld, P1 + x, Pm + y) * ej(y);
        }, ga, aa))
      return;
    push(w, F_MX, i + 1, j - 1, ga, aa);
    return;
  }
  int l1, l2;
  cdz_win(g1 - 1, l1, l2);
  const int k = i + 1 + l1, l = j - 1 - l2;
  const int dk = D.d[k], dL = D.d[l], Pk = D.P[k], Pl = D.P[l];
  if (l1 == 0 && l2 == 0) {
    if (!grid_decide(w, d1, dm, [&](int x, int y) {
          const int t2 = cdz_ptype(D.nt[k * 6 + x], D.nt[l * 6 + y]);
          return t2 < 0 ? 0.0 : ei(x) * Qv(D.Qb, ld, Pk + x, Pl + y) * ej(y) * (double)tab[TB_ST + t * 6 + t2];
        }, ga, aa))
      return;
    push(w, F_B, k, l, ga, aa);
    return;
  }
  if (l2 == 0) {  // left bulge: (a, b) groups, (x, y) alternatives
    const int db = D.d[k - 1], Pb = D.P[k - 1];
    if (!grid_decide(w, d1 * db, dk * dL, [&](int g, int x) {
          const int a = g / db, b = g % db, xx = x / dL, y = x % dL;
          return ei(a) * Qv(D.U, ld, P1 + a, Pb + b) * (double)D.e[(k - 1) * 36 + b * 6 + xx] *
                 Qv(D.Qb, ld, Pk + xx, Pl + y) * ej(y);
        }, ga, aa))
      return;
    push(w, F_B, k, l, aa / dL, aa % dL);
    push(w, F_RUN, i + 1, k - 1, ga / db, ga % db);
    return;
  }
  if (l1 == 0) {  // right bulge: (x, y) groups, (c, dd) alternatives
    const int dc = D.d[l + 1], Pc = D.P[l + 1];
    if (!grid_decide(w, dk * dL, dc * dm, [&](int g, int x) {
          const int xx = g / dL, y = g % dL, c = x / dm, dd = x % dm;
          return ei(xx) * Qv(D.Qb, ld, Pk + xx, Pl + y) * (double)D.e[l * 36 + y * 6 + c] *
                 Qv(D.U, ld, Pc + c, Pm + dd) * ej(dd);
        }, ga, aa))
      return;
    push(w, F_RUN, l + 1, j - 1, aa / dm, aa % dm);
    push(w, F_B, k, l, ga / dL, ga % dL);
    return;
  }
  // interior loop: (a, b) groups, (c, dd) alternatives; then the inner pair
  const int db = D.d[k - 1], Pb = D.P[k - 1], dc = D.d[l + 1], Pc = D.P[l + 1];
  if (!grid_decide(w, d1 * db, dc * dm, [&](int g, int x) {
        const int a = g / db, b = g % db, c = x / dm, dd = x % dm;
        return ei(a) * Qv(D.U, ld, P1 + a, Pb + b) * Qv(D.DI, ld, Pb + b, Pc + c) *
               Qv(D.U, ld, Pc + c, Pm + dd) * ej(dd) * mmo(a, dd);
      }, ga, aa))
    return;
  const int ca = ga / db, cb = ga % db, cc = aa / dm, cd = aa % dm;
  int gx, ay;
  if (!grid_decide(w, dk, dL, [&](int x, int y) {
        const int t2 = cdz_ptype(D.nt[l * 6 + y], D.nt[k * 6 + x]);
        if (t2 < 0) return 0.0;
        return (double)D.e[(k - 1) * 36 + cb * 6 + x] * Qv(D.Qb, ld, Pk + x, Pl + y) *
               (double)D.e[l * 36 + y * 6 + cc] *
               (double)tab[TB_MM + D.nt[(l + 1) * 6 + cc] * 24 + D.nt[(k - 1) * 6 + cb] * 6 + t2];
      }, gx, ay))
    return;
  push(w, F_RUN, l + 1, j - 1, cc, cd);
  push(w, F_B, k, l, gx, ay);
  push(w, F_RUN, i + 1, k - 1, ca, cb);
}

template <typename T>
__device__ __forceinline__ void f_split(W<T> &w, int i, int j, int s, int s2, bool with_m1p) {
  const DevProb<T> &D = w.S->D;
  const long long ld = D.ld;
  const int dl = j - i, Pi = D.P[i], Pj = D.P[j], E0 = D.E[dl];
  const int nu = j - 4 - (i + 5) + 1 > 0 ? j - 4 - (i + 5) + 1 : 0;
  const int G = nu + (with_m1p ? 1 : 0);
  auto cnt = [&](int g) { return g < nu ? D.d[i + 4 + g] * D.d[i + 5 + g] : 1; };
  auto alt = [&](int g, int a) -> double {
    if (g >= nu) return Qv(D.Qm1p, ld, Pi + s, Pj + s2);
    const int u = i + 5 + g, du = D.d[u], t = a / du, t2 = a % du;
    return Qv(D.Qm, ld, Pi + s, D.P[u - 1] + t) * (double)D.e[(u - 1) * 36 + t * 6 + t2] *
           Qv(D.Qm1, ld, D.P[u] + t2, Pj + s2) * ldexp(1.0, D.E[u - 1 - i] + D.E[j - u] - E0);
  };
  auto gsum = [&](int g) -> double {
    if (g >= nu) return Qv(D.Qm1p, ld, Pi + s, Pj + s2);
    const int u = i + 5 + g, du1 = D.d[u - 1], du = D.d[u], Pu1 = D.P[u - 1], Pu = D.P[u];
    double qa[6], qb[6];
#pragma unroll
    for (int t = 0; t < 6; t++) {
      qa[t] = t < du1 ? Qv(D.Qm, ld, Pi + s, Pu1 + t) : 0.0;
      qb[t] = t < du ? Qv(D.Qm1, ld, Pu + t, Pj + s2) : 0.0;
    }
    double x = 0;
#pragma unroll
    for (int t = 0; t < 6; t++)
#pragma unroll
      for (int t2 = 0; t2 < 6; t2++) x += qa[t] * (double)D.e[(u - 1) * 36 + t * 6 + t2] * qb[t2];
    return x * ldexp(1.0, D.E[u - 1 - i] + D.E[j - u] - E0);
  };
  auto scan = [&](int g, double run, double target) {
    const int c = cnt(g);
    int last = -1;
    for (int a = 0; a < c; a++) {
      const double v = alt(g, a);
      if (v > 0) last = a;
      if (run >= 0) {
        run += v;
        if (run > target) return a;
      }
    }
    return last;
  };
  int g, a;
  if (!decide(w, G, gsum, scan, g, a)) {
    w.bad = true;
    return;
  }
  if (g >= nu) {
    push(w, F_M1P, i, j, s, s2);
    return;
  }
  const int u = i + 5 + g, du = D.d[u];
  push(w, F_M1, u, j, a % du, s2);
  push(w, F_M, i, u - 1, s, a / du);
}

template <typename T>
__device__ __forceinline__ void f_m1(W<T> &w, int i, int j, int s, int s2) {
  const DevProb<T> &D = w.S->D;
  const long long ld = D.ld;
  set_state(w, i, s);
  set_state(w, j, s2);
  const int dl = j - i, Pi = D.P[i], Pj = D.P[j], dp = D.d[j - 1], Pp = D.P[j - 1];
  const double fe = ldexp(1.0, D.E[dl - 1] - D.E[dl]);
  const int a = small_decide(w, 1 + dp, [&](int x) -> double {
    if (x == 0) return Qv(D.Qb, ld, Pi + s, Pj + s2) * (double)D.tab[TB_MLB];
    const int t = x - 1;
    return Qv(D.Qm1, ld, Pi + s, Pp + t) * (double)D.e[(j - 1) * 36 + t * 6 + s2] *
           (double)D.v[j * 6 + s2] * (double)D.tab[TB_MLC] * fe;
  });
  if (a < 0) return;
  if (a == 0) push(w, F_B, i, j, s, s2);
  else push(w, F_M1, i, j - 1, s, a - 1);
}

template <typename T>
__device__ __forceinline__ void f_m1p(W<T> &w, int i, int j, int s, int s2) {
  const DevProb<T> &D = w.S->D;
  const long long ld = D.ld;
  set_state(w, i, s);
  set_state(w, j, s2);
  const int dl = j - i, Pi = D.P[i], Pj = D.P[j], d1 = D.d[i + 1], P1 = D.P[i + 1];
  const double fe = ldexp(1.0, D.E[dl - 1] - D.E[dl]);
  const int a = small_decide(w, 1 + d1, [&](int x) -> double {
    if (x == 0) return Qv(D.Qm1, ld, Pi + s, Pj + s2);
    const int t = x - 1;
    return (double)D.v[i * 6 + s] * (double)D.tab[TB_MLC] * (double)D.e[i * 36 + s * 6 + t] *
           Qv(D.Qm1p, ld, P1 + t, Pj + s2) * fe;
  });
  if (a < 0) return;
  if (a == 0) push(w, F_M1, i, j, s, s2);
  else push(w, F_M1P, i + 1, j, a - 1, s2);
}

}  // namespace

template <typename T>
__device__ __forceinline__ void sample_one(const Smp<T> &S, int sid) {
  const int lane = threadIdx.x & 63;
  const DevProb<T> &D = S.D;
  const int n = D.n, m = D.m;
  W<T> w;
  w.S = &S;
  w.sid = sid;
  w.lane = lane;
  w.top = 0;
  w.hk = -1;
  w.draw = 0;
  w.bad = false;
  w.stk = S.stack + (size_t)sid * S.cap * 5;
  w.gb = S.gbuf + (size_t)sid * S.gcap;
  w.st = S.state + (size_t)sid * n;
  w.pt = S.pairs + (size_t)sid * n;
  for (int p = lane; p < n; p += 64) {
    w.st[p] = -1;
    w.pt[p] = -1;
  }
  __threadfence_block();  // the lanes' initial stores are visible to the whole wave
  // slot of the last position
  {
    const int dn = D.d[n - 1];
    const int t = small_decide(w, dn, [&](int x) { return D.Z5[(n - 1) * 6 + x]; });
    if (t >= 0) push(w, F_EXT, n - 1, 0, t, 0);
  }
  // depth-first traversal; every wave ends when its stack is empty or on error
  while ((w.hk >= 0 || w.top > 0) && !w.bad) {
    int kind, i, j, s, t;
    if (w.hk >= 0) {
      kind = w.hk, i = w.hi, j = w.hj, s = w.hs, t = w.ht;
      w.hk = -1;
    } else {
      w.top--;
      const int *e = w.stk + 5 * w.top;
      kind = e[0], i = e[1], j = e[2], s = e[3], t = e[4];
    }
    switch (kind) {
      case F_EXT: f_ext(w, i, s); break;
      case F_B: f_pair(w, i, j, s, t); break;
      case F_M1: f_m1(w, i, j, s, t); break;
      case F_M1P: f_m1p(w, i, j, s, t); break;
      case F_MX: f_split(w, i, j, s, t, false); break;
      case F_M: f_split(w, i, j, s, t, true); break;
      case F_RUN: f_run(w, i, j, s, t); break;
      default: w.bad = true;
    }
  }
  if (lane == 0) {
    bool ok = !w.bad;
    for (int a = 0; a < m && ok; a++) {
      const int s0 = w.st[3 * a];
      if (s0 < 0 || w.st[3 * a + 1] != s0 || w.st[3 * a + 2] != s0) ok = false;
      else S.codons[(size_t)sid * m + a] = (uint8_t)s0;
    }
    S.err[sid] = ok ? 0 : 1;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void cdz_sample_kernel(Smp<T> S) {
  const int sid = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (sid < S.nsamp) sample_one<T>(S, sid);
}

// many problems in one launch: N samples of each, wavefront g runs sample
// g % N of problem g / N
template <typename T>
__global__ __launch_bounds__(256) void cdz_sample_batch_kernel(const Smp<T> *S, int N, int total) {
  const int g = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (g < total) sample_one<T>(S[g / N], g % N);
}

// Device scratch of cdz_sample_noalloc, one copy per device for the life of
// the process.  Host code never uses this name as an address: the per-device
// address comes from hipGetSymbolAddress (noalloc_scratch).
static __device__ __align__(256) unsigned char scratch[CDZ_NOALLOC_SCRATCH_BYTES];

void *noalloc_scratch(int device) {
  static std::mutex mu;
  static std::map<int, void *> addr;
  std::lock_guard<std::mutex> lock(mu);
  auto it = addr.find(device);
  if (it != addr.end()) return it->second;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != device) return nullptr;
  void *ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return nullptr;
  }
  addr[device] = ptr;
  return ptr;
}

// bytes of sampler workspace for N samples of a sequence of n positions, m
// residues (stacks, group sums, slots, codons, pairs, flags; 256-byte aligned)
static size_t sample_ws_bytes(int n, int m, int N, int &cap, int &gcap) {
  cap = n + 16;
  gcap = (n > CDZ_NWIN + 2 ? n : CDZ_NWIN + 2) + 64;
  return (size_t)N * cap * 5 * 4 + (size_t)N * gcap * 8 + (size_t)N * n + (size_t)N * m +
         (size_t)N * n * 4 + (size_t)N * 4 + 6 * 256;
}

// ws == nullptr: the handle's workspace (grown with hipMalloc as needed);
// else a caller-provided device buffer of ws_bytes (nothing is allocated)
template <typename T>
static cdz_status run_sample(cdz_handle *h, const DevProb<T> &D, uint64_t seed, int N,
                             uint8_t *codons, int32_t *pairs, char *ws = nullptr, size_t ws_bytes = 0) {
  const int n = D.n, m = D.m;
  Smp<T> S;
  S.D = D;
  S.seed = seed;
  S.nsamp = N;
  const size_t need = sample_ws_bytes(n, m, N, S.cap, S.gcap);
  if (ws) {
    if (need > ws_bytes)
      return cdz_fail(h, CDZ_ERR_BUDGET, std::to_string(N) + " samples of " + std::to_string(n) +
                                             " nt need " + std::to_string(need) +
                                             " bytes of scratch, above the " + std::to_string(ws_bytes) +
                                             " bytes of cdz_sample_noalloc");
  } else if (need > h->smp_bytes) {
    if (h->smp) (void)hipFree(h->smp);
    h->smp = nullptr;
    h->smp_bytes = 0;
    if (hipMalloc(&h->smp, need) != hipSuccess) {
      (void)hipGetLastError();
      return cdz_fail(h, CDZ_ERR_NOMEM, "sampler workspace allocation failed");
    }
    h->smp_bytes = need;
  }
  char *p = ws ? ws : (char *)h->smp;
  auto take = [&](size_t b) {
    char *r = p;
    p += (b + 255) / 256 * 256;
    return r;
  };
  S.stack = (int *)take((size_t)N * S.cap * 5 * 4);
  S.gbuf = (double *)take((size_t)N * S.gcap * 8);
  S.state = (signed char *)take((size_t)N * n);
  S.codons = (uint8_t *)take((size_t)N * m);
  S.pairs = (int32_t *)take((size_t)N * n * 4);
  S.err = (int *)take((size_t)N * 4);
  hipStream_t st = h->stream;
  HIPCHK(h, hipEventRecord(h->ev[4], st));
  hipLaunchKernelGGL(cdz_sample_kernel<T>, dim3((N + 3) / 4), dim3(256), 0, st, S);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipEventRecord(h->ev[5], st));
  std::vector<int> err(N);
  HIPCHK(h, hipMemcpyAsync(codons, S.codons, (size_t)N * m, hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipMemcpyAsync(pairs, S.pairs, (size_t)N * n * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipMemcpyAsync(err.data(), S.err, (size_t)N * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipStreamSynchronize(st));
  float ms = 0;
  HIPCHK(h, hipEventElapsedTime(&ms, h->ev[4], h->ev[5]));
  h->times[2] = ms;
  h->prof_smp_ms = ms;
  for (int k = 0; k < N; k++)
    if (err[k]) return cdz_fail(h, CDZ_ERR_NUMERIC, "sampling failed (sample " + std::to_string(k) + ")");
  return CDZ_OK;
}

// Samples of a batch of problems whose forward passes are on the device: N per
// problem, problem b drawn with seed + b (the same samples as cdz_sample of
// that problem alone with that seed).  Outputs concatenated in batch order.
template <typename T>
cdz_status sample_batch(cdz_handle *h, const std::vector<DevProb<T>> &Ds, uint64_t seed, int N, uint8_t *codons,
                        int32_t *pairs) {
  const int cnt = (int)Ds.size();
  if (cnt == 0 || N == 0) return CDZ_OK;
  std::vector<Smp<T>> S(cnt);
  std::vector<size_t> need(cnt);
  size_t tot = (size_t)cnt * sizeof(Smp<T>) + 4096;
  for (int b = 0; b < cnt; b++) {
    const int n = Ds[b].n, m = Ds[b].m;
    S[b].D = Ds[b];
    S[b].seed = seed + (uint64_t)b;
    S[b].nsamp = N;
    S[b].cap = n + 16;
    S[b].gcap = (n > CDZ_NWIN + 2 ? n : CDZ_NWIN + 2) + 64;
    need[b] = (size_t)N * S[b].cap * 5 * 4 + (size_t)N * S[b].gcap * 8 + (size_t)N * n + (size_t)N * m +
              (size_t)N * n * 4 + (size_t)N * 4 + 6 * 256;
    tot += need[b];
  }
  if (tot > h->smp_bytes) {
    if (h->smp) (void)hipFree(h->smp);
    h->smp = nullptr;
    h->smp_bytes = 0;
    if (hipMalloc(&h->smp, tot) != hipSuccess) {
      (void)hipGetLastError();
      return cdz_fail(h, CDZ_ERR_NOMEM, "sampler workspace allocation failed");
    }
    h->smp_bytes = tot;
  }
  char *p = (char *)h->smp;
  auto take = [&](size_t bytes) {
    char *r = p;
    p += (bytes + 255) / 256 * 256;
    return r;
  };
  Smp<T> *dS = (Smp<T> *)take((size_t)cnt * sizeof(Smp<T>));
  for (int b = 0; b < cnt; b++) {
    const int n = Ds[b].n, m = Ds[b].m;
    S[b].stack = (int *)take((size_t)N * S[b].cap * 5 * 4);
    S[b].gbuf = (double *)take((size_t)N * S[b].gcap * 8);
    S[b].state = (signed char *)take((size_t)N * n);
    S[b].codons = (uint8_t *)take((size_t)N * m);
    S[b].pairs = (int32_t *)take((size_t)N * n * 4);
    S[b].err = (int *)take((size_t)N * 4);
  }
  hipStream_t st = h->stream;
  HIPCHK(h, hipMemcpyAsync(dS, S.data(), (size_t)cnt * sizeof(Smp<T>), hipMemcpyHostToDevice, st));
  const int total = cnt * N;
  HIPCHK(h, hipEventRecord(h->ev[4], st));
  hipLaunchKernelGGL(cdz_sample_batch_kernel<T>, dim3((total + 3) / 4), dim3(256), 0, st, dS, N, total);
  HIPCHK(h, hipGetLastError());
  HIPCHK(h, hipEventRecord(h->ev[5], st));
  std::vector<std::vector<int>> err(cnt, std::vector<int>(N));
  size_t oc = 0, op = 0;
  for (int b = 0; b < cnt; b++) {
    const int n = Ds[b].n, m = Ds[b].m;
    HIPCHK(h, hipMemcpyAsync(codons + oc, S[b].codons, (size_t)N * m, hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipMemcpyAsync(pairs + op, S[b].pairs, (size_t)N * n * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipMemcpyAsync(err[b].data(), S[b].err, (size_t)N * 4, hipMemcpyDeviceToHost, st));
    oc += (size_t)N * m;
    op += (size_t)N * n;
  }
  HIPCHK(h, hipStreamSynchronize(st));
  float ms = 0;
  HIPCHK(h, hipEventElapsedTime(&ms, h->ev[4], h->ev[5]));
  h->times[2] += ms;
  for (int b = 0; b < cnt; b++)
    for (int k = 0; k < N; k++)
      if (err[b][k])
        return cdz_fail(h, CDZ_ERR_NUMERIC, "sampling failed (problem " + std::to_string(b) + ", sample " +
                                                std::to_string(k) + ")");
  return CDZ_OK;
}
template cdz_status sample_batch<float>(cdz_handle *, const std::vector<DevProb<float>> &, uint64_t, int, uint8_t *,
                                        int32_t *);
template cdz_status sample_batch<double>(cdz_handle *, const std::vector<DevProb<double>> &, uint64_t, int,
                                         uint8_t *, int32_t *);

// cdz_sample without device allocation: the forward pass must already be in
// the handle, and the sampler's workspace is the fixed per-device scratch.
extern "C" cdz_status cdz_sample_noalloc(cdz_handle *h, const cdz_problem *prob, uint64_t seed,
                                         int32_t n_samples, uint8_t *codons, int32_t *pairs) {
  if (!h || !prob) return cdz_fail(h, CDZ_ERR_ARG, "null argument");
  if (n_samples < 0) return cdz_fail(h, CDZ_ERR_ARG, "n_samples < 0");
  if (n_samples > 0 && (!codons || !pairs)) return cdz_fail(h, CDZ_ERR_ARG, "null output");
  HostTables t;
  cdz_status s = build_tables(h, prob->n_aa, prob->aa, prob->theta1, prob->theta2, t);
  if (s != CDZ_OK) return s;
  if (!h->have_fwd || h->fwd_key != t.key)
    return cdz_fail(h, CDZ_ERR_STATE, "cdz_sample_noalloc needs the forward pass of this problem in the handle "
                                      "(call cdz_partition or cdz_marginals first)");
  char *ws = (char *)noalloc_scratch(h->device);
  if (!ws) return cdz_fail(h, CDZ_ERR_HIP, "scratch address of this device is not available");
  if (n_samples == 0) return CDZ_OK;
  return h->opt.prec == CDZ_FP64
             ? run_sample<double>(h, h->pd, seed, n_samples, codons, pairs, ws, CDZ_NOALLOC_SCRATCH_BYTES)
             : run_sample<float>(h, h->pf, seed, n_samples, codons, pairs, ws, CDZ_NOALLOC_SCRATCH_BYTES);
}

extern "C" cdz_status cdz_sample(cdz_handle *h, const cdz_problem *prob, uint64_t seed,
                                 int32_t n_samples, uint8_t *codons, int32_t *pairs) {
  if (!h || !prob) return cdz_fail(h, CDZ_ERR_ARG, "null argument");
  if (n_samples < 0) return cdz_fail(h, CDZ_ERR_ARG, "n_samples < 0");
  if (n_samples > 0 && (!codons || !pairs)) return cdz_fail(h, CDZ_ERR_ARG, "null output");
  HostTables t;
  cdz_status s = build_tables(h, prob->n_aa, prob->aa, prob->theta1, prob->theta2, t);
  if (s != CDZ_OK) return s;
  s = ensure_forward(h, t, h->fwd_adjoint && h->have_fwd && h->fwd_key == t.key);
  if (s != CDZ_OK) return s;
  if (n_samples == 0) return CDZ_OK;
  return h->opt.prec == CDZ_FP64 ? run_sample<double>(h, h->pd, seed, n_samples, codons, pairs)
                                 : run_sample<float>(h, h->pf, seed, n_samples, codons, pairs);
}
