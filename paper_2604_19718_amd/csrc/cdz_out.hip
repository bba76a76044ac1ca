// cdz_out.hip -- outside (adjoint) pass; workspace carving for now.
#include "cdz_internal.h"

template <typename T>
void adj_carve(size_t &off, char *base, const HostTables &t, DevAdj<T> &A, size_t S2) {
  auto take = [&](size_t bytes) -> char * {
    off = (off + 255) / 256 * 256;
    char *p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  T **arrs[] = {&A.Qbb, &A.Qm1b, &A.Qm1pb, &A.QmXb, &A.QmXbt, &A.Qmb, &A.DIb, &A.Gb, &A.Fb, &A.Ub};
  for (T **a : arrs) *a = reinterpret_cast<T *>(take(S2 * sizeof(T)));
  A.eta = reinterpret_cast<double *>(take((size_t)t.n * 36 * sizeof(double)));
  A.out = reinterpret_cast<double *>(take(16 * sizeof(double)));
}
template void adj_carve<float>(size_t &, char *, const HostTables &, DevAdj<float> &, size_t);
template void adj_carve<double>(size_t &, char *, const HostTables &, DevAdj<double> &, size_t);
