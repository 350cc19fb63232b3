// Host build of the reverse-mode Riemann flux header, for a CPU test against
// the oracle's automatic differentiation.  Reads "DIM hllc count" and then,
// per case, qL qR n gF; prints gL gR, one case per line.
#include <cmath>
#include <cstdio>

#define __device__
namespace hfv {
using std::sqrt;
}
#include "../paper_2510_25906_amd/csrc/hfv_riemann_adj.hpp"

template <int DIM>
static int run(int hllc, int count) {
  constexpr int NV = DIM + 2;
  for (int c = 0; c < count; ++c) {
    double qL[NV], qR[NV], n[DIM], gF[NV], gL[NV], gR[NV];
    for (double &x : qL) if (scanf("%lf", &x) != 1) return 1;
    for (double &x : qR) if (scanf("%lf", &x) != 1) return 1;
    for (double &x : n) if (scanf("%lf", &x) != 1) return 1;
    for (double &x : gF) if (scanf("%lf", &x) != 1) return 1;
    hfv::riemann_vjp<DIM, double>(qL, qR, n, 1.4, hllc, gF, gL, gR);
    for (double x : gL) printf("%.17g ", x);
    for (double x : gR) printf("%.17g ", x);
    printf("\n");
  }
  return 0;
}

int main() {
  int dim, hllc, count;
  if (scanf("%d %d %d", &dim, &hllc, &count) != 3) return 1;
  return dim == 2 ? run<2>(hllc, count) : run<3>(hllc, count);
}
