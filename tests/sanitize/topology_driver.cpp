// Test driver (host only): runs the library's forest topology
// (paper_2605_07612_amd/csrc/topology.cpp) on a script read from stdin and
// prints every leaf table and remap list, so that a test can build it with
// AddressSanitizer and UndefinedBehaviorSanitizer and compare the output with
// the oracle's forest.
//
// stdin:  ndim nt0 nt1 nt2 per0 per1 per2 init_level lmin lmax n_regrids
//         then per regrid: n_blocks flags...
// stdout: per regrid "changed c nb", then nb lines "level g0 g1 g2 op src arg"
#include <cstdio>
#include <vector>

#include "foap4_internal.h"

int main() {
  int ndim, nt[3], per[3], init, lmin, lmax, n;
  if (std::scanf("%d %d %d %d %d %d %d %d %d %d %d", &ndim, &nt[0], &nt[1], &nt[2], &per[0], &per[1], &per[2],
                 &init, &lmin, &lmax, &n) != 11)
    return 2;
  f4::Topology t;
  t.init_uniform(ndim, nt, init);
  for (int a = 0; a < 3; a++) t.periodic[a] = per[a];
  std::printf("init %zu\n", t.leaves.size());
  for (const f4::Leaf &L : t.leaves) std::printf("%d %d %d %d\n", L.level, L.g[0], L.g[1], L.g[2]);
  for (int r = 0; r < n; r++) {
    long nb;
    if (std::scanf("%ld", &nb) != 1 || nb != (long)t.leaves.size()) return 3;
    std::vector<int8_t> flags(nb);
    for (long i = 0; i < nb; i++) {
      int f;
      if (std::scanf("%d", &f) != 1) return 4;
      flags[i] = (int8_t)f;
    }
    std::vector<f4::Leaf> out;
    std::vector<int32_t> op, src, arg;
    const bool changed = t.regrid(flags.data(), lmin, lmax, out, op, src, arg);
    std::printf("changed %d %zu\n", changed ? 1 : 0, changed ? out.size() : t.leaves.size());
    if (!changed) continue;
    for (size_t i = 0; i < out.size(); i++)
      std::printf("%d %d %d %d %d %d %d\n", out[i].level, out[i].g[0], out[i].g[1], out[i].g[2], op[i], src[i], arg[i]);
    t.leaves = out;
    t.sort_and_index();
  }
  return 0;
}
