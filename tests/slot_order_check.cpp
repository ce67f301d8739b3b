// Host check of the velocity slot order (test helper, built and run by
// test_slot_order_cpu.py): for many grids, with and without octants, the
// slots of all velocities are a permutation of 0 .. nv-1, decoding a slot
// gives back its node indices, and on the grids whose octants hold multiples
// of 64 velocities no 64-slot wave mixes signs of a transported component.
// Prints "ok" and exits 0 when every check holds.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <vector>

#include "../paper_2308_06196_amd/csrc/bgk_device.hpp"

using namespace bgk;

int main() {
  int bad = 0, cases = 0;
  const int grids[][3] = {{24, 24, 24}, {16, 16, 16}, {20, 20, 20}, {32, 32, 32}, {2, 2, 2},
                          {5, 5, 5},    {7, 6, 5},    {8, 3, 9},    {2, 4, 3},    {3, 2, 2}};
  const double ranges[][2] = {{-6, 6}, {-5, 5}, {-1, 3}, {0.5, 2}, {-2, -1}};
  for (int dim = 1; dim <= 3; ++dim)
    for (const auto& N : grids)
      for (const auto& r : ranges)
        for (int oct = 0; oct < 2; ++oct) {
          DevGeom g{};
          g.dim = dim;
          for (int k = 0; k < 3; ++k) {
            g.nv1[k] = N[k];
            g.vlo[k] = r[0];
            g.du[k] = (r[1] - r[0]) / (N[k] - 1);
          }
          set_velocity_slots(g, oct == 1);
          const int nv = N[0] * N[1] * N[2];
          ++cases;
          if (g.voct[8] != nv) {
            std::printf("dim %d grid %dx%dx%d: %d slots\n", dim, N[0], N[1], N[2], g.voct[8]);
            ++bad;
            continue;
          }
          std::vector<int> hits(nv, 0);
          for (int jc = 0; jc < nv; ++jc) {
            const int sl = vel_slot_of_canonical(g, jc);
            if (sl < 0 || sl >= nv) {
              ++bad;
              continue;
            }
            ++hits[sl];
            int b[3];
            slot_nodes(g, sl, b);
            if (b[0] + N[0] * (b[1] + N[1] * b[2]) != jc) ++bad;
            if (!oct && sl != jc) ++bad;  // no split: lexicographic
          }
          for (int i = 0; i < nv; ++i) bad += hits[i] != 1;
          const bool whole = oct && r[0] == -r[1] && N[0] == N[1] && N[1] == N[2] &&
                             (N[0] == 16 || N[0] == 24 || N[0] == 32);
          if (whole)
            for (int w0 = 0; w0 < nv; w0 += 64)
              for (int k = 0; k < dim; ++k) {
                int b[3];
                slot_nodes(g, w0, b);
                const bool p0 = g.vlo[k] + b[k] * g.du[k] > 0.0;
                for (int j = w0 + 1; j < w0 + 64 && j < nv; ++j) {
                  slot_nodes(g, j, b);
                  if ((g.vlo[k] + b[k] * g.du[k] > 0.0) != p0) {
                    std::printf("dim %d N %d: wave at %d mixes signs of u_%d\n", dim, N[0], w0, k);
                    ++bad;
                    break;
                  }
                }
              }
        }
  std::printf("%d grids, %d failures\n", cases, bad);
  if (bad == 0) std::printf("ok\n");
  return bad != 0;
}
