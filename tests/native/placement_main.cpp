// Placement of the pass-1 wave items (hdf::place_wave_items) on fixed and random weights: every
// item placed once, group sizes, and the busiest SIMD against the list-scheduling bound.  Built
// with the host compiler of the library at its optimisation level and, separately, under
// AddressSanitizer/UBSan.
#include <cstdio>
#include <random>
#include <vector>

#include "planner.hpp"

static int check(const std::vector<int>& loads, int wg, int ns, const char* name, int want_max = -1) {
  std::vector<int> order, nw;
  if (!hdf::place_wave_items(loads, wg, ns, order, nw)) {
    std::printf("%s: placement refused\n", name);
    return 1;
  }
  const int n = (int)loads.size(), G = (n + wg - 1) / wg;
  if ((int)nw.size() != G || (int)order.size() != n) {
    std::printf("%s: %zu groups, %zu items\n", name, nw.size(), order.size());
    return 1;
  }
  std::vector<int> seen(n, 0);
  for (int i : order) {
    if (i < 0 || i >= n || seen[i]++) {
      std::printf("%s: item %d placed twice or out of range\n", name, i);
      return 1;
    }
  }
  int total = 0, heaviest = 0, sum_nw = 0, busiest = 0;
  for (int v : loads) { total += v; heaviest = v > heaviest ? v : heaviest; }
  for (int g = 0, w0 = 0; g < G; w0 += nw[g], ++g) {
    if (nw[g] < 1 || nw[g] > wg || nw[g] < wg - (wg * G - n + G - 1) / G) {
      std::printf("%s: group %d has %d waves\n", name, g, nw[g]);
      return 1;
    }
    sum_nw += nw[g];
    for (int sm = 0; sm < ns; ++sm) {
      int l = 0;
      for (int w = sm; w < nw[g]; w += ns) l += loads[order[w0 + w]];
      busiest = l > busiest ? l : busiest;
    }
  }
  if (sum_nw != n) {
    std::printf("%s: %d waves for %d items\n", name, sum_nw, n);
    return 1;
  }
  // list scheduling: the last item placed on the busiest SIMD found it at or below the mean
  const int bins = G * ns, bound = (total + bins - 1) / bins + heaviest;
  if (busiest > bound || (want_max >= 0 && busiest != want_max)) {
    std::printf("%s: busiest SIMD %d (bound %d, expected %d)\n", name, busiest, bound, want_max);
    return 1;
  }
  return 0;
}

int main() {
  int bad = 0;
  // d = 5, degrees 0..8 (harmonics 1, 5, 14, 30, 55, 91, 140, 204, 285; radial functions 5, 5, 4,
  // 4, 3, 3, 2, 1, 1): 16-row tiles, radial ranges of at most three (one column tile) or the whole
  // degree at four column tiles with two radial functions per item
  const int nh[] = {1, 5, 14, 30, 55, 91, 140, 204, 285}, s[] = {5, 5, 4, 4, 3, 3, 2, 1, 1};
  std::vector<int> one, four;
  for (int k = 0; k < 9; ++k)
    for (int h0 = 0; h0 < nh[k]; h0 += 16) {
      for (int l0 = 0; l0 < s[k]; l0 += 3) one.push_back(s[k] - l0 < 3 ? s[k] - l0 : 3);
      for (int l0 = 0; l0 < s[k]; l0 += 2) four.push_back(4 * (s[k] - l0 < 2 ? s[k] - l0 : 2));
    }
  bad += check(one, 8, 4, "d5 one column tile", 4);
  bad += check(four, 8, 4, "d5 four column tiles");
  bad += check(one, 16, 4, "d5 sixteen waves");
  std::mt19937 rng(12345);
  for (int t = 0; t < 2000; ++t) {
    const int n = 1 + (int)(rng() % 300), top = 1 + (int)(rng() % 8);
    std::vector<int> loads(n);
    for (auto& v : loads) v = 1 + (int)(rng() % top);
    char name[64];
    std::snprintf(name, sizeof name, "random %d (n %d)", t, n);
    bad += check(loads, t % 3 == 0 ? 16 : 8, 4, name);
    if (bad) break;
  }
  // refused inputs
  std::vector<int> order, nw;
  if (hdf::place_wave_items({}, 8, 4, order, nw) || hdf::place_wave_items({1, 0, 2}, 8, 4, order, nw) ||
      hdf::place_wave_items({1, 2}, 6, 4, order, nw)) {
    std::printf("invalid inputs accepted\n");
    ++bad;
  }
  if (bad) return 1;
  std::printf("ok\n");
  return 0;
}
