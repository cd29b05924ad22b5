// ThreadSanitizer driver of the split search's worker threads (conv_split_search_many): twelve
// kernels on six threads, twice, so that the second pass reads the reduced-problem SVDs the first
// one cached in the shared context. Built with the split model's source alone (set_error stubbed).
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "convsplit.h"

namespace convreal {
void set_error(const std::string&) {}
}  // namespace convreal

int main() {
  const int lmax = 512, n = 12, ng = 6;
  std::vector<double> K(static_cast<size_t>(n) * (lmax + 1));
  for (int k = 0; k < n; ++k) {
    const double s = (15.0 + 5.0 * k) * M_PI / (180.0 * 60.0) / std::sqrt(8.0 * std::log(2.0));
    for (int l = 0; l <= lmax; ++l)
      K[k * (lmax + 1) + l] = l < 2 ? 0.0 : std::exp(-0.5 * l * (l + 1.0) * s * s) / std::sqrt(l * (l + 1.0));
  }
  conv_split_ctx* ctx = nullptr;
  if (conv_split_create(&ctx, lmax, nullptr, 0.3, 1e-6) != 0) return 1;
  if (conv_split_set_max_compensation(ctx, 1e-2) != 0) return 1;
  std::vector<double> bounds(n, 1e-5), grid(static_cast<size_t>(n) * ng), th(n), wl(n), sg(n);
  std::vector<int> lc(n);
  for (int k = 0; k < n; ++k)
    for (int g = 0; g < ng; ++g) grid[k * ng + g] = 0.02 + 0.045 * g;
  const conv_cost_model m{1e-4, 1e-13, 3e-12};
  for (int rep = 0; rep < 2; ++rep)
    if (conv_split_search_many(ctx, K.data(), n, 256, bounds.data(), 5.0, grid.data(), ng, 4, &m, 6, th.data(),
                               lc.data(), wl.data(), sg.data()) != 0)
      return 2;
  for (int k = 0; k < n; ++k) std::printf("%d %.4f %d %.3e\n", k, th[k], lc[k], sg[k]);
  conv_split_destroy(ctx);
  return 0;
}
