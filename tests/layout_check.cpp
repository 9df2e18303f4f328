// Host-side check of the kernel weight layouts in layout.hpp: every packed
// slot's gather source and every canonical weight's scatter position agree,
// and each canonical weight appears exactly once per region.
#include <cstdio>
#include <vector>

#include "layout.hpp"

using namespace nasg;

static int check_net(int H, int NH, int K, int S, int E) {
  NetDims d{H, NH, K, S, E};
  const int64_t nw = d.num_weights();
  int bad = 0;
  // permutations are bijections
  for (int n = 0; n < H; ++n) {
    if (phys_bf16(inv_phys_bf16(n)) != n) ++bad;
    if (phys_f32(inv_phys_f32(n)) != n) ++bad;
  }
  for (int R = 0; R < 8 * K + S; ++R)
    if (inv_canon_out_row(canon_out_row(R, K), K) != R) ++bad;
  for (int R = 8 * K + S; R < d.out_rows(); ++R)
    if (canon_out_row(R, K) != -1) ++bad;
  // bf16: gather source of every slot vs scatter position of every weight
  Bf16Layout bl{d};
  std::vector<int> seen_f(nw, 0), seen_b(nw, 0);
  for (int64_t e = 0; e < bl.total_elems(); ++e) {
    int l, n, k;
    bf16_source(bl, e, l, n, k);
    if (k < 0) continue;
    int64_t ci = d.canon_off(l) + (int64_t)n * d.cols(l) + k;
    if (ci < 0 || ci >= nw) { ++bad; continue; }
    bool fwd = e < bl.fwd_elems();
    int64_t back = fwd ? bf16_fwd_pos(bl, l, n, k) : bf16_bwd_pos(bl, l, n, k);
    if (back != e) ++bad;
    (fwd ? seen_f : seen_b)[ci]++;
  }
  for (int64_t i = 0; i < nw; ++i) {
    if (seen_f[i] != 1) ++bad;
    bool layer0 = i < d.canon_off(1);
    if (seen_b[i] != (layer0 ? 0 : 1)) ++bad;
  }
  // f32
  F32Layout fl{d};
  std::vector<int> seen(nw, 0);
  for (int64_t e = 0; e < fl.total_elems(); ++e) {
    int l, n, k;
    f32_source(fl, e, l, n, k);
    if (k < 0) continue;
    int64_t ci = d.canon_off(l) + (int64_t)n * d.cols(l) + k;
    if (f32_pos(fl, l, n, k) != e) ++bad;
    seen[ci]++;
  }
  for (int64_t i = 0; i < nw; ++i)
    if (seen[i] != 1) ++bad;
  printf("H=%d NH=%d K=%d S=%d E=%d weights=%lld bad=%d\n", H, NH, K, S, E, (long long)nw, bad);
  return bad;
}

int main() {
  int bad = 0;
  for (int H : {64, 128})
    for (int NH : {1, 2, 3, 4})
      for (int K : {4, 8, 16, 32})
        for (int S : {0, 1})
          for (int E : {0, 1}) bad += check_net(H, NH, K, S, E);
  return bad != 0;
}
