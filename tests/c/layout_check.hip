// Host-side check of the tile-interleaved layout of the FIR dictionary's bf16 signal slices
// (sig_index in the library's device helpers), built by the package build step and run by
// a CPU test.  For every column count Q = 1 .. 64 and two padded lengths it checks that
//   1. the Q real columns map one to one onto [0, Q Dp) (no gaps, no overlaps, so the
//      last tile, only w = min(16, Q - 16 (q / 16)) columns wide, takes no padding);
//   2. the filter kernels' signal loads, a lane's base sig_index(q, 8 g) plus 32 w per
//      32-sample block, land where sig_index puts sample 32 b + 8 g;
//   3. the anti-causal epilogue's reads of P's pair, sig_index(q, 4 g) plus 32 w m plus
//      16 par, land where sig_index puts sample 32 m + 16 par + 4 g;
//   4. a full 16-column tile is laid out as per tile, per 32-sample block, 16 columns of
//      32 samples.
// Exit status 0 and "layout ok" on success; the first mismatch is printed otherwise.
#include <cstdio>
#include <vector>

#include "device_common.h"

using cofem::sig_index;
using cofem::sig_tile_width;

static int fail(const char* what, long long Q, long long Dp, long long q, long long j) {
  std::printf("layout mismatch (%s): Q=%lld Dp=%lld q=%lld j=%lld\n", what, Q, Dp, q, j);
  return 1;
}

int main() {
  const int64_t lens[] = {1024, 3072};
  for (int64_t Dp : lens) {
    for (int64_t Q = 1; Q <= 64; ++Q) {
      std::vector<unsigned char> seen((size_t)(Q * Dp), 0);
      for (int64_t q = 0; q < Q; ++q) {
        const int64_t w = sig_tile_width(q, Q);
        if (w < 1 || w > 16) return fail("tile width", Q, Dp, q, 0);
        for (int64_t j = 0; j < Dp; ++j) {
          const int64_t o = sig_index(q, j, Dp, Q);
          if (o < 0 || o >= Q * Dp || seen[(size_t)o]) return fail("bijection", Q, Dp, q, j);
          seen[(size_t)o] = 1;
          if (w == 16 && o != ((((q >> 4) * (Dp >> 5) + (j >> 5)) * 16 + (q & 15)) * 32 + (j & 31)))
            return fail("full tile", Q, Dp, q, j);
        }
        for (int64_t g = 0; g < 4; ++g)
          for (int64_t b = 0; b < (Dp >> 5); ++b) {
            if (sig_index(q, 8 * g, Dp, Q) + 32 * w * b != sig_index(q, 32 * b + 8 * g, Dp, Q))
              return fail("signal load stride", Q, Dp, q, 32 * b + 8 * g);
            for (int64_t par = 0; par < 2; ++par)
              if (sig_index(q, 4 * g, Dp, Q) + 32 * w * b + 16 * par != sig_index(q, 32 * b + 16 * par + 4 * g, Dp, Q))
                return fail("epilogue P pair", Q, Dp, q, 32 * b + 16 * par + 4 * g);
          }
      }
    }
  }
  std::printf("layout ok\n");
  return 0;
}
