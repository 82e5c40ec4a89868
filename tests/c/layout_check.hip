// Host-side check of the tile-interleaved layout of the FIR dictionary's bf16 signal slices
// (sig_index in the library's device helpers), built by the package build step and run by
// a CPU test.  For every column count Q = 1 .. 64 and two padded lengths it checks that
//   1. the Q real columns map one to one onto [0, Q Dp) (no gaps, no overlaps, so the
//      last tile, only w = min(16, Q - 16 (q / 16)) columns wide, takes no padding);
//   2. the filter kernels' signal loads, a lane's base sig_index(q, 8 g) plus 32 w per
//      32-sample block, land where sig_index puts sample 32 b + 8 g;
//   3. a full 16-column tile is laid out as per tile, per 32-sample block, 16 columns of
//      32 samples;
// and, independent of Q, the two lane regroupings of the one-launch bf16 operator within a
// 32-sample block (operand lane g holds rows 8 g .. 8 g + 7; output lane g of half par
// holds rows 16 par + 4 g .. + 3):
//   4. V, output to operand: operand lane g' element j takes output lane 2 (g' & 1) + (j >> 2)
//      of half g' >> 1, element j & 3;
//   5. the epilogue's Pd, operand to output: output lane g of half par element e takes
//      operand lane 2 par + (g >> 1), element 4 (g & 1) + e.
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
          }
      }
    }
  }
  // the regroupings: rows of a 32-sample block
  auto operand_row = [](int g, int j) { return 8 * g + j; };
  auto output_row = [](int par, int g, int e) { return 16 * par + 4 * g + e; };
  for (int gp = 0; gp < 4; ++gp)
    for (int j = 0; j < 8; ++j)
      if (output_row(gp >> 1, 2 * (gp & 1) + (j >> 2), j & 3) != operand_row(gp, j))
        return fail("V regrouping", 0, 32, gp, j);
  for (int par = 0; par < 2; ++par)
    for (int g = 0; g < 4; ++g)
      for (int e = 0; e < 4; ++e)
        if (operand_row(2 * par + (g >> 1), 4 * (g & 1) + e) != output_row(par, g, e))
          return fail("epilogue Pd regrouping", par, 32, g, e);
  std::printf("layout ok\n");
  return 0;
}
