// Workgroup -> output tile schedule of the FP64 GEMM (host and device; no HIP runtime calls, so a
// host compiler can build it with __host__ and __device__ defined empty).
#pragma once
#include <cmath>
#include <cstdint>

namespace cf {

// Tile schedule.  Workgroups go to the 8 XCDs round-robin in launch order and every XCD has its
// own L2.  With remap, XCD x takes the contiguous range [x*per, (x+1)*per) of the (batch item,
// tile) sequence, and the tiles of one batch item are ordered in bands of 8 tile rows swept column
// by column, so that the tiles resident on one XCD at a time form compact blocks that share their
// A and B panels.  remap 2 enumerates only the lower trapezoid (diagonal included) of a grid with
// at least as many tile rows as tile columns -- row r holds min(r + 1, tiles_n) tiles -- so no
// workgroup is launched for a skipped tile.
__host__ __device__ inline bool tile_map(int remap, int tiles_m, int tiles_n, int64_t nx, int64_t nz,
                                         int64_t bx, int64_t bz, int64_t& z, int& tm, int& tn) {
  if (!remap) {
    tm = (int)(bx / tiles_n);
    tn = (int)(bx % tiles_n);
    z = bz;
    return true;
  }
  const int64_t gid = bz * nx + bx;
  const int64_t total = nx * nz;
  const int64_t base = total / 8, rem = total % 8, x = gid % 8;   // XCD x owns base (+1 if x < rem) items
  const int64_t tg = x * base + (x < rem ? x : rem) + gid / 8;
  if (tg >= total) return false;
  z = tg / nx;
  const int64_t t = tg % nx;
  constexpr int G = 8;
  if (remap == 2) {
    const int64_t tri = (int64_t)tiles_n * (tiles_n + 1) / 2;                     // the square's triangle
    auto T = [=](int64_t R) { return R <= tiles_n ? R * (R + 1) / 2 : tri + (R - tiles_n) * tiles_n; };
    auto S = [=](int64_t q) { return T(q * G < tiles_m ? q * G : tiles_m); };     // tiles in rows < qG
    const int64_t R = t < tri ? (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5)
                              : tiles_n + (t - tri) / tiles_n;                       // row of tile t, about
    int64_t q = R / G;
    while (q > 0 && S(q) > t) --q;
    while (S(q + 1) <= t) ++q;
    const int64_t r0 = q * G;
    const int rows = (int)(tiles_m - r0 < G ? tiles_m - r0 : G);
    int64_t u = t - S(q);
    if (u < rows * r0) {
      tn = (int)(u / rows);
      tm = (int)(r0 + u % rows);
    } else {
      u -= rows * r0;
      int c = 0;
      while (u >= rows - c) {
        u -= rows - c;
        ++c;
      }
      tn = (int)(r0 + c);
      tm = (int)(r0 + c + u);
    }
  } else {
    const int64_t span = (int64_t)G * tiles_n;
    const int64_t q = t / span;
    const int64_t r0 = q * G;
    const int rows = (int)(tiles_m - r0 < G ? tiles_m - r0 : G);
    const int64_t u = t - q * span;
    tn = (int)(u / rows);
    tm = (int)(r0 + u % rows);
  }
  return true;
}

}  // namespace cf
