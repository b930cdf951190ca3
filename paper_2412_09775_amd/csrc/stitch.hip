// Tiling of a field of view and stitching of restored tiles (Methods,
// "Cell-scale optical pooled screen data": a grid of tiles with 20 % overlap;
// "Organelle-scale optical pooled screen data": tiles stitched with linearly
// weighted Euclidean-distance-transform blending).
//
// A tile's weight at tile pixel (u, v) is its distance transform there -- the
// distance to the nearest pixel outside the tile, min(u + 1, T_y - u, v + 1,
// T_x - v) for a rectangle -- and the field is the weighted mean of the tiles
// that cover each pixel.
#include <math.h>

#include "../../include/waveorder.h"
#include "internal.hpp"

namespace wo {

constexpr int kMaxGrid = 32;   // tiles per axis

struct TileStarts {
  int y[kMaxGrid];
  int x[kMaxGrid];
};

// One thread per field pixel (y, x); every property plane p < P.
__global__ __launch_bounds__(256) void k_stitch(const float* __restrict__ tiles, int ny_t, int nx_t,
                                                int P, int ty, int tx, TileStarts st, int H, int W,
                                                float* __restrict__ out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)H * W) return;
  const int y = (int)(e / W), x = (int)(e - (long)y * W);
  const long tile_elems = (long)P * ty * tx;
  float den = 0.f;
  // covering tiles along each axis (starts ascend)
  int iy0 = ny_t, iy1 = -1, ix0 = nx_t, ix1 = -1;
  for (int i = 0; i < ny_t; ++i)
    if (st.y[i] <= y && y < st.y[i] + ty) { iy0 = min(iy0, i); iy1 = i; }
  for (int i = 0; i < nx_t; ++i)
    if (st.x[i] <= x && x < st.x[i] + tx) { ix0 = min(ix0, i); ix1 = i; }
  for (int iy = iy0; iy <= iy1; ++iy) {
    const int u = y - st.y[iy];
    const int du = min(u + 1, ty - u);
    for (int ix = ix0; ix <= ix1; ++ix) {
      const int v = x - st.x[ix];
      den += (float)min(du, min(v + 1, tx - v));
    }
  }
  for (int p = 0; p < P; ++p) {
    float num = 0.f;
    for (int iy = iy0; iy <= iy1; ++iy) {
      const int u = y - st.y[iy];
      const int du = min(u + 1, ty - u);
      for (int ix = ix0; ix <= ix1; ++ix) {
        const int v = x - st.x[ix];
        const float w = (float)min(du, min(v + 1, tx - v));
        const float* t = tiles + (long)(iy * nx_t + ix) * tile_elems + ((long)p * ty + u) * tx + v;
        num += w * *t;
      }
    }
    out[((long)p * H + y) * W + x] = den > 0.f ? num / den : 0.f;
  }
}

static bool smooth_even(int m) {
  if (m < 2 || (m & 1)) return false;
  for (int f : {2, 3, 5})
    while (m % f == 0) m /= f;
  return m == 1;
}

}  // namespace wo

extern "C" {

int wo_tile_grid(int32_t length, int32_t count, int32_t overlap, int32_t* tile, int32_t* starts) {
  if (length < 2 || count < 1 || count > wo::kMaxGrid || overlap < 0 || !tile || !starts)
    return WO_EINVAL;
  const long want = ((long)length + (long)(count - 1) * overlap + count - 1) / count;
  long T = want < 2 ? 2 : want;
  while (T <= 4096 && !wo::smooth_even((int)T)) ++T;
  if (T > length || T > 4096) return WO_EINVAL;
  *tile = (int32_t)T;
  for (int i = 0; i < count; ++i)
    starts[i] = count == 1 ? (int32_t)((length - T) / 2) : (int32_t)((long)i * (length - T) / (count - 1));
  return WO_OK;
}

int wo_stitch_tiles(const float* tiles, int32_t ny_t, int32_t nx_t, int32_t P, int32_t ty, int32_t tx,
                    const int32_t* ys, const int32_t* xs, int32_t H, int32_t W, float* out,
                    void* stream) {
  if (!tiles || !out || !ys || !xs || ny_t < 1 || nx_t < 1 || ny_t > wo::kMaxGrid ||
      nx_t > wo::kMaxGrid || P < 1 || ty < 1 || tx < 1 || H < 1 || W < 1)
    return WO_EINVAL;
  wo::TileStarts st;
  for (int i = 0; i < ny_t; ++i) {
    if (ys[i] < 0 || ys[i] + ty > H || (i && ys[i] < ys[i - 1])) return WO_EINVAL;
    st.y[i] = ys[i];
  }
  for (int i = 0; i < nx_t; ++i) {
    if (xs[i] < 0 || xs[i] + tx > W || (i && xs[i] < xs[i - 1])) return WO_EINVAL;
    st.x[i] = xs[i];
  }
  const long total = (long)H * W;
  wo::ScopedTiming _t("k_stitch", (hipStream_t)stream);
  hipLaunchKernelGGL(wo::k_stitch, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, tiles, ny_t, nx_t, P, ty, tx, st, H, W, out);
  return hipGetLastError() == hipSuccess ? WO_OK : WO_EHIP;
}

}  // extern "C"
