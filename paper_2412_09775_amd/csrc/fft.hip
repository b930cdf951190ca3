// FFT passes and the per-frequency operators of the linear model.
//
// A 3D real transform is three passes over HBM: rows along X (real <-> half
// spectrum, two real rows packed into one complex line), columns along Y
// (strided, tiles of W contiguous half-spectrum columns staged through LDS),
// and columns along Z.  The Z pass is fused with the per-frequency operator
// (forward H F, Tikhonov solve, or adjoint H^H R) and the inverse Z transform,
// so the spectrum of every channel visits HBM once between the Y passes.
#include "internal.hpp"

namespace wo {

// ------------------------------------------------------------------ rows

__device__ __forceinline__ long group_row(long r, long rpg, long stride) {
  const long g = r / rpg;
  return g * stride + (r - g * rpg);
}

template <int NS>
__global__ __launch_bounds__(1024) void k_rows_r2c(const float* __restrict__ in,
                                                   float2* __restrict__ out, int X, RowGroups g,
                                                   FftPlan plan, int lines_per_wg, long nlines,
                                                   int KT, int OP) {
  extern __shared__ float2 smem[];
  float2* tw = smem;
  float2* buf = smem + X;
  // element offsets of the line's rows (row index times the row pitch), -1
  // for a missing row: no 64-bit multiply per element
  __shared__ long rin[2 * 64], rout[2 * 64];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const long nrows = g.rows_per_group * g.ngroups;
  const long line0 = (long)blockIdx.x * lines_per_wg;
  const int nl = (int)min((long)lines_per_wg, nlines - line0);
  for (int t = tid; t < 2 * nl; t += nthr) {
    const long r = 2 * line0 + t;
    rin[t] = r < nrows ? group_row(r, g.rows_per_group, g.in_stride) * X : -1;
    rout[t] = r < nrows ? group_row(r, g.rows_per_group, g.out_stride) * OP : -1;
  }
  __syncthreads();
  const int Xc = NS > 0 ? NS : X;   // compile-time length for the index arithmetic
  const int PS = pad_shift(Xc);   // row padding
  const int LS = row_stride(Xc);    // padded line pitch in LDS
  // a missing second row (odd row count) loads the first row again and is
  // zeroed after the loads
  auto load = [&](int l, int i) {
    const long ra = rin[2 * l], rb = rin[2 * l + 1];
    return make_float2(in[ra + i], in[(rb >= 0 ? rb : ra) + i]);
  };
  auto finish = [&](int l, int, float2 v) { return make_float2(v.x, rin[2 * l + 1] >= 0 ? v.y : 0.f); };
  // the twiddle-table loads are issued first and written to LDS once the data
  // loads are in flight
  TwFetch twf;
  tw_begin(twf, tw, Xc, tid, nthr);
  if constexpr (NS > 0) {
    // first pass straight from memory; radices 8 ... 8 16 where that saves a
    // pass (the first radix is the same)
    static_assert(OrderedPlan<NS, false, true>::radix(0) == OrderedPlan<NS, false>::radix(0), "first pass");
    first_pass_in2<NS, 0, false, kEmax, true, false>(buf, nl, 1, LS, -1, -1.f, tid, nthr, load, finish,
                                                     [&] { tw_end(twf, tw, Xc, tid, nthr); });
    static_passes<NS, 0, false, kEmax, true, false, 1, StaticPlan<NS, true>::passes(), true>(
        buf, nl, 1, LS, -1, tw, -1.f, tid, nthr);
  } else {
    tw_end(twf, tw, Xc, tid, nthr);
    gather2_to_lds(buf, nl * Xc, tid, nthr, [&](int e) {
      const int l = e / Xc;
      return load(l, e - l * Xc);
    }, [&](int e, float2 v) { return finish(e / Xc, 0, v); }, [&](int e) {
      const int l = e / Xc;
      return l * LS + row_slot(e - l * Xc, PS);
    }, [] {});
    __syncthreads();
    fft_lines<NS, 0, false, kEmax, true>(buf, LdsLines{nl, 1, LS, false, -1, true}, plan, tw, -1.f, tid,
                                         nthr);
  }
  // half-spectrum columns k < KT (all Xh, or the band a caller keeps), row pitch OP
  const float inv_kt = 1.0f / (float)KT;
#pragma unroll
  for (int i = 0; i < kEmax; ++i) {
    const int e = tid + i * nthr;
    if (e < nl * KT) {
      const int l = div_small(e, inv_kt), k = e - l * KT;
      const float2 zk = buf[l * LS + row_slot(k, PS)];
      const float2 zm = buf[l * LS + row_slot(k == 0 ? 0 : Xc - k, PS)];
      const float2 A = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
      const float2 B = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
      out[rout[2 * l] + k] = A;
      if (rout[2 * l + 1] >= 0) out[rout[2 * l + 1] + k] = B;
    }
  }
}

template <int NS>
__global__ __launch_bounds__(1024) void k_rows_c2r(const float2* __restrict__ in,
                                                   float* __restrict__ out, int X, RowGroups g,
                                                   FftPlan plan, int lines_per_wg, long nlines,
                                                   float scale, int KT, int IP) {
  extern __shared__ float2 smem[];
  float2* tw = smem;
  float2* buf = smem + X;
  __shared__ long rin[2 * 64], rout[2 * 64];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const long nrows = g.rows_per_group * g.ngroups;
  const long line0 = (long)blockIdx.x * lines_per_wg;
  const int nl = (int)min((long)lines_per_wg, nlines - line0);
  for (int t = tid; t < 2 * nl; t += nthr) {   // element offsets, as in k_rows_r2c
    const long r = 2 * line0 + t;
    rin[t] = r < nrows ? group_row(r, g.rows_per_group, g.in_stride) * IP : -1;
    rout[t] = r < nrows ? group_row(r, g.rows_per_group, g.out_stride) * X : -1;
  }
  __syncthreads();
  const int Xc = NS > 0 ? NS : X;   // compile-time length for the index arithmetic
  const int PS = pad_shift(Xc);   // row padding
  const int LS = row_stride(Xc);    // padded line pitch in LDS
  auto slot = [&](int e) {
    const int l = e / Xc;
    return l * LS + row_slot(e - l * Xc, PS);
  };
  // input rows of pitch IP hold the half-spectrum columns k < KT; the
  // columns beyond are zero (the condition depends on the index only, so the
  // loads stay in flight together)
  auto load = [&](int l, int k) {
    const int kk = 2 * k > Xc ? Xc - k : k;
    const long ra = rin[2 * l], rb = rin[2 * l + 1];
    float2 A = make_float2(0.f, 0.f), B = A;
    if (kk < KT) {
      A = in[ra + kk];
      B = in[(rb >= 0 ? rb : ra) + kk];
    }
    return make_float4(A.x, A.y, B.x, B.y);
  };
  auto finish = [&](int l, int k, float4 v) {
    const bool mirror = 2 * k > Xc;
    const int kk = mirror ? Xc - k : k;
    float2 A = make_float2(v.x, v.y), B = make_float2(v.z, v.w);
    if (rin[2 * l + 1] < 0) B = make_float2(0.f, 0.f);
    if (kk == 0 || 2 * kk == Xc) { A.y = 0.f; B.y = 0.f; }   // Re of the inverse ignores them
    if (mirror) { A.y = -A.y; B.y = -B.y; }
    return make_float2(A.x - B.y, A.y + B.x);
  };
  // nontemporal stores: the real result is not read again by the call, so it
  // need not displace the spectra the next passes read from the caches
  // (label-free 96x512x512: 71 -> 58 us)
  auto store = [&](int l, int i, float2 v) {
    __builtin_nontemporal_store(v.x * scale, &out[rout[2 * l] + i]);
    if (rout[2 * l + 1] >= 0) __builtin_nontemporal_store(v.y * scale, &out[rout[2 * l + 1] + i]);
  };
  TwFetch twf;   // as in k_rows_r2c
  tw_begin(twf, tw, Xc, tid, nthr);
  if constexpr (NS > 0) {
    // first pass straight from memory, last pass straight to memory (the
    // 8 ... 8 16 plan of k_rows_r2c is slower here: its 16-point last pass
    // stores from half the threads, 320 -> 339 us on 4 x 64 x 1024 rows of 1024)
    constexpr int NP = StaticPlan<NS>::passes();
    first_pass_in2<NS, 0, false, kEmax, true, false>(buf, nl, 1, LS, -1, 1.f, tid, nthr, load, finish,
                                                     [&] { tw_end(twf, tw, Xc, tid, nthr); });
    static_passes<NS, 0, false, kEmax, true, false, 1, NP - 1>(buf, nl, 1, LS, -1, tw, 1.f, tid, nthr);
    last_pass_out<NS, 0, false, kEmax, true, false>(buf, nl, 1, LS, -1, tw, 1.f, tid, nthr, store);
  } else {
    tw_end(twf, tw, Xc, tid, nthr);
    gather2_to_lds(buf, nl * Xc, tid, nthr, [&](int e) {
      const int l = e / Xc;
      return load(l, e - l * Xc);
    }, [&](int e, float4 v) {
      const int l = e / Xc;
      return finish(l, e - l * Xc, v);
    }, slot, [] {});
    __syncthreads();
    fft_lines<NS, 0, false, kEmax, true>(buf, LdsLines{nl, 1, LS, false, -1, true}, plan, tw, 1.f, tid,
                                         nthr);
    scatter_from_lds_map(buf, nl * Xc, tid, nthr, slot, [&](int e, float2 v) {
      const int l = e / Xc;
      store(l, e - l * Xc, v);
    });
  }
}

// 2048 elements per workgroup (256 threads of 8): measured on the row passes
// of 1024- and 512-point rows against 1024 to 8192 elements and 2 to 8 per
// thread, the C2R pass is 3-4 % faster than with 4096 and the R2C pass equal
// within the run-to-run spread.
static int lines_per_wg_for(int X) {
  int L = 2048 / X;
  if (L < 1) L = 1;
  if (L > 64) L = 64;
  while (L > 1 && (long)L * X > kMaxElems) --L;
  return L;
}

// Lengths with compiled stages.
static bool compiled_length(int n) {
  switch (n) {
#define X_(NN) case NN:
    WO_ALL_SIZES(X_)
#undef X_
    return true;
    default:
      return false;
  }
}


static bool rows_choice_ok(int X, const FftChoice& c) {
  const long elems = (long)c.w * X;
  return c.w >= 1 && c.w <= 64 && elems <= kMaxElems && threads_ok(c.threads, elems) &&
         (long)(X + (long)c.w * row_stride(X)) * (long)sizeof(float2) <= lds_limit_bytes() &&
         c.plan >= 0 && c.plan <= 3;
}

static FftChoice rows_default(int X) {
  const int L = lines_per_wg_for(X);
  return FftChoice{L, threads_for((long)L * X), 0};
}

// Table entry for the launch, or the default; an entry the device cannot run
// falls back to the default.
static FftChoice rows_choice(const FftKey& k) {
  FftChoice c;
  if (fft_lookup(k, &c) && rows_choice_ok(k.n, c)) return c;
  return rows_default(k.n);
}

#define WO_CASE_ROWS(K, NN)                                                                      \
  case NN:                                                                                       \
    hipLaunchKernelGGL((K<NN>), dim3((unsigned)nwg), dim3(thr), lds, s, WO_ROWS_ARGS);          \
    return hipGetLastError();

hipError_t launch_rows_r2c(const float* in, float2* out, int X, const RowGroups& g, hipStream_t s,
                           int kt, int pitch, const char* tag) {
  const int Xh = X / 2 + 1;
  const int KT = kt > 0 ? kt : Xh, OP = pitch > 0 ? pitch : Xh;
  if (KT > Xh || OP < KT) return hipErrorInvalidValue;
  const long nrows = g.rows_per_group * g.ngroups;
  const FftKey key{kFftRowsR2C, X, 0, nrows, 0};
  if (fft_recording()) fft_record(key, [=] { return launch_rows_r2c(in, out, X, g, s, KT, OP, tag); });
  const FftChoice c = rows_choice(key);
  FftPlan plan;
  if (!make_plan_variant(X, c.plan, &plan)) return hipErrorInvalidValue;
  const long nlines = (nrows + 1) / 2;
  const int L = c.w;
  const long nwg = (nlines + L - 1) / L;
  const int thr = c.threads;
  const size_t lds = (size_t)(X + (long)L * row_stride(X)) * sizeof(float2);
  ScopedTiming _t(tag, s);
#define WO_ROWS_ARGS in, out, X, g, plan, L, nlines, KT, OP
#define X_(NN) WO_CASE_ROWS(k_rows_r2c, NN)
  if (c.plan == 0) switch (X) {
      WO_LATERAL_SIZES(X_)
      default:
        break;
    }
  hipLaunchKernelGGL((k_rows_r2c<0>), dim3((unsigned)nwg), dim3(thr), lds, s, WO_ROWS_ARGS);
#undef X_
#undef WO_ROWS_ARGS
  return hipGetLastError();
}

hipError_t launch_rows_c2r(const float2* in, float* out, int X, const RowGroups& g, float scale,
                           hipStream_t s, int kt, int pitch) {
  const int Xh = X / 2 + 1;
  const int KT = kt > 0 ? kt : Xh, IP = pitch > 0 ? pitch : Xh;
  if (KT > Xh || IP < KT) return hipErrorInvalidValue;
  const long nrows = g.rows_per_group * g.ngroups;
  const FftKey key{kFftRowsC2R, X, 0, nrows, 0};
  if (fft_recording()) fft_record(key, [=] { return launch_rows_c2r(in, out, X, g, scale, s, KT, IP); });
  const FftChoice c = rows_choice(key);
  FftPlan plan;
  if (!make_plan_variant(X, c.plan, &plan)) return hipErrorInvalidValue;
  const long nlines = (nrows + 1) / 2;
  const int L = c.w;
  const long nwg = (nlines + L - 1) / L;
  const int thr = c.threads;
  const size_t lds = (size_t)(X + (long)L * row_stride(X)) * sizeof(float2);
  ScopedTiming _t("k_rows_c2r", s);
#define WO_ROWS_ARGS in, out, X, g, plan, L, nlines, scale, KT, IP
#define X_(NN) WO_CASE_ROWS(k_rows_c2r, NN)
  if (c.plan == 0) switch (X) {
      WO_LATERAL_SIZES(X_)
      default:
        break;
    }
  hipLaunchKernelGGL((k_rows_c2r<0>), dim3((unsigned)nwg), dim3(thr), lds, s, WO_ROWS_ARGS);
#undef X_
#undef WO_ROWS_ARGS
  return hipGetLastError();
}

// ------------------------------------------------------------------ columns

// Band rows of a compact plane: index b of the nb = 2 ky + 1 band rows is row b
// (b <= ky) or row Y - nb + b; nb = Y (ky >= Y) is every row.
__device__ __forceinline__ int band_row(int b, int ky, int nb, int Y) {
  return b <= ky ? b : b + (Y - nb);
}
__device__ __forceinline__ bool in_band(int y, int ky, int nb, int Y) {
  return nb == Y || y <= ky || y >= Y - (nb - ky - 1);
}

// band: 0 every row; 1 stores only the band rows (ky, nb) of the transform;
// 2 loads only the band rows (the others are taken as zero).  At most 64
// VGPRs (8 waves per SIMD), so that two 1024-thread workgroups share a CU.
template <int NS, int WS>
__global__ __launch_bounds__(1024, 8) void k_cols(float2* __restrict__ data, int N, long M, int Wrt,
                                               long tiles_m, long planes_per_group,
                                               long group_stride, FftPlan plan, float sign,
                                               int band, int ky, int nb) {
  const int W = WS > 0 ? WS : Wrt;             // a power of two
  const int wsh = WS > 0 ? pow2_shift(WS) : pow2_shift(Wrt);
  extern __shared__ float2 smem[];
  float2* tw = smem;
  float2* buf = smem + N;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const long bid = xcd_block();
  const long tile = bid % tiles_m;
  const long plane = bid / tiles_m;
  const long pg = plane / planes_per_group, pi = plane - pg * planes_per_group;
  float2* base = data + (pg * group_stride + pi) * (long)N * M;
  const long m0 = tile * W;
  const int weff = (int)min((long)W, M - m0);
  const int Nc = NS > 0 ? NS : N;
  auto ld_ok = [&](int l, int n) { return l < weff && (band != 2 || in_band(n, ky, nb, Nc)); };
  auto st_ok = [&](int l, int n) { return l < weff && (band != 1 || in_band(n, ky, nb, Nc)); };
  TwFetch twf;   // as in the row passes
  tw_begin(twf, tw, Nc, tid, nthr);
  if constexpr (NS > 0) {
    // line l = column m0 + l; first pass straight from memory, last pass
    // straight to memory.  Element offsets within the plane in 32 bits (the
    // host launches the compiled lengths only for M < 2^24 and planes below
    // 2^32 elements): a 24-bit multiply-add per element instead of a 64-bit
    // product (about 9 VALU instructions per load or store before)
    const unsigned um = (unsigned)M, uc = (unsigned)m0;
    auto off = [&](int l, int n) { return __umul24((unsigned)n, um) + uc + (unsigned)l; };
    fft_direct<NS, WS, true, kEmax, false>(
        buf, W, W, 1, wsh, tw, sign, tid, nthr,
        [&](int l, int n) { return ld_ok(l, n) ? base[off(l, n)] : make_float2(0.f, 0.f); },
        [&] { tw_end(twf, tw, Nc, tid, nthr); },
        [&](int l, int n, float2 v) {
          if (st_ok(l, n)) base[off(l, n)] = v;
        });
  } else {
    tw_end(twf, tw, Nc, tid, nthr);
    gather_to_lds(buf, Nc * W, tid, nthr, [&](int e) {
      const int n = e >> wsh, w = e & (W - 1);
      return ld_ok(w, n) ? base[(long)n * M + m0 + w] : make_float2(0.f, 0.f);
    }, [] {});
    __syncthreads();
    fft_lines<NS, WS, true>(buf, LdsLines{W, W, 1, true, wsh}, plan, tw, sign, tid, nthr);
    scatter_from_lds(buf, Nc * W, tid, nthr, [&](int e, float2 v) {
      const int n = e >> wsh, w = e & (W - 1);
      if (st_ok(w, n)) base[(long)n * M + m0 + w] = v;
    });
  }
}

// k_cols for a compiled length and tile width as a loop over tiles: workgroup
// g of G transforms tiles g, g + G, ... and issues the loads of its next tile
// right after the first pass of the current one, so that they are in flight
// during its remaining passes and stores.
template <int NS, int WS>
__global__ __launch_bounds__(1024) void k_cols_loop(float2* __restrict__ data, long M, long tiles_m,
                                                    long planes_per_group, long group_stride,
                                                    long total, float sign, int band, int ky,
                                                    int nb) {
  static_assert(NS > 0 && WS > 0, "compiled length and tile width");
  constexpr int W = WS;
  constexpr int NP = StaticPlan<NS>::passes();
  const int wsh = pow2_shift(WS);
  extern __shared__ float2 smem[];
  float2* tw = smem;
  float2* buf = smem + NS;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const long G = gridDim.x;
  auto tile_at = [&](long t, long& m0, int& weff) {
    const long tile = t % tiles_m, plane = t / tiles_m;
    const long pg = plane / planes_per_group, pi = plane - pg * planes_per_group;
    m0 = tile * W;
    weff = (int)min((long)W, M - m0);
    return data + (pg * group_stride + pi) * (long)NS * M;
  };
  auto issue = [&](FirstPassRaw<NS, kEmax, false>& raw, long t) {
    long m0;
    int weff;
    const float2* base = tile_at(t, m0, weff);
    first_pass_load<NS, WS, true, kEmax, false, false>(raw, W, wsh, tid, nthr, [&](int l, int n) {
      return l < weff && (band != 2 || in_band(n, ky, nb, NS)) ? base[(long)n * M + m0 + l]
                                                               : make_float2(0.f, 0.f);
    });
  };
  fill_twiddles(tw, NS, tid, nthr);   // before the loads, as in the row passes
  FirstPassRaw<NS, kEmax, false> raw;
  long t = xcd_block();   // G <= total: every workgroup has a first tile
  issue(raw, t);
  while (t < total) {
    long m0;
    int weff;
    float2* base = tile_at(t, m0, weff);
    first_pass_store<NS, WS, true, kEmax, false, false>(raw, buf, W, W, 1, wsh, sign, tid, nthr,
                                                        [](int, int, float2 v) { return v; });
    const long tn = t + G;
    if (tn < total) issue(raw, tn);
    static_passes<NS, WS, true, kEmax, false, false, 1, NP - 1>(buf, W, W, 1, wsh, tw, sign, tid, nthr);
    last_pass_out<NS, WS, true, kEmax, false, false>(buf, W, W, 1, wsh, tw, sign, tid, nthr,
                                                     [&](int l, int n, float2 v) {
                                                       if (l < weff && (band != 1 || in_band(n, ky, nb, NS)))
                                                         base[(long)n * M + m0 + l] = v;
                                                     });
    t = tn;
  }
}

// Column tile width: W contiguous complex values per row (W = 16 is one
// 128-byte segment), limited by the elements a workgroup may own and by the
// device's LDS per workgroup (twiddles + tile).
static int tile_width(int n, int ch) {
  const long lim = lds_limit_bytes() / (long)sizeof(float2);
  int W = 16;
  while (W > 1 && ((long)W * n * ch > kMaxElems || n + (long)W * n * ch > lim)) W /= 2;
  return W;
}

// Static tile width for a compiled length: 16 columns when the tile fits the
// per-workgroup element budget, else the largest power of two that does.
constexpr int static_tile_width(int n) {
  int W = 16;
  while (W > 1 && W * n > kMaxElems) W /= 2;
  return W;
}

// Schedule plan 4: the compiled transform with the compiled tile width, as the
// tile loop k_cols_loop.
constexpr int kPlanColsLoop = 4;

static bool cols_choice_ok(int N, const FftChoice& c) {
  const long elems = (long)c.w * N;
  const bool loop_ok = c.plan == kPlanColsLoop && compiled_length(N) && c.w == static_tile_width(N);
  return pow2_shift(c.w) >= 0 && c.w <= 64 && elems <= kMaxElems && threads_ok(c.threads, elems) &&
         (long)(N + elems) * (long)sizeof(float2) <= lds_limit_bytes() && c.plan >= 0 &&
         (c.plan <= 3 || loop_ok);
}

// Workgroups of a tile loop: as many as are resident on the device at once
// (all of them when the occupancy query fails), at most one per tile.
static long loop_grid(const void* fn, int thr, size_t lds, long total) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, thr, lds) != hipSuccess || per < 1 || cus < 1)
    return total;
  return std::min(total, (long)per * cus);
}

static FftChoice cols_default(int N) {
  const int W = compiled_length(N) && (long)(N + static_tile_width(N) * N) * (long)sizeof(float2) <=
                                          lds_limit_bytes()
                    ? static_tile_width(N)
                    : tile_width(N, 1);
  return FftChoice{W, threads_for((long)N * W), 0};
}

hipError_t launch_cols(float2* data, int N, long M, long planes_per_group, long group_stride,
                       long ngroups, float sign, hipStream_t s, const char* tag, int band, int ky) {
  if (band < 0 || band > 2 || (band != 0 && ky < 0)) return hipErrorInvalidValue;
  const int nb = band == 0 || 2L * ky + 1 >= N ? N : 2 * ky + 1;
  const FftKey key{kFftCols, N, M, planes_per_group * ngroups, band};
  if (fft_recording())
    fft_record(key, [=] {
      return launch_cols(data, N, M, planes_per_group, group_stride, ngroups, sign, s, tag, band, ky);
    });
  FftChoice c;
  if (!fft_lookup(key, &c) || !cols_choice_ok(N, c)) c = cols_default(N);
  FftPlan plan;
  if (!make_plan_variant(N, c.plan, &plan)) return hipErrorInvalidValue;
  const int W = c.w;
  const long tiles = (M + W - 1) / W;
  const long nwg = tiles * planes_per_group * ngroups;
  const int thr = c.threads;
  const size_t lds = (size_t)(N + N * W) * sizeof(float2);
  ScopedTiming _t(tag, s);
#define X_(NN)                                                                                  \
  case NN:                                                                                      \
    if (c.plan == kPlanColsLoop) {                                                              \
      const void* fn = reinterpret_cast<const void*>(&k_cols_loop<NN, static_tile_width(NN)>);  \
      const long g = loop_grid(fn, thr, lds, nwg);                                              \
      hipLaunchKernelGGL((k_cols_loop<NN, static_tile_width(NN)>), dim3((unsigned)g), dim3(thr), lds, \
                         s, data, M, tiles, planes_per_group, group_stride, nwg, sign, band, ky, nb); \
    } else if (W == static_tile_width(NN))                                                      \
      hipLaunchKernelGGL((k_cols<NN, static_tile_width(NN)>), dim3((unsigned)nwg), dim3(thr), lds, \
                         s, data, N, M, W, tiles, planes_per_group, group_stride, plan, sign, band, \
                         ky, nb);                                                               \
    else                                                                                        \
      hipLaunchKernelGGL((k_cols<NN, 0>), dim3((unsigned)nwg), dim3(thr), lds, s, data, N, M, W, \
                         tiles, planes_per_group, group_stride, plan, sign, band, ky, nb);      \
    return hipGetLastError();
  // the compiled kernels index a plane in 32 bits
  const bool small_plane = M < (1L << 24) && (long)N * M < (1L << 32);
  if ((c.plan == 0 || c.plan == kPlanColsLoop) && small_plane) switch (N) {
      WO_ALL_SIZES(X_)
      default:
        break;
    }
#undef X_
  hipLaunchKernelGGL((k_cols<0, 0>), dim3((unsigned)nwg), dim3(thr), lds, s, data, N, M, W, tiles,
                     planes_per_group, group_stride, plan, sign, band, ky, nb);
  return hipGetLastError();
}

// FFT along N of the columns kx < kt of the band rows, from compact planes
// src [g][N][Ys][kt] into full planes dst [g][N][Y][Xh] (band row b is row
// band_row(b, .., Ys) of a source plane and band_row(b, .., Y) of a
// destination plane).  Workgroup: W
// consecutive columns of one band row of one plane group.  While its loads
// are in flight a workgroup also writes the zeros of its share (zrows rows
// from bid * zrows) of the rest of dst: rows outside the band, columns kx >= kt.
template <int NS, int WS>
__global__ __launch_bounds__(1024) void k_cols_expand(const float2* __restrict__ src,
                                                      float2* __restrict__ dst, int N, int Ys, int Y,
                                                      int Xh, int kt, int ky, int nb, int Wrt,
                                                      int tiles_row, long tiles_g, long zrows,
                                                      long zrows_total, int band_out, FftPlan plan,
                                                      float sign) {
  const int W = WS > 0 ? WS : Wrt;   // a power of two
  const int wsh = WS > 0 ? pow2_shift(WS) : pow2_shift(Wrt);
  extern __shared__ float2 smem[];
  float2* tw = smem;
  float2* buf = smem + N;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const long bid = xcd_block();
  const long g = bid / tiles_g;
  const long t = bid - g * tiles_g;
  const int b = (int)(t / tiles_row), j = (int)(t - (long)b * tiles_row);
  const int ys = band_row(b, ky, nb, Ys), y = band_row(b, ky, nb, Y);
  const int kx0 = j * W;
  const int weff = min(W, kt - kx0);
  // plane pitches; a band-layout destination holds the band rows in order
  const long ms = (long)Ys * kt, md = band_out ? (long)nb * kt : (long)Y * Xh;
  const float2* sb = src + g * N * ms + (long)ys * kt + kx0;
  float2* db = dst + g * N * md + (band_out ? (long)b * kt : (long)y * Xh) + kx0;
  const int Nc = NS > 0 ? NS : N;
  fill_twiddles(tw, Nc, tid, nthr);   // before the loads, as in the row passes
  auto mid = [&] {
    const long r0 = bid * zrows, r1 = min(r0 + zrows, zrows_total);
    int yr = (int)(r0 % Y);
    for (long row = r0; row < r1; ++row) {
      float2* rp = dst + row * Xh;
      for (int k = (in_band(yr, ky, nb, Y) ? kt : 0) + tid; k < Xh; k += nthr) rp[k] = make_float2(0.f, 0.f);
      if (++yr == Y) yr = 0;
    }
  };
  if constexpr (NS > 0) {
    fft_direct<NS, WS, true, kEmax, false>(
        buf, W, W, 1, wsh, tw, sign, tid, nthr,
        [&](int l, int n) { return l < weff ? sb[(long)n * ms + l] : make_float2(0.f, 0.f); }, mid,
        [&](int l, int n, float2 v) {
          if (l < weff) db[(long)n * md + l] = v;
        });
  } else {
    gather_to_lds(buf, Nc * W, tid, nthr, [&](int e) {
      const int n = e >> wsh, w = e & (W - 1);
      return w < weff ? sb[(long)n * ms + w] : make_float2(0.f, 0.f);
    }, mid);
    __syncthreads();
    fft_lines<NS, WS, true>(buf, LdsLines{W, W, 1, true, wsh}, plan, tw, sign, tid, nthr);
    scatter_from_lds(buf, Nc * W, tid, nthr, [&](int e, float2 v) {
      const int n = e >> wsh, w = e & (W - 1);
      if (w < weff) db[(long)n * md + w] = v;
    });
  }
}

hipError_t launch_cols_expand(const float2* src, float2* dst, int N, int Ys, int Y, int Xh, int kt,
                              int ky, long ngroups, float sign, hipStream_t s, bool band_out) {
  if (kt < 1 || kt > Xh || ky < 0 || Ys < 1 || Ys > Y) return hipErrorInvalidValue;
  const int nb = 2L * ky + 1 < Y ? 2 * ky + 1 : Y;
  if (nb > Ys || (nb == Y && Ys != Y)) return hipErrorInvalidValue;   // the band fits both
  const int kyn = nb == Y ? Y : ky;
  const FftChoice c = cols_default(N);
  FftPlan plan;
  if (!make_plan_variant(N, c.plan, &plan)) return hipErrorInvalidValue;
  const int W = c.w;
  const int tiles_row = (kt + W - 1) / W;
  const long tiles_g = (long)nb * tiles_row;
  const long nwg = tiles_g * ngroups;
  const int thr = c.threads;
  const size_t lds = (size_t)(N + N * W) * sizeof(float2);
  const long zrows_total = band_out ? 0 : ngroups * N * (long)Y;   // rows with zeros to write
  const long zrows = (zrows_total + nwg - 1) / nwg;
  const int bo = band_out ? 1 : 0;
  ScopedTiming _t(band_out ? "k_cols_z_band" : "k_cols_expand", s);
#define X_(NN)                                                                                  \
  case NN:                                                                                      \
    if (W == static_tile_width(NN))                                                             \
      hipLaunchKernelGGL((k_cols_expand<NN, static_tile_width(NN)>), dim3((unsigned)nwg), dim3(thr), \
                         lds, s, src, dst, N, Ys, Y, Xh, kt, kyn, nb, W, tiles_row, tiles_g,     \
                         zrows, zrows_total, bo, plan, sign);                                   \
    else                                                                                        \
      hipLaunchKernelGGL((k_cols_expand<NN, 0>), dim3((unsigned)nwg), dim3(thr), lds, s, src, dst, N, \
                         Ys, Y, Xh, kt, kyn, nb, W, tiles_row, tiles_g, zrows, zrows_total, bo,     \
                         plan, sign);                                                           \
    return hipGetLastError();
  if (c.plan == 0) switch (N) {
      WO_AXIAL_SIZES(X_)
      default:
        break;
    }
#undef X_
  hipLaunchKernelGGL((k_cols_expand<0, 0>), dim3((unsigned)nwg), dim3(thr), lds, s, src, dst, N, Ys, Y,
                     Xh, kt, kyn, nb, W, tiles_row, tiles_g, zrows, zrows_total, bo, plan, sign);
  return hipGetLastError();
}

// ------------------------------------------------------------------ polarisation bank expansion

// One thread per (z, y, k) of a patch's half-spectrum plane stack: reads the
// label-free pair there (zero off the band rows and columns k >= kt) and writes
// the 20 entries of the 5 x 4 bank, contiguous in k for each entry.
__global__ __launch_bounds__(256) void k_pol5_mix(const Coupling* __restrict__ cpl,
                                                  const float2* __restrict__ red,
                                                  float2* __restrict__ tf, int Z, int Y, int Xh,
                                                  int kt, int ky, int nb, long per_patch) {
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long patch = blockIdx.y;
  if (gid >= per_patch) return;
  const int k = (int)(gid % Xh);
  const long zy = gid / Xh;
  const int y = (int)(zy % Y), z = (int)(zy / Y);
  const bool on = k < kt && in_band(y, ky, nb, Y);
  float2 u = make_float2(0.f, 0.f), v = u;
  if (on) {
    const int b = (nb == Y || y <= ky) ? y : y - (Y - nb);
    const long rp = (long)Z * nb * kt;          // one reduced volume
    const float2* src = red + patch * 2 * rp + ((long)z * nb + b) * kt + k;
    u = src[0];
    v = src[rp];
  }
  const float* kf = &cpl[patch].k[0][0][0];
  float2* dst = tf + patch * 20 * per_patch + gid;
#pragma unroll
  for (int j = 0; j < 20; ++j)
    dst[j * per_patch] = on ? pol5_entry(kf[2 * j], kf[2 * j + 1], u, v) : make_float2(0.f, 0.f);
}

hipError_t launch_pol5_mix(const Coupling* cpl, const float2* red, float2* tf, int Z, int Y, int Xh,
                           int kt, int ky, int npatch, hipStream_t s) {
  if (kt < 1 || kt > Xh || ky < 0 || npatch < 1 || npatch > 65535) return hipErrorInvalidValue;
  const int nb = 2L * ky + 1 < Y ? 2 * ky + 1 : Y;
  const int kyn = nb == Y ? Y : ky;
  const long per_patch = (long)Z * Y * Xh;
  const long blocks = (per_patch + 255) / 256;
  if (blocks > 0x7fffffffL) return hipErrorInvalidValue;
  ScopedTiming _t("k_pol5_mix", s);
  hipLaunchKernelGGL(k_pol5_mix, dim3((unsigned)blocks, (unsigned)npatch), dim3(256), 0, s, cpl, red, tf,
                     Z, Y, Xh, kt, kyn, nb, per_patch);
  return hipGetLastError();
}

// ------------------------------------------------------------------ per-frequency operators
//
// Channel values of one frequency sit at cell[ch * cs].  H(c, p) returns the
// transfer-function value of channel c and property p at this frequency.
// forward: y_c = sum_p H_cp x_p (+ N b_c at DC)
// solve:   F = (H^H H + eta I)^-1 H^H (x - N b delta)      (Eq. tls_solution)
// adjoint: y_p = sum_c conj(H_cp) x_c
// Outputs are scaled by inv_n (the 1/N of the inverse transform).

// CT > 0 fixes the channel count at compile time (static register indexing);
// CT == 0 takes it from Crt.
template <int P, int CT, typename HF>
__device__ __forceinline__ void freq_op(float2* cell, long cs, HF H, int Crt, int mode, float eta,
                                        const float* __restrict__ bg, bool dc, float n_full,
                                        float inv_n) {
  const int C = CT > 0 ? CT : Crt;
  if (mode == kModeForward) {
    float2 x[P];
#pragma unroll
    for (int p = 0; p < P; ++p) x[p] = cell[p * cs];
    for (int c = 0; c < C; ++c) {
      float2 y = make_float2(0.f, 0.f);
#pragma unroll
      for (int p = 0; p < P; ++p) y = cadd(y, cmul(H(c, p), x[p]));
      if (dc && bg) y.x += n_full * bg[c];
      cell[c * cs] = cscale(y, inv_n);
    }
    return;
  }
  if (mode == kModeAdjoint) {
    float2 y[P];
#pragma unroll
    for (int p = 0; p < P; ++p) y[p] = make_float2(0.f, 0.f);
    for (int c = 0; c < C; ++c) {
      const float2 xc = cell[c * cs];
#pragma unroll
      for (int p = 0; p < P; ++p) y[p] = cadd(y[p], cmul(cconj(H(c, p)), xc));
    }
#pragma unroll
    for (int p = 0; p < P; ++p) cell[p * cs] = cscale(y[p], inv_n);
    return;
  }
  if constexpr (CT == 1) {
    // one channel: H is a row h, and (h^H h + eta I)^-1 h^H = h^H / (h h^H + eta)
    // (Sherman-Morrison), so F_p = conj(h_p) x / (sum_q |h_q|^2 + eta)
    float2 xc = cell[0];
    if (dc && bg) xc.x -= n_full * bg[0];
    float2 h[P];
    float den = eta;
#pragma unroll
    for (int p = 0; p < P; ++p) {
      h[p] = H(0, p);
      den += h[p].x * h[p].x + h[p].y * h[p].y;
    }
    const float sc = den > 0.f ? inv_n * __builtin_amdgcn_rcpf(den) : 0.f;   // hardware reciprocal
#pragma unroll
    for (int p = 0; p < P; ++p) cell[p * cs] = cscale(cmulconj(xc, h[p]), sc);
    return;
  }
  // solve: accumulate the lower triangle of M = H^H H, M_pq = sum_c conj(H_cp) H_cq,
  // and r = H^H x
  float2 m[P][P];
  float2 r[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    r[p] = make_float2(0.f, 0.f);
#pragma unroll
    for (int q = 0; q < P; ++q) m[p][q] = make_float2(0.f, 0.f);
  }
  for (int c = 0; c < C; ++c) {
    float2 xc = cell[c * cs];
    if (dc && bg) xc.x -= n_full * bg[c];
    float2 h[P];
#pragma unroll
    for (int p = 0; p < P; ++p) h[p] = H(c, p);
#pragma unroll
    for (int p = 0; p < P; ++p) {
      r[p] = cadd(r[p], cmul(cconj(h[p]), xc));
#pragma unroll
      for (int q = 0; q <= p; ++q) m[p][q] = cadd(m[p][q], cmul(cconj(h[p]), h[q]));
    }
  }
  float2 F[P];
  if (P == 1) {
    const float den = m[0][0].x + eta;
    F[0] = den > 0.f ? cscale(r[0], __builtin_amdgcn_rcpf(den)) : make_float2(0.f, 0.f);
  } else {
    chol_solve<P>(m, r, eta, F);
  }
#pragma unroll
  for (int p = 0; p < P; ++p) cell[p * cs] = cscale(F[p], inv_n);
}

// The polarisation solve from the reduced bank at one frequency: with
// H_cp = Kr_cp u + Ki_cp v (u = H_phase, v = H_abs there), H^H H has the entries
// A |u|^2 + B |v|^2 + S Re(conj(u) v) + i D Im(conj(u) v) (constants of the
// coupling) and H^H x = conj(u) Kr^T x + conj(v) Ki^T x, so the 5 x 4 bank is
// never formed.  Algebraically the solve of freq_op with that bank.
__device__ __forceinline__ void pol5_solve(float2* cell, long cs, float2 u, float2 v,
                                           const Coupling* __restrict__ cp, float eta,
                                           const float* __restrict__ bg, bool dc, float n_full,
                                           float inv_n) {
  float2 yr[4], yi[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) yr[p] = yi[p] = make_float2(0.f, 0.f);
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    float2 xc = cell[c * cs];
    if (dc && bg) xc.x -= n_full * bg[c];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      yr[p] = cadd(yr[p], cscale(xc, cp->k[c][p][0]));
      yi[p] = cadd(yi[p], cscale(xc, cp->k[c][p][1]));
    }
  }
  const float uu = u.x * u.x + u.y * u.y, vv = v.x * v.x + v.y * v.y;
  const float2 w = cmulconj(v, u);   // conj(u) v
  float2 m[4][4], r[4], F[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    r[p] = cadd(cmulconj(yr[p], u), cmulconj(yi[p], v));
#pragma unroll
    for (int q = 0; q <= p; ++q) {
      const int e = p * (p + 1) / 2 + q;
      m[p][q] = make_float2(cp->a[e] * uu + cp->b[e] * vv + cp->s[e] * w.x, cp->d[e] * w.y);
    }
  }
  chol_solve<4>(m, r, eta, F);
#pragma unroll
  for (int p = 0; p < 4; ++p) cell[p * cs] = cscale(F[p], inv_n);
}

constexpr int kTfPrefetch = 8;   // transfer-function values a thread may hold in registers

// Geometry of the fused Z pass.  A plane of the spectrum holds R rows of row
// pitch Ls (plane pitch Ms), a plane of the bank R rows of pitch Lt (plane
// pitch Mt), or only the band rows in band order (bank_band); the pass covers
// the columns k < kt of the band rows (band_row: ky, nb) in tiles of W columns
// that do not cross a row.  The plain layout is one row: R = 1,
// Ls = Lt = kt = Ms = Mt = M, nb = 1.
struct ZopGeom {
  long Ms, Mt, Ls, Lt, kt;
  int R, ky, nb, tiles_row, bank_band;
};

// With compiled stages at most 72 VGPRs (7 waves per SIMD, no spills); the
// runtime-plan instances keep their allocation (they would spill).
// RED: tf holds the polarisation bank in reduced form, [2][Z][..] per patch
// (H_phase, H_abs), and the coupling cpl[patch] forms H_cp per frequency.
template <int P, int CT, int NS, bool RED>
__global__ __launch_bounds__(1024, NS > 0 ? 7 : 1) void k_zop(float2* __restrict__ spec,
                                              const float2* __restrict__ tf, int C, int Z, ZopGeom gm,
                                              int slots, int W, long tiles_m, FftPlan plan,
                                              int mode, float eta, const float* __restrict__ bg,
                                              float inv_n, float n_full,
                                              const Coupling* __restrict__ cpl) {
  extern __shared__ float2 smem[];
  float2* tw = smem;
  float2* buf = smem + Z;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const long bid = xcd_block();
  const long tile = bid % tiles_m;
  const long patch = bid / tiles_m;
  const int Zc = NS > 0 ? NS : Z;   // compile-time length for the index arithmetic
  const int wsh = pow2_shift(W);    // W is a power of two
  const int cin = mode == kModeForward ? P : C;
  const int cout = mode == kModeForward ? C : P;
  const int CH = cin > cout ? cin : cout;
  const long Ms = gm.Ms, Mt = gm.Mt;
  float2* sp = spec + patch * (long)slots * Z * Ms;
  const float2* tp = tf + patch * (long)(RED ? 2 : C * P) * Z * Mt;
  const float* bp = bg ? bg + patch * C : nullptr;
  const int brow = (int)(tile / gm.tiles_row);
  const long col0 = (tile - (long)brow * gm.tiles_row) * W;
  const int row = band_row(brow, gm.ky, gm.nb, gm.R);
  const long m0 = row * gm.Ls + col0;        // tile start in a spectrum plane
  const long mt0 = (gm.bank_band ? brow : row) * gm.Lt + col0;   // and in a bank plane
  const bool dc_tile = row == 0 && col0 == 0;
  const int weff = (int)min((long)W, gm.kt - col0);
  // Element (plane, w) of the tile: a plane pitch is below 2^32 (checked on
  // the host), so its offset is one 32 x 32 -> 64-bit multiply, not a 64-bit
  // product per element.
  float2* const st = sp + m0;
  const float2* const tt = tp + mt0;
  const unsigned ums = (unsigned)Ms, umt = (unsigned)Mt;
  auto soff = [&](int plane) { return (long)((unsigned long)(unsigned)plane * ums); };
  auto toff = [&](int plane) { return (long)((unsigned long)(unsigned)plane * umt); };
  // Issue this thread's transfer-function loads first: they complete while the
  // data tile is loaded and transformed.  Frequency f = tid + i * nthr.
  const int nfreq = Zc * W;
  const int fpt = (nfreq + nthr - 1) / nthr;
  // entries of the bank a frequency reads: P (one channel) or the pair (reduced)
  constexpr int NE = RED ? 2 : P;
  constexpr int NPF = RED ? 4 : kTfPrefetch;   // registers for the prefetched entries
  const bool prefetch = (RED || CT == 1) && NE * fpt <= NPF;
  float2 hreg[NPF];
  if (prefetch) {
#pragma unroll
    for (int j = 0; j < NPF; ++j) {
      const int i = j / NE, cp = j - i * NE;
      const int f = tid + i * nthr;
      if (i < fpt && f < nfreq) {
        const int z = f >> wsh, w = f & (W - 1);
        hreg[j] = w < weff ? tt[toff(cp * Zc + z) + w] : make_float2(0.f, 0.f);
      }
    }
  }
  TwFetch twf;   // as in the row passes
  tw_begin(twf, tw, Zc, tid, nthr);
  // LDS holds [z][ch][w]: line l = ch W + w, element z at z CH W
  if constexpr (NS > 0) {
    // first pass of the forward Z transform straight from memory
    first_pass_in<NS, 0, true, kEmax, false, false>(
        buf, cin * W, CH * W, 1, pow2_shift(cin * W), -1.f, tid, nthr,
        [&](int l, int z) {
          const int ch = l >> wsh, w = l & (W - 1);
          return w < weff ? st[soff(ch * Zc + z) + w] : make_float2(0.f, 0.f);
        },
        [&] { tw_end(twf, tw, Zc, tid, nthr); });
    static_passes<NS, 0, true, kEmax, false, false, 1, StaticPlan<NS>::passes()>(
        buf, cin * W, CH * W, 1, pow2_shift(cin * W), tw, -1.f, tid, nthr);
  } else {
    tw_end(twf, tw, Zc, tid, nthr);
    // element e = (ch, z, w) of the global tile goes to LDS [z][ch][w]
    float2 t[kEmax];
#pragma unroll
    for (int i = 0; i < kEmax; ++i) {
      const int e = tid + i * nthr;
      if (e < cin * Zc * W) {
        const int w = e & (W - 1), r = e >> wsh;
        const int z = r % Zc, ch = r / Zc;
        t[i] = w < weff ? st[soff(ch * Zc + z) + w] : make_float2(0.f, 0.f);
      }
    }
#pragma unroll
    for (int i = 0; i < kEmax; ++i) {
      const int e = tid + i * nthr;
      if (e < cin * Zc * W) {
        const int w = e & (W - 1), r = e >> wsh;
        const int z = r % Zc, ch = r / Zc;
        buf[(z * CH + ch) * W + w] = t[i];
      }
    }
    __syncthreads();
    fft_lines<NS, 0, true>(buf, LdsLines{cin * W, CH * W, 1, true, pow2_shift(cin * W)}, plan, tw, -1.f,
                           tid, nthr);
  }
  if (prefetch) {
#pragma unroll
    for (int i = 0; i < NPF / NE; ++i) {
      const int f = tid + i * nthr;
      if (i < fpt && f < nfreq) {
        const int z = f >> wsh, w = f & (W - 1);
        if (w < weff) {
          const bool dcf = z == 0 && dc_tile && w == 0;
          if constexpr (RED) {
            const float2 hph = hreg[i * 2], hab = hreg[i * 2 + 1];
            const float* kf = &cpl[patch].k[0][0][0];
            if (mode == kModeSolve)
              pol5_solve(buf + (long)z * CH * W + w, W, hph, hab, cpl + patch, eta, bp, dcf, n_full, inv_n);
            else
              freq_op<P, CT>(buf + (long)z * CH * W + w, W,
                             [&](int c, int p) {
                               return pol5_entry(kf[(c * P + p) * 2], kf[(c * P + p) * 2 + 1], hph, hab);
                             },
                             C, mode, eta, bp, dcf, n_full, inv_n);
          } else {
            freq_op<P, 1>(buf + (long)z * CH * W + w, W,
                          [&](int c, int p) { return hreg[i * P + p]; }, C, mode, eta, bp, dcf, n_full,
                          inv_n);
          }
        }
      }
    }
  } else {
    for (int f = tid; f < nfreq; f += nthr) {
      const int z = f >> wsh, w = f & (W - 1);
      if (w >= weff) continue;
      const float2* hp = tt + w;
      if constexpr (RED) {
        const float2 hph = hp[toff(z)], hab = hp[toff(Zc + z)];
        const float* kf = &cpl[patch].k[0][0][0];
        if (mode == kModeSolve)
          pol5_solve(buf + (long)z * CH * W + w, W, hph, hab, cpl + patch, eta, bp,
                     z == 0 && dc_tile && w == 0, n_full, inv_n);
        else
          freq_op<P, CT>(buf + (long)z * CH * W + w, W,
                         [&](int c, int p) {
                           return pol5_entry(kf[(c * P + p) * 2], kf[(c * P + p) * 2 + 1], hph, hab);
                         },
                         C, mode, eta, bp, z == 0 && dc_tile && w == 0, n_full, inv_n);
      } else {
        freq_op<P, CT>(buf + (long)z * CH * W + w, W,
                       [&](int c, int p) { return hp[toff((c * P + p) * Zc + z)]; }, C, mode, eta, bp,
                       z == 0 && dc_tile && w == 0, n_full, inv_n);
      }
    }
  }
  __syncthreads();
  if constexpr (NS > 0) {
    // last pass of the inverse Z transform straight to memory
    static_passes<NS, 0, true, kEmax, false, false, 0, StaticPlan<NS>::passes() - 1>(
        buf, cout * W, CH * W, 1, pow2_shift(cout * W), tw, 1.f, tid, nthr);
    last_pass_out<NS, 0, true, kEmax, false, false>(
        buf, cout * W, CH * W, 1, pow2_shift(cout * W), tw, 1.f, tid, nthr,
        [&](int l, int z, float2 v) {
          const int ch = l >> wsh, w = l & (W - 1);
          if (w < weff) st[soff(ch * Zc + z) + w] = v;
        });
  } else {
    fft_lines<NS, 0, true>(buf, LdsLines{cout * W, CH * W, 1, true, pow2_shift(cout * W)}, plan, tw, 1.f,
                           tid, nthr);
    float2 t[kEmax];
#pragma unroll
    for (int i = 0; i < kEmax; ++i) {
      const int e = tid + i * nthr;
      if (e < cout * Zc * W) {
        const int w = e & (W - 1), r = e >> wsh;
        const int z = r % Zc, ch = r / Zc;
        t[i] = buf[(z * CH + ch) * W + w];
      }
    }
#pragma unroll
    for (int i = 0; i < kEmax; ++i) {
      const int e = tid + i * nthr;
      if (e < cout * Zc * W) {
        const int w = e & (W - 1), r = e >> wsh;
        const int z = r % Zc, ch = r / Zc;
        if (w < weff) st[soff(ch * Zc + z) + w] = t[i];
      }
    }
  }
}

template <int P, int CT, bool RED = false>
static void zop_launch(bool use_static, long nwg, int thr, size_t lds, hipStream_t s, float2* spec,
                       const float2* tf, int C, int Z, const ZopGeom& gm, int slots, int W, long tiles,
                       FftPlan plan, int mode, float eta, const float* bg, float inv_n, float nf,
                       const Coupling* cpl) {
#define X_(NN)                                                                                   \
  case NN:                                                                                       \
    hipLaunchKernelGGL((k_zop<P, CT, NN, RED>), dim3((unsigned)nwg), dim3(thr), lds, s, spec, tf, C, Z, \
                       gm, slots, W, tiles, plan, mode, eta, bg, inv_n, nf, cpl);                \
    return;
  if (use_static) switch (Z) {
      WO_AXIAL_SIZES(X_)
      default:
        break;
    }
#undef X_
  hipLaunchKernelGGL((k_zop<P, CT, 0, RED>), dim3((unsigned)nwg), dim3(thr), lds, s, spec, tf, C, Z, gm,
                     slots, W, tiles, plan, mode, eta, bg, inv_n, nf, cpl);
}

static bool zop_choice_ok(int Z, int CH, const FftChoice& c) {
  const long elems = (long)c.w * Z * CH;
  return pow2_shift(c.w) >= 0 && c.w <= 64 && elems <= kMaxElems && threads_ok(c.threads, elems) &&
         (long)(Z + elems) * (long)sizeof(float2) <= lds_limit_bytes() && c.plan >= 0 && c.plan <= 3;
}

// At most 4096 elements per workgroup (8 per thread, 512 threads): the pass
// waits on its loads and stores between short bursts of arithmetic, and
// smaller workgroups let more of them share a CU (5 channels x 64 planes:
// 8 columns 249 us, 16 columns 282 us on the 64x1024x1024 volume).
static FftChoice zop_default(int Z, int CH) {
  int W = tile_width(Z, CH);
  while (W > 1 && (long)W * Z * CH > 4096) W /= 2;
  return FftChoice{W, threads_for((long)CH * Z * W), 0};
}

bool zop_fits(int Z, int CH) { return zop_choice_ok(Z, CH, zop_default(Z, CH)); }

hipError_t launch_zop(float2* spec, const float2* tf, int C, int P, int Z, long M, int slots,
                      int npatch, int mode, float eta, const float* bg, float inv_n, double n_full,
                      hipStream_t s, const SpecBand* band, const Coupling* cpl) {
  if (cpl && (P != 4 || C != 5)) return hipErrorInvalidValue;
  if (band && (band->Y < 1 || M % band->Y != 0 || band->kt < 1 || band->kt > M / band->Y ||
               band->ky < 0))
    return hipErrorInvalidValue;
  const bool hb = band != nullptr;
  const SpecBand bc = hb ? *band : SpecBand{1, M, 0, 0};
  const int nbr = hb ? (2L * bc.ky + 1 >= bc.Y ? bc.Y : 2 * bc.ky + 1) : 1;
  const long mcov = hb ? (long)nbr * bc.kt : M;   // columns the pass covers per plane
  const FftKey key{kFftZop, Z, mcov, npatch,
                   P * 1000 + C * 10 + mode + (hb ? 100000 : 0) + (cpl ? 200000 : 0)};
  if (fft_recording())
    fft_record(key, [=] {
      return launch_zop(spec, tf, C, P, Z, M, slots, npatch, mode, eta, bg, inv_n, n_full, s,
                        hb ? &bc : nullptr, cpl);
    });
  const int cin = mode == kModeForward ? P : C;
  const int cout = mode == kModeForward ? C : P;
  const int CH = cin > cout ? cin : cout;
  FftChoice c;
  if (!fft_lookup(key, &c) || !zop_choice_ok(Z, CH, c)) c = zop_default(Z, CH);
  FftPlan plan;
  if (!make_plan_variant(Z, c.plan, &plan)) return hipErrorInvalidValue;
  const int W = c.w;
  ZopGeom gm;
  gm.R = bc.Y;
  gm.kt = bc.kt;
  gm.Ls = bc.kt;
  gm.bank_band = hb && bc.bank_band;
  gm.Lt = gm.bank_band ? bc.kt : M / bc.Y;
  gm.Ms = (long)bc.Y * bc.kt;
  gm.Mt = gm.bank_band ? (long)nbr * bc.kt : M;
  gm.nb = nbr;
  gm.ky = nbr == bc.Y ? bc.Y : bc.ky;
  if (gm.Ms >= (1L << 32) || gm.Mt >= (1L << 32)) return hipErrorInvalidValue;   // 32-bit plane offsets
  gm.tiles_row = (int)((bc.kt + W - 1) / W);
  const long tiles = (long)nbr * gm.tiles_row;
  const long nwg = tiles * npatch;
  const int thr = c.threads;
  const size_t lds = (size_t)(Z + CH * Z * W) * sizeof(float2);
  const float nf = (float)n_full;
  const bool st = c.plan == 0;
  ScopedTiming _t(P == 1 ? "k_zop<1>" : (P == 2 ? "k_zop<2>" : "k_zop<4>"), s);
#define WO_ZOP(PP, CC) \
  zop_launch<PP, CC>(st, nwg, thr, lds, s, spec, tf, C, Z, gm, slots, W, tiles, plan, mode, eta, bg, inv_n, nf, \
                     nullptr)
  if (cpl) zop_launch<4, 5, true>(st, nwg, thr, lds, s, spec, tf, C, Z, gm, slots, W, tiles, plan, mode, eta,
                                  bg, inv_n, nf, cpl);
  else if (P == 1) { if (C == 1) WO_ZOP(1, 1); else WO_ZOP(1, 0); }
  else if (P == 2) { if (C == 1) WO_ZOP(2, 1); else WO_ZOP(2, 0); }
  else if (P == 4) { if (C == 1) WO_ZOP(4, 1); else if (C == 5) WO_ZOP(4, 5); else WO_ZOP(4, 0); }
  else return hipErrorInvalidValue;
#undef WO_ZOP
  return hipGetLastError();
}

// ------------------------------------------------------------------ schedule candidates

static std::vector<int> thread_options(long elems) {
  std::vector<int> t;
  for (int per : {kEmax, kEmax / 2, kEmax / 4}) {
    long thr = (elems + per - 1) / per;
    thr = ((thr + 63) / 64) * 64;
    if (thr < 64) thr = 64;
    if (thr > kMaxThreads) continue;
    bool seen = false;
    for (int x : t) seen |= x == (int)thr;
    if (!seen) t.push_back((int)thr);
  }
  return t;
}

// Radix-plan variants of n whose pass sequences differ from each other (and,
// for compiled lengths, runtime plans other than the default order).
static std::vector<int> plan_options(int n) {
  std::vector<int> v{0};
  FftPlan p0, p;
  if (!make_plan_variant(n, 1, &p0)) return v;
  std::vector<unsigned long long> seen{p0.radices};
  for (int var : {2, 3}) {
    if (!make_plan_variant(n, var, &p)) continue;
    bool dup = false;
    for (auto r : seen) dup |= r == p.radices;
    if (!dup) {
      v.push_back(var);
      seen.push_back(p.radices);
    }
  }
  return v;
}

std::vector<FftChoice> fft_candidates(const FftKey& k) {
  std::vector<FftChoice> out;
  auto add = [&](const FftChoice& c) {
    for (auto& x : out)
      if (x.w == c.w && x.threads == c.threads && x.plan == c.plan) return;
    out.push_back(c);
  };
  std::vector<int> widths{1, 2, 4, 8, 16, 32, 64};
  const std::vector<int> plans = plan_options(k.n);
  if (k.kind == kFftRowsR2C || k.kind == kFftRowsC2R) {
    const FftChoice d = rows_default(k.n);
    add(d);
    widths.push_back(d.w);
    for (int pl : plans)
      for (int w : widths)
        for (int t : thread_options((long)w * k.n)) {
          const FftChoice c{w, t, pl};
          if (rows_choice_ok(k.n, c)) add(c);
        }
  } else if (k.kind == kFftCols) {
    const FftChoice d = cols_default(k.n);
    add(d);
    for (int pl : plans)
      for (int w : widths)
        for (int t : thread_options((long)w * k.n)) {
          const FftChoice c{w, t, pl};
          if (cols_choice_ok(k.n, c)) add(c);
        }
    for (int t : thread_options((long)static_tile_width(k.n) * k.n)) {
      const FftChoice c{static_tile_width(k.n), t, kPlanColsLoop};
      if (cols_choice_ok(k.n, c)) add(c);
    }
  } else if (k.kind == kFftTfRows) {
    const FftChoice d = tf_rows_default(k.n);
    add(d);
    for (int pl : plans)
      for (int w : {1, 2, 3, 4, 6, 8, 12, 16, 24, 32})
        for (int t : thread_options(2L * w * k.n)) {
          const FftChoice c{w, t, pl};
          if (tf_rows_choice_ok(k.n, c)) add(c);
        }
  } else if (k.kind == kFftTfFields) {
    const int Z = k.extra / 10;
    add(tf_fields_default(Z, k.m, k.batch));
    for (int w : {1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96}) {
      const FftChoice c{w, 0, 0};
      if (tf_fields_choice_ok(Z, c)) add(c);
    }
  } else if (k.kind == kFftZop) {
    const int P = (k.extra % 100000) / 1000, C = (k.extra / 10) % 100, mode = k.extra % 10;
    const int cin = mode == kModeForward ? P : C;
    const int cout = mode == kModeForward ? C : P;
    const int CH = cin > cout ? cin : cout;
    const FftChoice d = zop_default(k.n, CH);
    add(d);
    for (int pl : plans)
      for (int w : widths)
        for (int t : thread_options((long)w * k.n * CH)) {
          const FftChoice c{w, t, pl};
          if (zop_choice_ok(k.n, CH, c)) add(c);
        }
  }
  return out;
}

template <int P>
__global__ __launch_bounds__(256) void k_op2d(float2* __restrict__ spec,
                                              const float2* __restrict__ tf, int C, long M,
                                              int slots, int mode, float eta,
                                              const float* __restrict__ bg, float inv_n,
                                              float n_full, long blocks_per_patch,
                                              const float* __restrict__ eta_pp) {
  const long patch = blockIdx.x / blocks_per_patch;
  const long m = (blockIdx.x - patch * blocks_per_patch) * (long)blockDim.x + threadIdx.x;
  if (m >= M) return;
  if (eta_pp) eta = eta_pp[patch];
  float2* sp = spec + patch * (long)slots * M;
  const float2* tp = tf + patch * (long)C * P * M;
  const float* bp = bg ? bg + patch * C : nullptr;
  const float2* hp = tp + m;
  freq_op<P, 0>(sp + m, M, [&](int c, int p) { return hp[(long)(c * P + p) * M]; }, C, mode, eta,
                bp, m == 0, n_full, inv_n);
}

hipError_t launch_op2d(float2* spec, const float2* tf, int C, int P, long M, int slots, int npatch,
                       int mode, float eta, const float* bg, float inv_n, double n_full,
                       hipStream_t s, const float* eta_pp) {
  const long bpp = (M + 255) / 256;
  const long nwg = bpp * npatch;
  const float nf = (float)n_full;
  switch (P) {
    case 1:
      { ScopedTiming _t("k_op2d<1>", s);
      hipLaunchKernelGGL(k_op2d<1>, dim3((unsigned)nwg), dim3(256), 0, s, spec, tf, C, M, slots,
                         mode, eta, bg, inv_n, nf, bpp, eta_pp); }
      break;
    case 2:
      { ScopedTiming _t("k_op2d<2>", s);
      hipLaunchKernelGGL(k_op2d<2>, dim3((unsigned)nwg), dim3(256), 0, s, spec, tf, C, M, slots,
                         mode, eta, bg, inv_n, nf, bpp, eta_pp); }
      break;
    case 4:
      { ScopedTiming _t("k_op2d<4>", s);
      hipLaunchKernelGGL(k_op2d<4>, dim3((unsigned)nwg), dim3(256), 0, s, spec, tf, C, M, slots,
                         mode, eta, bg, inv_n, nf, bpp, eta_pp); }
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace wo
