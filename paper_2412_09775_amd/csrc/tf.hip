// Transfer-function synthesis (Table 1, scalar column) on the device.
//
// Label-free: per plane z, the direct field A_z = S P e^{i 2 pi kz (z - dz0)}
// and the scattered field B_z = P (i k_m / kz) e^{i 2 pi kz (z - dz0)} are
// generated on the lateral frequency grid (FP64 arithmetic, FP32 storage) and
// inverse-transformed along Y; a row kernel finishes the inverse transform
// along X, forms the point response c = b conj(a) / (X Y I_bg), transforms it
// forward along X and splits it into the half spectra of 2 Re c (phase) and
// -2 Im c (absorption).  The remaining Y (and, for 3D models, Z) transforms
// reuse the generic column passes.  Fluorescence does the same with the single
// field P e^{i 2 pi kz (z - dz0)} and the real PSF |h|^2 normalised to unit sum.
#include "internal.hpp"

namespace wo {

// ------------------------------------------------------------------ parameters

// Per-patch optics travel as kernel arguments (a batch of up to 8 records per
// launch), so setting them needs no host staging buffer and stays
// asynchronous on the stream.
struct OpticsBatch {
  DevOptics o[8];
};
static_assert(sizeof(OpticsBatch) <= 3584, "kernel arguments are limited to 4 KiB");

__global__ void k_set_params(DevOptics* dst, OpticsBatch b, int count) {
  const int i = threadIdx.x;
  if (i < count) dst[i] = b.o[i];
}

hipError_t launch_set_params(DevOptics* dst, const DevOptics* host, int n, hipStream_t s) {
  for (int i0 = 0; i0 < n; i0 += 8) {
    OpticsBatch b;
    const int cnt = n - i0 < 8 ? n - i0 : 8;
    for (int j = 0; j < cnt; ++j) b.o[j] = host[i0 + j];
    hipLaunchKernelGGL(k_set_params, dim3(1), dim3(64), 0, s, dst + i0, b, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

struct CouplingBatch {
  Coupling c[8];
};
static_assert(sizeof(CouplingBatch) <= 3584, "kernel arguments are limited to 4 KiB");

__global__ void k_set_coupling(Coupling* dst, CouplingBatch b, int count) {
  const int i = threadIdx.x;
  if (i < count) dst[i] = b.c[i];
}

hipError_t launch_set_coupling(Coupling* dst, const Coupling* host, int n, hipStream_t s) {
  for (int i0 = 0; i0 < n; i0 += 8) {
    CouplingBatch b;
    const int cnt = n - i0 < 8 ? n - i0 : 8;
    for (int j = 0; j < cnt; ++j) b.c[j] = host[i0 + j];
    hipLaunchKernelGGL(k_set_coupling, dim3(1), dim3(64), 0, s, dst + i0, b, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

struct TuneBatch {
  TuneState t[8];
};
static_assert(sizeof(TuneBatch) <= 3584, "kernel arguments are limited to 4 KiB");

__global__ void k_set_tune(TuneState* dst, TuneBatch b, int count) {
  const int i = threadIdx.x;
  if (i < count) dst[i] = b.t[i];
}

hipError_t launch_set_tune(TuneState* dst, const TuneState* host, int n, hipStream_t s) {
  for (int i0 = 0; i0 < n; i0 += 8) {
    TuneBatch b;
    const int cnt = n - i0 < 8 ? n - i0 : 8;
    for (int j = 0; j < cnt; ++j) b.t[j] = host[i0 + j];
    hipLaunchKernelGGL(k_set_tune, dim3(1), dim3(64), 0, s, dst + i0, b, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ------------------------------------------------------------------ reductions

// Deterministic workgroup sum of one double per thread (wave shuffles, then
// the wave partials in order).  Result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
  return t;
}

// ------------------------------------------------------------------ fields, inverse Y

// ab layout per patch: field 0 (A, or the fluorescence field) [z][y][ca],
// then field 1 (B) [z][y][c]: c the compact column of the lateral frequency kx
// among B's XC kept columns (see field_column; c = kx when XC = X), ca among
// A's XA (last non-negative column KPA; XA = XC: the same columns), y one of
// the LY points of the inverse Y transform.  LY = Y is the grid's own transform; a shorter LY (still longer
// than twice the support's extent along y) samples the same band-limited
// fields more coarsely: frequency index i of the LY-point transform stands for
// the grid's frequency (i or i - LY) / (Y dy).  A workgroup owns one column tile of one patch and a
// chunk of ZC consecutive planes: the pupil values, which do not depend on z,
// are evaluated once into registers; each plane then only needs its phase.
// The workgroup of the first chunk also writes the tile's share of the pupil
// sum (sum S P^2 for label-free, sum P^2 for fluorescence) to
// partials[patch * tiles_x + tile].
template <int NS, int NF, bool AB>
__global__ __launch_bounds__(1024) void k_tf_fields_y(const DevOptics* __restrict__ opt,
                                                      Sampling sm, float2* __restrict__ ab,
                                                      double* __restrict__ partials, int W,
                                                      long tiles_x, int ZC, int XC, int KP, int LY,
                                                      int XA, int KPA, FftPlan plan) {
  __shared__ double red[kMaxThreads / 64];
  extern __shared__ float2 smem[];
  const int Y = NS > 0 ? NS : LY;   // transform length
  const int X = sm.nx, Z = sm.nz;
  // field f of this patch at plane z, row y, compact column c of B's layout;
  // nullptr where A keeps no column
  auto field_at = [&](long patch, int f, int z, int y, int c) -> float2* {
    float2* pa = ab + patch * (long)Z * Y * (NF == 2 ? XA + XC : XC);
    if (NF == 1 || f == 1) return pa + (NF == 2 ? (long)Z * Y * XA : 0) + ((long)z * Y + y) * XC + c;
    const int ca = XA == XC ? c : compact_column(field_column(c, KP, X, XC), KPA, X, XA);
    return ca < 0 ? nullptr : pa + ((long)z * Y + y) * XA + ca;
  };
  // frequency of transform index i: the grid's spacing 1 / (ny dy), wrapped at Y
  auto freq_y = [&](int i) { return (double)(i < (Y + 1) / 2 ? i : i - Y) / ((double)sm.ny * sm.dy); };
  float2* tw = smem;
  float2* buf = smem + Y;
  const int tid = threadIdx.x, nthr = blockDim.x;
  fill_twiddles(tw, Y, tid, nthr);
  const long bid = xcd_block();
  const long tile = bid % tiles_x;
  const long rest = bid / tiles_x;
  const int zsplit = z_split(sm);
  const int nzc = z_chunk_count(Z, zsplit, ZC);
  const int zc = (int)(rest % nzc);
  const long patch = rest / nzc;
  int zbeg, zend;
  z_chunk_range(Z, zsplit, ZC, zc, &zbeg, &zend);
  const DevOptics o = opt[patch];
  constexpr bool fluor = NF == 1;   // one field (fluorescence) or A and B (label-free)
  constexpr int nf = NF;
  constexpr int EPT = kEmax / NF;   // elements of a thread: Y * W * NF <= threads * kEmax
  const int x0 = (int)(tile * W);
  const int wsh = pow2_shift(W);     // W is a power of two
  const int nl = nf * W;              // lines of the tile: field f, column w (l = f W + w)
  const int lsh = pow2_shift(nl);
  if constexpr (NS > 0) {
    // The first pass of the inverse Y transform takes its inputs from registers
    // (the fields are computed where the butterfly needs them) and the last
    // pass writes to memory from registers: LDS carries only the passes
    // between.  Butterfly j of the first pass: line l = j mod nl, elements
    // ky = k + r NB0 (k = j / nl); of the last pass: outputs ky = k + r NSL.
    constexpr int NP = StaticPlan<NS>::passes();
    constexpr int R0 = StaticPlan<NS>::radix(0), NB0 = NS / R0;
    constexpr int RL = StaticPlan<NS>::radix(NP - 1), NSL = NS / RL;
    constexpr int B0 = (kEmax + R0 - 1) / R0, BL = (kEmax + RL - 1) / RL;
    static_assert(NP >= 2, "compiled lateral lengths have at least two passes");
    double tkz[B0][R0];
    float fac[B0][R0];
    float ab2[AB ? B0 : 1][AB ? R0 : 1];   // 2 W(p): the aberration phase in units of pi
    {
      const double hw = soft_halfwidth(o, sm);
      const double km = o.n_medium / o.wavelength;
      const double ri = o.na_ill / o.wavelength;
      const DetAxis dax = det_axis(o);
      double cy, cx;
      source_centre(o, &cy, &cx);
      double psum = 0.0;
#pragma unroll
      for (int b = 0; b < B0; ++b) {
        const int j = tid + b * nthr;
        const int l = j & (nl - 1), k = j >> lsh;
        const int f = l >> wsh, c = x0 + (l & (W - 1));
        const int kx = field_column(c, KP, X, XC);
#pragma unroll
        for (int r = 0; r < R0; ++r) {
          tkz[b][r] = 0.0;
          fac[b][r] = 0.f;
          if constexpr (AB) ab2[b][r] = 0.f;
          if (j < nl * NB0 && c < XC) {
            const int ky = k + r * NB0;
            const double fy = freq_y(ky), fx = fftfreq(kx, X, sm.dx);
            const double P = det_pupil(o, dax, fy, fx, hw);
            if (P != 0.0) {
              const double kz = sqrt(fmax(km * km - (fy * fy + fx * fx), 0.0));
              tkz[b][r] = 2.0 * kz;
              if constexpr (AB) ab2[b][r] = (float)(2.0 * aberration_waves(o, fy, fx));
              if (fluor) {
                fac[b][r] = (float)P;
                psum += P * P;
              } else {
                double S = disc(fy - cy, fx - cx, ri, hw);
                if (o.sector >= 0 && octant(fy - cy, fx - cx) != o.sector) S = 0.0;
                if (f == 0) {
                  fac[b][r] = (float)(S * P);
                  psum += S * P * P;
                } else if (kz > 0.0) {
                  fac[b][r] = (float)(P * km / kz);   // P * (i k_m / kz)
                }
              }
            }
          }
        }
      }
      if (zc == 0) {
        const double tot = block_sum(psum, red);
        if (tid == 0) partials[patch * tiles_x + tile] = tot;
      }
    }
    // The phase pi arg(z), arg = 2 kz (z - dz0) (+ 2 W), is linear in the plane
    // position, which advances by dz within a chunk (chunks never cross the
    // jump of the wrapped axial order): each element carries its field value
    // of the current plane, the pupil factor times e^{i pi arg} (times i for
    // B), evaluated directly at the chunk's first plane (FP64 argument
    // reduction, FP32 sine and cosine) and then advanced plane by plane by
    // the step e^{i pi 2 kz dz}, one complex multiply.  Over at most ZC - 1
    // steps the products' rounding stays near 1e-6 relative.
    float2 ph[B0][R0], st[B0][R0];
    {
      const double dzr = plane_z(zbeg, sm) - o.defocus;
#pragma unroll
      for (int b = 0; b < B0; ++b) {
        const int j = tid + b * nthr;
        const bool fa = ((j & (nl - 1)) >> wsh) == 0;   // A (or the fluorescence field), else B
#pragma unroll
        for (int r = 0; r < R0; ++r) {
          ph[b][r] = st[b][r] = make_float2(0.f, 0.f);
          if (j < nl * NB0 && fac[b][r] != 0.f) {
            double arg = tkz[b][r] * dzr;
            if constexpr (AB) arg += (double)ab2[b][r];
            float sn, cs;
            sincospif((float)(arg - 2.0 * rint(0.5 * arg)), &sn, &cs);
            ph[b][r] = fa ? make_float2(fac[b][r] * cs, fac[b][r] * sn)
                          : make_float2(-fac[b][r] * sn, fac[b][r] * cs);   // e^{i phi} (i g)
            const double sa = tkz[b][r] * sm.dz;
            sincospif((float)(sa - 2.0 * rint(0.5 * sa)), &sn, &cs);
            st[b][r] = make_float2(cs, sn);
          }
        }
      }
    }
    for (int z = zbeg; z < zend; ++z) {
#pragma unroll
      for (int b = 0; b < B0; ++b) {
        const int j = tid + b * nthr;
        if (j < nl * NB0) {
          const int l = j & (nl - 1), k = j >> lsh;
          float2 v[R0];
#pragma unroll
          for (int r = 0; r < R0; ++r) {
            v[r] = ph[b][r];
            if (z + 1 < zend) ph[b][r] = cmul(ph[b][r], st[b][r]);
          }
          dft_small<R0>(v, 1.f);   // span 1: no twiddles
#pragma unroll
          for (int r = 0; r < R0; ++r) buf[l + (k * R0 + r) * nl] = v[r];
        }
      }
      __syncthreads();
      static_passes<NS, 0, true, kEmax, false, false, 1, NP - 1>(buf, nl, nl, 1, lsh, tw, 1.f, tid, nthr);
#pragma unroll
      for (int b = 0; b < BL; ++b) {
        const int j = tid + b * nthr;
        if (j < nl * NSL) {
          const int l = j & (nl - 1), k = j >> lsh;
          float2 w[RL];
          float2 w1 = tw[k];   // span NSL = NS / RL: twiddle stride 1; conjugate for the inverse
          w1.y = -w1.y;
          twiddle_powers<RL>(w, w1);
          float2 v[RL];
#pragma unroll
          for (int r = 0; r < RL; ++r) {
            v[r] = buf[l + (k + r * NSL) * nl];
            if (r > 0) v[r] = cmul(v[r], w[r]);
          }
          dft_small<RL>(v, 1.f);
          const int f = l >> wsh, c = x0 + (l & (W - 1));
          float2* dst = c < XC ? field_at(patch, f, z, 0, c) : nullptr;
          if (dst) {
            const int pitch = (NF == 2 && f == 0) ? XA : XC;
#pragma unroll
            for (int r = 0; r < RL; ++r) dst[(long)(k + r * NSL) * pitch] = v[r];
          }
        }
      }
      __syncthreads();   // the next plane's first pass writes the same LDS
    }
  } else {
    // z-independent factors of this thread's elements e = tid + i * nthr
    double tkz[EPT], sp[EPT], gg[fluor ? 1 : EPT];
    float ab2[AB ? EPT : 1];   // 2 W(p): the aberration phase in units of pi
    {
      const double hw = soft_halfwidth(o, sm);
      const double km = o.n_medium / o.wavelength;
      const double ri = o.na_ill / o.wavelength;
      const DetAxis dax = det_axis(o);
      double cy, cx;
      source_centre(o, &cy, &cx);
      double psum = 0.0;
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        tkz[i] = 0.0;
        sp[i] = 0.0;
        if constexpr (AB) ab2[i] = 0.f;
        if (!fluor) gg[i] = 0.0;
        const int e = tid + i * nthr;
        if (e < Y * W) {
          const int ky = e >> wsh, w = e & (W - 1);
          const int c = x0 + w;
          const int kx = field_column(c, KP, X, XC);
          if (c < XC) {
            const double fy = freq_y(ky), fx = fftfreq(kx, X, sm.dx);
            const double P = det_pupil(o, dax, fy, fx, hw);
            if (P != 0.0) {
              const double kz = sqrt(fmax(km * km - (fy * fy + fx * fx), 0.0));
              tkz[i] = 2.0 * kz;
              if constexpr (AB) ab2[i] = (float)(2.0 * aberration_waves(o, fy, fx));
              if (fluor) {
                sp[i] = P;
                psum += P * P;
              } else {
                double S = disc(fy - cy, fx - cx, ri, hw);
                if (o.sector >= 0 && octant(fy - cy, fx - cx) != o.sector) S = 0.0;
                psum += S * P * P;
                sp[i] = S * P;
                if (kz > 0.0) gg[i] = P * km / kz;   // P * (i k_m / kz)
              }
            }
          }
        }
      }
      if (zc == 0) {
        const double tot = block_sum(psum, red);
        if (tid == 0) partials[patch * tiles_x + tile] = tot;
      }
    }
    for (int z = zbeg; z < zend; ++z) {
      const double dzr = plane_z(z, sm) - o.defocus;
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * nthr;
        if (e < Y * W) {
          const int ky = e >> wsh, w = e & (W - 1);
          float2 A = make_float2(0.f, 0.f), B = make_float2(0.f, 0.f);
          if (sp[i] != 0.0 || (!fluor && gg[i] != 0.0)) {
            // phase 2 pi kz (z - dz0): reduce the argument (in units of pi) in FP64
            // to [-1, 1], then evaluate sin/cos in FP32
            double arg = tkz[i] * dzr;
            if constexpr (AB) arg += (double)ab2[i];
            const float rr = (float)(arg - 2.0 * rint(0.5 * arg));
            float snf, csf;
            sincospif(rr, &snf, &csf);
            const double sn = snf, cs = csf;
            A = make_float2((float)(sp[i] * cs), (float)(sp[i] * sn));
            if (!fluor) B = make_float2((float)(-gg[i] * sn), (float)(gg[i] * cs));   // e^{i phi} (i g)
          }
          buf[ky * nf * W + w] = A;
          if (!fluor) buf[ky * nf * W + W + w] = B;
        }
      }
      __syncthreads();
      fft_lines<NS, 0, true>(buf, LdsLines{nf * W, nf * W, 1, true, pow2_shift(nf * W)}, plan, tw, 1.f,
                             tid, nthr);
      scatter_from_lds(buf, Y * nf * W, tid, nthr, [&](int e, float2 v) {
        const int ky = e >> (wsh + nf - 1);
        const int r = e & (nf * W - 1);
        const int f = r >> wsh, w = r & (W - 1);
        const int c = x0 + w;
        float2* dst = c < XC ? field_at(patch, f, z, ky, c) : nullptr;
        if (dst) *dst = v;
      });
      __syncthreads();
    }
  }
}

// Planes per workgroup of the z-chunked kernels: about `target` workgroups
// per launch, at most 16 planes.
int tf_z_chunk(const Sampling& sm, long tiles_x, long npatch, long target) {
  const long wg_per_plane = tiles_x * npatch;
  long zc = (long)sm.nz * wg_per_plane / target;
  if (zc < 1) zc = 1;
  if (zc > 16) zc = 16;
  if (zc > sm.nz) zc = sm.nz;
  return (int)zc;
}

bool tf_fields_choice_ok(int Z, const FftChoice& c) {
  return c.w >= 1 && c.w <= Z && c.threads == 0 && c.plan == 0;
}

// Each workgroup evaluates the z-independent pupil factors of its tile once
// (FP64 square roots and divisions) and its first plane in full, then
// advances the others by one complex multiply.  Few planes per workgroup
// repeat that set-up, many leave too few waves to hide the passes' waits, and
// a short last chunk of a half of the axis (the chunks do not cross its wrap)
// costs nearly as much as a full one.  Measured over 4..16 planes, 12 is best
// on 96x512x512 (60 tiles: 4 planes 80 us, 8 64 us, 12 55 us, 16 64 us) and on
// 64x1024x1024 (76 tiles: 6 planes 67 us, 8 64 us, 10 74 us, 12 58 us, 16 65
// us).  The default aims at about 480 workgroups and raises a chunk below 12
// planes to 12 while that still leaves 256 workgroups; the tuner picks the
// chunk by timing.
FftChoice tf_fields_default(int Z, long tiles, long npatch) {
  Sampling sm{};
  sm.nz = Z;
  const int zc = tf_z_chunk(sm, tiles, npatch, 480);
  if (zc < 12 && Z >= 12 && tiles * npatch * z_chunk_count(Z, (Z + 1) / 2, 12) >= 256)
    return FftChoice{12, 0, 0};
  return FftChoice{zc, 0, 0};
}

// Column-tile width of the field kernel: at most 4096 elements (512 threads)
// per workgroup.  The kernel synchronises its workgroup several times per
// plane, so several smaller workgroups per CU hide those waits better than
// one large one (measured: 96x512x512, 8 columns x 2 fields 169 us, 4 columns
// 135 us).
int tf_tile_width(const Sampling& sm, int ly) {
  const int nf = sm.model == kFluor3D ? 1 : 2;
  const long n = ly > 0 ? ly : sm.ny;
  const long lim = lds_limit_bytes() / (long)sizeof(float2);
  int W = 16;
  while (W > 1 && ((long)W * nf * n > 4096 || n + (long)W * nf * n > lim)) W /= 2;
  return W;
}

hipError_t launch_tf_fields_y(const DevOptics* opt, const Sampling& sm, int npatch, float2* ab,
                              double* partials, hipStream_t s, const LatSupport* sup) {
  const LatSupport ls = sup ? *sup : full_support(sm);
  if (ls.xc < 1 || ls.xc > sm.nx || ls.kp < 0 || ls.kp >= ls.xc || ls.ly < 2 || ls.ly > sm.ny ||
      ls.xa < 1 || ls.xa > ls.xc || ls.kpa < 0 || ls.kpa > ls.kp ||
      ls.xa - ls.kpa > ls.xc - ls.kp)   // A's columns among B's
    return hipErrorInvalidValue;
  const int LY = ls.ly;
  const bool one_field = sm.model == kFluor3D;
  const int xa = one_field ? ls.xc : ls.xa, kpa = one_field ? ls.kp : ls.kpa;
  FftPlan plan;
  if (!make_plan(LY, &plan)) return hipErrorInvalidValue;
  const int nf = sm.model == kFluor3D ? 1 : 2;
  const int W = tf_tile_width(sm, LY);
  const long tiles = (ls.xc + W - 1) / W;
  const FftKey key{kFftTfFields, LY, tiles, (long)npatch, sm.nz * 10 + nf};
  if (fft_recording())
    fft_record(key, [=] { return launch_tf_fields_y(opt, sm, npatch, ab, partials, s, &ls); });
  FftChoice fc;
  if (!fft_lookup(key, &fc) || !tf_fields_choice_ok(sm.nz, fc)) fc = tf_fields_default(sm.nz, tiles, npatch);
  const int ZC = fc.w;
  const long nwg = tiles * z_chunk_count(sm.nz, z_split(sm), ZC) * (long)npatch;
  const int thr = threads_for((long)LY * nf * W);
  const size_t lds = (size_t)(LY + LY * nf * W) * sizeof(float2);
  ScopedTiming _t("k_tf_fields_y", s);
#define WO_FIELDS(NN, FF, AA)                                                                    \
  hipLaunchKernelGGL((k_tf_fields_y<NN, FF, AA>), dim3((unsigned)nwg), dim3(thr), lds, s, opt, sm, ab, \
                     partials, W, tiles, ZC, ls.xc, ls.kp, LY, xa, kpa, plan)
#define X_(NN)                                                                                   \
  case NN:                                                                                       \
    if (nf == 2) {                                                                               \
      if (sm.aberrated) WO_FIELDS(NN, 2, true); else WO_FIELDS(NN, 2, false);                    \
    } else {                                                                                     \
      if (sm.aberrated) WO_FIELDS(NN, 1, true); else WO_FIELDS(NN, 1, false);                    \
    }                                                                                            \
    return hipGetLastError();
  switch (LY) {
    WO_LATERAL_SIZES(X_)
    default:
      break;
  }
#undef X_
  if (nf == 2) {
    if (sm.aberrated) WO_FIELDS(0, 2, true); else WO_FIELDS(0, 2, false);
  } else {
    if (sm.aberrated) WO_FIELDS(0, 1, true); else WO_FIELDS(0, 1, false);
  }
#undef WO_FIELDS
  return hipGetLastError();
}

// ------------------------------------------------------------------ rows: label-free

// out[patch * patch_stride + p * pstride + z * zstride + y * OP + k], k < KT,
// y < LY, p = 0 phase, 1 absorption (pstride < 0: phase only).  The fields are
// read in the compact column layout of the field kernel (XC columns, last
// non-negative column KP) and placed on an LX-point transform (frequency kx
// at index kx or LX + kx); the columns it does not store are zero.

template <int NS>
__global__ __launch_bounds__(1024) void k_tf_rows_lf(const double* __restrict__ partials,
                                                     long tiles_x, Sampling sm,
                                                     const float2* __restrict__ ab,
                                                     float2* __restrict__ out, long patch_stride,
                                                     long pstride, long zstride, int rows_per_wg,
                                                     long wg_per_patch, int XC, int KP, int KT,
                                                     int OP, int LY, int LX, int XA, int KPA,
                                                     FftPlan plan) {
  __shared__ double ibg_s;
  extern __shared__ float2 smem[];
  // transform lengths: LY rows per plane (the field kernel's), X = LX points
  // per row (compile-time for the index arithmetic)
  const int Y = LY, Z = sm.nz;
  const int X = NS > 0 ? NS : LX;
  float2* tw = smem;
  float2* buf = smem + X;
  const int tid = threadIdx.x, nthr = blockDim.x;
  fill_twiddles(tw, X, tid, nthr);
  const long patch = blockIdx.x / wg_per_patch;
  const long rpp = (long)Z * Y;
  const long row0 = (blockIdx.x - patch * wg_per_patch) * (long)rows_per_wg;
  const int nr = (int)min((long)rows_per_wg, rpp - row0);
  const int z0 = (int)(row0 / Y), y0 = (int)(row0 - (long)z0 * Y);
  const float2* a_src = ab + patch * rpp * (XA + XC);
  const float2* b_src = a_src + rpp * XA;
  const int PS = pad_shift(X);   // row padding
  const int LS = row_stride(X);      // padded line pitch in LDS
  // line 2r holds a (XA columns, last non-negative KPA), line 2r + 1 holds b
  // (XC, KP) of row r.  A column the field kernel does not store loads the
  // line's last non-negative column (a valid address, no branch, so the loads
  // of a thread stay in flight together) and is zeroed after the loads.
  auto load = [&](int t, int i) {
    const bool isb = t & 1;
    const int xc = isb ? XC : XA, kp = isb ? KP : KPA;
    const float2* src = (isb ? b_src : a_src) + (row0 + (t >> 1)) * xc;
    return src[i <= kp ? i : max(i - (X - xc), kp)];
  };
  auto kept = [&](int t, int i, float2 v) {
    const bool isb = t & 1;
    const int xc = isb ? XC : XA, kp = isb ? KP : KPA;
    return (i <= kp || i >= X - (xc - kp - 1)) ? v : make_float2(0.f, 0.f);
  };
  if constexpr (NS > 0) {
    // Inverse transforms of a and b in reversed radix order, the first pass
    // straight from memory; their last pass, the product c = b conj(a) /
    // (X Y I_bg) and the first pass of the forward transform of c run in
    // registers (the outputs of the one are the inputs of the other,
    // k + i NB); c goes to line 2r.
    constexpr int NP = StaticPlan<NS>::passes();
    constexpr int R0 = StaticPlan<NS>::radix(0);
    constexpr int NB = NS / R0;
    constexpr int BPF = (kEmax + 2 * R0 - 1) / (2 * R0);   // butterflies of a thread
    first_pass_in2<NS, 0, false, kEmax, true, true>(
        buf, 2 * nr, 1, LS, -1, 1.f, tid, nthr, load, kept,
        [&] { wave0_sum(partials + patch * tiles_x, tiles_x, &ibg_s); });   // sum S P^2
    const float cs = (float)(1.0 / ((double)X * (double)Y * ibg_s));
    static_passes<NS, 0, false, kEmax, true, true, 1, NP - 1>(buf, 2 * nr, 1, LS, -1, tw, 1.f, tid,
                                                              nthr);
    float2 cv[BPF][R0];
    int cr[BPF], ck[BPF];
#pragma unroll
    for (int b = 0; b < BPF; ++b) {
      const int j = tid + b * nthr;
      cr[b] = -1;
      if (j < nr * NB) {
        const int r = j / NB, k = j - r * NB;
        float2 w[R0];
        if constexpr (NP > 1) {
          float2 w1 = tw[k];   // span NB, twiddle stride 1; conjugate for the inverse
          w1.y = -w1.y;
          twiddle_powers<R0>(w, w1);
        }
        float2 va[R0], vb[R0];
#pragma unroll
        for (int i = 0; i < R0; ++i) {
          const int sl = row_slot(k + i * NB, PS);
          va[i] = buf[2 * r * LS + sl];
          vb[i] = buf[(2 * r + 1) * LS + sl];
          if constexpr (NP > 1) {
            if (i > 0) {
              va[i] = cmul(va[i], w[i]);
              vb[i] = cmul(vb[i], w[i]);
            }
          }
        }
        dft_small<R0>(va, 1.f);
        dft_small<R0>(vb, 1.f);
#pragma unroll
        for (int i = 0; i < R0; ++i) cv[b][i] = cscale(cmulconj(vb[i], va[i]), cs);
        dft_small<R0>(cv[b], -1.f);
        cr[b] = r;
        ck[b] = k;
      }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < BPF; ++b) {
      if (cr[b] >= 0) {
#pragma unroll
        for (int i = 0; i < R0; ++i) buf[2 * cr[b] * LS + row_slot(ck[b] * R0 + i, PS)] = cv[b][i];
      }
    }
    __syncthreads();
    static_passes<NS, 0, false, kEmax, true, false, 1, NP>(buf, nr, 1, 2 * LS, -1, tw, -1.f, tid, nthr);
  } else {
    gather_to_lds_map(buf, nr * 2 * X, tid, nthr, [&](int e) {
      const int t = e / X, i = e - t * X;
      return kept(t, i, load(t, i));
    }, [&](int e) {
      const int t = e / X;
      return t * LS + row_slot(e - t * X, PS);
    }, [&] { wave0_sum(partials + patch * tiles_x, tiles_x, &ibg_s); });   // sum S P^2
    __syncthreads();
    const float cs = (float)(1.0 / ((double)X * (double)Y * ibg_s));
    fft_lines<NS, 0, false, kEmax, true>(buf, LdsLines{2 * nr, 1, LS, false, -1, true}, plan, tw, 1.f,
                                         tid, nthr);
    for (int e = tid; e < nr * X; e += nthr) {
      const int r = e / X, i = row_slot(e - r * X, PS);
      const float2 a = buf[2 * r * LS + i], b = buf[(2 * r + 1) * LS + i];
      buf[2 * r * LS + i] = cscale(cmulconj(b, a), cs);
    }
    __syncthreads();
    fft_lines<NS, 0, false, kEmax, true>(buf, LdsLines{nr, 1, 2 * LS, false, -1, true}, plan, tw, -1.f,
                                         tid, nthr);
  }
  float2* op = out + patch * patch_stride;
  const float inv_kt = 1.0f / (float)KT;
  for (int e = tid; e < nr * KT; e += nthr) {
    const int r = div_small(e, inv_kt), k = e - r * KT;
    const float2 Ck = buf[2 * r * LS + row_slot(k, PS)];
    const float2 Cm = buf[2 * r * LS + row_slot(k == 0 ? 0 : X - k, PS)];
    int y = y0 + r, z = z0;
    while (y >= Y) { y -= Y; ++z; }
    const float2 U = make_float2(Ck.x + Cm.x, Ck.y - Cm.y);          // C + conj(C(-k))
    const float2 V = make_float2(-(Ck.y + Cm.y), Ck.x - Cm.x);       // i (C - conj(C(-k)))
    op[(long)z * zstride + (long)y * OP + k] = U;
    if (pstride >= 0) op[pstride + (long)z * zstride + (long)y * OP + k] = V;
  }
}

bool tf_rows_choice_ok(int X, const FftChoice& c) {
  const long elems = 2L * c.w * X;
  return c.w >= 1 && c.w <= 64 && elems <= kMaxElems && threads_ok(c.threads, elems) &&
         (long)(X + 2L * c.w * row_stride(X)) * (long)sizeof(float2) <= lds_limit_bytes() &&
         c.plan >= 0 && c.plan <= 3;
}

FftChoice tf_rows_default(int X) {
  int R = 2048 / X;                       // rows per workgroup (2 lines each)
  if (R < 1) R = 1;
  while (R > 1 && (2L * R * X > kMaxElems ||
                   (long)(X + 2L * R * row_stride(X)) * (long)sizeof(float2) > lds_limit_bytes()))
    --R;
  return FftChoice{R, threads_for(2L * R * X), 0};
}

hipError_t launch_tf_rows_labelfree(const double* partials, const Sampling& sm, int npatch,
                                    const float2* ab, float2* out, long patch_stride,
                                    long pstride, long zstride, hipStream_t s,
                                    const LatSupport* sup, int pitch) {
  const LatSupport ls = sup ? *sup : full_support(sm);
  const int LX = ls.lx, LY = ls.ly;
  if (ls.xc < 1 || ls.xc > LX || ls.kp < 0 || ls.kp >= ls.xc || ls.kt < 1 || 2 * (ls.kt - 1) > LX ||
      LX > sm.nx || LY < 2 || LY > sm.ny || ls.xa < 1 || ls.xa > ls.xc || ls.kpa < 0 ||
      ls.kpa > ls.kp || ls.xa - ls.kpa > ls.xc - ls.kp)
    return hipErrorInvalidValue;
  const int OP = pitch > 0 ? pitch : sm.nx / 2 + 1;
  if (OP < ls.kt) return hipErrorInvalidValue;
  const FftKey key{kFftTfRows, LX, LY, (long)npatch * sm.nz, pstride < 0 ? 1 : 0};
  if (fft_recording())
    fft_record(key, [=] {
      return launch_tf_rows_labelfree(partials, sm, npatch, ab, out, patch_stride, pstride, zstride, s,
                                      &ls, OP);
    });
  FftChoice c;
  if (!fft_lookup(key, &c) || !tf_rows_choice_ok(LX, c)) c = tf_rows_default(LX);
  const long tiles_x = (ls.xc + tf_tile_width(sm, LY) - 1) / tf_tile_width(sm, LY);
  FftPlan plan;
  if (!make_plan_variant(LX, c.plan, &plan)) return hipErrorInvalidValue;
  const int R = c.w;
  const long rpp = (long)sm.nz * LY;
  const long wpp = (rpp + R - 1) / R;
  const long nwg = wpp * npatch;
  const int thr = c.threads;
  const size_t lds = (size_t)(LX + 2L * R * row_stride(LX)) * sizeof(float2);
  ScopedTiming _t("k_tf_rows_lf", s);
#define X_(NN)                                                                                   \
  case NN:                                                                                       \
    hipLaunchKernelGGL((k_tf_rows_lf<NN>), dim3((unsigned)nwg), dim3(thr), lds, s, partials, tiles_x, \
                       sm, ab, out, patch_stride, pstride, zstride, R, wpp, ls.xc, ls.kp, ls.kt, OP, \
                       LY, LX, ls.xa, ls.kpa, plan);                                             \
    return hipGetLastError();
  if (c.plan == 0) switch (LX) {
      WO_LATERAL_SIZES(X_)
      default:
        break;
    }
#undef X_
  hipLaunchKernelGGL((k_tf_rows_lf<0>), dim3((unsigned)nwg), dim3(thr), lds, s, partials, tiles_x, sm,
                     ab, out, patch_stride, pstride, zstride, R, wpp, ls.xc, ls.kp, ls.kt, OP, LY, LX,
                     ls.xa, ls.kpa, plan);
  return hipGetLastError();
}

// ------------------------------------------------------------------ rows: fluorescence

// h: [patch][z][y][x] complex (after the inverse Y pass); out: [patch][z][y][Xh]
template <int NS>
__global__ __launch_bounds__(1024) void k_tf_rows_fl(const double* __restrict__ partials,
                                                     long tiles_x, Sampling sm,
                                                     const float2* __restrict__ h,
                                                     float2* __restrict__ out, int pairs_per_wg,
                                                     long wg_per_patch, FftPlan plan) {
  __shared__ double ibg_s;
  extern __shared__ float2 smem[];
  const int Y = sm.ny, X = sm.nx, Z = sm.nz, Xh = X / 2 + 1;
  float2* tw = smem;
  float2* buf = smem + X;
  const int tid = threadIdx.x, nthr = blockDim.x;
  fill_twiddles(tw, X, tid, nthr);
  const long patch = blockIdx.x / wg_per_patch;
  const long rpp = (long)Z * Y;
  const long row0 = (blockIdx.x - patch * wg_per_patch) * 2L * pairs_per_wg;
  const int nrows = (int)min(2L * pairs_per_wg, rpp - row0);
  const int np = (nrows + 1) / 2;
  const float2* src = h + patch * rpp * X;
  gather_to_lds(buf, 2 * np * X, tid, nthr, [&](int e) {
    const int l = e / X, i = e - l * X;
    return l < nrows ? src[(row0 + l) * X + i] : make_float2(0.f, 0.f);
  }, [&] { wave0_sum(partials + patch * tiles_x, tiles_x, &ibg_s); });   // sum P^2
  __syncthreads();
  fft_lines<NS, 0, false>(buf, LdsLines{2 * np, 1, X, false}, plan, tw, 1.f, tid, nthr);
  const double norm = 1.0 / ((double)Z * (double)X * (double)Y * ibg_s);
  const float nm = (float)norm;
  for (int e = tid; e < np * X; e += nthr) {
    const int q = e / X, i = e - q * X;
    const float2 u = buf[2 * q * X + i], v = buf[(2 * q + 1) * X + i];
    buf[2 * q * X + i] = make_float2((u.x * u.x + u.y * u.y) * nm, (v.x * v.x + v.y * v.y) * nm);
  }
  __syncthreads();
  fft_lines<NS, 0, false>(buf, LdsLines{np, 1, 2 * X, false}, plan, tw, -1.f, tid, nthr);
  float2* op = out + patch * rpp * Xh;
  for (int e = tid; e < np * Xh; e += nthr) {
    const int q = e / Xh, k = e - q * Xh;
    const float2 zk = buf[2 * q * X + k];
    const float2 zm = buf[2 * q * X + (k == 0 ? 0 : X - k)];
    const long r0 = row0 + 2 * q;
    op[r0 * Xh + k] = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
    if (r0 + 1 < rpp && 2 * q + 1 < nrows)
      op[(r0 + 1) * Xh + k] = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
  }
}

hipError_t launch_tf_rows_fluor(const double* partials, const Sampling& sm, int npatch,
                                const float2* h, float2* out, hipStream_t s) {
  const long tiles_x = (sm.nx + tf_tile_width(sm) - 1) / tf_tile_width(sm);
  FftPlan plan;
  if (!make_plan(sm.nx, &plan)) return hipErrorInvalidValue;
  int Q = 2048 / sm.nx;                       // row pairs per workgroup
  if (Q < 1) Q = 1;
  while (Q > 1 && 2L * Q * sm.nx > kMaxElems) --Q;
  const long rpp = (long)sm.nz * sm.ny;
  const long wpp = (rpp + 2 * Q - 1) / (2 * Q);
  const long nwg = wpp * npatch;
  const int thr = threads_for(2L * Q * sm.nx);
  const size_t lds = (size_t)(sm.nx + 2 * Q * sm.nx) * sizeof(float2);
  ScopedTiming _t("k_tf_rows_fl", s);
#define X_(NN)                                                                                   \
  case NN:                                                                                       \
    hipLaunchKernelGGL((k_tf_rows_fl<NN>), dim3((unsigned)nwg), dim3(thr), lds, s, partials, tiles_x, \
                       sm, h, out, Q, wpp, plan);                                                \
    return hipGetLastError();
  switch (sm.nx) {
    WO_LATERAL_SIZES(X_)
    default:
      break;
  }
#undef X_
  hipLaunchKernelGGL((k_tf_rows_fl<0>), dim3((unsigned)nwg), dim3(thr), lds, s, partials, tiles_x, sm, h,
                     out, Q, wpp, plan);
  return hipGetLastError();
}

}  // namespace wo
