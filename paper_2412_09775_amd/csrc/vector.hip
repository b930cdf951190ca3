// Vector label-free transfer functions (Table 1, vector column, label-free row).
//
// The bank correlates two tensor-valued fields per plane z.  The detected
// scattered field of a unit dipole along n, u_i'n = IFFT2[P_i'j G_jn prop],
// and the detected direct field of the source times the conjugate incident
// field that drives the dipole, v_ik = IFFT2[S P_ik' e_k' conj(e_k) prop].
// The aplanatic pupil map Q(p) (3 x 2) gives both: the incident field of
// source point q is e = Q J, the detection tensor is P E Q^T, and its
// columns are transverse to the wave, so P E Q^T (I - k^ k^T) g = P E g Q^T.
// The direct light reaches the detector as P E J, so v_ik = J_i w_k with
// w_k = IFFT2[S P E conj(e_k) prop]: six u fields and three w fields per
// illumination state.  A channel c (state s, analyser M_c) then responds to
// property p (tensor T_p) with
//   R_cp = 1 / (Y X I_bg) sum_n,k beta_n T_p^{nk} conj(w_k),
//   beta_n = sum_i' alpha_c,i' u_i'n,  alpha_c = J_s^H M_c,
// and H_cp = FFT3(2 Re R_cp).  The spectra vanish outside the detection
// pupil's columns: they are written on those columns only and inverse-
// transformed along Y there (column passes).  With a compiled row length the
// X transform and the products are fused per row (k_vec_rows_all or
// k_vec_rows_resp) on the support's shortened transforms; otherwise a complex
// row pass writes the fields on the grid and k_vec_products multiplies them
// per voxel.  The real responses are transformed forward by the row and
// column passes of the linear model, on the bank's support.
#include <algorithm>

#include "internal.hpp"

namespace wo {

struct VecBatch {
  VecRec r[4];
};
static_assert(sizeof(VecBatch) <= 3584, "kernel arguments are limited to 4 KiB");

__global__ void k_set_vec(VecRec* dst, VecBatch b, int count) {
  const int i = threadIdx.x;
  if (i < count) dst[i] = b.r[i];
}

hipError_t launch_set_vec(VecRec* dst, const VecRec* host, int n, hipStream_t s) {
  for (int i0 = 0; i0 < n; i0 += 4) {
    VecBatch b;
    const int cnt = n - i0 < 4 ? n - i0 : 4;
    for (int j = 0; j < cnt; ++j) b.r[j] = host[i0 + j];
    hipLaunchKernelGGL(k_set_vec, dim3(1), dim3(64), 0, s, dst + i0, b, cnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// One thread per lateral frequency (ky, kx) of one patch: the pupil values
// and the map Q in FP64, then every plane's propagator phase.  Q is written
// without angles: with w = 1 / (k_m (k_m + kz)),
//   Q = [[1 - px^2 w, -px py w], [-px py w, 1 - py^2 w], [-px / k_m, -py / k_m]].
// NS (1 or 5 illumination states) is a template parameter so that the
// per-state arrays stay in registers (a runtime bound indexed them from
// scratch memory).
// LY rows: row i of the LY-point transform stands for the grid's frequency
// (i or i - LY) / (ny dy); LY = ny is the grid's own transform, a shorter one
// (longer than twice the band) samples the same band-limited fields more
// coarsely along y.
template <int NS>
__global__ __launch_bounds__(256) void k_vec_spectra(const DevOptics* __restrict__ opt,
                                                     const VecRec* __restrict__ rec, Sampling sm,
                                                     float2* __restrict__ fields, int XC, int KP, int LY) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int ky = blockIdx.y;
  const long patch = blockIdx.z;
  const int X = sm.nx, Z = sm.nz;
  if (c >= XC) return;
  const int kx = field_column(c, KP, X, XC);
  const DevOptics o = opt[patch];
  const int F = 6 + 3 * NS;
  const long plane = (long)LY * XC;
  float2* base = fields + patch * (long)F * Z * plane + (long)ky * XC + c;
  const double fy = (double)(ky < (LY + 1) / 2 ? ky : ky - LY) / ((double)sm.ny * sm.dy);
  const double fx = fftfreq(kx, X, sm.dx);
  const double hw = soft_halfwidth(o, sm);
  const double km = o.n_medium / o.wavelength;
  const DetAxis dax = det_axis(o);
  const double P = det_pupil(o, dax, fy, fx, hw);
  double cy, cx;
  source_centre(o, &cy, &cx);
  const double S = disc(fy - cy, fx - cx, o.na_ill / o.wavelength, hw);
  const double kz = sqrt(fmax(km * km - (fy * fy + fx * fx), 0.0));
  // u_i'n spectrum: i (P k_m / kz) Q_n,i' e^{i phi}; w_k: S P conj(e_k) e^{i phi}
  float q[3][2] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
  float gp = 0.f, sp = 0.f;
  float2 ce[NS][3];
  if (P != 0.0 && kz > 0.0) {
    const double w = 1.0 / (km * (km + kz));
    q[0][0] = (float)(1.0 - fx * fx * w);
    q[0][1] = (float)(-fx * fy * w);
    q[1][0] = q[0][1];
    q[1][1] = (float)(1.0 - fy * fy * w);
    q[2][0] = (float)(-fx / km);
    q[2][1] = (float)(-fy / km);
    gp = (float)(P * km / kz);
    sp = (float)(S * P);
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const float2 jx = make_float2(rec[patch].J[s][0][0], rec[patch].J[s][0][1]);
    const float2 jy = make_float2(rec[patch].J[s][1][0], rec[patch].J[s][1][1]);
#pragma unroll
    for (int k = 0; k < 3; ++k)   // conj(e_k) = conj(Q_k0 Jx + Q_k1 Jy)
      ce[s][k] = make_float2(q[k][0] * jx.x + q[k][1] * jy.x, -(q[k][0] * jx.y + q[k][1] * jy.y));
  }
  const double ab2 = (gp != 0.f) ? 2.0 * aberration_waves(o, fy, fx) : 0.0;
  for (int z = 0; z < Z; ++z) {
    float sn = 0.f, cs = 0.f;
    if (gp != 0.f) {
      const double arg = 2.0 * kz * (plane_z(z, sm) - o.defocus) + ab2;   // phase / pi
      sincospif((float)(arg - 2.0 * rint(0.5 * arg)), &sn, &cs);
    }
    float2* pz = base + (long)z * plane;
#pragma unroll
    for (int ip = 0; ip < 2; ++ip)
#pragma unroll
      for (int n = 0; n < 3; ++n) {
        const float a = gp * q[n][ip];
        pz[(long)(3 * ip + n) * Z * plane] = make_float2(-a * sn, a * cs);   // i a e^{i phi}
      }
#pragma unroll
    for (int s = 0; s < NS; ++s)
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float2 c = ce[s][k];
        const float2 e = make_float2(sp * cs, sp * sn);
        pz[(long)(6 + 3 * s + k) * Z * plane] = make_float2(e.x * c.x - e.y * c.y, e.x * c.y + e.y * c.x);
      }
  }
}

hipError_t launch_vec_spectra(const DevOptics* opt, const VecRec* rec, const Sampling& sm, int npatch, int NS,
                              float2* fields, int XC, int KP, int LY, hipStream_t s) {
  if (NS < 1 || NS > 5 || npatch < 1 || npatch > 65535 || LY < 2 || LY > sm.ny) return hipErrorInvalidValue;
  if (XC < 1 || XC > sm.nx || KP < 0 || KP >= XC) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((XC + 255) / 256), (unsigned)LY, (unsigned)npatch);
  ScopedTiming _t("k_vec_spectra", s);
  if (NS == 1)
    hipLaunchKernelGGL(k_vec_spectra<1>, grid, dim3(256), 0, s, opt, rec, sm, fields, XC, KP, LY);
  else if (NS == 5)
    hipLaunchKernelGGL(k_vec_spectra<5>, grid, dim3(256), 0, s, opt, rec, sm, fields, XC, KP, LY);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Complex FFT along X of L rows per workgroup (unnormalised; sign -1 forward,
// +1 inverse): row r of src holds the XC kept columns of the spectrum
// (field_column order, the others zero), row r of dst receives all X values.
// Compiled lengths (NS > 0) take the first pass from memory and write the
// last one to memory from registers, as the real row passes do; other
// lengths use the runtime plan.
template <int NS>
__global__ __launch_bounds__(1024) void k_rows_c2c(const float2* __restrict__ src, float2* __restrict__ dst,
                                                   int X, int XC, int KP, long nrows, FftPlan plan, int L,
                                                   float sign) {
  extern __shared__ float2 smem[];
  float2* tw = smem;
  float2* buf = smem + X;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const long row0 = (long)blockIdx.x * L;
  const int nl = (int)min((long)L, nrows - row0);
  const int Xc = NS > 0 ? NS : X;
  const int PS = pad_shift(Xc), LS = row_stride(Xc);
  const float2* in = src + row0 * XC;
  float2* out = dst + row0 * Xc;
  // the condition depends on the index only, so the loads stay in flight together
  auto load = [&](int l, int k) {
    const int c = compact_column(k, KP, Xc, XC);
    return c >= 0 ? in[(long)l * XC + c] : make_float2(0.f, 0.f);
  };
  fill_twiddles(tw, Xc, tid, nthr);
  if constexpr (NS > 0) {
    constexpr int NP = StaticPlan<NS>::passes();
    auto finish = [](int, int, float2 v) { return v; };
    auto store = [&](int l, int i, float2 v) { out[(long)l * NS + i] = v; };
    first_pass_in2<NS, 0, false, kEmax, true, false>(buf, nl, 1, LS, -1, sign, tid, nthr, load, finish,
                                                     [] {});
    static_passes<NS, 0, false, kEmax, true, false, 1, NP - 1>(buf, nl, 1, LS, -1, tw, sign, tid, nthr);
    last_pass_out<NS, 0, false, kEmax, true, false>(buf, nl, 1, LS, -1, tw, sign, tid, nthr, store);
  } else {
    auto slot = [&](int e) {
      const int l = e / Xc;
      return l * LS + row_slot(e - l * Xc, PS);
    };
    gather2_to_lds(buf, nl * Xc, tid, nthr, [&](int e) {
      const int l = e / Xc;
      return load(l, e - l * Xc);
    }, [](int, float2 v) { return v; }, slot, [] {});
    __syncthreads();
    fft_lines<0, 0, false, kEmax, true>(buf, LdsLines{nl, 1, LS, false, -1, true}, plan, tw, sign, tid,
                                        nthr);
    __syncthreads();
    scatter_from_lds_map(buf, nl * Xc, tid, nthr, slot, [&](int e, float2 v) { out[e] = v; });
  }
}

hipError_t launch_rows_c2c(const float2* src, float2* dst, int X, int XC, int KP, long nrows, float sign,
                           hipStream_t s) {
  if (X < 2 || nrows < 1 || XC < 1 || XC > X || KP < 0 || KP >= XC) return hipErrorInvalidValue;
  FftPlan plan;
  if (!make_plan(X, &plan)) return hipErrorInvalidValue;
  int L = 2048 / X;   // 2048 elements per workgroup, as the real row passes
  if (L < 1) L = 1;
  while (L > 1 && (long)L * X > kMaxElems) --L;
  if ((long)L * X > kMaxElems) return hipErrorInvalidValue;
  const size_t lds = (size_t)(X + (long)L * row_stride(X)) * sizeof(float2);
  if ((long)lds > lds_limit_bytes()) return hipErrorInvalidValue;
  const long nwg = (nrows + L - 1) / L;
  const int thr = threads_for((long)L * X);
  ScopedTiming _t("k_rows_c2c", s);
#define X_(NN)                                                                                       \
  case NN:                                                                                           \
    hipLaunchKernelGGL((k_rows_c2c<NN>), dim3((unsigned)nwg), dim3(thr), lds, s, src, dst, X, XC, KP, \
                       nrows, plan, L, sign);                                                        \
    return hipGetLastError();
  switch (X) {
    WO_LATERAL_SIZES(X_)
    default:
      break;
  }
#undef X_
  hipLaunchKernelGGL((k_rows_c2c<0>), dim3((unsigned)nwg), dim3(thr), lds, s, src, dst, X, XC, KP, nrows, plan,
                     L, sign);
  return hipGetLastError();
}

// One thread per voxel of one patch: beta_n = sum_i' alpha_c,i' u_i'n for
// every channel, then 2 Re(sum_n,k T_p^{nk} beta_n conj(w_k)) / (Y X I_bg)
// for every property.  NS illumination states: one (the four Stokes channels
// share it) or five (channel c uses state c); compile-time, so that every
// array index is static and the fields stay in registers.
template <int NS>
__global__ __launch_bounds__(256) void k_vec_products(const VecRec* __restrict__ rec,
                                                      const float2* __restrict__ fields,
                                                      float* __restrict__ out, long vox) {
  constexpr int C = NS == 1 ? 4 : 5, F = 6 + 3 * NS;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long patch = blockIdx.y;
  if (i >= vox) return;
  const VecRec& r = rec[patch];
  const int P = r.P;
  const float2* fp = fields + patch * (long)F * vox + i;
  float2 u[6], w[NS][3];
#pragma unroll
  for (int f = 0; f < 6; ++f) u[f] = fp[(long)f * vox];
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int k = 0; k < 3; ++k) w[s][k] = fp[(long)(6 + 3 * s + k) * vox];
  const float sc = 2.f * r.scale;
  float* op = out + patch * (long)C * P * vox + i;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const int s = NS == 1 ? 0 : c;
    const float2 a0 = make_float2(r.alpha[c][0][0], r.alpha[c][0][1]);
    const float2 a1 = make_float2(r.alpha[c][1][0], r.alpha[c][1][1]);
    float2 qm[3][3];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const float2 b = cadd(cmul(a0, u[n]), cmul(a1, u[3 + n]));
#pragma unroll
      for (int k = 0; k < 3; ++k) qm[n][k] = cmul(b, make_float2(w[s][k].x, -w[s][k].y));
    }
    for (int p = 0; p < P; ++p) {
      float acc = 0.f;
#pragma unroll
      for (int e = 0; e < 9; ++e) {
        const float2 t = make_float2(r.T[p][e][0], r.T[p][e][1]);
        acc += t.x * qm[e / 3][e % 3].x - t.y * qm[e / 3][e % 3].y;
      }
      op[(long)(c * P + p) * vox] = sc * acc;
    }
  }
}

hipError_t launch_vec_products(const VecRec* rec, const float2* fields, float* out, long vox, int F, int npatch,
                               hipStream_t s) {
  if (vox < 1 || npatch < 1 || npatch > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((vox + 255) / 256), (unsigned)npatch);
  ScopedTiming _t("k_vec_products", s);
  if (F == 9)
    hipLaunchKernelGGL(k_vec_products<1>, grid, dim3(256), 0, s, rec, fields, out, vox);
  else if (F == 21)
    hipLaunchKernelGGL(k_vec_products<5>, grid, dim3(256), 0, s, rec, fields, out, vox);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// Channel responses straight from the Y-transformed spectra (compiled row
// lengths N, the grid's X or a shorter length holding the responses'
// band without wrap-around): one workgroup per row (patch, z, y) and channel c.  beta_n =
// sum_i' alpha_c,i' u_i'n is linear in the fields, so its three lines are
// formed from the u spectra as they are loaded; with the three w lines of
// the channel's state they are inverse-transformed along X in LDS (six
// lines), and each x then gets the channel's P responses.  This replaces the
// full-grid fields' round trip through HBM (the X pass writing them, the
// products reading them) by a re-read of the compact spectra per channel.
template <int NS, int N>
__global__ __launch_bounds__(1024) void k_vec_rows_resp(const VecRec* __restrict__ rec,
                                                        const float2* __restrict__ spec,
                                                        float* __restrict__ out, int XC, int KP, long zy) {
  constexpr int C = NS == 1 ? 4 : 5, F = 6 + 3 * NS, NL = 6;
  extern __shared__ float2 smem[];
  float2* tw = smem;
  float2* buf = smem + N;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const long rowid = blockIdx.x / C;
  const int c = (int)(blockIdx.x - rowid * C);
  const long patch = rowid / zy, r = rowid - patch * zy;
  const VecRec& rv = rec[patch];
  const int s = NS == 1 ? 0 : c;
  const float2 a0 = make_float2(rv.alpha[c][0][0], rv.alpha[c][0][1]);
  const float2 a1 = make_float2(rv.alpha[c][1][0], rv.alpha[c][1][1]);
  const float2* sp = spec + patch * (long)F * zy * XC + r * XC;
  const int PS = pad_shift(N), LS = row_stride(N);
  fill_twiddles(tw, N, tid, nthr);
  // line l < 3: beta_l = alpha_0 u_0l + alpha_1 u_1l; l >= 3: w_{l-3} of state s
  auto load = [&](int l, int k) {
    const int cc = compact_column(k, KP, N, XC);
    float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
    if (cc >= 0) {
      if (l < 3) {
        const float2 u0 = sp[(long)l * zy * XC + cc], u1 = sp[(long)(3 + l) * zy * XC + cc];
        v = make_float4(u0.x, u0.y, u1.x, u1.y);
      } else {
        const float2 w = sp[(long)(6 + 3 * s + l - 3) * zy * XC + cc];
        v = make_float4(w.x, w.y, 0.f, 0.f);
      }
    }
    return v;
  };
  auto finish = [&](int l, int, float4 v) {
    if (l >= 3) return make_float2(v.x, v.y);
    return cadd(cmul(a0, make_float2(v.x, v.y)), cmul(a1, make_float2(v.z, v.w)));
  };
  constexpr int NP = StaticPlan<N>::passes();
  first_pass_in2<N, 0, false, kEmax, true, false>(buf, NL, 1, LS, -1, 1.f, tid, nthr, load, finish, [] {});
  static_passes<N, 0, false, kEmax, true, false, 1, NP>(buf, NL, 1, LS, -1, tw, 1.f, tid, nthr);
  __syncthreads();
  const int P = rv.P;
  const float sc = 2.f * rv.scale_short;
  const long vox = zy * N;
  float* op = out + (patch * (long)C + c) * P * vox + r * N;
  for (int x = tid; x < N; x += nthr) {
    const int sl = row_slot(x, PS);
    float2 qm[3][3];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const float2 b = buf[n * LS + sl];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float2 w = buf[(3 + k) * LS + sl];
        qm[n][k] = cmul(b, make_float2(w.x, -w.y));
      }
    }
    for (int p = 0; p < P; ++p) {
      float acc = 0.f;
#pragma unroll
      for (int e = 0; e < 9; ++e) {
        const float2 t = make_float2(rv.T[p][e][0], rv.T[p][e][1]);
        acc += t.x * qm[e / 3][e % 3].x - t.y * qm[e / 3][e % 3].y;
      }
      op[(long)p * vox + x] = sc * acc;
    }
  }
}

// The same for every channel of a row in one workgroup, where the row's six u
// lines and 3 NS w lines fit LDS (each set transformed in one batch): the
// spectra are read once per row instead of once per channel, and beta is
// formed per x from the transformed u lines.
template <int NS, int N>
__global__ __launch_bounds__(1024) void k_vec_rows_all(const VecRec* __restrict__ rec,
                                                       const float2* __restrict__ spec,
                                                       float* __restrict__ out, int XC, int KP, long zy) {
  constexpr int C = NS == 1 ? 4 : 5, F = 6 + 3 * NS, NW = 3 * NS;
  extern __shared__ float2 smem[];
  float2* tw = smem;
  const int LS = row_stride(N), PS = pad_shift(N);
  float2* bu = smem + N;            // 6 u lines
  float2* bw = bu + 6 * LS;         // 3 NS w lines
  const int tid = threadIdx.x, nthr = blockDim.x;
  const long rowid = blockIdx.x;
  const long patch = rowid / zy, r = rowid - patch * zy;
  const VecRec& rv = rec[patch];
  const float2* sp = spec + patch * (long)F * zy * XC + r * XC;
  fill_twiddles(tw, N, tid, nthr);
  auto finish = [](int, int, float2 v) { return v; };
  constexpr int NP = StaticPlan<N>::passes();
  auto load_u = [&](int l, int k) {
    const int cc = compact_column(k, KP, N, XC);
    return cc >= 0 ? sp[(long)l * zy * XC + cc] : make_float2(0.f, 0.f);
  };
  auto load_w = [&](int l, int k) {
    const int cc = compact_column(k, KP, N, XC);
    return cc >= 0 ? sp[(long)(6 + l) * zy * XC + cc] : make_float2(0.f, 0.f);
  };
  first_pass_in2<N, 0, false, kEmax, true, false>(bu, 6, 1, LS, -1, 1.f, tid, nthr, load_u, finish, [] {});
  static_passes<N, 0, false, kEmax, true, false, 1, NP>(bu, 6, 1, LS, -1, tw, 1.f, tid, nthr);
  first_pass_in2<N, 0, false, kEmax, true, false>(bw, NW, 1, LS, -1, 1.f, tid, nthr, load_w, finish, [] {});
  static_passes<N, 0, false, kEmax, true, false, 1, NP>(bw, NW, 1, LS, -1, tw, 1.f, tid, nthr);
  __syncthreads();
  const int P = rv.P;
  const float sc = 2.f * rv.scale_short;
  const long vox = zy * N;
  float* op = out + patch * (long)C * P * vox + r * N;
  // one (channel, x) pair per thread and step: every thread busy, x contiguous
  // across a wave for the stores
  for (int e = tid; e < C * N; e += nthr) {
    const int c = e / N, x = e - c * N;
    const int sl = row_slot(x, PS);
    const int s = NS == 1 ? 0 : c;
    const float2 a0 = make_float2(rv.alpha[c][0][0], rv.alpha[c][0][1]);
    const float2 a1 = make_float2(rv.alpha[c][1][0], rv.alpha[c][1][1]);
    float2 cw[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float2 w = bw[(3 * s + k) * LS + sl];
      cw[k] = make_float2(w.x, -w.y);
    }
    float2 qm[3][3];
#pragma unroll
    for (int n = 0; n < 3; ++n) {
      const float2 b = cadd(cmul(a0, bu[n * LS + sl]), cmul(a1, bu[(3 + n) * LS + sl]));
#pragma unroll
      for (int k = 0; k < 3; ++k) qm[n][k] = cmul(b, cw[k]);
    }
    for (int p = 0; p < P; ++p) {
      float acc = 0.f;
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const float2 t = make_float2(rv.T[p][q][0], rv.T[p][q][1]);
        acc += t.x * qm[q / 3][q % 3].x - t.y * qm[q / 3][q % 3].y;
      }
      op[(long)(c * P + p) * vox + x] = sc * acc;
    }
  }
}

// Whether every channel of a row fits one workgroup of k_vec_rows_all.
static bool vec_rows_all_fits(int X, int NS) {
  const long nw = 3L * NS * X;
  return 6L * X <= kMaxElems && nw <= kMaxElems &&
         (long)(X + (6L + 3L * NS) * row_stride(X)) * (long)sizeof(float2) <= lds_limit_bytes();
}

bool vec_rows_fused(int X) {
  switch (X) {
#define X_(NN) case NN:
    WO_LATERAL_SIZES(X_)
#undef X_
    return true;
    default:
      return false;
  }
}

hipError_t launch_vec_rows_resp(const VecRec* rec, const float2* spec, float* out, int X, int XC, int KP, long zy,
                                int NS, int npatch, hipStream_t s) {
  if (!vec_rows_fused(X) || (NS != 1 && NS != 5) || zy < 1 || npatch < 1 || XC < 1 || XC > X || KP < 0 ||
      KP >= XC)
    return hipErrorInvalidValue;
  const int C = NS == 1 ? 4 : 5;
  if (vec_rows_all_fits(X, NS)) {
    const long nwg = (long)npatch * zy;
    if (nwg > 0x7fffffffL) return hipErrorInvalidValue;
    const int thr = threads_for(std::max(6L, 3L * NS) * X);
    const size_t lds = (size_t)(X + (6L + 3L * NS) * row_stride(X)) * sizeof(float2);
    ScopedTiming _t("k_vec_rows_resp", s);
#define X_(NN)                                                                                       \
  case NN:                                                                                           \
    if (NS == 1)                                                                                     \
      hipLaunchKernelGGL((k_vec_rows_all<1, NN>), dim3((unsigned)nwg), dim3(thr), lds, s, rec, spec, out, XC, \
                         KP, zy);                                                                    \
    else                                                                                             \
      hipLaunchKernelGGL((k_vec_rows_all<5, NN>), dim3((unsigned)nwg), dim3(thr), lds, s, rec, spec, out, XC, \
                         KP, zy);                                                                    \
    return hipGetLastError();
    switch (X) {
      WO_LATERAL_SIZES(X_)
      default:
        break;
    }
#undef X_
    return hipErrorInvalidValue;
  }
  const long nwg = (long)npatch * zy * C;
  if (nwg > 0x7fffffffL) return hipErrorInvalidValue;
  const int thr = threads_for(6L * X);
  const size_t lds = (size_t)(X + 6L * row_stride(X)) * sizeof(float2);
  if ((long)lds > lds_limit_bytes()) return hipErrorInvalidValue;
  ScopedTiming _t("k_vec_rows_resp", s);
#define X_(NN)                                                                                       \
  case NN:                                                                                           \
    if (NS == 1)                                                                                     \
      hipLaunchKernelGGL((k_vec_rows_resp<1, NN>), dim3((unsigned)nwg), dim3(thr), lds, s, rec, spec, out, XC, \
                         KP, zy);                                                                    \
    else                                                                                             \
      hipLaunchKernelGGL((k_vec_rows_resp<5, NN>), dim3((unsigned)nwg), dim3(thr), lds, s, rec, spec, out, XC, \
                         KP, zy);                                                                    \
    return hipGetLastError();
  switch (X) {
    WO_LATERAL_SIZES(X_)
    default:
      break;
  }
#undef X_
  return hipErrorInvalidValue;
}

}  // namespace wo
