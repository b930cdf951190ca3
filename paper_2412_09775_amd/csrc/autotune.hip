// Mid-band loss, its parameter gradient through the thin-model transfer
// function, and the Adam auto-tune step (Results, "Physics-guided ML
// auto-tunes multi-contrast blind deconvolution"; Methods, "Cell-scale optical
// pooled screen data"; Ext. Data Fig. 3).
//
// Per iteration, for every (virtual) patch v with parameters theta_v =
// (defocus, NA_det, tilt zenith, tilt azimuth):
//   forward   A_z, B_z -> a, b (inverse 2D FFT) -> c = s b conj(a), s = N / I_bg
//             H_z = [FFT2(2 Re c), FFT2(-2 Im c)]
//             F = (H^H H + eta I)^-1 H^H D per 2D frequency (D = FFT2 of the stack)
//             L = -(1/|B|) sum_{nu in band} |F_phase(nu)|^2
//   backward  G_H = dL/dH* = r Y^H - (H Y) F^H, Y = M^-1 dL/dF*, r = D - H F
//             Gamma = Re N IFFT2(G_phase) + i Re N IFFT2(G_abs)
//             dL = 4 Re sum Gamma dc
//                = 4 Re sum_p dB(p) IFFT2(s Gamma conj a)(p)
//                + 4 Re sum_q dA(q) IFFT2(s conj(Gamma b))(q)
//                + 4 Re sum Gamma b conj(a) ds
//             with analytic dA/dtheta, dB/dtheta and dI_bg/dtheta.
// The transfer function is recomputed every iteration, never stored across
// iterations.
#include "internal.hpp"

namespace wo {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ double block_sum_d(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
  return t;
}

// ------------------------------------------------------------------ loss and dL/dH*

// One thread per half-spectrum frequency m = ky * Xh + kx of virtual patch v.
// D: [n][Z][Y][Xh] (patch v reads data patch v / data_div), bank: [v][Z][2][Y][Xh],
// overwritten with dL/dH*.  lpart[v * bpp + block] = sum of w |F_phase|^2.
__global__ __launch_bounds__(256) void k_loss_grad(const DevOptics* __restrict__ opt,
                                                   const TuneState* __restrict__ st, Sampling sm,
                                                   const float2* __restrict__ D,
                                                   float2* __restrict__ bank,
                                                   double* __restrict__ lpart, long bpp,
                                                   int data_div) {
  __shared__ double red[4];
  const int Z = sm.nz, Y = sm.ny, X = sm.nx, Xh = X / 2 + 1;
  const long M = (long)Y * Xh;
  const long v = blockIdx.x / bpp;
  const long blk = blockIdx.x - v * bpp;
  const long m = blk * blockDim.x + threadIdx.x;
  double lsum = 0.0;
  if (m < M) {
    const int ky = (int)(m / Xh), kx = (int)(m - (long)ky * Xh);
    const double fy = fftfreq(ky, Y, sm.dy), fx = fftfreq(kx, X, sm.dx);
    const double r = sqrt(fy * fy + fx * fx);
    const TuneState& s = st[v];
    const bool band = r >= s.nu_c / 8.0 && r <= s.nu_c / 4.0;
    const float eta = (float)s.eta;
    const float2* dp = D + (v / data_div) * (long)Z * M + m;
    float2* hp = bank + v * (long)Z * 2 * M + m;
    // pass 1: normal matrix and right-hand side
    float m00 = 0.f, m11 = 0.f;
    float2 m10 = make_float2(0.f, 0.f), r0 = make_float2(0.f, 0.f), r1 = make_float2(0.f, 0.f);
#pragma unroll 4
    for (int c = 0; c < Z; ++c) {
      const float2 h0 = hp[(long)(2 * c) * M], h1 = hp[(long)(2 * c + 1) * M];
      const float2 x = dp[(long)c * M];
      m00 += h0.x * h0.x + h0.y * h0.y;
      m11 += h1.x * h1.x + h1.y * h1.y;
      m10 = cadd(m10, cmul(cconj(h1), h0));
      r0 = cadd(r0, cmul(cconj(h0), x));
      r1 = cadd(r1, cmul(cconj(h1), x));
    }
    const float a00 = m00 + eta, a11 = m11 + eta;
    const float det = a00 * a11 - (m10.x * m10.x + m10.y * m10.y);
    const float idet = __builtin_amdgcn_rcpf(det);   // hardware reciprocal (about 1 ulp)
    // F = M^-1 r with M = [[a00, conj(m10)], [m10, a11]]
    const float2 F0 = cscale(csub(cscale(r0, a11), cmul(cconj(m10), r1)), idet);
    const float2 F1 = cscale(csub(cscale(r1, a00), cmul(m10, r0)), idet);
    if (band) {
      const double w = (kx == 0 || 2 * kx == X) ? 1.0 : 2.0;
      lsum = w * ((double)F0.x * F0.x + (double)F0.y * F0.y);
      const float ib = (float)(1.0 / s.band_count);
      const float2 g0 = cscale(F0, -ib);                  // dL/dF_phase*
      const float2 Y0 = cscale(cscale(g0, a11), idet);    // Y = M^-1 (g0, 0)
      const float2 Y1 = cscale(cmul(m10, g0), -idet);
#pragma unroll 4
      for (int c = 0; c < Z; ++c) {
        const float2 h0 = hp[(long)(2 * c) * M], h1 = hp[(long)(2 * c + 1) * M];
        const float2 x = dp[(long)c * M];
        const float2 rc = csub(x, cadd(cmul(h0, F0), cmul(h1, F1)));
        const float2 hy = cadd(cmul(h0, Y0), cmul(h1, Y1));
        hp[(long)(2 * c) * M] = csub(cmulconj(rc, Y0), cmulconj(hy, F0));
        hp[(long)(2 * c + 1) * M] = csub(cmulconj(rc, Y1), cmulconj(hy, F1));
      }
    } else {
      for (int c = 0; c < 2 * Z; ++c) hp[(long)c * M] = make_float2(0.f, 0.f);
    }
  }
  const double tot = block_sum_d(lsum, red);
  if (threadIdx.x == 0) lpart[v * bpp + blk] = tot;
}

hipError_t launch_loss_grad(const DevOptics* opt, const TuneState* st, const Sampling& sm, int nv,
                            const float2* D, float2* bank, double* lpart, int data_div,
                            hipStream_t s) {
  const long M = (long)sm.ny * (sm.nx / 2 + 1);
  const long bpp = (M + 255) / 256;
  { ScopedTiming _t("k_loss_grad", s);
  hipLaunchKernelGGL(k_loss_grad, dim3((unsigned)(bpp * nv)), dim3(256), 0, s, opt, st, sm, D, bank,
                     lpart, bpp, data_div); }
  return hipGetLastError();
}

long loss_blocks(const Sampling& sm) {
  const long M = (long)sm.ny * (sm.nx / 2 + 1);
  return (M + 255) / 256;
}

// ------------------------------------------------------------------ gradient of a loss of the 3D reconstruction

// One thread per 3D half-spectrum frequency (kz, m) of patch v (grid y).  bank:
// [v][Z][2][M] the label-free pair after its Z transform (POL: the 5 x 4 bank is
// pol5_entry(coupling, pair)); D: [v][C][Z][M] the data spectrum; G: [v][P][Z][M]
// the spectrum of dL/df.  Per frequency, with x = D - N b delta,
// M = H^H H (+ eta I), F = M^-1 H^H x, Y = M^-1 G, R = x - H F:
//   dL/dH* = (R Y^H - H Y F^H) / (2N)   (dL/dF* = G / (2N))
// overwrites the pair in bank (POL: its coefficients summed through the
// coupling, dL/dH_phase* = sum_cp Re(kappa_cp) dL/dH_cp*, dL/dH_abs* with
// Im(kappa_cp)), and, if want_dd, D by H Y, the spectrum of dL/dd.
template <bool POL>
__global__ __launch_bounds__(256) void k_recon_grad(float2* __restrict__ bank, float2* __restrict__ D,
                                                    const float2* __restrict__ G,
                                                    const float* __restrict__ bg,
                                                    const Coupling* __restrict__ cpl, int Z, long M,
                                                    float eta, float n_full, int want_dd) {
  constexpr int C = POL ? 5 : 1, P = POL ? 4 : 2;
  const long per = (long)Z * M;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long v = blockIdx.y;
  if (gid >= per) return;
  const int z = (int)(gid / M);
  const long m = gid - (long)z * M;
  float2* hp = bank + ((v * Z + z) * 2) * M + m;
  const float2 u = hp[0], w = hp[M];
  float2 H[C][P];
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int p = 0; p < P; ++p)
      H[c][p] = POL ? pol5_entry(cpl[v].k[c][p][0], cpl[v].k[c][p][1], u, w) : (p == 0 ? u : w);
  const bool dc = z == 0 && m == 0;
  float2 x[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    x[c] = D[((v * C + c) * Z + z) * M + m];
    if (dc && bg) x[c].x -= n_full * bg[v * C + c];
  }
  float2 g[P], mm[P][P], r[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    g[p] = G[((v * P + p) * Z + z) * M + m];
    r[p] = make_float2(0.f, 0.f);
#pragma unroll
    for (int q = 0; q <= p; ++q) mm[p][q] = make_float2(0.f, 0.f);
  }
#pragma unroll
  for (int c = 0; c < C; ++c)
#pragma unroll
    for (int p = 0; p < P; ++p) {
      r[p] = cadd(r[p], cmul(cconj(H[c][p]), x[c]));
#pragma unroll
      for (int q = 0; q <= p; ++q) mm[p][q] = cadd(mm[p][q], cmul(cconj(H[c][p]), H[c][q]));
    }
  float2 L[P][P], F[P], Yv[P];
  float dinv[P];
  chol_factor<P>(mm, eta, L, dinv);
  chol_apply<P>(L, dinv, r, F);
  chol_apply<P>(L, dinv, g, Yv);
  const float s = 0.5f / n_full;
  float2 pair[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
#pragma unroll
  for (int c = 0; c < C; ++c) {
    float2 R = x[c], HY = make_float2(0.f, 0.f);
#pragma unroll
    for (int p = 0; p < P; ++p) {
      R = csub(R, cmul(H[c][p], F[p]));
      HY = cadd(HY, cmul(H[c][p], Yv[p]));
    }
#pragma unroll
    for (int p = 0; p < P; ++p) {
      const float2 Wcp = cscale(csub(cmulconj(R, Yv[p]), cmulconj(HY, F[p])), s);
      if (POL) {
        pair[0] = cadd(pair[0], cscale(Wcp, cpl[v].k[c][p][0]));
        pair[1] = cadd(pair[1], cscale(Wcp, cpl[v].k[c][p][1]));
      } else {
        pair[p] = Wcp;
      }
    }
    if (want_dd) D[((v * C + c) * Z + z) * M + m] = HY;
  }
  hp[0] = pair[0];
  hp[M] = pair[1];
}

hipError_t launch_recon_grad(float2* bank, float2* D, const float2* G, const float* bg, const Coupling* cpl,
                             const Sampling& sm, int npatch, float eta, double n_full, int want_dd,
                             hipStream_t s) {
  const long M = (long)sm.ny * (sm.nx / 2 + 1);
  const long per = (long)sm.nz * M;
  const long blocks = (per + 255) / 256;
  if (npatch < 1 || npatch > 65535 || blocks > 0x7fffffffL) return hipErrorInvalidValue;
  ScopedTiming _t("k_recon_grad", s);
  if (cpl)
    hipLaunchKernelGGL(k_recon_grad<true>, dim3((unsigned)blocks, (unsigned)npatch), dim3(256), 0, s, bank,
                       D, G, bg, cpl, sm.nz, M, eta, (float)n_full, want_dd);
  else
    hipLaunchKernelGGL(k_recon_grad<false>, dim3((unsigned)blocks, (unsigned)npatch), dim3(256), 0, s, bank,
                       D, G, bg, cpl, sm.nz, M, eta, (float)n_full, want_dd);
  return hipGetLastError();
}

// ------------------------------------------------------------------ backward rows

// ab: [v][2][Z][Y][XC] (field 0 = a, 1 = b after the inverse Y pass, complex,
// in the compact columns of the field kernel: XC kept, last non-negative KP;
// the others are zero, and so are u_A, u_B there: only the kept columns are
// written back);
// g: [v][Z][2][Y][Xh], the half spectra of dL/dH* after the inverse Y pass.  For
// each row the kernel forms Gamma = Gamma_phase + i Gamma_abs in one inverse X
// transform (the two real rows packed into one complex line), then replaces
// field 0 by the inverse X transform of u_A = conj(Gamma b)/(N I_bg) and field 1
// by that of u_B = Gamma conj(a)/(N I_bg); dpart[v * wpp + wg] =
// sum Re(Gamma b conj(a)).
template <int NS>
__global__ __launch_bounds__(1024) void k_tf_rows_bwd(const double* __restrict__ partials,
                                                      long tiles_x, Sampling sm,
                                                      float2* __restrict__ ab,
                                                      const float2* __restrict__ g,
                                                      double* __restrict__ dpart, int rows_per_wg,
                                                      long wg_per_patch, int XC, int KP, FftPlan plan) {
  extern __shared__ float2 smem[];
  __shared__ double red[kMaxThreads / 64];
  __shared__ double ibg_s;
  const int Y = sm.ny, Z = sm.nz;
  const int X = NS > 0 ? NS : sm.nx;   // compile-time length for the index arithmetic
  const int Xh = X / 2 + 1;
  float2* tw = smem;
  float2* buf = smem + X;
  const int tid = threadIdx.x, nthr = blockDim.x;
  fill_twiddles(tw, X, tid, nthr);
  const long v = blockIdx.x / wg_per_patch;
  const long rpp = (long)Z * Y;
  const long wg = blockIdx.x - v * wg_per_patch;
  const long row0 = wg * (long)rows_per_wg;
  const int nr = (int)min((long)rows_per_wg, rpp - row0);
  const int z0 = (int)(row0 / Y), y0 = (int)(row0 - (long)z0 * Y);
  float2* a_src = ab + (v * 2 + 0) * rpp * XC;
  float2* b_src = ab + (v * 2 + 1) * rpp * XC;
  const float2* g_src = g + v * rpp * 2 * Xh;
  const int neg0 = X - (XC - KP - 1);   // first kept negative-frequency column
  auto kept = [&](int i) { return i <= KP || i >= neg0; };
  auto ccol = [&](int i) { return i <= KP ? i : max(i - (X - XC), KP); };   // clamped compact column
  const int PS = pad_shift(X);   // row padding
  const int LS = row_stride(X);      // padded line pitch in LDS
  // lines 2r, 2r + 1: a (then u_A), b (then u_B) of row r; line 2 nr + r: Gamma of row r
  auto slot = [&](int e) {
    const int t = e / X;
    return t * LS + row_slot(e - t * X, PS);
  };
  // All loads of a thread first, then the selections and the Hermitian
  // extension, so the loads stay in flight together: the field lines (one
  // load per element), then the Gamma lines (the phase and absorption half
  // spectra, packed as Z_k = P_k + i A_k).  The workgroup has at least
  // 3 nr X / kEmax threads, so a thread owns at most 6 field and 3 Gamma
  // elements.
  {
    constexpr int EF = 6, EG = 3;
    const int nf = 2 * nr * X, ng = nr * X;
    float2 vf[EF];
    float4 vg[EG];
#pragma unroll
    for (int q = 0; q < EF; ++q) {
      const int e = tid + q * nthr;
      if (e < nf) {
        const int t = e / X, i = e - t * X;
        vf[q] = ((t & 1) ? b_src : a_src)[(row0 + (t >> 1)) * XC + ccol(i)];
      }
    }
#pragma unroll
    for (int q = 0; q < EG; ++q) {
      const int e = tid + q * nthr;
      if (e < ng) {
        const int r = e / X, i = e - r * X;
        int y = y0 + r, z = z0;
        while (y >= Y) { y -= Y; ++z; }
        const int kk = 2 * i > X ? X - i : i;
        const float2* gp = g_src + ((long)(z * 2 + 0) * Y + y) * Xh + kk;   // absorption: Y Xh on
        const float2 P = gp[0], A = gp[(long)Y * Xh];
        vg[q] = make_float4(P.x, P.y, A.x, A.y);
      }
    }
    wave0_sum(partials + v * tiles_x, tiles_x, &ibg_s);   // sum S P^2
#pragma unroll
    for (int q = 0; q < EF; ++q) {
      const int e = tid + q * nthr;
      if (e < nf) {
        const int t = e / X, i = e - t * X;
        buf[t * LS + row_slot(i, PS)] = kept(i) ? vf[q] : make_float2(0.f, 0.f);
      }
    }
#pragma unroll
    for (int q = 0; q < EG; ++q) {
      const int e = tid + q * nthr;
      if (e < ng) {
        const int r = e / X, i = e - r * X;
        const bool mirror = 2 * i > X;
        const int kk = mirror ? X - i : i;
        float2 P = make_float2(vg[q].x, vg[q].y), A = make_float2(vg[q].z, vg[q].w);
        if (kk == 0 || 2 * kk == X) { P.y = 0.f; A.y = 0.f; }   // Re of the inverse ignores them
        if (mirror) { P.y = -P.y; A.y = -A.y; }
        buf[(2 * nr + r) * LS + row_slot(i, PS)] = make_float2(P.x - A.y, P.y + A.x);
      }
    }
  }
  __syncthreads();
  const float k = (float)(1.0 / ((double)X * (double)Y * ibg_s));
  double dsum = 0.0;
  fft_lines<NS, 0, false, kEmax, true>(buf, LdsLines{3 * nr, 1, LS, false, -1, true}, plan, tw, 1.f,
                                       tid, nthr);
  for (int e = tid; e < nr * X; e += nthr) {
    const int r = e / X, i = e - r * X;
    const int si = row_slot(i, PS);
    const float2 G = buf[(2 * nr + r) * LS + si];   // (Gamma_phase, Gamma_abs)
    const float2 a = buf[2 * r * LS + si], b = buf[(2 * r + 1) * LS + si];
    const float2 gb = cmul(G, b);
    dsum += (double)gb.x * a.x + (double)gb.y * a.y;     // Re(G b conj(a))
    buf[2 * r * LS + si] = cscale(cconj(gb), k);          // u_A
    buf[(2 * r + 1) * LS + si] = cscale(cmulconj(G, a), k);  // u_B
  }
  const double tot = block_sum_d(dsum, red);
  if (tid == 0) dpart[v * wg_per_patch + wg] = tot;
  __syncthreads();
  auto store = [&](int t, int i, float2 val) {
    if (kept(i)) ((t & 1) ? b_src : a_src)[(row0 + (t >> 1)) * XC + ccol(i)] = val;
  };
  if constexpr (NS > 0) {
    // last pass straight to memory
    static_passes<NS, 0, false, kEmax, true, false, 0, StaticPlan<NS>::passes() - 1>(
        buf, 2 * nr, 1, LS, -1, tw, 1.f, tid, nthr);
    last_pass_out<NS, 0, false, kEmax, true, false>(buf, 2 * nr, 1, LS, -1, tw, 1.f, tid, nthr, store);
  } else {
    fft_lines<NS, 0, false, kEmax, true>(buf, LdsLines{2 * nr, 1, LS, false, -1, true}, plan, tw, 1.f,
                                         tid, nthr);
    scatter_from_lds_map(buf, nr * 2 * X, tid, nthr, slot, [&](int e, float2 val) {
      const int t = e / X;
      store(t, e - t * X, val);
    });
  }
}

// Rows per workgroup of the backward row kernel (three LDS lines per row):
// about 1024 elements per row group keeps several workgroups per CU.
int bwd_rows_per_wg(const Sampling& sm) {
  int R = 1024 / sm.nx;
  if (R < 1) R = 1;
  while (R > 1 && 3L * R * sm.nx > kMaxElems) --R;
  return R;
}

long bwd_wg_per_patch(const Sampling& sm) {
  const int R = bwd_rows_per_wg(sm);
  return ((long)sm.nz * sm.ny + R - 1) / R;
}

hipError_t launch_tf_rows_bwd(const double* partials, const Sampling& sm, int nv, float2* ab,
                              const float2* g, double* dpart, hipStream_t s, const LatSupport* sup) {
  if (3L * sm.nx > kMaxElems) return hipErrorInvalidValue;
  const LatSupport ls = sup ? *sup : full_support(sm);
  if (ls.xc < 1 || ls.xc > sm.nx || ls.kp < 0 || ls.kp >= ls.xc || ls.ly != sm.ny || ls.lx != sm.nx)
    return hipErrorInvalidValue;
  FftPlan plan;
  if (!make_plan(sm.nx, &plan)) return hipErrorInvalidValue;
  const int R = bwd_rows_per_wg(sm);
  const long wpp = bwd_wg_per_patch(sm);
  const long tiles_x = pupil_tiles(sm, ls);
  const int thr = threads_for(3L * R * sm.nx);
  const size_t lds = (size_t)(sm.nx + 3L * R * row_stride(sm.nx)) * sizeof(float2);
  ScopedTiming _t("k_tf_rows_bwd", s);
#define X_(NN)                                                                                   \
  case NN:                                                                                       \
    hipLaunchKernelGGL((k_tf_rows_bwd<NN>), dim3((unsigned)(wpp * nv)), dim3(thr), lds, s, partials, \
                       tiles_x, sm, ab, g, dpart, R, wpp, ls.xc, ls.kp, plan);                 \
    return hipGetLastError();
  switch (sm.nx) {
    WO_LATERAL_SIZES(X_)
    default:
      break;
  }
#undef X_
  hipLaunchKernelGGL((k_tf_rows_bwd<0>), dim3((unsigned)(wpp * nv)), dim3(thr), lds, s, partials,
                     tiles_x, sm, ab, g, dpart, R, wpp, ls.xc, ls.kp, plan);
  return hipGetLastError();
}

// ------------------------------------------------------------------ backward columns + contraction

// Inverse Y transform of u_A, u_B columns, then per lateral frequency the
// contraction 4 Re(U_B dB/dtheta + U_A dA/dtheta).  A workgroup owns one column
// tile and a chunk of ZC planes; the pupils and their derivatives, which do not
// depend on z, are evaluated once.  gpart[((v*nzc + chunk)*tiles + tile)*KG + j]
// with KG = TH (+ 7 aberration coefficients when AB), TH = 4 theta components
// (+ det_tilt, det_azimuth when DT); the first chunk also writes dI_bg/dtheta
// partials to ipart[(v*tiles + tile)*TH + j].
template <int NS, bool AB, bool DT>
__global__ __launch_bounds__(1024) void k_tf_grad_y(const DevOptics* __restrict__ opt, Sampling sm,
                                                    const float2* __restrict__ ab,
                                                    double* __restrict__ gpart,
                                                    double* __restrict__ ipart, int W,
                                                    long tiles_x, int ZC, int XC, int KP,
                                                    FftPlan plan) {
  extern __shared__ float2 smem[];
  __shared__ double red[kMaxThreads / 64];
  constexpr int EPT = 2;   // lateral frequencies of a thread: Y * W <= 2 * threads
  const int Y = sm.ny, X = sm.nx, Z = sm.nz;
  float2* tw = smem;
  float2* buf = smem + Y;
  const int tid = threadIdx.x, nthr = blockDim.x;
  fill_twiddles(tw, Y, tid, nthr);
  const long bid = xcd_block();
  const long tile = bid % tiles_x;
  const long rest = bid / tiles_x;
  const int nzc = (Z + ZC - 1) / ZC;
  const int zc = (int)(rest % nzc);
  const long v = rest / nzc;
  const DevOptics o = opt[v];
  const int x0 = (int)(tile * W);
  const int wsh = pow2_shift(W);     // W is a power of two
  // per element: phase rate 2 kz (FP64, the phase needs it) and the pupil
  // products of the contraction (FP32)
  constexpr int TH = DT ? kThetaAll : 4;
  double tkz[EPT];
  float SP[EPT], gkP[EPT], SdP[EPT], gkdP[EPT], dSzP[EPT], dSaP[EPT];
  // with DT: the detection pupil's derivatives along the tilt and azimuth of its
  // axis, in the same products as dP/dNA
  float SdPt[DT ? EPT : 1], gkdPt[DT ? EPT : 1], SdPa[DT ? EPT : 1], gkdPa[DT ? EPT : 1];
  // aberration-aware (AB): the aberration phase 2 W in units of pi, and
  // Q = sum_z (S P Im(U_A e) + gk P Re(U_B e)), which every derivative of the
  // aberration phase multiplies (d/dc_j: -2 pi Z_j; the NA term: -2 pi dW/dNA)
  float ab2[AB ? EPT : 1];
  double Qe[AB ? EPT : 1];
  {
    const double hw = soft_halfwidth(o, sm);
    const double km = o.n_medium / o.wavelength;
    const double ri = o.na_ill / o.wavelength;
    const DetAxis dax = det_axis(o);
    double cy, cx;
    source_centre(o, &cy, &cx);
    const double rq0 = o.n_medium * sin(o.tilt_zenith) / o.wavelength;
    const double drq0 = o.n_medium * cos(o.tilt_zenith) / o.wavelength;
    const double sa = sin(o.tilt_azimuth), ca = cos(o.tilt_azimuth);
    double di[kThetaAll] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      tkz[i] = 0.0;
      SP[i] = gkP[i] = SdP[i] = gkdP[i] = dSzP[i] = dSaP[i] = 0.f;
      if constexpr (DT) SdPt[i] = gkdPt[i] = SdPa[i] = gkdPa[i] = 0.f;
      if constexpr (AB) {
        ab2[i] = 0.f;
        Qe[i] = 0.0;
      }
      const int e = tid + i * nthr;
      if (e >= Y * W) continue;
      const int ky = e >> wsh, w = e & (W - 1);
      const int c = x0 + w;   // compact column of the fields
      if (c >= XC) continue;
      const int kx = field_column(c, KP, X, XC);
      const double fy = fftfreq(ky, Y, sm.dy), fx = fftfreq(kx, X, sm.dx);
      const double rp = sqrt(fy * fy + fx * fx);
      const double P = det_pupil(o, dax, fy, fx, hw);
      double dP, dPt, dPa;                                           // dP / d(NA_det, tilt, azimuth)
      det_pupil_derivs(o, dax, fy, fx, hw, &dP, &dPt, &dPa);
      const double qy = fy - cy, qx = fx - cx;
      const double rq = sqrt(qy * qy + qx * qx);
      const double S = disc(qy, qx, ri, hw);
      const double sl = edge_slope(ri - rq, hw);
      const double uy = rq > 0.0 ? qy / rq : 0.0, ux = rq > 0.0 ? qx / rq : 0.0;
      const double dSy = sl * uy, dSx = sl * ux;                     // dS / d(cy, cx)
      const double dSz = dSy * drq0 * sa + dSx * drq0 * ca;          // dS / d zenith
      const double dSa = dSy * rq0 * ca - dSx * rq0 * sa;            // dS / d azimuth
      di[1] += 2.0 * S * P * dP;
      di[2] += dSz * P * P;
      di[3] += dSa * P * P;
      if constexpr (DT) {
        di[4] += 2.0 * S * P * dPt;
        di[5] += 2.0 * S * P * dPa;
      }
      if (P == 0.0 && dP == 0.0 && (!DT || (dPt == 0.0 && dPa == 0.0))) continue;
      const double kz = sqrt(fmax(km * km - rp * rp, 0.0));
      const double gk = kz > 0.0 ? km / kz : 0.0;
      tkz[i] = 2.0 * kz;
      if constexpr (AB) ab2[i] = (float)(2.0 * aberration_waves(o, fy, fx));
      // A = S P e, B = P (i km / kz) e with e = e^{i 2 pi kz (z - dz0)}
      SP[i] = (float)(S * P);
      gkP[i] = (float)(gk * P);
      SdP[i] = (float)(S * dP);
      gkdP[i] = (float)(gk * dP);
      dSzP[i] = (float)(dSz * P);
      dSaP[i] = (float)(dSa * P);
      if constexpr (DT) {
        SdPt[i] = (float)(S * dPt);
        gkdPt[i] = (float)(gk * dPt);
        SdPa[i] = (float)(S * dPa);
        gkdPa[i] = (float)(gk * dPa);
      }
    }
    if (zc == 0) {
#pragma unroll
      for (int j = 0; j < TH; ++j) {
        const double t = block_sum_d(di[j], red);
        if (tid == 0) ipart[(v * tiles_x + tile) * TH + j] = t;
      }
    }
  }
  double g[kThetaAll] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int zend = min(Z, (zc + 1) * ZC);
  // the tile of plane z: element e = (ky, field, w) from ab; plane z + 1 is loaded
  // into registers while plane z is transformed and contracted
  const int ntile = Y * 2 * W;
  auto load_plane = [&](int z, float2* t) {
#pragma unroll
    for (int i = 0; i < 2 * EPT; ++i) {
      const int e = tid + i * nthr;
      if (e < ntile) {
        const int ky = e >> (wsh + 1);
        const int r = e & (2 * W - 1);
        const int f = r >> wsh, w = r & (W - 1);
        const int c = x0 + w;
        t[i] = c < XC ? ab[(((v * 2 + f) * Z + z) * (long)Y + ky) * XC + c] : make_float2(0.f, 0.f);
      }
    }
  };
  float2 nxt[2 * EPT];
  if (zc * ZC < zend) load_plane(zc * ZC, nxt);
  for (int z = zc * ZC; z < zend; ++z) {
#pragma unroll
    for (int i = 0; i < 2 * EPT; ++i) {
      const int e = tid + i * nthr;
      if (e < ntile) buf[e] = nxt[i];
    }
    __syncthreads();
    if (z + 1 < zend) load_plane(z + 1, nxt);
    fft_lines<NS, 0, true, 2 * EPT>(buf, LdsLines{2 * W, 2 * W, 1, true, pow2_shift(2 * W)}, plan, tw,
                                    1.f, tid, nthr);
    const double dzr = plane_z(z, sm) - o.defocus;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * nthr;
      if (e >= Y * W || (tkz[i] == 0.0 && SP[i] == 0.f && SdP[i] == 0.f && gkdP[i] == 0.f &&
                         dSzP[i] == 0.f && dSaP[i] == 0.f &&
                         (!DT || (SdPt[i] == 0.f && gkdPt[i] == 0.f && SdPa[i] == 0.f && gkdPa[i] == 0.f))))
        continue;
      const int ky = e >> wsh, w = e & (W - 1);
      double arg = tkz[i] * dzr;
      if constexpr (AB) arg += (double)ab2[i];
      const float red_arg = (float)(arg - 2.0 * rint(0.5 * arg));
      float snf, csf;
      sincospif(red_arg, &snf, &csf);
      const float2 UA = buf[ky * 2 * W + w];
      const float2 UB = buf[ky * 2 * W + W + w];
      // per-term products in FP32 (their inputs are FP32), sums in FP64
      const float ua_re = UA.x * csf - UA.y * snf, ua_im = UA.x * snf + UA.y * csf;   // U_A e^{i phi}
      const float ub_re = UB.x * csf - UB.y * snf, ub_im = UB.x * snf + UB.y * csf;   // U_B e^{i phi}
      const float tpk = (float)(M_PI * tkz[i]);                                       // 2 pi kz
      // d/d defocus multiplies A and B by -i 2 pi kz:
      //   Re(U_A A (-i tpk)) = tpk S P Im(U_A e); Re(U_B B (-i tpk)) = tpk gk P Re(U_B e)
      const float qv = SP[i] * ua_im + gkP[i] * ub_re;
      g[0] += (double)(tpk * qv);
      if constexpr (AB) Qe[i] += (double)qv;
      // d/dNA: A' = S dP e, B' = dP i gk e -> Re(U_B e i gk dP) = -gk dP Im(U_B e)
      g[1] += (double)(SdP[i] * ua_re - gkdP[i] * ub_im);
      g[2] += (double)(dSzP[i] * ua_re);
      g[3] += (double)(dSaP[i] * ua_re);
      if constexpr (DT) {
        // the detection axis moves P as NA does: S dP e in A, i gk dP e in B
        g[4] += (double)(SdPt[i] * ua_re - gkdPt[i] * ub_im);
        g[5] += (double)(SdPa[i] * ua_re - gkdPa[i] * ub_im);
      }
    }
    __syncthreads();
  }
  constexpr int KG = TH + (AB ? 7 : 0);
  double ga[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if constexpr (AB) {
    const double tp = 2.0 * M_PI;
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * nthr;
      if (e >= Y * W || Qe[i] == 0.0) continue;
      const int ky = e >> wsh, kx = field_column(x0 + (e & (W - 1)), KP, X, XC);
      double zj[7], dwdna;
      zernike_terms(o, fftfreq(ky, Y, sm.dy), fftfreq(kx, X, sm.dx), zj, &dwdna);
      g[1] -= tp * dwdna * Qe[i];
#pragma unroll
      for (int j = 0; j < 7; ++j) ga[j] -= tp * zj[j] * Qe[i];
    }
  }
#pragma unroll
  for (int j = 0; j < KG; ++j) {
    const double t = block_sum_d(4.0 * (j < TH ? g[j] : ga[j - TH]), red);
    if (tid == 0) gpart[((v * nzc + zc) * tiles_x + tile) * KG + j] = t;
  }
}

// Column tile of the gradient kernel: two lateral frequencies per thread (and
// four LDS elements), so that each thread keeps the z-independent factors of
// its frequencies in registers; at most 1024 threads (Y W <= 2048).
static int grad_tile_width(const Sampling& sm) {
  int W = 16;
  while (W > 1 && (long)W * sm.ny > 2048) W /= 2;
  return W;
}

static int grad_threads(const Sampling& sm) {
  long t = ((long)grad_tile_width(sm) * sm.ny + 1) / 2;
  t = (t + 63) / 64 * 64;
  return (int)(t < 64 ? 64 : t);
}

long grad_tiles(const Sampling& sm, const LatSupport* sup) {
  const int W = grad_tile_width(sm);
  return ((sup ? sup->xc : sm.nx) + W - 1) / W;
}

long pupil_tiles(const Sampling& sm, const LatSupport& ls) {
  const int W = tf_tile_width(sm, ls.ly);
  return (ls.xc + W - 1) / W;
}

// z chunk of the gradient kernel (the reduction reads ceil(nz / chunk) * tiles
// partials per patch).
int grad_z_chunk(const Sampling& sm, int nv) {
  // the pupil derivatives cost more than the planes' work: favour longer chunks
  return tf_z_chunk(sm, grad_tiles(sm), nv, 512);
}

hipError_t launch_tf_grad_y(const DevOptics* opt, const Sampling& sm, int nv, const float2* ab,
                            double* gpart, double* ipart, hipStream_t s, const LatSupport* sup) {
  FftPlan plan;
  if (!make_plan(sm.ny, &plan)) return hipErrorInvalidValue;
  if (sm.ny > 2048) return hipErrorInvalidValue;
  const LatSupport ls = sup ? *sup : full_support(sm);
  if (ls.xc < 1 || ls.xc > sm.nx || ls.kp < 0 || ls.kp >= ls.xc) return hipErrorInvalidValue;
  const int W = grad_tile_width(sm);
  const long tiles = grad_tiles(sm, &ls);
  const int ZC = grad_z_chunk(sm, nv);
  const long nwg = tiles * ((sm.nz + ZC - 1) / ZC) * (long)nv;
  const int thr = grad_threads(sm);
  const size_t lds = (size_t)(sm.ny + sm.ny * 2 * W) * sizeof(float2);
  ScopedTiming _t("k_tf_grad_y", s);
#define WO_GRAD(NN, AA)                                                                          \
  do {                                                                                           \
    if (sm.det_grad)                                                                             \
      hipLaunchKernelGGL((k_tf_grad_y<NN, AA, true>), dim3((unsigned)nwg), dim3(thr), lds, s, opt, sm, ab, \
                         gpart, ipart, W, tiles, ZC, ls.xc, ls.kp, plan);                        \
    else                                                                                         \
      hipLaunchKernelGGL((k_tf_grad_y<NN, AA, false>), dim3((unsigned)nwg), dim3(thr), lds, s, opt, sm, ab, \
                         gpart, ipart, W, tiles, ZC, ls.xc, ls.kp, plan);                        \
  } while (0)
#define X_(NN)                                                                                   \
  case NN:                                                                                       \
    if (sm.aberrated) WO_GRAD(NN, true); else WO_GRAD(NN, false);                                \
    return hipGetLastError();
  switch (sm.ny) {
    WO_LATERAL_SIZES(X_)
    default:
      break;
  }
#undef X_
  if (sm.aberrated) WO_GRAD(0, true); else WO_GRAD(0, false);
#undef WO_GRAD
  return hipGetLastError();
}

// ------------------------------------------------------------------ reduction + Adam

// One workgroup per virtual patch: total loss and gradient from the partials,
// then (if update) one Adam step with bias correction, mask and box.
__global__ __launch_bounds__(256) void k_adam(DevOptics* __restrict__ opt,
                                              TuneState* __restrict__ st, Sampling sm,
                                              const double* __restrict__ ppart, long tiles_x,
                                              long gtiles,
                                              const double* __restrict__ lpart, long lbpp,
                                              const double* __restrict__ dpart, long dwpp,
                                              const double* __restrict__ gpart, long gn,
                                              const double* __restrict__ ipart, int update) {
  __shared__ double red[4];
  const long v = blockIdx.x;
  const int tid = threadIdx.x;
  double acc;
  acc = 0.0;
  for (long i = tid; i < lbpp; i += blockDim.x) acc += lpart[v * lbpp + i];
  const double lsum = block_sum_d(acc, red);
  acc = 0.0;
  for (long i = tid; i < dwpp; i += blockDim.x) acc += dpart[v * dwpp + i];
  const double dsum = block_sum_d(acc, red);
  acc = 0.0;
  for (long i = tid; i < tiles_x; i += blockDim.x) acc += ppart[v * tiles_x + i];
  const double ibg = block_sum_d(acc, red);
  const int TH = sm.det_grad ? kThetaAll : 4;
  const int KG = TH + (sm.aberrated ? 7 : 0);
  double gj[kGradAll], dij[kThetaAll];
  for (int j = 0; j < KG; ++j) {
    acc = 0.0;
    for (long i = tid; i < gn; i += blockDim.x) acc += gpart[(v * gn + i) * KG + j];
    gj[j] = block_sum_d(acc, red);
  }
  for (int j = 0; j < TH; ++j) {
    acc = 0.0;
    for (long i = tid; i < gtiles; i += blockDim.x) acc += ipart[(v * gtiles + i) * TH + j];
    dij[j] = block_sum_d(acc, red);
  }
  if (tid != 0) return;
  TuneState s = st[v];
  const double N = (double)sm.ny * sm.nx;
  const double loss = -lsum / s.band_count;
  double grad[kThetaAll] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int j = 0; j < TH; ++j) grad[j] = gj[j] - 4.0 * dsum / (N * ibg * ibg) * dij[j];
  s.loss = loss;
  for (int j = 0; j < kThetaAll; ++j) s.grad[j] = grad[j];
  // I_bg = sum S |P|^2 does not depend on the aberration
  for (int j = 0; j < 7; ++j) s.gab[j] = KG > TH ? gj[TH + j] : 0.0;
  if (update) {
    DevOptics o = opt[v];
    double th[4] = {o.defocus, o.na_det, o.tilt_zenith, o.tilt_azimuth};
    s.t += 1;
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    const double c1 = 1.0 - pow(b1, (double)s.t), c2 = 1.0 - pow(b2, (double)s.t);
    for (int j = 0; j < 4; ++j) {
      const double gm = ((s.mask >> j) & 1) ? grad[j] : 0.0;
      s.m[j] = b1 * s.m[j] + (1.0 - b1) * gm;
      s.v[j] = b2 * s.v[j] + (1.0 - b2) * gm * gm;
      const double mh = s.m[j] / c1, vh = s.v[j] / c2;
      double t = th[j] - s.lr[j] * mh / (sqrt(vh) + eps);
      t = t < s.lo[j] ? s.lo[j] : (t > s.hi[j] ? s.hi[j] : t);
      th[j] = t;
    }
    opt[v].defocus = th[0];
    opt[v].na_det = th[1];
    opt[v].tilt_zenith = th[2];
    opt[v].tilt_azimuth = th[3];
    for (int j = 0; j < 7; ++j) {
      if (!((s.mask >> (4 + j)) & 1)) continue;
      const double gm = s.gab[j];
      s.mab[j] = b1 * s.mab[j] + (1.0 - b1) * gm;
      s.vab[j] = b2 * s.vab[j] + (1.0 - b2) * gm * gm;
      const double mh = s.mab[j] / c1, vh = s.vab[j] / c2;
      double t = (double)o.zern[j] - s.lr_ab * mh / (sqrt(vh) + eps);
      t = t < -s.bound_ab ? -s.bound_ab : (t > s.bound_ab ? s.bound_ab : t);
      opt[v].zern[j] = (float)t;
    }
  }
  st[v] = s;
}

hipError_t launch_adam(DevOptics* opt, TuneState* st, const Sampling& sm, int nv,
                       const double* ppart, const double* lpart, const double* dpart,
                       const double* gpart, const double* ipart, int update, hipStream_t s,
                       const LatSupport* sup) {
  const LatSupport ls = sup ? *sup : full_support(sm);
  const long tiles_x = pupil_tiles(sm, ls);
  { ScopedTiming _t("k_adam", s);
  const int ZC = grad_z_chunk(sm, nv);
  const long gt = grad_tiles(sm, &ls);
  const long gn = (long)((sm.nz + ZC - 1) / ZC) * gt;
  hipLaunchKernelGGL(k_adam, dim3(nv), dim3(256), 0, s, opt, st, sm, ppart, tiles_x, gt, lpart,
                     loss_blocks(sm), dpart, bwd_wg_per_patch(sm), gpart, gn, ipart, update); }
  return hipGetLastError();
}

// ------------------------------------------------------------------ best start

// One thread per patch; ties keep the earliest start, and a start whose loss
// is not finite is taken only when no start's is.
__global__ __launch_bounds__(64) void k_pick_best(const DevOptics* __restrict__ opt,
                                                  const TuneState* __restrict__ st, int starts,
                                                  int npatch, DevOptics* __restrict__ ropt,
                                                  float* __restrict__ eta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npatch) return;
  const long v0 = (long)i * starts;
  long best = v0;
  for (int s = 1; s < starts; ++s) {
    const double lb = st[best].loss, ls = st[v0 + s].loss;
    if (ls < lb || (!isfinite(lb) && isfinite(ls))) best = v0 + s;
  }
  ropt[i] = opt[best];
  eta[i] = (float)st[v0].eta;
}

hipError_t launch_pick_best(const DevOptics* opt, const TuneState* st, int starts, int npatch,
                            DevOptics* ropt, float* eta, hipStream_t s) {
  { ScopedTiming _t("k_pick_best", s);
  hipLaunchKernelGGL(k_pick_best, dim3((unsigned)((npatch + 63) / 64)), dim3(64), 0, s, opt, st, starts,
                     npatch, ropt, eta); }
  return hipGetLastError();
}

}  // namespace wo
