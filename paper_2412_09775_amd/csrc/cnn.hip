// Parameter-regression CNN on BF16 MFMA (gfx950): the learned initialiser of
// the auto-tune.  4 blocks of [3x3x3 convolution, stride 2, padding 1, bias,
// GELU] (channels 1 -> 32 -> 64 -> 128 -> 256), global average pooling and a
// linear head to 3 normalised parameters; MSE loss; AdamW.
//
// Every convolution (forward, input gradient, weight gradient) is one
// implicit GEMM on v_mfma_f32_16x16x32_bf16 with FP32 accumulation:
//   forward  C[pos_out][co]  = sum_{tap,ci} x(im2col)        * w[co][tap][ci]
//   dgrad    C[pos_in][ci]   = sum_{tap,co} gz(col2im)       * w[co][tap][ci]
//   wgrad    C[co][tap,ci]   = sum_{pos_out} gz[pos_out][co] * x(im2col)
// Operands are gathered on the fly into LDS tiles (no im2col buffer).
// Activations are channels-last BF16, pre-activations FP32.
// Lane layout of the 16x16x32 MFMA (checked on the device): lane l holds
// A[l%16][(l/16)*8 + i] and B[(l/16)*8 + i][l%16], i < 8; accumulator
// register r of lane l is C[(l/16)*4 + r][l%16].
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/waveorder.h"
#include "internal.hpp"

namespace wo {

typedef unsigned short u16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ u16 f2bf(float f) {  // round to nearest even
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (u16)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (u16)(u >> 16);
}
__device__ __forceinline__ float bf2f(u16 b) { return __uint_as_float(((unsigned)b) << 16); }

// ------------------------------------------------------------------ operand gathers
//
// A gather exposes row(i) -> a per-row context computed once per kernel (the
// thread's row of the tile never changes), then at(ctx, k) for the K index.
// K indices walk (tap, channel) with the channel fastest.

struct ConvGeom {
  int D, H, W, C;     // input volume and channels
  int Do, Ho, Wo;     // output volume
};

struct TapCh {  // (tap, channel) of a K index, advanced incrementally
  int tap, ch;
};

// A(m, k) of the forward GEMM: m = output position, k = tap * Cin + ci.
struct GatherIm2col {
  const u16* x;
  ConvGeom g;
  // positions (batch included) stay below 2^31 (checked on the host): 32-bit
  // index arithmetic, one widening multiply per address
  struct Row { int n, d0, h0, w0; };
  __device__ __forceinline__ Row row(long m) const {
    Row r;
    unsigned q = (unsigned)m;
    const unsigned wo = (unsigned)g.Wo, ho = (unsigned)g.Ho, dd = (unsigned)g.Do;
    unsigned q1 = q / wo;
    const int ow = (int)(q - q1 * wo);
    unsigned q2 = q1 / ho;
    const int oh = (int)(q1 - q2 * ho);
    const unsigned q3 = q2 / dd;
    const int od = (int)(q2 - q3 * dd);
    r.n = (int)q3;
    r.d0 = 2 * od - 1; r.h0 = 2 * oh - 1; r.w0 = 2 * ow - 1;
    return r;
  }
  __device__ __forceinline__ int chans() const { return g.C; }
  __device__ __forceinline__ const u16* ptr(const Row& r, TapCh t) const {
    const int kw = t.tap % 3, kh = (t.tap / 3) % 3, kd = t.tap / 9;
    const int id = r.d0 + kd, ih = r.h0 + kh, iw = r.w0 + kw;
    if (id < 0 || id >= g.D || ih < 0 || ih >= g.H || iw < 0 || iw >= g.W) return nullptr;
    const unsigned pos = (((unsigned)r.n * g.D + id) * g.H + ih) * g.W + iw;
    return x + (long)((unsigned long)pos * (unsigned)g.C) + t.ch;
  }
  __device__ __forceinline__ u16 at(const Row& r, TapCh t) const {
    const u16* p = ptr(r, t);
    return p ? *p : (u16)0;
  }
  // the next output position's row (positions in order: w fastest, then h, d, n)
  __device__ __forceinline__ Row next(Row r) const {
    r.w0 += 2;
    if (r.w0 == 2 * g.Wo - 1) {
      r.w0 = -1;
      r.h0 += 2;
      if (r.h0 == 2 * g.Ho - 1) {
        r.h0 = -1;
        r.d0 += 2;
        if (r.d0 == 2 * g.Do - 1) { r.d0 = -1; ++r.n; }
      }
    }
    return r;
  }
  // 8 consecutive k (channels t.ch .. t.ch + 7 of one tap), when g.C % 8 == 0
  static constexpr int kMode = 1;
  static constexpr bool kPositions = false;
  __host__ __device__ __forceinline__ bool vec() const { return g.C % 8 == 0; }
  __device__ __forceinline__ uint4 load8(const Row& r, TapCh t) const {
    const u16* p = ptr(r, t);
    return p ? *(const uint4*)p : make_uint4(0, 0, 0, 0);
  }
};

// B(k, n) = w[n * K + k] (weights stored [Cout][tap][Cin]).
struct GatherRows {
  const u16* w;
  long K;
  int C;  // channels per tap along k
  struct Row { const u16* p; };
  __device__ __forceinline__ Row row(long n) const { return Row{w + n * K}; }
  __device__ __forceinline__ int chans() const { return C; }
  __device__ __forceinline__ u16 at(const Row& r, TapCh t) const { return r.p[(long)t.tap * C + t.ch]; }
  static constexpr int kMode = 1;
  static constexpr bool kPositions = false;
  __host__ __device__ __forceinline__ bool vec() const { return C % 8 == 0; }
  __device__ __forceinline__ uint4 load8(const Row& r, TapCh t) const {
    return *(const uint4*)(r.p + (long)t.tap * C + t.ch);
  }
};

// A(m, k) of the input-gradient GEMM restricted to one parity class of input
// positions (pd, ph, pw): m enumerates the class, k = j * Cout + co runs over
// the taps that reach an output position from this class (kd = 1 for even d,
// kd in {0, 2} for odd d, per axis).
struct GatherCol2imClass {
  const u16* gz;
  ConvGeom g;     // g.C = Cout
  int pd, ph, pw; // parity of the class
  int cd, ch, cw; // class extents: positions with that parity
  int nd, nh, nw; // valid taps per axis (1 or 2)
  struct Row { int n, d, h, w; };   // 32-bit, as in GatherIm2col
  __device__ __forceinline__ Row row(long m) const {
    Row r;
    const unsigned q = (unsigned)m;
    const unsigned q1 = q / (unsigned)cw;
    const int iw = (int)(q - q1 * (unsigned)cw);
    const unsigned q2 = q1 / (unsigned)ch;
    const int ih = (int)(q1 - q2 * (unsigned)ch);
    const unsigned q3 = q2 / (unsigned)cd;
    const int id = (int)(q2 - q3 * (unsigned)cd);
    r.n = (int)q3;
    r.d = 2 * id + pd; r.h = 2 * ih + ph; r.w = 2 * iw + pw;
    return r;
  }
  __device__ __forceinline__ int chans() const { return g.C; }
  __device__ __forceinline__ const u16* ptr(const Row& r, TapCh t) const {
    const int jw = t.tap % nw, jh = (t.tap / nw) % nh, jd = t.tap / (nw * nh);
    const int kd = nd == 1 ? 1 : 2 * jd, kh = nh == 1 ? 1 : 2 * jh, kw = nw == 1 ? 1 : 2 * jw;
    const int od2 = r.d + 1 - kd, oh2 = r.h + 1 - kh, ow2 = r.w + 1 - kw;
    if (od2 < 0 || oh2 < 0 || ow2 < 0) return nullptr;
    const int od = od2 >> 1, oh = oh2 >> 1, ow = ow2 >> 1;
    if (od >= g.Do || oh >= g.Ho || ow >= g.Wo) return nullptr;
    const unsigned pos = (((unsigned)r.n * g.Do + od) * g.Ho + oh) * g.Wo + ow;
    return gz + (long)((unsigned long)pos * (unsigned)g.C) + t.ch;
  }
  __device__ __forceinline__ u16 at(const Row& r, TapCh t) const {
    const u16* p = ptr(r, t);
    return p ? *p : (u16)0;
  }
  static constexpr int kMode = 1;
  static constexpr bool kPositions = false;
  __host__ __device__ __forceinline__ bool vec() const { return g.C % 8 == 0; }
  __device__ __forceinline__ uint4 load8(const Row& r, TapCh t) const {
    const u16* p = ptr(r, t);
    return p ? *(const uint4*)p : make_uint4(0, 0, 0, 0);
  }
  // the global input position of class row m (output row mapping)
  __device__ __forceinline__ long out_row(long m) const {
    const Row r = row(m);
    return (long)((((unsigned)r.n * g.D + r.d) * g.H + r.h) * g.W + r.w);
  }
};

// B(k, n) of the class input-gradient GEMM: w[co][tap(j)][ci], k = j * Cout + co, n = ci.
struct GatherWTClass {
  const u16* w;
  int Cin, Cout;
  int nd, nh, nw;
  struct Row { int ci; };
  __device__ __forceinline__ Row row(long n) const { return Row{(int)n}; }
  __device__ __forceinline__ int chans() const { return Cout; }
  __device__ __forceinline__ long off(TapCh t) const {
    const int jw = t.tap % nw, jh = (t.tap / nw) % nh, jd = t.tap / (nw * nh);
    const int kd = nd == 1 ? 1 : 2 * jd, kh = nh == 1 ? 1 : 2 * jh, kw = nw == 1 ? 1 : 2 * jw;
    const int tap = (kd * 3 + kh) * 3 + kw;
    return (long)((t.ch * 27 + tap) * Cin);
  }
  __device__ __forceinline__ u16 at(const Row& r, TapCh t) const { return w[off(t) + r.ci]; }
  // 8 consecutive rows (ci .. ci + 7) at one k, when Cin % 8 == 0
  static constexpr int kMode = 2;
  static constexpr bool kPositions = false;
  __host__ __device__ __forceinline__ bool vec() const { return Cin % 8 == 0; }
  __device__ __forceinline__ uint4 load_rows8(long n0, TapCh t) const {
    return *(const uint4*)(w + off(t) + n0);
  }
};

// A(m, k) of the weight-gradient GEMM: gz[k][m] (k = output position, m = co).
// K here is a position index (chans() = 1, tap = position).
struct GatherT {
  const u16* gz;
  int Cout;
  struct Row { int co; };
  __device__ __forceinline__ Row row(long m) const { return Row{(int)m}; }
  __device__ __forceinline__ int chans() const { return 1; }
  __device__ __forceinline__ long off(TapCh t) const { return (long)((unsigned long)(unsigned)t.tap * (unsigned)Cout); }
  __device__ __forceinline__ u16 at(const Row& r, TapCh t) const { return gz[off(t) + r.co]; }
  static constexpr int kMode = 2;
  static constexpr bool kPositions = false;
  __host__ __device__ __forceinline__ bool vec() const { return Cout % 8 == 0; }
  __device__ __forceinline__ uint4 load_rows8(long m0, TapCh t) const {
    return *(const uint4*)(gz + off(t) + m0);
  }
};

// B(k, n) of the weight-gradient GEMM: im2col(x)(position k, n = tap * Cin + ci).
struct GatherIm2colT {
  GatherIm2col a;
  struct Row { int tap, ci; };
  __device__ __forceinline__ Row row(long n) const { return Row{(int)(n / a.g.C), (int)(n % a.g.C)}; }
  __device__ __forceinline__ int chans() const { return 1; }
  __device__ __forceinline__ u16 at(const Row& r, TapCh t) const {
    return a.at(a.row(t.tap), TapCh{r.tap, r.ci});
  }
  // rows n0 .. n0 + 7 (channels of one tap) at position k, when Cin % 8 == 0
  static constexpr int kMode = 2;
  // K indices are output positions: eight consecutive ones from one decode,
  // stepping to the next position (no division per element)
  static constexpr bool kPositions = true;
  __device__ __forceinline__ uint4 at_run(const Row& r, long k, long kend, bool ok) const {
    uint4 v = make_uint4(0, 0, 0, 0);
    u16* pv = (u16*)&v;
    GatherIm2col::Row p = a.row(ok ? k : 0);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      pv[e] = (ok && k + e < kend) ? a.at(p, TapCh{r.tap, r.ci}) : (u16)0;
      p = a.next(p);
    }
    return v;
  }
  __host__ __device__ __forceinline__ bool vec() const { return a.g.C % 8 == 0; }
  __device__ __forceinline__ uint4 load_rows8(long n0, TapCh t) const {
    const Row r = row(n0);
    return a.load8(a.row(t.tap), TapCh{r.tap, r.ci});
  }
};

struct IdentityRows {
  __device__ __forceinline__ long operator()(long m) const { return m; }
};
struct ClassRows {
  GatherCol2imClass c;
  __device__ __forceinline__ long operator()(long m) const { return c.out_row(m); }
};

// ------------------------------------------------------------------ GEMM

constexpr int kBM = 64, kBN = 64, kBK = 32, kLdsPad = 8;   // kBM x kBN: the default tile

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// Where a tile's FP32 results go.  StoreC: C_z[orow][n] (z the split-K chunk,
// Mout rows per chunk).  StoreBiasGelu (forward convolutions): the
// pre-activation z = v + b[n] in FP32 and a = BF16(GELU(z)), the same
// arithmetic as a separate bias-GELU pass over C.
struct StoreC {
  float* C;
  long Mout, N;
  __device__ __forceinline__ void operator()(int zi, long orow, long col, float v) const {
    C[((long)zi * Mout + orow) * N + col] = v;
  }
};
struct StoreBiasGelu {
  float* z;
  u16* a;
  const float* b;
  long N;
  __device__ __forceinline__ void operator()(int, long orow, long col, float v) const {
    const float t = v + b[col];
    const long i = orow * N + col;
    z[i] = t;
    a[i] = f2bf(gelu_f(t));
  }
};

// (tap, channel) of K index k with `ch` channels per tap; K indices stay
// below 2^31 (checked on the host), so 32-bit arithmetic.
__device__ __forceinline__ TapCh tapch(long k, int ch) {
  const unsigned u = (unsigned)k, c = (unsigned)ch;
  const unsigned q = u / c;
  return TapCh{(int)q, (int)(u - q * c)};
}
// the same advanced by kBK (q = kBK / ch, r = kBK % ch)
__device__ __forceinline__ void tapch_step(TapCh& t, int ch, int q, int r) {
  t.tap += q;
  t.ch += r;
  if (t.ch >= ch) { t.ch -= ch; ++t.tap; }
}

// C[rowmap(m)][n] = sum_{k in [kbeg, kend)} A(m, k) B(k, n) for the TM x TN
// tile at (m0, n0): 64 x 64, or 128 x 32 for narrow N (no MFMA on padding);
// each of the 4 waves computes a 32 x 32 block as 2 x 2 MFMA tiles.  Operand
// tiles are staged in LDS as [row][k], each operand in slots of 64 rows per
// thread.  Load modes per operand: 0 one element at a time; 1 eight
// consecutive k of a row in one 16-byte load; 2 eight consecutive rows at one
// k in one 16-byte load (the operand is contiguous along its rows).  Each
// thread's next K-tile is loaded into registers before the current tile's
// MFMAs, so the global loads are in flight while the matrix cores run.
template <class G, int MODE, int ROWS>
struct Stage {
  static constexpr int S = ROWS >= 64 ? ROWS / 64 : 1;   // 64-row slots per thread
  typename G::Row r[S];
  bool ok[S], ok8[S];
  long row8[S];
  uint4 v[S];
  int lr, lk, kk, lr8, ch;
  __device__ __forceinline__ bool mine(int i) const {   // this thread stages slot i
    return (MODE == 2 ? lr8 : lr) + 64 * i < ROWS;
  }
  __device__ __forceinline__ void init(const G& g, long r0, long R, int t) {
    lr = t >> 2; lk = (t & 3) * 8; kk = t & 31; lr8 = (t >> 5) * 8;
    ch = g.chans();
#pragma unroll
    for (int i = 0; i < S; ++i) {
      const long rr = r0 + lr + 64 * i;
      ok[i] = mine(i) && rr < R;
      row8[i] = r0 + lr8 + 64 * i;
      ok8[i] = mine(i) && row8[i] < R;
      r[i] = g.row(ok[i] ? rr : 0);
    }
  }
  __device__ __forceinline__ int koff() const { return MODE == 2 ? kk : lk; }
  __device__ __forceinline__ void fetch(const G& g, long k, long kend, TapCh tc) {
#pragma unroll
    for (int i = 0; i < S; ++i) {
      uint4 x = make_uint4(0, 0, 0, 0);
      if constexpr (MODE == 2) {
        if (ok8[i] && k < kend) x = g.load_rows8(row8[i], tc);
      } else if constexpr (MODE == 1) {
        if (ok[i] && k < kend) x = g.load8(r[i], tc);
      } else if constexpr (G::kPositions) {
        x = g.at_run(r[i], k, kend, ok[i]);
      } else {
        u16* pv = (u16*)&x;
        TapCh c = tc;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          pv[e] = (ok[i] && k + e < kend) ? g.at(r[i], c) : (u16)0;
          if (++c.ch == ch) { c.ch = 0; ++c.tap; }
        }
      }
      v[i] = x;
    }
  }
  __device__ __forceinline__ void put(u16 (*T)[kBK + kLdsPad]) const {
#pragma unroll
    for (int i = 0; i < S; ++i) {
      if (!mine(i)) continue;
      if constexpr (MODE == 2) {
        const u16* pv = (const u16*)&v[i];
#pragma unroll
        for (int e = 0; e < 8; ++e) T[lr8 + 64 * i + e][kk] = pv[e];
      } else {
        *(uint4*)&T[lr + 64 * i][lk] = v[i];
      }
    }
  }
};

template <int TM, int TN, class GA, class GB, class RM, class EP, int AM, int BM>
__device__ __forceinline__ void gemm_tile(const GA& ga, const GB& gb, const RM& rowmap, const EP& ep, int zi,
                                          long M, long N, long kbeg, long kend, long m0, long n0) {
  static_assert(TM * TN == 4 * 32 * 32, "four waves of 32 x 32");
  __shared__ __attribute__((aligned(16))) u16 As[TM][kBK + kLdsPad];
  __shared__ __attribute__((aligned(16))) u16 Bs[TN][kBK + kLdsPad];
  constexpr int WN = TN / 32;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave / WN, wn = wave % WN;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  Stage<GA, AM, TM> sa;
  Stage<GB, BM, TN> sb;
  sa.init(ga, m0, M, t);
  sb.init(gb, n0, N, t);
  const int ca = sa.ch, cb = sb.ch;
  const int qa = kBK / ca, rma = kBK % ca, qb = kBK / cb, rmb = kBK % cb;
  TapCh ta = tapch(kbeg + sa.koff(), ca), tb = tapch(kbeg + sb.koff(), cb);
  sa.fetch(ga, kbeg + sa.koff(), kend, ta);
  sb.fetch(gb, kbeg + sb.koff(), kend, tb);
  for (long k0 = kbeg; k0 < kend; k0 += kBK) {
    sa.put(As);
    sb.put(Bs);
    __syncthreads();
    if (k0 + kBK < kend) {
      tapch_step(ta, ca, qa, rma);
      tapch_step(tb, cb, qb, rmb);
      sa.fetch(ga, k0 + kBK + sa.koff(), kend, ta);
      sb.fetch(gb, k0 + kBK + sb.koff(), kend, tb);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const bf16x8 a = *(const bf16x8*)&As[wm * 32 + i * 16 + (lane & 15)][(lane >> 4) * 8];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const bf16x8 b = *(const bf16x8*)&Bs[wn * 32 + j * 16 + (lane & 15)][(lane >> 4) * 8];
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const long row = m0 + wm * 32 + i * 16 + (lane >> 4) * 4 + r;
      if (row >= M) continue;
      const long orow = rowmap(row);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const long col = n0 + wn * 32 + j * 16 + (lane & 15);
        if (col < N) ep(zi, orow, col, acc[i][j][r]);
      }
    }
}

// One GEMM, split-K chunk z = blockIdx.z of kchunk K indices.
template <int TM, int TN, class GA, class GB, class RM, class EP, int AM, int BM>
__global__ __launch_bounds__(256) void k_gemm_bf16(GA ga, GB gb, RM rowmap, EP ep, long M, long N, long K,
                                                   long kchunk) {
  const long kbeg = (long)blockIdx.z * kchunk;
  gemm_tile<TM, TN, GA, GB, RM, EP, AM, BM>(ga, gb, rowmap, ep, (int)blockIdx.z, M, N, kbeg,
                                            min(K, kbeg + kchunk), (long)blockIdx.x * TM,
                                            (long)blockIdx.y * TN);
}

// Every gather states its vector mode (kMode) and when it applies (vec()).
template <class G>
static int load_mode(const G& g) {
  return g.vec() ? G::kMode : 0;
}

template <class GA, class GB, class RM = IdentityRows, class EP>
static hipError_t gemm_ep(GA ga, GB gb, EP ep, long M, long N, long K, int splits, hipStream_t s,
                          const char* tag, RM rowmap = RM()) {
  if (K >= (1L << 31)) return hipErrorInvalidValue;   // 32-bit K indices
  long kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + kBK - 1) / kBK * kBK;
  const int z = (int)((K + kchunk - 1) / kchunk);
  const bool narrow = N <= 32;   // 128 x 32 tiles: no MFMA on padding columns
  const long tm = narrow ? 128 : kBM, tn = narrow ? 32 : kBN;
  dim3 grid((unsigned)((M + tm - 1) / tm), (unsigned)((N + tn - 1) / tn), (unsigned)z);
  const int am = load_mode(ga), bm = load_mode(gb);
  ScopedTiming _t(tag, s);
#define WO_GEMM(A_, B_)                                                                                  \
  do {                                                                                                   \
    if (narrow)                                                                                          \
      hipLaunchKernelGGL((k_gemm_bf16<128, 32, GA, GB, RM, EP, A_, B_>), grid, dim3(256), 0, s, ga, gb,  \
                         rowmap, ep, M, N, K, kchunk);                                                   \
    else                                                                                                 \
      hipLaunchKernelGGL((k_gemm_bf16<kBM, kBN, GA, GB, RM, EP, A_, B_>), grid, dim3(256), 0, s, ga, gb, \
                         rowmap, ep, M, N, K, kchunk);                                                   \
  } while (0)
  if (am && bm) WO_GEMM(GA::kMode, GB::kMode);
  else if (am) WO_GEMM(GA::kMode, 0);
  else if (bm) WO_GEMM(0, GB::kMode);
  else WO_GEMM(0, 0);
#undef WO_GEMM
  return hipGetLastError();
}

template <class GA, class GB>
static hipError_t gemm(GA ga, GB gb, float* C, long M, long N, long K, int splits, hipStream_t s,
                       const char* tag) {
  return gemm_ep(ga, gb, StoreC{C, M, N}, M, N, K, splits, s, tag);
}

// Input gradient: the 8 GEMMs of the parity classes of input positions in one
// launch, class = blockIdx.z (workgroups past a class's rows exit).
struct DgradClasses {
  GatherCol2imClass a[8];
  GatherWTClass b[8];
  long M[8], K[8];
};

// blockIdx.z = split * nc + class; with splits > 1 split q of every class's K
// range writes its partial sums to out + q * Mout * N (summed afterwards in a
// fixed order), each output row exactly once per split.
template <int TM, int TN, int AM, int BM>
__global__ __launch_bounds__(256) void k_gemm_dgrad(DgradClasses cl, float* __restrict__ out, long N,
                                                    long Mout, int nc, int splits) {
  const int c = (int)(blockIdx.z % nc), q = (int)(blockIdx.z / nc);
  const long m0 = (long)blockIdx.x * TM;
  if (m0 >= cl.M[c]) return;
  long kchunk = (cl.K[c] + splits - 1) / splits;
  kchunk = (kchunk + kBK - 1) / kBK * kBK;
  const long kbeg = min(cl.K[c], (long)q * kchunk), kend = min(cl.K[c], kbeg + kchunk);
  gemm_tile<TM, TN, GatherCol2imClass, GatherWTClass, ClassRows, StoreC, AM, BM>(
      cl.a[c], cl.b[c], ClassRows{cl.a[c]}, StoreC{out + (long)q * Mout * N, Mout, N}, 0, cl.M[c], N, kbeg,
      kend, m0, (long)blockIdx.y * TN);
}

// Split-K count of an input gradient: only when its tiles (over all parity
// classes) cannot fill the GPU, up to 8 chunks of at least 256 K indices.
static int dgrad_splits(long tiles, long kmax) {
  if (tiles >= 1024) return 1;
  return (int)std::max<long>(1, std::min<long>({8, (2048 + tiles - 1) / tiles, kmax / 256}));
}

// The parity classes of an input gradient (nc of them, the longest M and K,
// and the tile count at the tile shape gemm_ep would take).
struct DgradPlan {
  DgradClasses cl;
  int nc = 0;
  long mmax = 0, kmax = 0, tiles = 0;
  bool narrow = false;
};

static DgradPlan dgrad_plan(const u16* gz, const u16* w, ConvGeom gout, int Cin, int N) {
  DgradPlan pl;
  DgradClasses& cl = pl.cl;
  int& nc = pl.nc;
  for (int cls = 0; cls < 8; ++cls) {
    GatherCol2imClass a;
    a.gz = gz;
    a.g = gout;
    a.pd = cls >> 2; a.ph = (cls >> 1) & 1; a.pw = cls & 1;
    a.cd = (gout.D - a.pd + 1) / 2; a.ch = (gout.H - a.ph + 1) / 2; a.cw = (gout.W - a.pw + 1) / 2;
    if (a.cd <= 0 || a.ch <= 0 || a.cw <= 0) continue;
    a.nd = a.pd ? 2 : 1; a.nh = a.ph ? 2 : 1; a.nw = a.pw ? 2 : 1;
    cl.a[nc] = a;
    cl.b[nc] = GatherWTClass{w, Cin, gout.C, a.nd, a.nh, a.nw};
    cl.M[nc] = (long)N * a.cd * a.ch * a.cw;
    cl.K[nc] = (long)a.nd * a.nh * a.nw * gout.C;
    pl.mmax = std::max(pl.mmax, cl.M[nc]);
    ++nc;
  }
  pl.narrow = Cin <= 32;   // 128 x 32 tiles, as in gemm_ep
  const long tm = pl.narrow ? 128 : kBM, tn = pl.narrow ? 32 : kBN;
  for (int c = 0; c < nc; ++c) {
    pl.tiles += ((cl.M[c] + tm - 1) / tm) * ((Cin + tn - 1) / tn);
    pl.kmax = std::max(pl.kmax, cl.K[c]);
  }
  return pl;
}

static hipError_t reduce_parts(const float* part, int z, long n, float* out, hipStream_t s);

// Input gradient into out (Mout x Cin): directly, or (part not null, few
// tiles) split over K into the partials in part and summed in a fixed order.
static hipError_t dgrad_classes(const u16* gz, const u16* w, ConvGeom gout, int Cin, int N,
                                float* out, float* part, hipStream_t s, const char* tag = "k_gemm_conv_dgrad") {
  const DgradPlan pl = dgrad_plan(gz, w, gout, Cin, N);
  const DgradClasses& cl = pl.cl;
  const int nc = pl.nc;
  const long mmax = pl.mmax;
  if (nc == 0) return hipSuccess;
  const long Mout = (long)N * gout.D * gout.H * gout.W;
  if (Mout >= (1L << 31)) return hipErrorInvalidValue;   // 32-bit position arithmetic
  const bool narrow = pl.narrow;
  const long tm = narrow ? 128 : kBM, tn = narrow ? 32 : kBN;
  const int splits = part ? dgrad_splits(pl.tiles, pl.kmax) : 1;
  float* dst = splits > 1 ? part : out;
  dim3 grid((unsigned)((mmax + tm - 1) / tm), (unsigned)((Cin + tn - 1) / tn), (unsigned)(nc * splits));
  const int am = load_mode(cl.a[0]), bm = load_mode(cl.b[0]);
  {
  ScopedTiming _t(tag, s);
#define WO_DG(A_, B_)                                                                                  \
  do {                                                                                                 \
    if (narrow)                                                                                        \
      hipLaunchKernelGGL((k_gemm_dgrad<128, 32, A_, B_>), grid, dim3(256), 0, s, cl, dst, (long)Cin, Mout, nc, \
                         splits);                                                                      \
    else                                                                                               \
      hipLaunchKernelGGL((k_gemm_dgrad<kBM, kBN, A_, B_>), grid, dim3(256), 0, s, cl, dst, (long)Cin, Mout, nc, \
                         splits);                                                                      \
  } while (0)
  if (am && bm) WO_DG(GatherCol2imClass::kMode, GatherWTClass::kMode);
  else if (am) WO_DG(GatherCol2imClass::kMode, 0);
  else if (bm) WO_DG(0, GatherWTClass::kMode);
  else WO_DG(0, 0);
#undef WO_DG
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splits == 1) return e;
  ScopedTiming _t("k_reduce_parts", s);
  return reduce_parts(part, splits, Mout * Cin, out, s);
}

static int splits_used(long K, int splits) {
  long kchunk = (K + splits - 1) / splits;
  kchunk = (kchunk + kBK - 1) / kBK * kBK;
  return (int)((K + kchunk - 1) / kchunk);
}

// out[i] = sum_q part[q * n + i] for q < z, in a fixed order: a workgroup
// takes CW consecutive outputs and 256 / CW phases; phase h adds q = h, h + PH,
// ... with four independent accumulators (loads in flight), then a tree over
// the phases.  Many phases per output keep the serial chains short when n is
// small and z large.
static inline unsigned blocks(long n, int t) { return (unsigned)((n + t - 1) / t); }

template <int CW>
__global__ __launch_bounds__(256) void k_reduce_parts(const float* __restrict__ part, int z, long n,
                                                      float* __restrict__ out) {
  constexpr int PH = 256 / CW;
  __shared__ float red[256];
  const int t = threadIdx.x, c = t % CW, h = t / CW;
  const long i = (long)blockIdx.x * CW + c;
  float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
  if (i < n) {
    int q = h;
    for (; q + 3 * PH < z; q += 4 * PH) {
      a0 += part[(long)q * n + i];
      a1 += part[(long)(q + PH) * n + i];
      a2 += part[(long)(q + 2 * PH) * n + i];
      a3 += part[(long)(q + 3 * PH) * n + i];
    }
    for (; q < z; q += PH) a0 += part[(long)q * n + i];
  }
  red[t] = (a0 + a1) + (a2 + a3);
  __syncthreads();
  for (int st = PH / 2; st > 0; st >>= 1) {
    if (h < st) red[t] += red[t + st * CW];
    __syncthreads();
  }
  if (h == 0 && i < n) out[i] = red[c];
}

static hipError_t reduce_parts(const float* part, int z, long n, float* out, hipStream_t s) {
  if (n >= 64L * 512)
    hipLaunchKernelGGL(k_reduce_parts<64>, dim3(blocks(n, 64)), dim3(256), 0, s, part, z, n, out);
  else if (n >= 16L * 256)
    hipLaunchKernelGGL(k_reduce_parts<16>, dim3(blocks(n, 16)), dim3(256), 0, s, part, z, n, out);
  else
    hipLaunchKernelGGL(k_reduce_parts<4>, dim3(blocks(n, 4)), dim3(256), 0, s, part, z, n, out);
  return hipGetLastError();
}

// ------------------------------------------------------------------ elementwise

// z = z + b[c] (FP32), a = BF16(GELU(z)): the forward epilogue after a split-K
// sum (StoreBiasGelu's arithmetic).
__global__ void k_bias_gelu(float* __restrict__ z, const float* __restrict__ b, long P, int Co,
                            u16* __restrict__ a) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P * Co) return;
  const float v = z[i] + b[i % Co];
  z[i] = v;
  a[i] = f2bf(gelu_f(v));
}

// gz = BF16(ga * GELU'(z)) over P positions x Co channels (Co divides 256), and
// the bias gradient's first stage: workgroup g sums the rounded gz of its rows
// [g R, g R + R) per channel in a fixed order into part[g][c].  Lanes run along
// the channels, so every load and store is coalesced.
__global__ __launch_bounds__(256) void k_gelu_bwd_bias(const float* __restrict__ ga,
                                                       const float* __restrict__ z, long P, int Co,
                                                       long R, u16* __restrict__ gz,
                                                       float* __restrict__ part) {
  __shared__ float red[256];
  const int t = threadIdx.x, step = 256 / Co;
  const int c = t % Co;
  const long r0 = (long)blockIdx.x * R, r1 = min(P, r0 + R);
  float s = 0.f;
  // four rows per iteration, their loads issued before any is used (the sum
  // still adds the rows in order)
  for (long p = r0 + t / Co; p < r1; p += 4 * step) {
    float gv[4], zv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long q = p + u * step;
      const long i = q * Co + c;
      gv[u] = q < r1 ? ga[i] : 0.f;
      zv[u] = q < r1 ? z[i] : 0.f;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long q = p + u * step;
      if (q < r1) {
        const u16 b = f2bf(gv[u] * gelu_grad_f(zv[u]));
        gz[q * Co + c] = b;
        s += bf2f(b);
      }
    }
  }
  red[t] = s;
  __syncthreads();
  if (t < Co) {
    float acc = 0.f;
    for (int k = 0; k < step; ++k) acc += red[k * Co + t];
    part[(long)blockIdx.x * Co + t] = acc;
  }
}

// Rows per workgroup of k_gelu_bwd_bias: a multiple of 256 / Co, at most
// kBiasPartsMax workgroups.
constexpr int kBiasPartsMax = 1024;
static long bias_rows(long P, int Co) {
  const long step = 256 / Co;
  long R = std::max<long>(4 * step, (P + kBiasPartsMax - 1) / kBiasPartsMax);
  return (R + step - 1) / step * step;
}

// Per-sample input scaling x / rms(x) -> BF16 channels-last (C = 1), in two
// steps so that every sample spreads over many workgroups: FP64 sums of squares
// of kNormSlices slices per sample, then the scaling, each workgroup adding its
// sample's slice sums in a fixed order.
constexpr int kNormSlices = 32;
__global__ __launch_bounds__(256) void k_sumsq_slices(const float* __restrict__ x, long vol,
                                                      double* __restrict__ part) {
  __shared__ double red[256];
  const long n = blockIdx.y;
  const long len = (vol + kNormSlices - 1) / kNormSlices;
  const long i0 = blockIdx.x * len, i1 = min(vol, i0 + len);
  const float* xs = x + n * vol;
  double s = 0.0;
  for (long i = i0 + threadIdx.x; i < i1; i += blockDim.x) s += (double)xs[i] * xs[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[n * kNormSlices + blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_scale_bf16(const float* __restrict__ x, long vol,
                                                    const double* __restrict__ part,
                                                    u16* __restrict__ out) {
  __shared__ float inv_s;
  const long n = blockIdx.y;
  if (threadIdx.x == 0) {
    double ss = 0.0;
    for (int k = 0; k < kNormSlices; ++k) ss += part[n * kNormSlices + k];
    const double rms = sqrt(ss / (double)vol);
    inv_s = rms > 0.0 ? (float)(1.0 / rms) : 1.f;
  }
  __syncthreads();
  const float inv = inv_s;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < vol) out[n * vol + i] = f2bf(x[n * vol + i] * inv);
}

// Head per sample: feat = mean over positions of a (BF16), y = Wh feat + bh.
// With targets: dy = 2 (y - t) / (3 N), lossp[n] = sum (y - t)^2, and
// ga[n][p][c] = (Wh^T dy)[c] / npos.
__global__ __launch_bounds__(256) void k_head(const u16* __restrict__ a, long npos, int Cf,
                                              const float* __restrict__ wh, const float* __restrict__ bh,
                                              const float* __restrict__ target, int N,
                                              float* __restrict__ y_out, float* __restrict__ feat_out,
                                              float* __restrict__ dy_out, float* __restrict__ lossp,
                                              float* __restrict__ ga) {
  __shared__ float feat[256];
  __shared__ float dys[kCnnOut];
  const int n = blockIdx.x, c = threadIdx.x;
  if (c < Cf) {
    float s = 0.f;
    for (long p = 0; p < npos; ++p) s += bf2f(a[((long)n * npos + p) * Cf + c]);
    feat[c] = s / (float)npos;
    if (feat_out) feat_out[(long)n * Cf + c] = feat[c];
  }
  __syncthreads();
  if (c < kCnnOut) {
    float y = bh[c];
    for (int k = 0; k < Cf; ++k) y += wh[c * Cf + k] * feat[k];
    y_out[n * kCnnOut + c] = y;
    if (target) {
      const float d = y - target[n * kCnnOut + c];
      dys[c] = 2.f * d / (float)(kCnnOut * N);
      dy_out[n * kCnnOut + c] = dys[c];
    }
  }
  __syncthreads();
  if (target) {
    if (c == 0) {
      float l = 0.f;
      for (int j = 0; j < kCnnOut; ++j) {
        const float d = y_out[n * kCnnOut + j] - target[n * kCnnOut + j];
        l += d * d;
      }
      lossp[n] = l;
    }
    if (c < Cf) {
      float g = 0.f;
      for (int j = 0; j < kCnnOut; ++j) g += wh[j * Cf + c] * dys[j];
      g /= (float)npos;
      for (long p = 0; p < npos; ++p) ga[((long)n * npos + p) * Cf + c] = g;
    }
  }
}

// Head gradients (single workgroup): gwh = dy^T feat, gbh = sum dy, loss = mean.
__global__ __launch_bounds__(256) void k_head_grads(const float* __restrict__ dy,
                                                    const float* __restrict__ feat,
                                                    const float* __restrict__ lossp, int N, int Cf,
                                                    float* __restrict__ gwh, float* __restrict__ gbh,
                                                    float* __restrict__ loss) {
  for (int i = threadIdx.x; i < kCnnOut * Cf; i += blockDim.x) {
    const int j = i / Cf, c = i - j * Cf;
    float s = 0.f;
    for (int n = 0; n < N; ++n) s += dy[n * kCnnOut + j] * feat[(long)n * Cf + c];
    gwh[i] = s;
  }
  if (threadIdx.x < kCnnOut) {
    float s = 0.f;
    for (int n = 0; n < N; ++n) s += dy[n * kCnnOut + threadIdx.x];
    gbh[threadIdx.x] = s;
  }
  if (threadIdx.x == 0 && loss) {
    float s = 0.f;
    for (int n = 0; n < N; ++n) s += lossp[n];
    *loss = s / (float)(N * kCnnOut);
  }
}

// AdamW on the flat FP32 parameters; refreshes the BF16 copy of conv weights.
__global__ void k_adamw(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                        float* __restrict__ v, long n, float lr, float wd, float c1, float c2,
                        u16* __restrict__ pbf) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float upd = (mi / c1) / (sqrtf(vi / c2) + eps) + wd * p[i];
  const float np = p[i] - lr * upd;
  p[i] = np;
  pbf[i] = f2bf(np);
}

__global__ void k_to_bf16(const float* __restrict__ p, long n, u16* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = f2bf(p[i]);
}


// ------------------------------------------------------------------ network plan

struct Layer {
  ConvGeom g;
  int Cin, Cout;
  long P_in, P_out;   // positions (batch included)
  long w_off, b_off;  // offsets into the flat parameters
};

struct Net {
  int N;
  Layer L[kCnnLayers];
  long wh_off, bh_off, nparam;
  long npos_last;
};

static Net make_net(int N, int Z, int Y, int X) {
  Net net;
  net.N = N;
  int D = Z, H = Y, W = X;
  long off = 0;
  for (int l = 0; l < kCnnLayers; ++l) {
    Layer& L = net.L[l];
    L.Cin = kCnnChannels[l];
    L.Cout = kCnnChannels[l + 1];
    L.g.D = D; L.g.H = H; L.g.W = W; L.g.C = L.Cin;
    L.g.Do = (D - 1) / 2 + 1; L.g.Ho = (H - 1) / 2 + 1; L.g.Wo = (W - 1) / 2 + 1;
    L.P_in = (long)N * D * H * W;
    L.P_out = (long)N * L.g.Do * L.g.Ho * L.g.Wo;
    L.w_off = off;
    off += (long)L.Cout * 27 * L.Cin;
    L.b_off = off;
    off += L.Cout;
    D = L.g.Do; H = L.g.Ho; W = L.g.Wo;
  }
  net.wh_off = off;
  off += (long)kCnnOut * kCnnChannels[kCnnLayers];
  net.bh_off = off;
  off += kCnnOut;
  net.nparam = off;
  net.npos_last = (long)D * H * W;
  return net;
}

long cnn_param_count() { return make_net(1, 32, 64, 64).nparam; }

// Workspace for a batch: BF16 input and activations, FP32 pre-activations,
// FP32 input gradients, BF16 gradients, split-K partials, head buffers, BF16
// weights.
struct CnnWs {
  size_t x, a[kCnnLayers], z[kCnnLayers], gz, ga, part, pbf, grad, head, nrm, total;
};

static size_t al(size_t x) { return (x + 255) / 256 * 256; }
constexpr int kWgradSplitsMax = 1024;

// Split-K count of a weight gradient (Co x K outputs) over P output positions:
// about 2048 workgroups in all, at least 256 positions per split.
static int wgrad_splits(long P, long Co, long K) {
  const long tiles = ((Co + kBM - 1) / kBM) * ((K + kBN - 1) / kBN);
  const long want = (2048 + tiles - 1) / tiles;
  return (int)std::max<long>(1, std::min<long>({kWgradSplitsMax, P / 256, want}));
}

// Split-K count of a forward convolution: only when its tiles cannot fill the
// GPU (fewer than 512), up to 8 chunks of at least 256 K indices.
static int fwd_splits(long P, long Co, long K) {
  const long tiles = ((P + kBM - 1) / kBM) * ((Co + kBN - 1) / kBN);
  if (tiles >= 512) return 1;
  return (int)std::max<long>(1, std::min<long>({8, (1024 + tiles - 1) / tiles, K / 256}));
}

static CnnWs cnn_ws(const Net& net) {
  CnnWs w;
  size_t b = 0;
  auto take = [&](size_t bytes) { size_t o = b; b += al(bytes); return o; };
  w.x = take(net.L[0].P_in * sizeof(u16));
  long maxc = 0, maxg = 0, maxpart = 0;
  for (int l = 0; l < kCnnLayers; ++l) {
    const Layer& L = net.L[l];
    w.a[l] = take(L.P_out * L.Cout * sizeof(u16));
    w.z[l] = take(L.P_out * L.Cout * sizeof(float));
    maxc = std::max(maxc, std::max(L.P_out * L.Cout, L.P_in * L.Cin));
    maxg = std::max(maxg, L.P_out * L.Cout);
    maxpart = std::max(maxpart, (long)splits_used(L.P_out, wgrad_splits(L.P_out, L.Cout, 27L * L.Cin)) * L.Cout * 27 * L.Cin);
    maxpart = std::max(maxpart, (long)kBiasPartsMax * L.Cout);
    const long kf = 27L * L.Cin;
    maxpart = std::max(maxpart, (long)splits_used(kf, fwd_splits(L.P_out, L.Cout, kf)) * L.P_out * L.Cout);
    if (l > 0) {   // the input gradient's split-K partials
      ConvGeom gd = L.g;
      gd.C = L.Cout;
      const DgradPlan pl = dgrad_plan(nullptr, nullptr, gd, L.Cin, net.N);
      if (pl.nc > 0) maxpart = std::max(maxpart, (long)dgrad_splits(pl.tiles, pl.kmax) * L.P_in * L.Cin);
    }
  }
  w.gz = take(maxg * sizeof(u16));
  w.ga = take(maxc * sizeof(float));
  w.part = take(maxpart * sizeof(float));
  w.pbf = take(net.nparam * sizeof(u16));
  w.grad = take(net.nparam * sizeof(float));
  w.head = take((size_t)net.N * (kCnnOut * 3 + kCnnChannels[kCnnLayers] + 2) * sizeof(float));
  w.nrm = take((size_t)net.N * kNormSlices * sizeof(double));
  w.total = b;
  return w;
}

size_t cnn_workspace_size(int N, int Z, int Y, int X) { return cnn_ws(make_net(N, Z, Y, X)).total; }

// Forward through the convolutions (and, with targets, the backward pass that
// fills the flat FP32 gradient).  params: FP32 flat; the BF16 copy of the
// weights is refreshed from it at the start.
// Timing tags of the GEMMs per layer (the library's per-kernel report).
static const char* const kFwdTag[kCnnLayers] = {"k_gemm_conv_fwd_l0", "k_gemm_conv_fwd_l1", "k_gemm_conv_fwd_l2",
                                                "k_gemm_conv_fwd_l3"};
static const char* const kWgradTag[kCnnLayers] = {"k_gemm_conv_wgrad_l0", "k_gemm_conv_wgrad_l1",
                                                  "k_gemm_conv_wgrad_l2", "k_gemm_conv_wgrad_l3"};
static const char* const kDgradTag[kCnnLayers] = {"k_gemm_conv_dgrad_l0", "k_gemm_conv_dgrad_l1",
                                                  "k_gemm_conv_dgrad_l2", "k_gemm_conv_dgrad_l3"};

int cnn_run(const float* params, const float* x, int N, int Z, int Y, int X, const float* target,
            float* y_out, float* loss_out, float* grad_out, void* ws, hipStream_t s) {
  const Net net = make_net(N, Z, Y, X);
  const CnnWs W = cnn_ws(net);
  char* w = (char*)ws;
  u16* xb = (u16*)(w + W.x);
  u16* gz = (u16*)(w + W.gz);
  float* ga = (float*)(w + W.ga);
  float* part = (float*)(w + W.part);
  u16* pbf = (u16*)(w + W.pbf);
  float* grad = grad_out ? grad_out : (float*)(w + W.grad);
  float* head = (float*)(w + W.head);
  float* dy = head;
  float* lossp = dy + (long)N * kCnnOut;
  float* feat = lossp + N;
  const int Cf = kCnnChannels[kCnnLayers];
  { ScopedTiming _tm("k_to_bf16", s);
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks(net.nparam, 256)), dim3(256), 0, s, params, net.nparam, pbf);
  }
  {
    const long vol = (long)Z * Y * X;
    double* nrm = (double*)(w + W.nrm);
    ScopedTiming _tm("k_normalise", s);
    hipLaunchKernelGGL(k_sumsq_slices, dim3(kNormSlices, N), dim3(256), 0, s, x, vol, nrm);
    hipLaunchKernelGGL(k_scale_bf16, dim3(blocks(vol, 256), N), dim3(256), 0, s, x, vol, nrm, xb);
  }
  WO_HIP_CHECK(hipGetLastError());
  const u16* a_in = xb;
  for (int l = 0; l < kCnnLayers; ++l) {
    const Layer& L = net.L[l];
    const long K = 27L * L.Cin;
    float* z = (float*)(w + W.z[l]);
    u16* a = (u16*)(w + W.a[l]);
    const int fs = fwd_splits(L.P_out, L.Cout, K);
    if (fs == 1) {
      // the GEMM's epilogue adds the bias and applies GELU (z and a written directly)
      WO_HIP_CHECK(gemm_ep(GatherIm2col{a_in, L.g}, GatherRows{pbf + L.w_off, K, L.Cin},
                           StoreBiasGelu{z, a, params + L.b_off, L.Cout}, L.P_out, L.Cout, K, 1, s,
                           kFwdTag[l]));
    } else {
      // few tiles: split K, sum the partials in a fixed order into z, then bias and GELU
      WO_HIP_CHECK(gemm(GatherIm2col{a_in, L.g}, GatherRows{pbf + L.w_off, K, L.Cin}, part, L.P_out, L.Cout,
                        K, fs, s, kFwdTag[l]));
      { ScopedTiming _tm("k_reduce_parts", s);
      WO_HIP_CHECK(reduce_parts(part, splits_used(K, fs), L.P_out * L.Cout, z, s));
      }
      { ScopedTiming _tm("k_bias_gelu", s);
      hipLaunchKernelGGL(k_bias_gelu, dim3(blocks(L.P_out * L.Cout, 256)), dim3(256), 0, s, z,
                         params + L.b_off, L.P_out, L.Cout, a);
      }
    }
    a_in = a;
  }
  { ScopedTiming _tm("k_head", s);
  hipLaunchKernelGGL(k_head, dim3(N), dim3(256), 0, s, a_in, net.npos_last, Cf, params + net.wh_off,
                     params + net.bh_off, target, N, y_out, feat, dy, lossp, ga);
  }
  WO_HIP_CHECK(hipGetLastError());
  if (!target) return WO_OK;
  { ScopedTiming _tm("k_head_grads", s);
  hipLaunchKernelGGL(k_head_grads, dim3(1), dim3(256), 0, s, dy, feat, lossp, N, Cf,
                     grad + net.wh_off, grad + net.bh_off, loss_out);
  }
  for (int l = kCnnLayers - 1; l >= 0; --l) {
    const Layer& L = net.L[l];
    const long K = 27L * L.Cin;
    const float* z = (const float*)(w + W.z[l]);
    {
      // gz and the bias gradient: partials in part, summed before the weight
      // gradient reuses part
      const long R = bias_rows(L.P_out, L.Cout);
      const int G = (int)((L.P_out + R - 1) / R);
      ScopedTiming _tm("k_gelu_bwd_bias", s);
      hipLaunchKernelGGL(k_gelu_bwd_bias, dim3(G), dim3(256), 0, s, ga, z, L.P_out, L.Cout, R, gz, part);
      WO_HIP_CHECK(reduce_parts(part, G, (long)L.Cout, grad + L.b_off, s));
    }
    const u16* a_prev = l == 0 ? xb : (const u16*)(w + W.a[l - 1]);
    // weight gradient, split over output positions
    const int splits = wgrad_splits(L.P_out, L.Cout, K);
    const int zs = splits_used(L.P_out, splits);
    WO_HIP_CHECK(gemm(GatherT{gz, L.Cout}, GatherIm2colT{GatherIm2col{a_prev, L.g}}, part, L.Cout, K,
                      L.P_out, splits, s, kWgradTag[l]));
    { ScopedTiming _tm("k_reduce_parts", s);
    WO_HIP_CHECK(reduce_parts(part, zs, (long)L.Cout * K, grad + L.w_off, s));
    }
    if (l > 0) {
      ConvGeom gd = L.g;
      gd.C = L.Cout;
      WO_HIP_CHECK(dgrad_classes(gz, pbf + L.w_off, gd, L.Cin, net.N, ga, part, s, kDgradTag[l]));
    }
  }
  return WO_OK;
}

// AdamW step on the flat parameters (t >= 1).
hipError_t cnn_adamw(float* p, const float* g, float* m, float* v, long n, int t, float lr, float wd,
                     void* ws_pbf, hipStream_t s) {
  const float c1 = 1.f - powf(0.9f, (float)t), c2 = 1.f - powf(0.999f, (float)t);
  { ScopedTiming _tm("k_adamw", s);
  hipLaunchKernelGGL(k_adamw, dim3(blocks(n, 256)), dim3(256), 0, s, p, g, m, v, n, lr, wd, c1, c2,
                     (u16*)ws_pbf);
  }
  return hipGetLastError();
}

size_t cnn_pbf_offset(int N, int Z, int Y, int X) { return cnn_ws(make_net(N, Z, Y, X)).pbf; }
size_t cnn_grad_offset(int N, int Z, int Y, int X) { return cnn_ws(make_net(N, Z, Y, X)).grad; }

// Single convolution GEMMs for parity tests.
hipError_t conv_fwd_raw(const u16* x, const u16* w, int N, int D, int H, int W, int Cin, int Cout,
                        float* out, hipStream_t s) {
  ConvGeom g{D, H, W, Cin, (D - 1) / 2 + 1, (H - 1) / 2 + 1, (W - 1) / 2 + 1};
  const long P = (long)N * g.Do * g.Ho * g.Wo;
  return gemm(GatherIm2col{x, g}, GatherRows{w, 27L * Cin, Cin}, out, P, Cout, 27L * Cin, 1, s,
              "k_gemm_conv_fwd");
}

hipError_t conv_dgrad_raw(const u16* gz, const u16* w, int N, int D, int H, int W, int Cin, int Cout,
                          float* out, hipStream_t s) {
  ConvGeom g{D, H, W, Cout, (D - 1) / 2 + 1, (H - 1) / 2 + 1, (W - 1) / 2 + 1};
  return dgrad_classes(gz, w, g, Cin, N, out, nullptr, s);
}

hipError_t conv_wgrad_raw(const u16* x, const u16* gz, int N, int D, int H, int W, int Cin, int Cout,
                          float* out, float* part, long part_elems, hipStream_t s) {
  ConvGeom g{D, H, W, Cin, (D - 1) / 2 + 1, (H - 1) / 2 + 1, (W - 1) / 2 + 1};
  const long P = (long)N * g.Do * g.Ho * g.Wo;
  const long K = 27L * Cin;
  int splits = wgrad_splits(P, Cout, K);
  while (splits > 1 && (long)splits_used(P, splits) * Cout * K > part_elems) splits /= 2;
  const int zs = splits_used(P, splits);
  if ((long)zs * Cout * K > part_elems) return hipErrorInvalidValue;
  hipError_t e = gemm(GatherT{gz, Cout}, GatherIm2colT{GatherIm2col{x, g}}, part, Cout, K, P, splits,
                      s, "k_gemm_conv_wgrad");
  if (e != hipSuccess) return e;
  return reduce_parts(part, zs, (long)Cout * K, out, s);
}

}  // namespace wo

// ------------------------------------------------------------------ training-data generators

namespace wo {

// SplitMix64 finaliser: a counter-based hash giving independent 64-bit words.
__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ double u01(unsigned long long h) {  // (0, 1)
  return ((double)(h >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

// Thin cells: per patch, `ncells` randomly oriented ellipses (semi-axes
// U(0.8, 2.5) um, phase U(0.1, 0.5) rad, absorption U(0, 0.02)) with a dome
// profile 1 - rho^2 / 2, wrapping at the tile edges; out [n][2][Y][X].
__global__ void k_synth_cells(float* __restrict__ out, int Y, int X, double pixel, int ncells,
                              unsigned long long seed) {
  const long n = blockIdx.y;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)Y * X) return;
  const int y = (int)(idx / X), x = (int)(idx - (long)y * X);
  const double Ly = Y * pixel, Lx = X * pixel;
  double ph = 0.0, ab = 0.0;
  for (int c = 0; c < ncells; ++c) {
    const unsigned long long base = seed * 0x100000001b3ull + ((unsigned long long)n << 20) + (unsigned long long)c * 16;
    const double cy = u01(mix64(base + 0)) * Ly, cx = u01(mix64(base + 1)) * Lx;
    const double a = 0.8 + 1.7 * u01(mix64(base + 2)), b = 0.8 + 1.7 * u01(mix64(base + 3));
    const double t = M_PI * u01(mix64(base + 4));
    const double p0 = 0.1 + 0.4 * u01(mix64(base + 5)), a0 = 0.02 * u01(mix64(base + 6));
    double dy = y * pixel - cy + 0.5 * Ly, dx = x * pixel - cx + 0.5 * Lx;
    dy = dy - floor(dy / Ly) * Ly - 0.5 * Ly;
    dx = dx - floor(dx / Lx) * Lx - 0.5 * Lx;
    const double u = dx * cos(t) + dy * sin(t), v = -dx * sin(t) + dy * cos(t);
    const double r2 = (u / a) * (u / a) + (v / b) * (v / b);
    if (r2 <= 1.0) {
      ph += p0 * (1.0 - 0.5 * r2);
      ab += a0 * (1.0 - 0.5 * r2);
    }
  }
  out[(n * 2 + 0) * (long)Y * X + idx] = (float)ph;
  out[(n * 2 + 1) * (long)Y * X + idx] = (float)ab;
}

// x += sigma * N(0, 1) (Box-Muller on hashed counters)
__global__ void k_add_noise(float* __restrict__ x, long n, float sigma, unsigned long long seed) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const unsigned long long h1 = mix64(seed ^ (2ull * (unsigned long long)i));
  const unsigned long long h2 = mix64(seed ^ (2ull * (unsigned long long)i + 1ull));
  const double r = sqrt(-2.0 * log(u01(h1)));
  x[i] += sigma * (float)(r * cos(2.0 * M_PI * u01(h2)));
}

// One thread per output voxel: the window of each stack at (z0, y0, x0),
// zero outside the input and outside the central keep[i] planes.
__global__ void k_crop(const float* __restrict__ in, int nz, int ny, int nx, float* out, int oz,
                       int oy, int ox, int z0, int y0, int x0, const int* __restrict__ keep,
                       long total) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int x = (int)(e % ox);
  const long r = e / ox;
  const int y = (int)(r % oy);
  const long r2 = r / oy;
  const int z = (int)(r2 % oz);
  const long i = r2 / oz;
  const int zi = z + z0, yi = y + y0, xi = x + x0;
  bool in_win = zi >= 0 && zi < nz && yi >= 0 && yi < ny && xi >= 0 && xi < nx;
  if (keep) in_win = in_win && abs(2 * z - (oz - 1)) < keep[i];
  out[e] = in_win ? in[((i * nz + zi) * (long)ny + yi) * nx + xi] : 0.f;
}

// Centred network windows of packed patches of uneven shapes: record j of a
// launch gives patch j's offset in the packed stacks and its shape; the
// window's first voxel sits at floor((n - o) / 2) along each axis (central
// planes of deeper patches, symmetric zero padding of shallower ones).
struct CropRec {
  long off;
  int nz, ny, nx;
};
constexpr int kCropRecs = 16;
struct CropBatch {
  CropRec r[kCropRecs];
};
__device__ __forceinline__ int floor_half(int v) { return v >= 0 ? v / 2 : -((1 - v) / 2); }
__global__ void k_crop_packed(const float* __restrict__ in, CropBatch b, int nrec, float* __restrict__ out,
                              int oz, int oy, int ox) {
  const long per = (long)oz * oy * ox;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nrec * per) return;
  const int j = (int)(e / per);
  const long w = e - j * per;
  const int x = (int)(w % ox), y = (int)((w / ox) % oy), z = (int)(w / ((long)ox * oy));
  const CropRec c = b.r[j];
  const int zi = z + floor_half(c.nz - oz), yi = y + floor_half(c.ny - oy), xi = x + floor_half(c.nx - ox);
  const bool in_win = zi >= 0 && zi < c.nz && yi >= 0 && yi < c.ny && xi >= 0 && xi < c.nx;
  out[e] = in_win ? in[c.off + ((long)zi * c.ny + yi) * c.nx + xi] : 0.f;
}

// The learned initialiser's prior box (normalised outputs -1 .. 1 span it).
constexpr double kPriorLo[3] = {-2.0, 1.0, 0.0};
constexpr double kPriorHi[3] = {2.0, 1.3, 0.52359877559829887};   // 30 degrees
constexpr int kNetZ = 32, kNetY = 64, kNetX = 64;

struct CnnInitWs {
  size_t x, net, y, total;
};
static CnnInitWs cnn_init_ws(int n) {
  CnnInitWs w;
  size_t b = 0;
  auto take = [&](size_t bytes) { size_t o = b; b += al(bytes); return o; };
  w.x = take((size_t)n * kNetZ * kNetY * kNetX * sizeof(float));
  w.net = take(cnn_workspace_size(n, kNetZ, kNetY, kNetX));
  w.y = take((size_t)n * kCnnOut * sizeof(float));
  w.total = b;
  return w;
}

}  // namespace wo

// ------------------------------------------------------------------ C ABI

extern "C" {

int64_t wo_cnn_param_count(void) { return wo::cnn_param_count(); }

int wo_synth_thin_cells(float* out, int32_t n, int32_t ny, int32_t nx, double pixel, int32_t ncells,
                        uint64_t seed, void* stream) {
  if (!out || n < 1 || n > 65535 || ny < 1 || nx < 1 || !(pixel > 0) || ncells < 0) return WO_EINVAL;
  dim3 grid(wo::blocks((long)ny * nx, 256), n);
  hipLaunchKernelGGL(wo::k_synth_cells, grid, dim3(256), 0, (hipStream_t)stream, out, ny, nx, pixel,
                     ncells, (unsigned long long)seed);
  WO_HIP_CHECK(hipGetLastError());
  return WO_OK;
}

int wo_add_gaussian_noise(float* x, int64_t n, double sigma, uint64_t seed, void* stream) {
  if (!x || n < 0) return WO_EINVAL;
  if (n == 0) return WO_OK;
  hipLaunchKernelGGL(wo::k_add_noise, dim3(wo::blocks(n, 256)), dim3(256), 0, (hipStream_t)stream, x,
                     (long)n, (float)sigma, (unsigned long long)seed);
  WO_HIP_CHECK(hipGetLastError());
  return WO_OK;
}

int wo_crop_stacks(const float* in, int32_t n, int32_t nz, int32_t ny, int32_t nx, float* out,
                   int32_t oz, int32_t oy, int32_t ox, int32_t z0, int32_t y0, int32_t x0,
                   const int32_t* keep_z, void* stream) {
  if (!in || !out || n < 1 || nz < 1 || ny < 1 || nx < 1 || oz < 1 || oy < 1 || ox < 1)
    return WO_EINVAL;
  if (in == out && (nz != oz || ny != oy || nx != ox || z0 || y0 || x0)) return WO_EALIAS;
  const long total = (long)n * oz * oy * ox;
  hipLaunchKernelGGL(wo::k_crop, dim3(wo::blocks(total, 256)), dim3(256), 0, (hipStream_t)stream, in,
                     nz, ny, nx, out, oz, oy, ox, z0, y0, x0, keep_z, total);
  WO_HIP_CHECK(hipGetLastError());
  return WO_OK;
}

void wo_cnn_prior(double lo[3], double hi[3]) {
  for (int j = 0; j < 3; ++j) {
    lo[j] = wo::kPriorLo[j];
    hi[j] = wo::kPriorHi[j];
  }
}

size_t wo_cnn_init_workspace_size(int32_t n) {
  if (n < 1 || (long)n * wo::kNetZ * wo::kNetY * wo::kNetX >= (1L << 31)) return 0;
  return wo::cnn_init_ws(n).total;
}

int wo_cnn_init_theta(const float* params, const wo_optics* o, int32_t n, const float* d, double* theta_out,
                      void* ws, size_t ws_bytes, void* stream) {
  if (!params || !o || !d || !theta_out || !ws || n < 1) return WO_EINVAL;
  const size_t need = wo_cnn_init_workspace_size(n);
  if (need == 0) return WO_EINVAL;
  if (ws_bytes < need) return WO_ENOMEM;
  for (int i = 0; i < n; ++i)
    if (o[i].nz < 1 || o[i].ny < 1 || o[i].nx < 1) return WO_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const wo::CnnInitWs W = wo::cnn_init_ws(n);
  char* w = (char*)ws;
  float* x = (float*)(w + W.x);
  float* y = (float*)(w + W.y);
  const long per = (long)wo::kNetZ * wo::kNetY * wo::kNetX;
  long off = 0;
  for (int i0 = 0; i0 < n; i0 += wo::kCropRecs) {
    const int nr = std::min(wo::kCropRecs, n - i0);
    wo::CropBatch b{};
    for (int j = 0; j < nr; ++j) {
      const wo_optics& oi = o[i0 + j];
      b.r[j] = wo::CropRec{off, oi.nz, oi.ny, oi.nx};
      off += (long)oi.nz * oi.ny * oi.nx;
    }
    hipLaunchKernelGGL(wo::k_crop_packed, dim3(wo::blocks(nr * per, 256)), dim3(256), 0, s, d, b, nr,
                       x + (long)i0 * per, wo::kNetZ, wo::kNetY, wo::kNetX);
    WO_HIP_CHECK(hipGetLastError());
  }
  const int r = wo::cnn_run(params, x, n, wo::kNetZ, wo::kNetY, wo::kNetX, nullptr, y, nullptr, nullptr,
                            w + W.net, s);
  if (r) return r;
  std::vector<float> h((size_t)n * wo::kCnnOut);
  WO_HIP_CHECK(hipMemcpyAsync(h.data(), y, h.size() * sizeof(float), hipMemcpyDeviceToHost, s));
  WO_HIP_CHECK(hipStreamSynchronize(s));
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < 3; ++j)
      theta_out[4 * i + j] = wo::kPriorLo[j] + 0.5 * ((double)h[(size_t)wo::kCnnOut * i + j] + 1.0) *
                                                    (wo::kPriorHi[j] - wo::kPriorLo[j]);
    theta_out[4 * i + 3] = o[i].tilt_azimuth;
  }
  return WO_OK;
}

// the kernels index positions (batch included) in 32 bits
static bool cnn_shape_ok(int32_t batch, int32_t nz, int32_t ny, int32_t nx) {
  return batch >= 1 && batch <= 65535 && nz >= 1 && ny >= 1 && nx >= 1 && nz <= 1024 && ny <= 4096 &&
         nx <= 4096 && (long)batch * nz * ny * nx < (1L << 31);
}

size_t wo_cnn_workspace_size(int32_t batch, int32_t nz, int32_t ny, int32_t nx) {
  if (!cnn_shape_ok(batch, nz, ny, nx)) return 0;
  return wo::cnn_workspace_size(batch, nz, ny, nx);
}

int wo_cnn_forward(const float* params, const float* x, int32_t batch, int32_t nz, int32_t ny,
                   int32_t nx, float* y_out, void* ws, size_t ws_bytes, void* stream) {
  if (!params || !x || !y_out || !ws || !cnn_shape_ok(batch, nz, ny, nx)) return WO_EINVAL;
  if (ws_bytes < wo::cnn_workspace_size(batch, nz, ny, nx)) return WO_ENOMEM;
  return wo::cnn_run(params, x, batch, nz, ny, nx, nullptr, y_out, nullptr, nullptr, ws,
                     (hipStream_t)stream);
}

int wo_cnn_gradient(const float* params, const float* x, const float* target, int32_t batch,
                    int32_t nz, int32_t ny, int32_t nx, float* y_out, float* loss_out,
                    float* grad_out, void* ws, size_t ws_bytes, void* stream) {
  if (!params || !x || !target || !y_out || !ws || !cnn_shape_ok(batch, nz, ny, nx)) return WO_EINVAL;
  if (ws_bytes < wo::cnn_workspace_size(batch, nz, ny, nx)) return WO_ENOMEM;
  return wo::cnn_run(params, x, batch, nz, ny, nx, target, y_out, loss_out, grad_out, ws,
                     (hipStream_t)stream);
}

int wo_cnn_train_step(float* params, float* adam_m, float* adam_v, int32_t t, double lr,
                      double weight_decay, const float* x, const float* target, int32_t batch,
                      int32_t nz, int32_t ny, int32_t nx, float* y_out, float* loss_out, void* ws,
                      size_t ws_bytes, void* stream) {
  if (!params || !adam_m || !adam_v || t < 1 || !(lr >= 0) || !(weight_decay >= 0)) return WO_EINVAL;
  int st = wo_cnn_gradient(params, x, target, batch, nz, ny, nx, y_out, loss_out, nullptr, ws,
                           ws_bytes, stream);
  if (st) return st;
  char* w = (char*)ws;
  const float* g = (const float*)(w + wo::cnn_grad_offset(batch, nz, ny, nx));
  void* pbf = w + wo::cnn_pbf_offset(batch, nz, ny, nx);
  WO_HIP_CHECK(wo::cnn_adamw(params, g, adam_m, adam_v, wo::cnn_param_count(), t, (float)lr,
                             (float)weight_decay, pbf, (hipStream_t)stream));
  return WO_OK;
}

static bool conv_ok(int N, int D, int H, int W, int Cin, int Cout) {
  return N >= 1 && D >= 1 && H >= 1 && W >= 1 && Cin >= 1 && Cout >= 1 && Cin <= 4096 &&
         Cout <= 4096 && (long)N * D * H * W < (1L << 31);
}

int wo_conv3d_forward(const uint16_t* x, const uint16_t* w, int32_t N, int32_t D, int32_t H,
                      int32_t W, int32_t Cin, int32_t Cout, float* out, void* stream) {
  if (!x || !w || !out || !conv_ok(N, D, H, W, Cin, Cout)) return WO_EINVAL;
  WO_HIP_CHECK(wo::conv_fwd_raw(x, w, N, D, H, W, Cin, Cout, out, (hipStream_t)stream));
  return WO_OK;
}

int wo_conv3d_input_grad(const uint16_t* gz, const uint16_t* w, int32_t N, int32_t D, int32_t H,
                         int32_t W, int32_t Cin, int32_t Cout, float* out, void* stream) {
  if (!gz || !w || !out || !conv_ok(N, D, H, W, Cin, Cout)) return WO_EINVAL;
  WO_HIP_CHECK(wo::conv_dgrad_raw(gz, w, N, D, H, W, Cin, Cout, out, (hipStream_t)stream));
  return WO_OK;
}

int wo_conv3d_weight_grad(const uint16_t* x, const uint16_t* gz, int32_t N, int32_t D, int32_t H,
                          int32_t W, int32_t Cin, int32_t Cout, float* out, void* ws,
                          size_t ws_bytes, void* stream) {
  if (!x || !gz || !out || !ws || !conv_ok(N, D, H, W, Cin, Cout)) return WO_EINVAL;
  WO_HIP_CHECK(wo::conv_wgrad_raw(x, gz, N, D, H, W, Cin, Cout, out, (float*)ws,
                                  (long)(ws_bytes / sizeof(float)), (hipStream_t)stream));
  return WO_OK;
}

}  // extern "C"
