// Shared device helpers: complex arithmetic, the LDS Stockham FFT core and
// the per-patch optics record used by the transfer-function kernels.
//
// FFT core: a mixed-radix (2, 3, 4, 5, 8) Stockham autosort transform of
// `nl` lines held in LDS.  Each pass reads every butterfly's inputs into
// registers, synchronises, and writes the outputs back in place, so one LDS
// buffer suffices.  Radices are a runtime plan (one switch per pass); the
// per-thread register arrays are sized statically from EMAX, the maximum
// number of elements a thread owns (lines * n <= threads * EMAX).
// Twiddles W_n^m are generated per workgroup in FP64 and stored in LDS as
// FP32, so the FFT needs no global table.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wo {

constexpr int kMaxPasses = 16;
constexpr int kEmax = 8;                   // elements owned by one thread in an LDS FFT
constexpr int kMaxThreads = 1024;
constexpr int kMaxElems = kEmax * kMaxThreads;  // elements one workgroup may own

// Threads for a workgroup owning `elems` elements: a multiple of 64 with
// threads * kEmax >= elems (callers keep elems <= kMaxElems).
inline int threads_for(long elems) {
  long t = (elems + kEmax - 1) / kEmax;
  t = ((t + 63) / 64) * 64;
  if (t < 64) t = 64;
  if (t > kMaxThreads) t = kMaxThreads;
  return (int)t;
}

// Radix sequence of one transform length, packed 4 bits per pass (the radix
// itself) so that device code reads it with shifts instead of indexing an
// array (which would force the plan into private memory).
struct FftPlan {
  int n;
  int npass;
  unsigned long long radices;
};

__host__ __device__ inline int plan_radix(const FftPlan& p, int q) {
  return (int)((p.radices >> (4 * q)) & 15ull);
}

// Host-side factorisation: as many radix-8 passes as possible, then 4, 2, 3, 5.
// Returns false when n has a prime factor other than 2, 3, 5.
inline bool make_plan(int n, FftPlan* p) {
  p->n = n;
  p->npass = 0;
  p->radices = 0;
  int m = n;
  if (n < 1) return false;
  const int order[5] = {8, 4, 2, 3, 5};
  for (int f : order) {
    while (m % f == 0 && p->npass < kMaxPasses) {
      p->radices |= (unsigned long long)f << (4 * p->npass);
      p->npass++;
      m /= f;
    }
  }
  return m == 1;
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulconj(float2 a, float2 b) {  // a * conj(b)
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 ctimes_i(float2 a, float s) {  // (s * i) * a, s = +-1
  return make_float2(-s * a.y, s * a.x);
}

// ---------------------------------------------------------------- small DFTs
// sign = -1: forward (exp(-2 pi i nk/R)); +1: inverse (unnormalised).

__device__ __forceinline__ void dft2(float2* v) {
  float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

__device__ __forceinline__ void dft4(float2* v, float s) {
  float2 a = cadd(v[0], v[2]), b = csub(v[0], v[2]);
  float2 c = cadd(v[1], v[3]), d = csub(v[1], v[3]);
  float2 id = ctimes_i(d, s);
  v[0] = cadd(a, c);
  v[2] = csub(a, c);
  v[1] = cadd(b, id);
  v[3] = csub(b, id);
}

__device__ __forceinline__ void dft3(float2* v, float s) {
  const float h = 0.86602540378443864676f;  // sin(2 pi / 3)
  float2 a = cadd(v[1], v[2]);
  float2 t = make_float2(v[0].x - 0.5f * a.x, v[0].y - 0.5f * a.y);
  float2 u = ctimes_i(cscale(csub(v[1], v[2]), h), s);
  v[0] = cadd(v[0], a);
  v[1] = cadd(t, u);
  v[2] = csub(t, u);
}

__device__ __forceinline__ void dft5(float2* v, float s) {
  const float c1 = 0.30901699437494742410f;   // cos(2 pi / 5)
  const float c2 = -0.80901699437494742410f;  // cos(4 pi / 5)
  const float s1 = 0.95105651629515357212f;   // sin(2 pi / 5)
  const float s2 = 0.58778525229247312917f;   // sin(4 pi / 5)
  float2 a1 = cadd(v[1], v[4]), a2 = cadd(v[2], v[3]);
  float2 b1 = csub(v[1], v[4]), b2 = csub(v[2], v[3]);
  float2 x0 = v[0];
  float2 t1 = make_float2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
  float2 t2 = make_float2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
  float2 u1 = make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y);
  float2 u2 = make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y);
  float2 iu1 = ctimes_i(u1, s), iu2 = ctimes_i(u2, s);
  v[0] = make_float2(x0.x + a1.x + a2.x, x0.y + a1.y + a2.y);
  v[1] = cadd(t1, iu1);
  v[4] = csub(t1, iu1);
  v[2] = cadd(t2, iu2);
  v[3] = csub(t2, iu2);
}

__device__ __forceinline__ void dft8(float2* v, float s) {
  const float r = 0.70710678118654752440f;
  float2 a[4], b[4];
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    a[n] = cadd(v[n], v[n + 4]);
    b[n] = csub(v[n], v[n + 4]);
  }
  // b_n *= W8^n, W8 = exp(s 2 pi i / 8)
  b[1] = make_float2(r * (b[1].x - s * b[1].y), r * (b[1].y + s * b[1].x));
  b[2] = ctimes_i(b[2], s);
  b[3] = make_float2(r * (-b[3].x - s * b[3].y), r * (-b[3].y + s * b[3].x));
  dft4(a, s);
  dft4(b, s);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[2 * k] = a[k];
    v[2 * k + 1] = b[k];
  }
}

// 6 = 2 x 3: DFTs of the even and odd samples, E and O, then
// X[k] = E[k] + W6^k O[k] and X[k + 3] = E[k] - W6^k O[k], W6 = exp(s i pi / 3).
__device__ __forceinline__ void dft6(float2* v, float s) {
  const float h = 0.86602540378443864676f;  // sin(pi / 3)
  float2 e[3] = {v[0], v[2], v[4]}, o[3] = {v[1], v[3], v[5]};
  dft3(e, s);
  dft3(o, s);
  const float2 t1 = make_float2(0.5f * o[1].x - s * h * o[1].y, 0.5f * o[1].y + s * h * o[1].x);
  const float2 t2 = make_float2(-0.5f * o[2].x - s * h * o[2].y, -0.5f * o[2].y + s * h * o[2].x);
  v[0] = cadd(e[0], o[0]);
  v[3] = csub(e[0], o[0]);
  v[1] = cadd(e[1], t1);
  v[4] = csub(e[1], t1);
  v[2] = cadd(e[2], t2);
  v[5] = csub(e[2], t2);
}

// 16 = 4 x 4: with n = 4 n1 + n2 and k = k1 + 4 k2, Y_n2[k1] = DFT4 over n1 of
// v[4 n1 + n2] times W16^(n2 k1), and X[k1 + 4 k2] = DFT4 over n2 of Y_n2[k1]
// (W16 = exp(s 2 pi i / 16); the products n2 k1 are 1, 2, 3, 4, 6 and 9).
__device__ __forceinline__ void dft16(float2* v, float s) {
  const float c1 = 0.92387953251128675613f;   // cos(pi / 8)
  const float s1 = 0.38268343236508977173f;   // sin(pi / 8)
  const float r = 0.70710678118654752440f;
  auto rot = [](float2 x, float c, float sn) {   // x (c + i sn)
    return make_float2(c * x.x - sn * x.y, c * x.y + sn * x.x);
  };
  float2 y[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
#pragma unroll
    for (int n1 = 0; n1 < 4; ++n1) y[n2][n1] = v[4 * n1 + n2];
    dft4(y[n2], s);
  }
  y[1][1] = rot(y[1][1], c1, s * s1);     // W^1
  y[1][2] = rot(y[1][2], r, s * r);       // W^2
  y[1][3] = rot(y[1][3], s1, s * c1);     // W^3
  y[2][1] = rot(y[2][1], r, s * r);       // W^2
  y[2][2] = ctimes_i(y[2][2], s);         // W^4
  y[2][3] = rot(y[2][3], -r, s * r);      // W^6
  y[3][1] = rot(y[3][1], s1, s * c1);     // W^3
  y[3][2] = rot(y[3][2], -r, s * r);      // W^6
  y[3][3] = rot(y[3][3], -c1, -s * s1);   // W^9
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    float2 z[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
    dft4(z, s);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = z[k2];
  }
}

template <int R>
__device__ __forceinline__ void dft_small(float2* v, float s) {
  if constexpr (R == 2) dft2(v);
  else if constexpr (R == 3) dft3(v, s);
  else if constexpr (R == 4) dft4(v, s);
  else if constexpr (R == 5) dft5(v, s);
  else if constexpr (R == 6) dft6(v, s);
  else if constexpr (R == 8) dft8(v, s);
  else if constexpr (R == 16) dft16(v, s);
}

// Twiddle tables of the compiled transform lengths, evaluated by the compiler:
// tw_n[m] = exp(-2 pi i m / n) rounded to FP32 from FP64 Taylor sums of sin
// and cos on [0, pi/4] (error below 1e-16 there), the other octants by the
// symmetries of compute_twiddles below.  A workgroup copies its table from
// memory (it stays in the caches) instead of evaluating n/8 + 1 FP64 sines
// and cosines.
struct TwPair {
  float c, s;
};
constexpr int kTwSizes[] = {16, 24, 32, 48, 64, 96, 128, 160, 192, 240, 256, 320, 384, 480, 512, 1024};
constexpr int kTwCount = sizeof(kTwSizes) / sizeof(kTwSizes[0]);
constexpr int tw_offset(int n) {
  int off = 0;
  for (int i = 0; i < kTwCount; ++i) {
    if (kTwSizes[i] == n) return off;
    off += kTwSizes[i];
  }
  return -1;
}
constexpr int kTwTotal = [] {
  int t = 0;
  for (int i = 0; i < kTwCount; ++i) t += kTwSizes[i];
  return t;
}();
constexpr double cx_sin(double x) {   // |x| <= pi/4: terms to x^29
  double x2 = x * x, term = x, sum = x;
  for (int k = 1; k < 15; ++k) {
    term *= -x2 / (double)((2 * k) * (2 * k + 1));
    sum += term;
  }
  return sum;
}
constexpr double cx_cos(double x) {
  double x2 = x * x, term = 1.0, sum = 1.0;
  for (int k = 1; k < 15; ++k) {
    term *= -x2 / (double)((2 * k - 1) * (2 * k));
    sum += term;
  }
  return sum;
}
struct TwTables {
  TwPair v[kTwTotal];
};
constexpr TwTables make_tw_tables() {
  TwTables t{};
  int off = 0;
  for (int i = 0; i < kTwCount; ++i) {
    const int n = kTwSizes[i], e = n >> 3, qn = n >> 2;
    TwPair* tw = t.v + off;
    for (int r = 0; r <= e; ++r) {
      const double a = 2.0 * 3.14159265358979323846 * (double)r / (double)n;
      const float c = (float)cx_cos(a), s = (float)cx_sin(a);
      tw[r] = TwPair{c, -s};
      tw[qn + r] = TwPair{-s, -c};
      tw[2 * qn + r] = TwPair{-c, s};
      tw[3 * qn + r] = TwPair{s, c};
      if (r > 0 && r < e) {
        tw[qn - r] = TwPair{s, -c};
        tw[2 * qn - r] = TwPair{-c, -s};
        tw[3 * qn - r] = TwPair{-s, c};
        tw[n - r] = TwPair{c, s};
      }
    }
    off += n;
  }
  return t;
}
static __device__ const TwTables kTwTables = make_tw_tables();

// Twiddles tw[m] = exp(-2 pi i m / n), m < n, from FP64 sines and cosines.
// When 8 divides n only the angles a = 2 pi r / n in [0, pi/4] (r <= n/8) are
// evaluated: with (c, s) = (cos a, sin a), the angles q pi/2 + a and
// q pi/2 - a (q = 0..3, 1..4) have cos and sin equal to c and s up to swaps
// and signs, so each evaluation fills up to eight entries exactly, and a
// workgroup computes n/8 + 1 sine-cosine pairs instead of n.
__device__ __forceinline__ void compute_twiddles(float2* tw, int n, int tid, int nthr) {
  if ((n & 7) != 0) {
    for (int m = tid; m < n; m += nthr) {
      double sn, cs;
      sincospi(-2.0 * (double)m / (double)n, &sn, &cs);
      tw[m] = make_float2((float)cs, (float)sn);
    }
    return;
  }
  const int e = n >> 3, qn = n >> 2;
  for (int r = tid; r <= e; r += nthr) {
    double sd, cd;
    sincospi(2.0 * (double)r / (double)n, &sd, &cd);
    const float c = (float)cd, s = (float)sd;
    // exp(-i t) = (cos t, -sin t) for t = q pi/2 + a
    tw[r] = make_float2(c, -s);
    tw[qn + r] = make_float2(-s, -c);
    tw[2 * qn + r] = make_float2(-c, s);
    tw[3 * qn + r] = make_float2(s, c);
    if (r > 0 && r < e) {   // t = q pi/2 - a (r = 0 and r = n/8 coincide with the above)
      tw[qn - r] = make_float2(s, -c);
      tw[2 * qn - r] = make_float2(-c, -s);
      tw[3 * qn - r] = make_float2(-s, c);
      tw[n - r] = make_float2(c, s);
    }
  }
}

// The table copy in two steps, so that a kernel can issue its data loads in
// between and the two wait on memory together: tw_begin issues this thread's
// loads of the table of length n (at most kTwFetch entries a thread), or
// evaluates the twiddles when n has no table or the workgroup is too small;
// tw_end writes the fetched entries to LDS.
constexpr int kTwFetch = 4;
struct TwFetch {
  float2 v[kTwFetch];
  bool fetched;
};
__device__ __forceinline__ void tw_begin(TwFetch& f, float2* tw, int n, int tid, int nthr) {
  const int off = tw_offset(n);
  f.fetched = off >= 0 && n <= kTwFetch * nthr;
  if (!f.fetched) {
    compute_twiddles(tw, n, tid, nthr);
    return;
  }
#pragma unroll
  for (int i = 0; i < kTwFetch; ++i) {
    const int m = tid + i * nthr;
    if (m < n) {
      const TwPair p = kTwTables.v[off + m];
      f.v[i] = make_float2(p.c, p.s);
    }
  }
}
__device__ __forceinline__ void tw_end(const TwFetch& f, float2* tw, int n, int tid, int nthr) {
  if (!f.fetched) return;
#pragma unroll
  for (int i = 0; i < kTwFetch; ++i) {
    const int m = tid + i * nthr;
    if (m < n) tw[m] = f.v[i];
  }
}
// The whole table of length n in LDS (visible after the caller's next
// barrier), evaluated: for kernels that cannot overlap a table copy with
// their own loads (a copy waited on at once costs them more than the FP64
// evaluation, e.g. the TF field pass at 384 points: 55 -> 58 us).
__device__ __forceinline__ void fill_twiddles(float2* tw, int n, int tid, int nthr) {
  compute_twiddles(tw, n, tid, nthr);
}

// Cooperative copy of `total` (<= kEmax * nthr) elements into LDS, element e
// taken from src(e).  Every load of a thread is issued before its LDS stores,
// so the loads of one thread are in flight together.
template <int EM = kEmax, typename F>
__device__ __forceinline__ void gather_to_lds(float2* buf, int total, int tid, int nthr, F src) {
  float2 t[EM];
#pragma unroll
  for (int i = 0; i < EM; ++i) {
    const int e = tid + i * nthr;
    if (e < total) t[i] = src(e);
  }
#pragma unroll
  for (int i = 0; i < EM; ++i) {
    const int e = tid + i * nthr;
    if (e < total) buf[e] = t[i];
  }
}

// As above, running mid() after the loads are issued and before the LDS stores
// (e.g. to generate twiddles while the loads are in flight).
template <typename F, typename G>
__device__ __forceinline__ void gather_to_lds(float2* buf, int total, int tid, int nthr, F src,
                                              G mid) {
  float2 t[kEmax];
#pragma unroll
  for (int i = 0; i < kEmax; ++i) {
    const int e = tid + i * nthr;
    if (e < total) t[i] = src(e);
  }
  mid();
#pragma unroll
  for (int i = 0; i < kEmax; ++i) {
    const int e = tid + i * nthr;
    if (e < total) buf[e] = t[i];
  }
}

// As gather_to_lds, element e stored at buf[slot(e)].
template <typename F, typename S, typename G>
__device__ __forceinline__ void gather_to_lds_map(float2* buf, int total, int tid, int nthr, F src,
                                                  S slot, G mid) {
  float2 t[kEmax];
#pragma unroll
  for (int i = 0; i < kEmax; ++i) {
    const int e = tid + i * nthr;
    if (e < total) t[i] = src(e);
  }
  mid();
#pragma unroll
  for (int i = 0; i < kEmax; ++i) {
    const int e = tid + i * nthr;
    if (e < total) buf[slot(e)] = t[i];
  }
}

// Two-phase gather: load(e) only issues the global loads of element e and
// returns them raw; finish(e, raw) turns them into the LDS value after every
// load of the thread has been issued.  Data-dependent branches or uses of a
// loaded value inside load() would make the compiler wait for each load in
// turn; keep them in finish().
template <typename L, typename F, typename S, typename G>
__device__ __forceinline__ void gather2_to_lds(float2* buf, int total, int tid, int nthr, L load,
                                               F finish, S slot, G mid) {
  using T = decltype(load(0));
  T t[kEmax];
#pragma unroll
  for (int i = 0; i < kEmax; ++i) {
    const int e = tid + i * nthr;
    if (e < total) t[i] = load(e);
  }
  mid();
#pragma unroll
  for (int i = 0; i < kEmax; ++i) {
    const int e = tid + i * nthr;
    if (e < total) buf[slot(e)] = finish(e, t[i]);
  }
}

// As scatter_from_lds, element e read from buf[slot(e)].
template <typename F, typename S>
__device__ __forceinline__ void scatter_from_lds_map(const float2* buf, int total, int tid, int nthr,
                                                     S slot, F dst) {
  float2 t[kEmax];
#pragma unroll
  for (int i = 0; i < kEmax; ++i) {
    const int e = tid + i * nthr;
    if (e < total) t[i] = buf[slot(e)];
  }
#pragma unroll
  for (int i = 0; i < kEmax; ++i) {
    const int e = tid + i * nthr;
    if (e < total) dst(e, t[i]);
  }
}

// Cooperative write-out of `total` (<= kEmax * nthr) elements: dst(e, value).
template <typename F>
__device__ __forceinline__ void scatter_from_lds(const float2* buf, int total, int tid, int nthr,
                                                 F dst) {
  float2 t[kEmax];
#pragma unroll
  for (int i = 0; i < kEmax; ++i) {
    const int e = tid + i * nthr;
    if (e < total) t[i] = buf[e];
  }
#pragma unroll
  for (int i = 0; i < kEmax; ++i) {
    const int e = tid + i * nthr;
    if (e < total) dst(e, t[i]);
  }
}

// Line layout in LDS: element i of line l lives at lds[line_base(l) + i * es].
// linefast == true maps consecutive butterfly slots to consecutive lines
// (use when lines are adjacent in LDS, es = number of lines); otherwise
// consecutive slots walk along a line (use for row layouts, es = 1).
struct LdsLines {
  int nl;     // number of lines
  int es;     // element stride
  int ls;     // line stride
  bool linefast;
  int shift = -1;   // log2(nl) when nl is a power of two (slot -> line by masks), else -1
  bool pad = false; // padded row layout (see row_slot)
};

// Row layout (lines contiguous in LDS): element i of a line of length n sits
// at row_slot(i, pad_shift(n)) = i + (i >> pad_shift(n)), one padding slot per
// 8 or 16 elements.  LDS serves a 64-bit access 16 lanes at a time over 32
// four-byte banks.  A Stockham pass writes its first outputs with a stride of
// R elements (16 R bytes, every lane of a group on the same banks); the
// padding staggers them.  One slot per 16 elements keeps 16 consecutive
// elements (a unit-stride access) on 32 distinct banks; one per 8 splits such
// groups but suits short rows (measured: 512-point rows run about 3 % faster
// with 16, the 128-point backward rows of the auto-tune 7 % faster with 8).
// row_stride(n) is the line pitch that holds n padded elements.
__host__ __device__ constexpr int pad_shift(int n) { return n <= 128 ? 3 : 4; }
__host__ __device__ __forceinline__ int row_slot(int i, int ps) { return i + (i >> ps); }
__host__ __device__ __forceinline__ int row_stride(int n) { return n + (n >> pad_shift(n)) + 1; }

// log2(n) for a power of two n, else -1.
__host__ __device__ inline int pow2_shift(int n) {
  if (n <= 0 || (n & (n - 1))) return -1;
  int s = 0;
  while ((1 << s) < n) ++s;
  return s;
}

// Twiddles w^r (r < R) of one butterfly from w = w1: products of lower powers
// (at most three deep), so a butterfly reads one table entry instead of R - 1.
template <int R>
__device__ __forceinline__ void twiddle_powers(float2 (&w)[R], float2 w1) {
  w[0] = make_float2(1.f, 0.f);
  if constexpr (R > 1) w[1] = w1;
#pragma unroll
  for (int r = 2; r < R; ++r) w[r] = cmul(w[r / 2], w[r - r / 2]);
}

template <int R>
__device__ __forceinline__ void stockham_pass(float2* lds, const LdsLines L, int n, int ns,
                                              const float2* tw, float s, int tid, int nthr) {
  constexpr int BPT = (kEmax + R - 1) / R;
  const int nb = n / R;
  const int total = L.nl * nb;
  const int twstep = n / (ns * R);
  float2 v[BPT][R];
  int base[BPT], kk[BPT];
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = tid + b * nthr;
    base[b] = -1;
    if (j < total) {
      int l, k;
      if (L.linefast) {
        if (L.shift >= 0) { l = j & (L.nl - 1); k = j >> L.shift; }
        else { l = j % L.nl; k = j / L.nl; }
      } else { k = j % nb; l = j / nb; }
      const int lb = l * L.ls;
      const int km = k % ns;
      base[b] = lb;
      kk[b] = k;
      float2 w[R];
      if (ns > 1) {
        float2 w1 = tw[km * twstep];
        if (s > 0.f) w1.y = -w1.y;
        twiddle_powers<R>(w, w1);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int idx = k + r * nb;
        float2 x = lds[lb + (L.pad ? row_slot(idx, pad_shift(n)) : idx * L.es)];
        if (r > 0 && ns > 1) x = cmul(x, w[r]);
        v[b][r] = x;
      }
      dft_small<R>(v[b], s);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    if (base[b] >= 0) {
      const int k = kk[b];
      const int d0 = (k / ns) * ns * R + (k % ns);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int idx = d0 + r * ns;
        lds[base[b] + (L.pad ? row_slot(idx, pad_shift(n)) : idx * L.es)] = v[b][r];
      }
    }
  }
  __syncthreads();
}

// In-place FFT of all lines.  Caller must have synchronised after filling LDS
// (data and twiddles).  s = -1 forward, +1 inverse (unnormalised).
__device__ __forceinline__ void lds_fft(float2* lds, const LdsLines L, const FftPlan& p,
                                        const float2* tw, float s, int tid, int nthr) {
  int ns = 1;
  for (int q = 0; q < p.npass; ++q) {
    const int R = plan_radix(p, q);
    switch (R) {
      case 8: stockham_pass<8>(lds, L, p.n, ns, tw, s, tid, nthr); break;
      case 4: stockham_pass<4>(lds, L, p.n, ns, tw, s, tid, nthr); break;
      case 2: stockham_pass<2>(lds, L, p.n, ns, tw, s, tid, nthr); break;
      case 3: stockham_pass<3>(lds, L, p.n, ns, tw, s, tid, nthr); break;
      case 5: stockham_pass<5>(lds, L, p.n, ns, tw, s, tid, nthr); break;
      default: break;
    }
    ns *= R;
  }
}

// Workgroup index remapped so that each XCD (accelerator die, own L2) runs a
// contiguous range of logical indices: the hardware hands workgroups to the 8
// XCDs in turn, so physical index b runs on XCD b % 8.  Neighbouring column
// tiles then share an L2 and the halves of cache lines they split.
constexpr unsigned kXcds = 8;
__device__ __forceinline__ long xcd_block() {
  const unsigned n = gridDim.x, b = blockIdx.x;
  const unsigned q = n / kXcds, r = n % kXcds;
  const unsigned x = b % kXcds, k = b / kXcds;
  return (long)(x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k);
}

// Sum of p[0..n) by wave 0 of the workgroup in a fixed order (lane-strided
// sums, then a shuffle tree); lane 0 stores it to *out, other waves return at
// once.  Called between issuing a tile's loads and storing them to LDS, its
// loads overlap theirs.  The caller synchronises before reading *out.
__device__ __forceinline__ void wave0_sum(const double* p, long n, double* out) {
  if (threadIdx.x >= 64) return;
  double v = 0.0;
  for (long i = threadIdx.x; i < n; i += 64) v += p[i];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (threadIdx.x == 0) *out = v;
}

// ---------------------------------------------------------------- optics

enum Model { kFluor3D = 0, kLabelFree3D = 1, kLabelFreeThin = 2, kPol5 = 3, kSectors9 = 4 };

// Per-patch optical parameters on the device (float64).  ``ibg`` is written
// by the pupil-sum kernel: sum S P^2 (label-free) or sum P^2 (fluorescence).
struct DevOptics {
  double wavelength, na_ill, na_det, n_medium;
  double defocus, tilt_zenith, tilt_azimuth;
  double edge_width;       // half-width of the soft edge, in frequency pixels
  double ibg;
  int sector;              // illumination aperture: -1 the full disc, 0..7 an azimuthal sector
  float zern[7];           // detection aberration, waves, Noll j = 5..11
  double det_tilt, det_azimuth;   // oblique detection: zenith and azimuth of the detection axis
};

// Polarisation coupling kappa_cp of one patch in FP32, (re, im) per channel c
// and property p: the values every kernel that forms the 5 x 4 bank uses.
struct Coupling {
  float k[5][4][2];
  // Gram constants of the 4 x 4 solve from the reduced bank, lower triangles
  // (entry p (p + 1) / 2 + q, q <= p): A = Kr^T Kr, B = Ki^T Ki, S = G + G^T,
  // D = G - G^T with G = Kr^T Ki, Kr = Re kappa, Ki = Im kappa (5 x 4 each)
  float a[10], b[10], s[10], d[10];
};

// One entry of the polarisation bank from the label-free pair at a frequency:
// H_cp = Re(kappa_cp) H_phase + Im(kappa_cp) H_abs (the paraxial Jones
// reduction of Table 1's vector row).  Each product and the sum are rounded
// on their own (no fused multiply-add), so the bank expansion, the fused Z
// pass and a plain FP32 evaluation on the host give the same bits.
__device__ __forceinline__ float2 pol5_entry(float kr, float ki, float2 hp, float2 ha) {
#pragma clang fp contract(off)
  return make_float2(kr * hp.x + ki * ha.x, kr * hp.y + ki * ha.y);
}

// Cholesky factor of M + eta I = L L^H for a Hermitian positive semi-definite
// M given by its lower triangle (m[p][q], q <= p): L below the diagonal and
// the reciprocals of its diagonal, which is all the solves use, so each comes
// from one hardware reciprocal square root (about 1 ulp) instead of a
// correctly rounded square root and division (some 26 instructions).
template <int P>
__device__ __forceinline__ void chol_factor(const float2 (&m)[P][P], float eta, float2 (&L)[P][P],
                                            float (&dinv)[P]) {
#pragma unroll
  for (int j = 0; j < P; ++j) {
    float d = m[j][j].x + eta;
#pragma unroll
    for (int k = 0; k < j; ++k) d -= L[j][k].x * L[j][k].x + L[j][k].y * L[j][k].y;
    dinv[j] = __builtin_amdgcn_rsqf(fmaxf(d, 1e-37f));
#pragma unroll
    for (int i = j + 1; i < P; ++i) {
      float2 v = m[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) v = csub(v, cmulconj(L[i][k], L[j][k]));
      L[i][j] = cscale(v, dinv[j]);
    }
  }
}

// F = (L L^H)^-1 r by the two triangular solves.
template <int P>
__device__ __forceinline__ void chol_apply(const float2 (&L)[P][P], const float (&dinv)[P],
                                           const float2 (&r)[P], float2 (&F)[P]) {
  float2 y[P];
#pragma unroll
  for (int i = 0; i < P; ++i) {
    float2 v = r[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v = csub(v, cmul(L[i][k], y[k]));
    y[i] = cscale(v, dinv[i]);
  }
#pragma unroll
  for (int i = P - 1; i >= 0; --i) {
    float2 v = y[i];
#pragma unroll
    for (int k = i + 1; k < P; ++k) v = csub(v, cmul(cconj(L[k][i]), F[k]));
    F[i] = cscale(v, dinv[i]);
  }
}

// (M + eta I) F = r.
template <int P>
__device__ __forceinline__ void chol_solve(const float2 (&m)[P][P], const float2 (&r)[P], float eta,
                                           float2 (&F)[P]) {
  float2 L[P][P];
  float dinv[P];
  chol_factor<P>(m, eta, L, dinv);
  chol_apply<P>(L, dinv, r, F);
}

// Detection aberration W(p) in waves: sum of zern[j - 5] Z_j over Noll's
// unit-RMS Zernike polynomials j = 5..11 at rho = |p| / (NA_det / lambda0),
// with cos(m phi), sin(m phi) formed from p / |p| (phi = atan2(p_y, p_x)).
__host__ __device__ inline double aberration_waves(const DevOptics& o, double fy, double fx) {
  bool any = false;
  for (int j = 0; j < 7; ++j) any |= o.zern[j] != 0.f;
  if (!any) return 0.0;
  const double pr = sqrt(fy * fy + fx * fx);
  const double r = pr / (o.na_det / o.wavelength), r2 = r * r, r3 = r2 * r;
  const double s1 = pr > 0.0 ? fy / pr : 0.0, c1 = pr > 0.0 ? fx / pr : 1.0;
  const double s2 = 2.0 * s1 * c1, c2 = c1 * c1 - s1 * s1;            // sin, cos of 2 phi
  const double s3 = s2 * c1 + c2 * s1, c3 = c2 * c1 - s2 * s1;        // sin, cos of 3 phi
  const double k6 = 2.449489742783178, k8 = 2.8284271247461903, k5 = 2.23606797749979;
  const double coma = k8 * (3.0 * r3 - 2.0 * r);
  return o.zern[0] * k6 * r2 * s2 + o.zern[1] * k6 * r2 * c2 + o.zern[2] * coma * s1 +
         o.zern[3] * coma * c1 + o.zern[4] * k8 * r3 * s3 + o.zern[5] * k8 * r3 * c3 +
         o.zern[6] * k5 * (6.0 * r2 * r2 - 6.0 * r2 + 1.0);
}

// The seven polynomials Z_5..Z_11 at p (zj) and dW/dNA_det of the aberration
// (W depends on NA_det through rho = |p| lambda0 / NA_det: dW/dNA = -(rho /
// NA) sum_j c_j dZ_j/drho).
__host__ __device__ inline void zernike_terms(const DevOptics& o, double fy, double fx, double zj[7],
                                              double* dw_dna) {
  const double pr = sqrt(fy * fy + fx * fx);
  const double r = pr / (o.na_det / o.wavelength), r2 = r * r, r3 = r2 * r;
  const double s1 = pr > 0.0 ? fy / pr : 0.0, c1 = pr > 0.0 ? fx / pr : 1.0;
  const double s2 = 2.0 * s1 * c1, c2 = c1 * c1 - s1 * s1;
  const double s3 = s2 * c1 + c2 * s1, c3 = c2 * c1 - s2 * s1;
  const double k6 = 2.449489742783178, k8 = 2.8284271247461903, k5 = 2.23606797749979;
  zj[0] = k6 * r2 * s2;
  zj[1] = k6 * r2 * c2;
  zj[2] = k8 * (3.0 * r3 - 2.0 * r) * s1;
  zj[3] = k8 * (3.0 * r3 - 2.0 * r) * c1;
  zj[4] = k8 * r3 * s3;
  zj[5] = k8 * r3 * c3;
  zj[6] = k5 * (6.0 * r2 * r2 - 6.0 * r2 + 1.0);
  const double d[7] = {2.0 * k6 * r * s2, 2.0 * k6 * r * c2, k8 * (9.0 * r2 - 2.0) * s1,
                       k8 * (9.0 * r2 - 2.0) * c1, 3.0 * k8 * r2 * s3, 3.0 * k8 * r2 * c3,
                       k5 * (24.0 * r3 - 12.0 * r)};
  double dw = 0.0;
  for (int j = 0; j < 7; ++j) dw += o.zern[j] * d[j];
  *dw_dna = -(r / o.na_det) * dw;
}

// Azimuthal sector k of the direction (dy, dx): the azimuth, from +x towards +y,
// lies in [k pi/4, (k+1) pi/4); the origin is in sector 0.  Comparisons only.
__host__ __device__ __forceinline__ int octant(double dy, double dx) {
  if (dy == 0.0 && dx == 0.0) return 0;
  if (dy >= 0.0 && dx > 0.0) return dy < dx ? 0 : 1;
  if (dx <= 0.0 && dy > 0.0) return dy > -dx ? 2 : 3;
  if (dy <= 0.0 && dx < 0.0) return dy > dx ? 4 : 5;
  return dx < -dy ? 6 : 7;
}

// Auto-tune state of one (virtual) patch: Adam moments and hyper-parameters,
// Tikhonov eta, the mid-band cutoff and band size, and the last loss/gradient.
struct TuneState {
  double m[4], v[4];
  double lr[4], lo[4], hi[4];
  double eta, nu_c, band_count;
  double loss, grad[6];    // defocus, na_det, tilt_zenith, tilt_azimuth, det_tilt, det_azimuth
  double gab[7];   // dL / d zernike[j] (filled when the gradient is aberration-aware)
  // Adam on the aberration coefficients (mask bits 4..10): moments, one rate
  // and the box [-bound, bound] shared by the seven
  double mab[7], vab[7], lr_ab, bound_ab;
  int t, mask;
  int pad[2];
};

// Gradient components per partial: theta (4), then the 7 aberration coefficients
// when the gradient kernels run aberration-aware.
constexpr int kGradAll = 13;
// Parameter gradient components before the aberration coefficients: theta
// (4), then the detection axis (2) when the gradient kernels compute them.
constexpr int kThetaAll = 6;

// Sampling shared by every patch of a call.
struct Sampling {
  int model;
  int nz, ny, nx;
  double dz, dy, dx;
  int aberrated = 0;   // some patch has detection aberrations (selects the kernel variant)
  int det_grad = 0;    // the gradient kernels also form d/d(det_tilt, det_azimuth)
};

__host__ __device__ __forceinline__ double fftfreq(int k, int n, double d) {
  const double val = 1.0 / ((double)n * d);
  const int ks = (k < (n + 1) / 2) ? k : k - n;
  return (double)ks * val;
}

// e / d for 0 <= e < 2^20 and 1 <= d <= 2^13, given inv_d = 1.0f / d: the exact
// quotient of e + 0.5 lies at least 0.5 / d from an integer, far more than the
// rounding error of the float product (a runtime integer division costs
// dozens of instructions per element).
__device__ __forceinline__ int div_small(int e, float inv_d) {
  return (int)(((float)e + 0.5f) * inv_d);
}

// Compact column layout of a band-limited lateral axis: of the X frequency
// columns only kx <= KP (zero and positive frequencies) and the XC - KP - 1
// highest (negative frequencies) are stored; column c holds kx = c for
// c <= KP and kx = c + X - XC beyond.  XC = X with KP = X - 1 is the plain
// layout.  compact_column is the inverse (-1: a column that is not stored).
__host__ __device__ __forceinline__ int field_column(int c, int KP, int X, int XC) {
  return c <= KP ? c : c + (X - XC);
}
__host__ __device__ __forceinline__ int compact_column(int kx, int KP, int X, int XC) {
  return kx <= KP ? kx : (kx >= X - (XC - KP - 1) ? kx - (X - XC) : -1);
}

__host__ __device__ __forceinline__ double edge_profile(double inside, double hw) {
  if (hw == 0.0) return inside >= 0.0 ? 1.0 : 0.0;
  double t = (inside / hw + 1.0) * 0.5;
  t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
  return t * t * (3.0 - 2.0 * t);
}

// d edge / d inside (0 for the hard edge)
__device__ __forceinline__ double edge_slope(double inside, double hw) {
  if (hw == 0.0) return 0.0;
  const double t = (inside / hw + 1.0) * 0.5;
  if (t <= 0.0 || t >= 1.0) return 0.0;
  return 6.0 * t * (1.0 - t) * (0.5 / hw);
}

__host__ __device__ __forceinline__ double disc(double fy, double fx, double radius, double hw) {
  const double r2 = fy * fy + fx * fx;
  if (hw == 0.0) return r2 <= radius * radius ? 1.0 : 0.0;
  return edge_profile(radius - sqrt(r2), hw);
}

// Detection pupil (Ext. Data Fig. 3b, calc_det_pupil): the disc of radius
// NA_det / lambda0 or, with oblique detection, the cap of the shell within that
// NA about the detection axis a tilted by det_tilt in the azimuth det_azimuth,
// a = (sin t sin az, sin t cos az, cos t) in (y, x, z): P = edge(NA_det/lambda0 - |p'|)
// with |p'|^2 = k_m^2 - (k . a)^2 the lateral distance in the tilted frame,
// k = (p, kz(p)), and k . a > 0.
struct DetAxis {
  double ay, ax, az;
};
__host__ __device__ __forceinline__ DetAxis det_axis(const DevOptics& o) {
  const double st = sin(o.det_tilt);
  return DetAxis{st * sin(o.det_azimuth), st * cos(o.det_azimuth), cos(o.det_tilt)};
}

__host__ __device__ __forceinline__ double det_pupil(const DevOptics& o, const DetAxis& a, double fy,
                                                     double fx, double hw) {
  const double rd = o.na_det / o.wavelength;
  if (o.det_tilt == 0.0) return disc(fy, fx, rd, hw);
  const double km = o.n_medium / o.wavelength;
  const double p2 = fy * fy + fx * fx;
  if (!(p2 < km * km)) return 0.0;
  const double kz = sqrt(km * km - p2);
  const double ka = fy * a.ay + fx * a.ax + kz * a.az;
  if (!(ka > 0.0)) return 0.0;
  const double pp2 = km * km - ka * ka;
  if (hw == 0.0) return pp2 <= rd * rd ? 1.0 : 0.0;
  return edge_profile(rd - sqrt(fmax(pp2, 0.0)), hw);
}

// Partial derivatives of det_pupil with respect to NA_det, det_tilt and
// det_azimuth: P = edge(rd - |p'|), d|p'| = -(k . a)(k . da) / |p'| (all zero
// for the hard edge).
__device__ __forceinline__ void det_pupil_derivs(const DevOptics& o, const DetAxis& a, double fy,
                                                 double fx, double hw, double* dna, double* dt,
                                                 double* daz) {
  *dna = *dt = *daz = 0.0;
  const double km = o.n_medium / o.wavelength;
  const double p2 = fy * fy + fx * fx;
  if (!(p2 < km * km) || hw == 0.0) return;
  const double kz = sqrt(km * km - p2);
  const double ka = fy * a.ay + fx * a.ax + kz * a.az;
  if (!(ka > 0.0)) return;
  const double pp = sqrt(fmax(km * km - ka * ka, 0.0));
  const double sl = edge_slope(o.na_det / o.wavelength - pp, hw);
  *dna = sl / o.wavelength;
  if (sl == 0.0 || !(pp > 0.0)) return;
  const double ct = cos(o.det_tilt), st = sin(o.det_tilt);
  const double ca = cos(o.det_azimuth), sa = sin(o.det_azimuth);
  const double kdt = fy * ct * sa + fx * ct * ca - kz * st;   // k . da/dt
  const double kda = fy * st * ca - fx * st * sa;             // k . da/daz
  *dt = sl * ka * kdt / pp;
  *daz = sl * ka * kda / pp;
}

// Radius about p = 0 of a disc holding the detection pupil (without its soft
// edge): NA_det / lambda0, or k_m sin(det_tilt + asin(NA_det / n)).
__host__ __device__ __forceinline__ double det_radius(const DevOptics& o) {
  if (o.det_tilt == 0.0) return o.na_det / o.wavelength;
  const double a = fabs(o.det_tilt) + asin(fmin(o.na_det / o.n_medium, 1.0));
  return (o.n_medium / o.wavelength) * (a < 0.5 * M_PI ? sin(a) : 1.0);
}

__device__ __forceinline__ double soft_halfwidth(const DevOptics& o, const Sampling& sm) {
  const double dnu = fmin(1.0 / ((double)sm.nx * sm.dx), 1.0 / ((double)sm.ny * sm.dy));
  return o.edge_width * dnu;
}

__host__ __device__ __forceinline__ void source_centre(const DevOptics& o, double* cy, double* cx) {
  const double r = o.n_medium * sin(o.tilt_zenith) / o.wavelength;
  *cy = r * sin(o.tilt_azimuth);
  *cx = r * cos(o.tilt_azimuth);
}

// Axial PSF coordinate of plane k: FFT order for 3D models, centred planes for thin.
// Plane chunks of the field kernel: runs of at most ZC consecutive planes that
// never cross the jump of the wrapped axial order (3D models: plane
// (nz + 1) / 2 follows the last non-negative z), so within a chunk the plane
// position advances by dz from one plane to the next.
__host__ __device__ __forceinline__ int z_split(const Sampling& sm) {
  return sm.model == kLabelFreeThin ? 0 : (sm.nz + 1) / 2;
}
__host__ __device__ __forceinline__ int z_chunk_count(int Z, int zs, int ZC) {
  return (zs + ZC - 1) / ZC + (Z - zs + ZC - 1) / ZC;
}
__host__ __device__ __forceinline__ void z_chunk_range(int Z, int zs, int ZC, int zc, int* zb, int* ze) {
  const int n1 = (zs + ZC - 1) / ZC;
  if (zc < n1) {
    *zb = zc * ZC;
    *ze = *zb + ZC < zs ? *zb + ZC : zs;
  } else {
    *zb = zs + (zc - n1) * ZC;
    *ze = *zb + ZC < Z ? *zb + ZC : Z;
  }
}

__device__ __forceinline__ double plane_z(int k, const Sampling& sm) {
  if (sm.model == kLabelFreeThin) return sm.dz * ((double)k - 0.5 * (double)(sm.nz - 1));
  const int ks = (k < (sm.nz + 1) / 2) ? k : k - sm.nz;
  return sm.dz * (double)ks;
}

}  // namespace wo

namespace wo {

// ---------------------------------------------------------------- static-length FFT
//
// The same Stockham passes with the length, radices, spans and (optionally)
// the line count fixed at compile time, so index arithmetic becomes constants
// and shifts.  Used for the transform lengths of the workloads; other lengths
// take the runtime plan above.

template <int N, bool W16 = false>
struct StaticPlan {
  // radices in the order 8, 4, 6, 2, 3, 5: a radix-6 butterfly (two radix-3
  // DFTs in registers) replaces a radix-2 and a radix-3 pass, one LDS round
  // trip fewer (384 = 8 8 6, 240 = 8 6 5, 48 = 8 6)
  // W16, for 2^t with t = 3a + 1 >= 7 (128, 1024): 8 ... 8 then 16, one LDS
  // round trip fewer than 8 ... 8 then 2, for kernels with the registers for
  // a 16-point butterfly (about 20 more VGPRs)
  static constexpr bool last16() {
    int t = 0;
    while ((1 << t) < N) ++t;
    return W16 && (1 << t) == N && t >= 7 && t % 3 == 1;
  }
  static constexpr int radix(int q) {
    if (last16()) {
      int t = 0;
      while ((1 << t) < N) ++t;
      const int np = (t - 4) / 3 + 1;
      return q < np - 1 ? 8 : (q == np - 1 ? 16 : 0);
    }
    int m = N, p = 0;
    const int order[6] = {8, 4, 6, 2, 3, 5};
    for (int i = 0; i < 6; ++i) {
      const int f = order[i];
      while (m % f == 0) {
        if (p == q) return f;
        m /= f;
        ++p;
      }
    }
    return 0;
  }
  static constexpr int passes() {
    int p = 0;
    while (radix(p)) ++p;
    return p;
  }
  static constexpr int span(int q) {
    int s = 1;
    for (int i = 0; i < q; ++i) s *= radix(i);
    return s;
  }
};

template <int N, int R, int NS, int NL, bool LF, int EM, bool PD>
__device__ __forceinline__ void static_pass(float2* lds, int nl_rt, int es, int ls, int shift,
                                            const float2* tw, float s, int tid, int nthr) {
  constexpr int NB = N / R;
  constexpr int BPT = (EM + R - 1) / R;
  constexpr int TWS = N / (NS * R);
  const int nl = NL > 0 ? NL : nl_rt;
  const int total = nl * NB;
  float2 v[BPT][R];
  int base[BPT], kk[BPT];
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = tid + b * nthr;
    base[b] = -1;
    if (j < total) {
      int l, k;
      if (LF) {
        if (NL == 0 && shift >= 0) { l = j & (nl - 1); k = j >> shift; }
        else { l = j % nl; k = j / nl; }
      } else { k = j % NB; l = j / NB; }
      const int lb = l * ls;
      const int km = k % NS;
      base[b] = lb;
      kk[b] = k;
      float2 w[R];
      if constexpr (NS > 1) {
        float2 w1 = tw[km * TWS];
        if (s > 0.f) w1.y = -w1.y;
        twiddle_powers<R>(w, w1);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int idx = k + r * NB;
        float2 x = lds[lb + (PD ? row_slot(idx, pad_shift(N)) : idx * es)];
        if constexpr (NS > 1) {
          if (r > 0) x = cmul(x, w[r]);
        }
        v[b][r] = x;
      }
      dft_small<R>(v[b], s);
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    if (base[b] >= 0) {
      const int k = kk[b];
      const int d0 = (k / NS) * NS * R + (k % NS);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int idx = d0 + r * NS;
        lds[base[b] + (PD ? row_slot(idx, pad_shift(N)) : idx * es)] = v[b][r];
      }
    }
  }
  __syncthreads();
}

template <int N, int NL, bool LF, int EM, bool PD, int Q = 0>
__device__ __forceinline__ void static_fft(float2* lds, int nl_rt, int es, int ls, int shift,
                                           const float2* tw, float s, int tid, int nthr) {
  if constexpr (Q < StaticPlan<N>::passes()) {
    static_pass<N, StaticPlan<N>::radix(Q), StaticPlan<N>::span(Q), NL, LF, EM, PD>(
        lds, nl_rt, es, ls, shift, tw, s, tid, nthr);
    static_fft<N, NL, LF, EM, PD, Q + 1>(lds, nl_rt, es, ls, shift, tw, s, tid, nthr);
  }
}

// Radix order of the compiled stages, forward (REV false) or reversed.  Any
// order is a valid Stockham sequence (the span of a pass is the product of the
// radices before it); a transform in reversed order ends with a pass whose
// outputs, k + r N/R0, are the inputs of the first pass (radix R0, span 1) of
// a transform in forward order, so the two can meet in registers.
template <int N, bool REV, bool W16 = false>
struct OrderedPlan {
  static constexpr int passes() { return StaticPlan<N, W16>::passes(); }
  static constexpr int radix(int q) { return StaticPlan<N, W16>::radix(REV ? passes() - 1 - q : q); }
  static constexpr int span(int q) {
    int s = 1;
    for (int i = 0; i < q; ++i) s *= radix(i);
    return s;
  }
};

// Passes [Q, QE) of the compiled transform of length N in the given order.
template <int N, int NL, bool LF, int EM, bool PD, bool REV, int Q, int QE, bool W16 = false>
__device__ __forceinline__ void static_passes(float2* lds, int nl_rt, int es, int ls, int shift,
                                              const float2* tw, float s, int tid, int nthr) {
  if constexpr (Q < QE) {
    using PL = OrderedPlan<N, REV, W16>;
    static_pass<N, PL::radix(Q), PL::span(Q), NL, LF, EM, PD>(lds, nl_rt, es, ls, shift, tw, s, tid,
                                                             nthr);
    static_passes<N, NL, LF, EM, PD, REV, Q + 1, QE, W16>(lds, nl_rt, es, ls, shift, tw, s, tid, nthr);
  }
}

// First and last pass of a compiled transform through registers.
//
// first_pass_in: the first pass (span 1, no twiddles) of the lines of length N
// in the given radix order takes its inputs from load(l, i) (line l, element
// i; first_pass_in2: finish(l, i, load(l, i)), finish applied after every load
// of the thread is issued) and writes its outputs to LDS (layout as in LdsLines: line base l * ls,
// element i at i * es, or the padded row slot); load() is called for every
// input of the thread before any butterfly (keep it free of data-dependent
// branches so the loads are in flight together) and mid() runs after the
// loads are issued (fill the twiddle table there or before).  Ends with a
// barrier.
//
// last_pass_out: the last pass reads LDS and hands its outputs to
// store(l, i, v) (memory or registers, not the same LDS: other threads may
// still read it).  Ends with a barrier.
//
// Between them static_passes runs the passes in LDS; fft_direct is the three
// together, which halves the LDS traffic of a three-pass length.
template <int N, int NL, bool LF, bool PD>
__device__ __forceinline__ void line_of(int j, int nl, int nb, int shift, int& l, int& k) {
  if (LF) {
    if (NL == 0 && shift >= 0) { l = j & (nl - 1); k = j >> shift; }
    else { l = j % nl; k = j / nl; }
  } else {
    k = j % nb;
    l = j / nb;
  }
}

// The loaded inputs of a thread's first-pass butterflies (B0 butterflies of
// radix R0), held between first_pass_load and first_pass_store.
template <int N, int EM, bool REV, typename T = float2>
struct FirstPassRaw {
  static constexpr int R0 = OrderedPlan<N, REV>::radix(0);
  static constexpr int B0 = (EM + R0 - 1) / R0;
  T v[B0][R0];
};

// Issues every load of the thread's first-pass butterflies (load(l, i) as in
// first_pass_in2).
template <int N, int NL, bool LF, int EM, bool PD, bool REV, typename T, typename LD>
__device__ __forceinline__ void first_pass_load(FirstPassRaw<N, EM, REV, T>& raw, int nl_rt, int shift,
                                                int tid, int nthr, LD load) {
  using FR = FirstPassRaw<N, EM, REV, T>;
  constexpr int NB0 = N / FR::R0;
  const int nl = NL > 0 ? NL : nl_rt;
#pragma unroll
  for (int b = 0; b < FR::B0; ++b) {
    const int j = tid + b * nthr;
    if (j < nl * NB0) {
      int l, k;
      line_of<N, NL, LF, PD>(j, nl, NB0, shift, l, k);
#pragma unroll
      for (int r = 0; r < FR::R0; ++r) raw.v[b][r] = load(l, k + r * NB0);
    }
  }
}

// The first pass on loaded inputs (finish(l, i, v) applied to each) into LDS;
// ends with a barrier.
template <int N, int NL, bool LF, int EM, bool PD, bool REV, typename T, typename FIN>
__device__ __forceinline__ void first_pass_store(const FirstPassRaw<N, EM, REV, T>& raw, float2* lds,
                                                 int nl_rt, int es, int ls, int shift, float s, int tid,
                                                 int nthr, FIN finish) {
  using FR = FirstPassRaw<N, EM, REV, T>;
  constexpr int R0 = FR::R0, NB0 = N / R0;
  const int nl = NL > 0 ? NL : nl_rt;
#pragma unroll
  for (int b = 0; b < FR::B0; ++b) {
    const int j = tid + b * nthr;
    if (j < nl * NB0) {
      int l, k;
      line_of<N, NL, LF, PD>(j, nl, NB0, shift, l, k);
      float2 v[R0];
#pragma unroll
      for (int r = 0; r < R0; ++r) v[r] = finish(l, k + r * NB0, raw.v[b][r]);
      dft_small<R0>(v, s);
#pragma unroll
      for (int r = 0; r < R0; ++r)
        lds[l * ls + (PD ? row_slot(k * R0 + r, pad_shift(N)) : (k * R0 + r) * es)] = v[r];
    }
  }
  __syncthreads();
}

template <int N, int NL, bool LF, int EM, bool PD, bool REV, typename LD, typename FIN, typename MID>
__device__ __forceinline__ void first_pass_in2(float2* lds, int nl_rt, int es, int ls, int shift,
                                               float s, int tid, int nthr, LD load, FIN finish,
                                               MID mid) {
  FirstPassRaw<N, EM, REV, decltype(load(0, 0))> raw;
  first_pass_load<N, NL, LF, EM, PD, REV>(raw, nl_rt, shift, tid, nthr, load);
  mid();
  first_pass_store<N, NL, LF, EM, PD, REV>(raw, lds, nl_rt, es, ls, shift, s, tid, nthr, finish);
}

// As first_pass_in2 with the loaded values used as they are.
template <int N, int NL, bool LF, int EM, bool PD, bool REV, typename LD, typename MID>
__device__ __forceinline__ void first_pass_in(float2* lds, int nl_rt, int es, int ls, int shift,
                                              float s, int tid, int nthr, LD load, MID mid) {
  first_pass_in2<N, NL, LF, EM, PD, REV>(lds, nl_rt, es, ls, shift, s, tid, nthr, load,
                                         [](int, int, float2 v) { return v; }, mid);
}

template <int N, int NL, bool LF, int EM, bool PD, bool REV, bool W16 = false, typename ST>
__device__ __forceinline__ void last_pass_out(const float2* lds, int nl_rt, int es, int ls, int shift,
                                              const float2* tw, float s, int tid, int nthr, ST store) {
  using PL = OrderedPlan<N, REV, W16>;
  constexpr int NP = PL::passes();
  constexpr int RL = PL::radix(NP - 1), NSL = N / RL;
  constexpr int BL = (EM + RL - 1) / RL;
  const int nl = NL > 0 ? NL : nl_rt;
  // every butterfly of the thread first, then the stores: a register that a
  // store reads is not reused by the next butterfly, which would make the
  // compiler wait for the stores to complete (vmcnt) between butterflies
  float2 x[BL][RL];
  int ll[BL], kk[BL];
#pragma unroll
  for (int b = 0; b < BL; ++b) {
    const int j = tid + b * nthr;
    kk[b] = -1;
    if (j < nl * NSL) {
      int l, k;
      line_of<N, NL, LF, PD>(j, nl, NSL, shift, l, k);
      float2 w[RL];
      float2 w1 = tw[k];   // span NSL = N / RL: twiddle stride 1
      if (s > 0.f) w1.y = -w1.y;
      twiddle_powers<RL>(w, w1);
#pragma unroll
      for (int r = 0; r < RL; ++r) {
        const int i = k + r * NSL;
        x[b][r] = lds[l * ls + (PD ? row_slot(i, pad_shift(N)) : i * es)];
        if (r > 0) x[b][r] = cmul(x[b][r], w[r]);
      }
      dft_small<RL>(x[b], s);
      ll[b] = l;
      kk[b] = k;
    }
  }
#pragma unroll
  for (int b = 0; b < BL; ++b) {
    if (kk[b] >= 0) {
#pragma unroll
      for (int r = 0; r < RL; ++r) store(ll[b], kk[b] + r * NSL, x[b][r]);
    }
  }
  __syncthreads();
}

template <int N, int NL, bool LF, int EM, bool PD, typename LD, typename MID, typename ST>
__device__ __forceinline__ void fft_direct(float2* lds, int nl_rt, int es, int ls, int shift,
                                           const float2* tw, float s, int tid, int nthr, LD load,
                                           MID mid, ST store) {
  constexpr int NP = StaticPlan<N>::passes();
  static_assert(NP >= 2, "fft_direct needs at least two passes");
  first_pass_in<N, NL, LF, EM, PD, false>(lds, nl_rt, es, ls, shift, s, tid, nthr, load, mid);
  static_passes<N, NL, LF, EM, PD, false, 1, NP - 1>(lds, nl_rt, es, ls, shift, tw, s, tid, nthr);
  last_pass_out<N, NL, LF, EM, PD, false>(lds, nl_rt, es, ls, shift, tw, s, tid, nthr, store);
}

// FFT of the lines described by L: static length NSTAT (> 0) or the runtime plan
// (NSTAT == 0).  NL > 0 fixes the number of lines; LF must equal L.linefast.
// EM bounds the elements a thread owns (lines * n <= threads * EM) for the
// compiled stages; the runtime plan assumes kEmax.
// PD must equal L.pad (the padded row layout).
template <int NSTAT, int NL, bool LF, int EM = kEmax, bool PD = false>
__device__ __forceinline__ void fft_lines(float2* lds, const LdsLines& L, const FftPlan& p,
                                          const float2* tw, float s, int tid, int nthr) {
  if constexpr (NSTAT > 0)
    static_fft<NSTAT, NL, LF, EM, PD>(lds, L.nl, L.es, L.ls, L.shift, tw, s, tid, nthr);
  else
    lds_fft(lds, L, p, tw, s, tid, nthr);
}

}  // namespace wo

// Transform lengths with compiled FFT stages (lateral sizes and axial sizes).
#define WO_LATERAL_SIZES(X) X(64) X(128) X(160) X(192) X(240) X(256) X(320) X(384) X(480) X(512) X(1024)
#define WO_AXIAL_SIZES(X) X(16) X(24) X(32) X(48) X(64) X(96)
#define WO_ALL_SIZES(X) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(160) X(192) X(240) X(256) X(320) X(384) X(480) X(512) X(1024)
