// Host-side launchers shared between the translation units of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <functional>
#include <vector>

#include "common.hpp"

namespace wo {

#define WO_HIP_CHECK(expr)                  \
  do {                                      \
    hipError_t _e = (expr);                 \
    if (_e != hipSuccess) return WO_EHIP;   \
  } while (0)

// Parameter-regression CNN: channels of the 4 convolution blocks and outputs.
constexpr int kCnnLayers = 4;
constexpr int kCnnOut = 3;
constexpr int kCnnChannels[kCnnLayers + 1] = {1, 32, 64, 128, 256};

// Dynamic LDS bytes one workgroup may use on the current device (queried once).
long lds_limit_bytes();

// Optional per-kernel timing: when enabled, launches are bracketed by HIP
// events on their own stream; wo_timing_report() sums the elapsed times.
bool timing_enabled();
void timing_begin(const char* name, hipStream_t s, void** token);
void timing_end(void* token, hipStream_t s);

struct ScopedTiming {
  void* token = nullptr;
  hipStream_t s;
  ScopedTiming(const char* name, hipStream_t st) : s(st) {
    if (timing_enabled()) timing_begin(name, st, &token);
  }
  ~ScopedTiming() {
    if (token) timing_end(token, s);
  }
};

// ---------------------------------------------------------------- FFT plan table
//
// Launch schedule of one FFT pass for one problem shape, chosen by timing
// (wo_fft_tune) or by the default heuristics when the table has no entry.
enum FftKind { kFftRowsR2C = 0, kFftRowsC2R = 1, kFftCols = 2, kFftZop = 3, kFftTfRows = 4,
               kFftTfFields = 5 };
constexpr int kFftKinds = 6;
// plan: 0 = the compiled stages of the length when there are some, else the
// runtime plan in the default radix order; 1 = runtime plan, default order
// (8, 4, 2, 3, 5); 2 = runtime plan, reversed pass order; 3 = runtime plan,
// odd radices first (5, 3, 8, 4, 2).
struct FftKey {
  int kind, n;
  long m, batch;   // cols/zop: columns per plane (M); rows: 0.  batch: rows,
                   // planes or patches of the launch
  int extra;       // zop: P * 1000 + C * 10 + mode
  bool operator<(const FftKey& o) const {
    if (kind != o.kind) return kind < o.kind;
    if (n != o.n) return n < o.n;
    if (m != o.m) return m < o.m;
    if (batch != o.batch) return batch < o.batch;
    return extra < o.extra;
  }
};
struct FftChoice {
  int w;        // rows: lines per workgroup; cols/zop: tile width (columns)
  int threads;  // workgroup size
  int plan;
};
// Table entry for k, if any.
bool fft_lookup(const FftKey& k, FftChoice* c);
void fft_store(const FftKey& k, const FftChoice& c);
// Changes whenever the table changes (graphs captured before are stale).
unsigned long long fft_table_version();
// Every schedule the launcher of k accepts (the first is the default).
// Schedules of the label-free transfer-function row pass (w = rows per
// workgroup, two LDS lines each).
bool tf_rows_choice_ok(int X, const FftChoice& c);
FftChoice tf_rows_default(int X);
// Schedules of the field kernel: w = planes per workgroup (the z-independent
// pupil factors are evaluated once per workgroup), for Z planes, `tiles`
// column tiles and `npatch` field sets (key: n = transform length, m = tiles,
// batch = npatch, extra = Z * 10 + fields).
bool tf_fields_choice_ok(int Z, const FftChoice& c);
FftChoice tf_fields_default(int Z, long tiles, long npatch);
// A workgroup of `thr` threads can own `elems` elements (kEmax per thread).
inline bool threads_ok(int thr, long elems) {
  return thr >= 64 && thr <= kMaxThreads && thr % 64 == 0 && (long)thr * kEmax >= elems;
}
std::vector<FftChoice> fft_candidates(const FftKey& k);
// While a tuning run records, each tunable launch registers its key and a
// closure that repeats it.
bool fft_recording();
void fft_record(const FftKey& k, std::function<hipError_t()> relaunch);
bool make_plan_variant(int n, int variant, FftPlan* p);

// Grouped row addressing: row i of group g lives at row g * stride + i.
struct RowGroups {
  long rows_per_group;
  long in_stride;   // rows between consecutive groups of the input
  long out_stride;  // rows between consecutive groups of the output
  long ngroups;
};

// Real rows -> half-spectrum rows (forward, unnormalised): the columns k < kt
// (0: all X/2 + 1) of each output row, row pitch `pitch` (0: X/2 + 1).
hipError_t launch_rows_r2c(const float* in, float2* out, int X, const RowGroups& g, hipStream_t s,
                           int kt = 0, int pitch = 0, const char* tag = "k_rows_r2c");
// Half-spectrum rows -> real rows times `scale` (inverse); input rows of
// pitch `pitch` hold the columns k < kt, the others are taken as zero.
hipError_t launch_rows_c2r(const float2* in, float* out, int X, const RowGroups& g, float scale,
                           hipStream_t s, int kt = 0, int pitch = 0);
// In-place FFT along the middle axis of planes [N][M]; plane p of group g
// starts at data + (g * group_stride + p) * N * M.
// band: 0 every row; 1 stores only the band rows n <= ky or n >= N - ky of
// the transform; 2 loads only those (the others are taken as zero).
hipError_t launch_cols(float2* data, int N, long M, long planes_per_group, long group_stride,
                       long ngroups, float sign, hipStream_t s, const char* tag = "k_cols",
                       int band = 0, int ky = -1);
// FFT along N of the band rows (y <= ky or y >= rows - ky) of compact planes
// src [g][N][Ys][kt] into the full half-spectrum planes dst [g][N][Y][Xh];
// every other value of dst (rows outside the band, columns kx >= kt) is set
// to zero.  band_out: dst planes hold the band rows only, [g][N][nb][kt] in
// band order (no zeros written).
hipError_t launch_cols_expand(const float2* src, float2* dst, int N, int Ys, int Y, int Xh, int kt,
                              int ky, long ngroups, float sign, hipStream_t s, bool band_out = false);

enum SpectralMode { kModeForward = 0, kModeSolve = 1, kModeAdjoint = 2 };

// Whether one Z line of CH channels fits a workgroup of the fused Z pass.
bool zop_fits(int Z, int CH);
// Lateral band of a compact spectrum: planes of Y rows holding the
// half-spectrum columns k < kt; the band rows are y <= ky and y >= Y - ky.
// bank_band: the bank, too, holds only the band rows (in band order) of kt
// columns per plane instead of Y rows of Xh.
struct SpecBand {
  int Y;
  long kt;
  int ky;
  int bank_band;
};
// 3D: forward Z-FFT, per-frequency op, inverse Z-FFT, fused.  spec holds
// `slots` channel slots of [Z][M] per patch; tf holds [C][P][Z][M] per patch.
// With a band, spec holds `slots` slots of [Z][Y][kt] instead (M = Y * Xh
// stays the bank's plane) and only the band rows' columns k < kt are
// transformed; the rest of spec is left as it is.
// cpl (not NULL; P = 4, C = 5): tf holds the polarisation bank in reduced
// form, [2][Z][..] per patch (H_phase, H_abs) in the layout the band gives, and
// H_cp = pol5_entry(cpl[patch].k[c][p], H_phase, H_abs) is formed per frequency.
hipError_t launch_zop(float2* spec, const float2* tf, int C, int P, int Z, long M, int slots,
                      int npatch, int mode, float eta, const float* bg, float inv_n, double n_full,
                      hipStream_t s, const SpecBand* band = nullptr, const Coupling* cpl = nullptr);
// The 5 x 4 polarisation bank tf [patch][5][4][Z][Y][Xh] from its reduced form
// red [patch][2][Z][nb][kt] (H_phase, H_abs on the band rows of kt columns; nb =
// Y and kt = Xh: the full layout): H_cp = pol5_entry(kappa_cp, ...) on the
// support, exact zeros elsewhere.
hipError_t launch_pol5_mix(const Coupling* cpl, const float2* red, float2* tf, int Z, int Y, int Xh,
                           int kt, int ky, int npatch, hipStream_t s);
// 2D (thin) per-frequency op: spec [slots][M] per patch, tf [C][P][M] per patch.
// eta_pp (device [npatch], may be NULL) overrides eta per patch.
hipError_t launch_op2d(float2* spec, const float2* tf, int C, int P, long M, int slots, int npatch,
                       int mode, float eta, const float* bg, float inv_n, double n_full,
                       hipStream_t s, const float* eta_pp = nullptr);

// Transfer-function synthesis.
hipError_t launch_set_params(DevOptics* dst, const DevOptics* host, int n, hipStream_t s);
// Lateral support of the label-free fields and transfer function.  The field
// kernel stores xc compact columns of its fields (field_column, last
// non-negative column kp); the label-free row kernel writes the transfer
// function's half-spectrum columns kx < kt; the band Z pass transforms rows
// y <= ky or y >= Y - ky (ky = Y: every row).  full_support is the plain
// layout.
// The label-free transfer function is the 2D correlation of the fields' spectra
// A and B, so a transform of ly x lx points (at least the correlation's
// extent) yields it exactly: the field kernel's inverse Y transform has ly
// points, the row kernel's X transforms lx (ly = ny, lx = nx: the grid's own).
// The label-free field A = S P e^{..} vanishes outside the source's support
// too: it is kept on its own xa compact columns (last non-negative column
// kpa), a subset of B's xc columns (xa = xc: the same layout).
struct LatSupport {
  int xc, kp;
  int kt;
  int ky;
  int ly, lx;
  int xa, kpa;
};
inline LatSupport full_support(const Sampling& sm) {
  return LatSupport{sm.nx, sm.nx - 1, sm.nx / 2 + 1, sm.ny, sm.ny, sm.nx, sm.nx, sm.nx - 1};
}
// Column tile width of the field kernel for a transform of ly points (0: ny);
// the pupil-sum partials hold ceil(xc / width) doubles per patch.
int tf_tile_width(const Sampling& sm, int ly = 0);
// Planes per workgroup of the z-chunked field and gradient kernels.
int tf_z_chunk(const Sampling& sm, long tiles_x, long npatch, long target);
hipError_t launch_tf_fields_y(const DevOptics* opt, const Sampling& sm, int npatch, float2* ab,
                              double* partials, hipStream_t s, const LatSupport* sup = nullptr);
// out[patch * patch_stride + p * pstride + z * zstride + y * pitch + k], k < sup->kt
// (pitch: Xh, or sup->kt when the caller keeps the compact columns).
hipError_t launch_tf_rows_labelfree(const double* partials, const Sampling& sm, int npatch,
                                    const float2* ab, float2* out, long patch_stride,
                                    long pstride, long zstride, hipStream_t s,
                                    const LatSupport* sup = nullptr, int pitch = 0);
hipError_t launch_tf_rows_fluor(const double* partials, const Sampling& sm, int npatch,
                                const float2* h, float2* out, hipStream_t s);
hipError_t launch_set_coupling(Coupling* dst, const Coupling* host, int n, hipStream_t s);

// Auto-tune (thin model).
hipError_t launch_set_tune(TuneState* dst, const TuneState* host, int n, hipStream_t s);
long loss_blocks(const Sampling& sm);
long bwd_wg_per_patch(const Sampling& sm);
// Column tiles of the gradient kernel over the support's compact columns (all
// columns: sup = NULL); its partials hold nz * tiles * 4 (at most) and
// tiles * 4 doubles per virtual patch.
long grad_tiles(const Sampling& sm, const LatSupport* sup = nullptr);
// Column tiles of the field kernel over the support's compact columns: the
// pupil-sum partials per patch.
long pupil_tiles(const Sampling& sm, const LatSupport& ls);
hipError_t launch_loss_grad(const DevOptics* opt, const TuneState* st, const Sampling& sm, int nv,
                            const float2* D, float2* bank, double* lpart, int data_div,
                            hipStream_t s);
// Gradient of a loss of the 3D reconstruction per frequency (bank [v][Z][2][M]
// the label-free pair after its Z transform, D [v][C][Z][M] the data spectrum,
// G [v][P][Z][M] the spectrum of dL/df; cpl: the polarisation bank): the pair
// becomes dL/dH*, and D the spectrum of dL/dd if want_dd.
hipError_t launch_recon_grad(float2* bank, float2* D, const float2* G, const float* bg, const Coupling* cpl,
                             const Sampling& sm, int npatch, float eta, double n_full, int want_dd,
                             hipStream_t s);
// The backward kernels and Adam take the fields' compact columns (sup; NULL:
// every column), as the field kernel wrote them.
hipError_t launch_tf_rows_bwd(const double* partials, const Sampling& sm, int nv, float2* ab,
                              const float2* g, double* dpart, hipStream_t s,
                              const LatSupport* sup = nullptr);
hipError_t launch_tf_grad_y(const DevOptics* opt, const Sampling& sm, int nv, const float2* ab,
                            double* gpart, double* ipart, hipStream_t s, const LatSupport* sup = nullptr);
hipError_t launch_adam(DevOptics* opt, TuneState* st, const Sampling& sm, int nv,
                       const double* ppart, const double* lpart, const double* dpart,
                       const double* gpart, const double* ipart, int update, hipStream_t s,
                       const LatSupport* sup = nullptr);
// Per patch, the start with the lowest loss: its optics into ropt[i] and the
// patch's eta into eta[i].
hipError_t launch_pick_best(const DevOptics* opt, const TuneState* st, int starts, int npatch,
                            DevOptics* ropt, float* eta, hipStream_t s);

// ---------------------------------------------------------------- vector label-free bank

// Constants of one patch of the vector model, computed on the host: the
// Jones vector of each illumination state, each channel's analysed direct
// state alpha_c = J_s^H M_c and its state s, the property tensors T_p
// ([p][3 n + k]) and 1 / (Y X I_bg).
struct VecRec {
  float J[5][2][2];
  float alpha[5][2][2];
  int state[5];
  float T[8][9][2];
  float scale;         // 1 / (Y X I_bg): responses on the grid
  float scale_short;   // 1 / (LY LX I_bg): responses on the shortened transforms
  int C, P, NS;
};
hipError_t launch_set_vec(VecRec* dst, const VecRec* host, int n, hipStream_t s);
// Field spectra fields [patch][f][z][y][c] on the XC kept columns c (column kx
// = field_column(c, KP, X, XC)) and LY rows (row i the grid's frequency (i or
// i - LY) / (ny dy)): f < 6 the detected scattered field of a unit
// dipole, u_i'n (f = 3 i' + n), then for each illumination state s the direct
// arm S P E conj(e_k) (f = 6 + 3 s + k), each times the propagator of plane z.
hipError_t launch_vec_spectra(const DevOptics* opt, const VecRec* rec, const Sampling& sm, int npatch, int NS,
                              float2* fields, int XC, int KP, int LY, hipStream_t s);
// Unnormalised complex FFT along X (sign -1 forward, +1 inverse) of nrows rows:
// src rows hold the XC kept columns (the others zero), dst rows all X values.
hipError_t launch_rows_c2c(const float2* src, float2* dst, int X, int XC, int KP, long nrows, float sign,
                           hipStream_t s);
// The real channel responses out [patch][C][P][vox] = 2 Re R_cp from the
// transformed fields [patch][F][vox].
hipError_t launch_vec_products(const VecRec* rec, const float2* fields, float* out, long vox, int F, int npatch,
                               hipStream_t s);
// Whether the row length has the fused X pass + responses kernel (compiled lengths).
bool vec_rows_fused(int X);
// The same responses straight from the Y-transformed spectra [patch][F][zy][XC]
// (zy = Z * Y rows of the kept columns): X inverse transforms and products
// fused per row and channel.
hipError_t launch_vec_rows_resp(const VecRec* rec, const float2* spec, float* out, int X, int XC, int KP, long zy,
                                int NS, int npatch, hipStream_t s);

}  // namespace wo
