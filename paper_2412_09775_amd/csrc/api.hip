// C ABI: validation, workspace layout and the launch sequence of each call.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <complex>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/waveorder.h"
#include "internal.hpp"

using namespace wo;

namespace wo {

long lds_limit_bytes() {
  static long cached = 0;
  if (cached == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        v > 0)
      cached = v;
    else
      cached = 65536;
  }
  return cached;
}

// ---------------------------------------------------------------- timing

namespace {
struct TimingRec {
  const char* name;
  hipEvent_t a, b;
};
std::mutex g_tmu;
bool g_timing = false;
std::string g_tsel;   // kernel name the events are restricted to (empty: all)
std::vector<TimingRec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
  if (!g_pool.empty()) {
    hipEvent_t e = g_pool.back();
    g_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

bool timing_enabled() { return g_timing; }

void timing_begin(const char* name, hipStream_t s, void** token) {
  std::lock_guard<std::mutex> lk(g_tmu);
  if (!g_tsel.empty() && g_tsel != name) {
    *token = nullptr;
    return;
  }
  TimingRec* r = new TimingRec{name, take_event(), take_event()};
  if (!r->a || !r->b) {
    delete r;
    *token = nullptr;
    return;
  }
  (void)hipEventRecord(r->a, s);   // instrumentation: a failed record only loses the sample
  *token = r;
}

void timing_end(void* token, hipStream_t s) {
  TimingRec* r = (TimingRec*)token;
  (void)hipEventRecord(r->b, s);
  std::lock_guard<std::mutex> lk(g_tmu);
  g_recs.push_back(*r);
  delete r;
}

}  // namespace wo

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool smooth235(int n) {
  if (n < 1 || n > 4096) return false;
  for (int f : {2, 3, 5})
    while (n % f == 0) n /= f;
  return n == 1;
}

struct Shape {
  int C, P, dims;
  bool thin;
  bool pol5 = false;   // the polarisation model (its bank has a reduced form)
  long Z, Y, X, Xh;
};

bool bank_shape(const wo_optics* o, Shape* s) {
  s->Z = o->nz;
  s->Y = o->ny;
  s->X = o->nx;
  s->Xh = o->nx / 2 + 1;
  s->thin = false;
  s->dims = 3;
  switch (o->model) {
    case WO_MODEL_FLUOR_3D: s->C = 1; s->P = 1; break;
    case WO_MODEL_LABELFREE_3D: s->C = 1; s->P = 2; break;
    case WO_MODEL_LABELFREE_THIN: s->C = o->nz; s->P = 2; s->thin = true; s->dims = 2; break;
    case WO_MODEL_POL5_3D: s->C = 5; s->P = 4; break;
    case WO_MODEL_SECTORS9_3D: s->C = 9; s->P = 1; break;
    case WO_MODEL_VECTOR_3D:
      if (o->vec_channels != 0 && o->vec_channels != 1) return false;
      if (o->vec_nprops < 1 || o->vec_nprops > 8) return false;
      s->C = o->vec_channels == 0 ? 4 : 5;
      s->P = o->vec_nprops;
      break;
    default: return false;
  }
  s->pol5 = o->model == WO_MODEL_POL5_3D;
  return true;
}

long bank_elems(const Shape& s) {
  return s.thin ? (long)s.C * s.P * s.Y * s.Xh : (long)s.C * s.P * s.Z * s.Y * s.Xh;
}

int check_sampling(const wo_optics* o) {
  if (!o) return WO_EINVAL;
  if (o->model < 0 || o->model > 5) return WO_EINVAL;
  if (o->model == WO_MODEL_VECTOR_3D) {
    if ((o->vec_channels != 0 && o->vec_channels != 1) || o->vec_nprops < 1 || o->vec_nprops > 8)
      return WO_EINVAL;
    for (int k = 0; k < o->vec_nprops; ++k)
      if (o->vec_props[k] < 0 || o->vec_props[k] > 17) return WO_EINVAL;
  }
  if (!(o->dz > 0 && o->dy > 0 && o->dx > 0 && o->wavelength > 0)) return WO_EINVAL;
  if (!smooth235(o->nz) || !smooth235(o->ny) || !smooth235(o->nx)) return WO_EUNSUPPORTED;
  if (o->nx % 2 || o->ny % 2) return WO_EUNSUPPORTED;
  if (o->model == WO_MODEL_LABELFREE_THIN && o->nz > 64) return WO_EUNSUPPORTED;
  return WO_OK;
}

bool same_sampling(const wo_optics* a, const wo_optics* b) {
  if (!(a->model == b->model && a->nz == b->nz && a->ny == b->ny && a->nx == b->nx &&
        a->dz == b->dz && a->dy == b->dy && a->dx == b->dx))
    return false;
  if (a->model != WO_MODEL_VECTOR_3D) return true;
  if (a->vec_channels != b->vec_channels || a->vec_nprops != b->vec_nprops) return false;
  for (int k = 0; k < a->vec_nprops && k < 8; ++k)
    if (a->vec_props[k] != b->vec_props[k]) return false;
  return true;
}

// Validity of the sampled model (same conditions as the FP64 oracle).
int check_optics(const wo_optics* o) {
  if (!(o->na_det >= 0 && o->na_ill >= 0 && o->n_medium > 0 && o->edge_width >= 0))
    return WO_EINVAL;
  if (!(isfinite(o->defocus) && isfinite(o->tilt_zenith) && isfinite(o->tilt_azimuth) &&
        isfinite(o->det_tilt) && isfinite(o->det_azimuth)))
    return WO_EINVAL;
  const double km = o->n_medium / o->wavelength;
  const double dnu = fmin(1.0 / (o->nx * o->dx), 1.0 / (o->ny * o->dy));
  const double hw = o->edge_width * dnu;
  // the detection pupil (the cap about a tilted detection axis) inside the shell
  DevOptics dd;
  memset(&dd, 0, sizeof(dd));
  dd.wavelength = o->wavelength;
  dd.na_det = o->na_det;
  dd.n_medium = o->n_medium;
  dd.det_tilt = o->det_tilt;
  const double rdet = det_radius(dd);
  if (rdet + hw >= km || fabs(o->det_tilt) + asin(fmin(o->na_det / o->n_medium, 1.0)) >= 0.5 * M_PI)
    return WO_EINVAL;
  if (o->det_tilt != 0.0)
    for (int j = 0; j < 7; ++j)
      if (o->zernike[j] != 0.0) return WO_EUNSUPPORTED;   // aberrations on a tilted pupil
  const double q0 = fabs(o->n_medium * sin(o->tilt_zenith) / o->wavelength);
  if (o->model != WO_MODEL_FLUOR_3D && o->na_ill / o->wavelength + q0 + hw >= km) return WO_EINVAL;
  const double nyq = fmin(0.5 / o->dx, 0.5 / o->dy);
  double lat, ax;
  const double kd = fmin(rdet + hw, km);
  if (o->model == WO_MODEL_FLUOR_3D) {
    lat = 2.0 * (rdet + hw);
  } else {
    lat = rdet + o->na_ill / o->wavelength + q0 + 2.0 * hw;
  }
  ax = km - sqrt(km * km - kd * kd);
  if (lat >= nyq) return WO_EALIAS;
  if (o->model != WO_MODEL_LABELFREE_THIN && ax >= 0.5 / o->dz) return WO_EALIAS;
  if ((o->model == WO_MODEL_POL5_3D || o->model == WO_MODEL_VECTOR_3D) && !(isfinite(o->swing)))
    return WO_EINVAL;
  if (o->model == WO_MODEL_VECTOR_3D) {
    if (o->det_tilt != 0.0) return WO_EUNSUPPORTED;   // the pupil map is the untilted objective's
    for (int j = 0; j < 4; ++j)
      if (!isfinite(o->ill_jones[j])) return WO_EINVAL;
  }
  for (int j = 0; j < 7; ++j)
    if (!isfinite(o->zernike[j])) return WO_EINVAL;
  return WO_OK;
}

bool aberrated(const wo_optics& o) {
  for (int j = 0; j < 7; ++j)
    if (o.zernike[j] != 0.0) return true;
  return false;
}

// Every aperture of the 9-aperture model must pass direct light (sum_q S_c P^2 > 0),
// evaluated with the device's pupil functions.
bool sectors_lit(const wo_optics& oo) {
  DevOptics d;
  memset(&d, 0, sizeof(d));
  d.wavelength = oo.wavelength;
  d.na_ill = oo.na_ill;
  d.n_medium = oo.n_medium;
  d.tilt_zenith = oo.tilt_zenith;
  d.tilt_azimuth = oo.tilt_azimuth;
  d.na_det = oo.na_det;
  d.det_tilt = oo.det_tilt;
  d.det_azimuth = oo.det_azimuth;
  const DetAxis da = det_axis(d);
  double cy, cx;
  source_centre(d, &cy, &cx);
  const double dnu = fmin(1.0 / (oo.nx * oo.dx), 1.0 / (oo.ny * oo.dy));
  const double hw = oo.edge_width * dnu;
  // S vanishes beyond the tilted source disc widened by the soft edge: only the
  // rows and columns of its bounding box (one spare frequency pixel) can add
  // to the sums, in the same order as a scan of the whole grid
  const double rs = oo.na_ill / oo.wavelength + hw + dnu;
  std::vector<int> kxs;
  for (int kx = 0; kx < oo.nx; ++kx)
    if (fabs(fftfreq(kx, oo.nx, oo.dx) - cx) <= rs) kxs.push_back(kx);
  double bg[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int ky = 0; ky < oo.ny; ++ky) {
    const double fy = fftfreq(ky, oo.ny, oo.dy);
    if (fabs(fy - cy) > rs) continue;
    for (int kx : kxs) {
      const double fx = fftfreq(kx, oo.nx, oo.dx);
      const double P = det_pupil(d, da, fy, fx, hw);
      const double S = disc(fy - cy, fx - cx, oo.na_ill / oo.wavelength, hw);
      bg[octant(fy - cy, fx - cx)] += S * P * P;
    }
  }
  for (double b : bg)
    if (!(b > 0.0)) return false;
  return true;
}

int validate(const wo_optics* o, int32_t n) {
  if (!o || n < 1) return WO_EINVAL;
  int st = check_sampling(&o[0]);
  if (st) return st;
  for (int i = 0; i < n; ++i) {
    if (!same_sampling(&o[0], &o[i])) return WO_EINVAL;
    st = check_optics(&o[i]);
    if (st) return st;
    if (o[i].model == WO_MODEL_SECTORS9_3D && !sectors_lit(o[i])) return WO_EINVAL;
  }
  return WO_OK;
}

// Polarisation coupling kappa_cp = conj(a^H e_c) (a^H B_p e_c), FP64 on the host.
typedef std::complex<double> cd;

// The five illumination states of the swing: e_0 = (1, i)/sqrt2 and
// e_c = J(2 pi swing, alpha_c) e_0, alpha_c in {0, pi/4, pi/2, 3 pi/4}.
void pol5_states(double swing, cd states[5][2]) {
  const double r2 = 1.0 / sqrt(2.0);
  const cd I(0.0, 1.0);
  cd e0[2] = {cd(r2, 0), cd(0, r2)};
  states[0][0] = e0[0];
  states[0][1] = e0[1];
  const double delta = 2.0 * M_PI * swing;
  const double alphas[4] = {0.0, M_PI / 4, M_PI / 2, 3 * M_PI / 4};
  for (int s = 0; s < 4; ++s) {
    const double c = cos(alphas[s]), sn = sin(alphas[s]);
    // R(a) = [[c, s], [-s, c]]; J = R(-a) diag(e^{-i d/2}, e^{i d/2}) R(a)
    cd v0 = c * e0[0] + sn * e0[1];
    cd v1 = -sn * e0[0] + c * e0[1];
    v0 *= std::exp(-0.5 * I * delta);
    v1 *= std::exp(0.5 * I * delta);
    states[s + 1][0] = c * v0 - sn * v1;
    states[s + 1][1] = sn * v0 + c * v1;
  }
}

void pol5_kappa(double swing, double out[5][4][2]) {
  const double r2 = 1.0 / sqrt(2.0);
  const cd I(0.0, 1.0);
  cd states[5][2];
  pol5_states(swing, states);
  const cd ah[2] = {cd(r2, 0), cd(0, r2)};  // a^H for a = (1, -i)/sqrt2
  const cd B[4][2][2] = {
      {{1.0, 0.0}, {0.0, 1.0}},
      {{0.5, 0.0}, {0.0, -0.5}},
      {{0.0, 0.5}, {0.5, 0.0}},
      {{I, 0.0}, {0.0, I}},
  };
  for (int c = 0; c < 5; ++c) {
    const cd direct = ah[0] * states[c][0] + ah[1] * states[c][1];
    for (int p = 0; p < 4; ++p) {
      const cd be0 = B[p][0][0] * states[c][0] + B[p][0][1] * states[c][1];
      const cd be1 = B[p][1][0] * states[c][0] + B[p][1][1] * states[c][1];
      const cd k = std::conj(direct) * (ah[0] * be0 + ah[1] * be1);
      out[c][p][0] = k.real();
      out[c][p][1] = k.imag();
    }
  }
}

// The FP32 coupling the kernels use (each FP64 value rounded once).
Coupling coupling_of(double swing) {
  double k[5][4][2];
  pol5_kappa(swing, k);
  Coupling c;
  for (int i = 0; i < 5; ++i)
    for (int p = 0; p < 4; ++p)
      for (int r = 0; r < 2; ++r) c.k[i][p][r] = (float)k[i][p][r];
  // Gram constants: with H_cp = Kr_cp u + Ki_cp v, (H^H H)_pq = A_pq |u|^2 +
  // B_pq |v|^2 + G_pq conj(u) v + G_qp u conj(v), G = Kr^T Ki
  for (int p = 0; p < 4; ++p)
    for (int q = 0; q <= p; ++q) {
      double a = 0, b = 0, gpq = 0, gqp = 0;
      for (int i = 0; i < 5; ++i) {
        a += k[i][p][0] * k[i][q][0];
        b += k[i][p][1] * k[i][q][1];
        gpq += k[i][p][0] * k[i][q][1];
        gqp += k[i][q][0] * k[i][p][1];
      }
      const int e = p * (p + 1) / 2 + q;
      c.a[e] = (float)a;
      c.b[e] = (float)b;
      c.s[e] = (float)(gpq + gqp);
      c.d[e] = (float)(gpq - gqp);
    }
  return c;
}

bool is_pol5(const Shape& s) { return s.pol5; }

// Spherical-harmonic tensor Y_b of the vector model in (x, y, z), entry 3 n + k:
// b = 0 the identity, 1..3 (yz - zy)/2, (zx - xz)/2, (xy - yx)/2, 4..8
// (xy + yx)/2, (yz + zy)/2, (2zz - xx - yy)/(2 sqrt 3), (xz + zx)/2, (xx - yy)/2.
void sh_tensor(int b, double T[9]) {
  for (int e = 0; e < 9; ++e) T[e] = 0.0;
  auto sym = [&](int a, int c) { T[3 * a + c] += 0.5; T[3 * c + a] += 0.5; };
  auto asym = [&](int a, int c) { T[3 * a + c] += 0.5; T[3 * c + a] -= 0.5; };
  switch (b) {
    case 0: T[0] = T[4] = T[8] = 1.0; break;
    case 1: asym(1, 2); break;
    case 2: asym(2, 0); break;
    case 3: asym(0, 1); break;
    case 4: sym(0, 1); break;
    case 5: sym(1, 2); break;
    case 6: {
      const double r = 1.0 / (2.0 * sqrt(3.0));
      T[0] = -r;
      T[4] = -r;
      T[8] = 2.0 * r;
      break;
    }
    case 7: sym(0, 2); break;
    case 8: T[0] = 0.5; T[4] = -0.5; break;
    default: break;
  }
}

DevOptics dev_optics(const wo_optics& o);

// Direct-direct intensity I_bg = sum_q S(q) P(q)^2 on the grid (FP64), over
// the rows and columns of the source disc's bounding box (one spare pixel).
double host_ibg(const wo_optics& oo) {
  const DevOptics d = dev_optics(oo);
  const DetAxis da = det_axis(d);
  double cy, cx;
  source_centre(d, &cy, &cx);
  const double dnu = fmin(1.0 / (oo.nx * oo.dx), 1.0 / (oo.ny * oo.dy));
  const double hw = oo.edge_width * dnu;
  const double rs = oo.na_ill / oo.wavelength + hw + dnu;
  double bg = 0.0;
  for (int ky = 0; ky < oo.ny; ++ky) {
    const double fy = fftfreq(ky, oo.ny, oo.dy);
    if (fabs(fy - cy) > rs) continue;
    for (int kx = 0; kx < oo.nx; ++kx) {
      const double fx = fftfreq(kx, oo.nx, oo.dx);
      if (fabs(fx - cx) > rs) continue;
      const double P = det_pupil(d, da, fy, fx, hw);
      bg += disc(fy - cy, fx - cx, oo.na_ill / oo.wavelength, hw) * P * P;
    }
  }
  return bg;
}

// Constants of one patch of the vector model (channels, property tensors,
// normalisation on the grid and on LY x LX shortened transforms); false if no
// direct light reaches the detector.
bool vec_rec(const wo_optics& o, VecRec* r, int LY, int LX) {
  memset(r, 0, sizeof(*r));
  const cd I(0.0, 1.0);
  cd J[5][2];
  cd M[5][2][2];
  int NS, C;
  if (o.vec_channels == 0) {
    NS = 1;
    C = 4;
    J[0][0] = cd(o.ill_jones[0], o.ill_jones[1]);
    J[0][1] = cd(o.ill_jones[2], o.ill_jones[3]);
    const cd sig[4][2][2] = {{{1.0, 0.0}, {0.0, 1.0}},
                             {{1.0, 0.0}, {0.0, -1.0}},
                             {{0.0, 1.0}, {1.0, 0.0}},
                             {{0.0, -I}, {I, 0.0}}};
    for (int c = 0; c < 4; ++c) {
      r->state[c] = 0;
      for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 2; ++k) M[c][i][k] = sig[c][i][k];
    }
  } else {
    NS = 5;
    C = 5;
    pol5_states(o.swing, J);
    const double r2 = 1.0 / sqrt(2.0);
    const cd a[2] = {cd(r2, 0), cd(0, -r2)};   // the circular analyser (1, -i)/sqrt2
    for (int c = 0; c < 5; ++c) {
      r->state[c] = c;
      for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 2; ++k) M[c][i][k] = a[i] * std::conj(a[k]);
    }
  }
  for (int s = 0; s < NS; ++s)
    for (int i = 0; i < 2; ++i) {
      r->J[s][i][0] = (float)J[s][i].real();
      r->J[s][i][1] = (float)J[s][i].imag();
    }
  for (int c = 0; c < C; ++c)
    for (int ip = 0; ip < 2; ++ip) {
      cd al = 0.0;
      for (int i = 0; i < 2; ++i) al += std::conj(J[r->state[c]][i]) * M[c][i][ip];
      r->alpha[c][ip][0] = (float)al.real();
      r->alpha[c][ip][1] = (float)al.imag();
    }
  for (int p = 0; p < o.vec_nprops; ++p) {
    double T[9];
    sh_tensor(o.vec_props[p] / 2, T);
    const bool im = o.vec_props[p] % 2 == 1;
    for (int e = 0; e < 9; ++e) {
      r->T[p][e][0] = im ? 0.f : (float)T[e];
      r->T[p][e][1] = im ? (float)T[e] : 0.f;
    }
  }
  const double ibg = host_ibg(o);
  if (!(ibg > 0.0)) return false;
  r->scale = (float)(1.0 / ((double)o.ny * o.nx * ibg));
  r->scale_short = (float)(1.0 / ((double)LY * LX * ibg));
  r->C = C;
  r->P = o.vec_nprops;
  r->NS = NS;
  return true;
}

Sampling sampling_of(const wo_optics* o) {
  Sampling s;
  s.model = o->model;
  s.nz = o->nz;
  s.ny = o->ny;
  s.nx = o->nx;
  s.dz = o->dz;
  s.dy = o->dy;
  s.dx = o->dx;
  return s;
}

size_t params_bytes(int32_t n) { return align_up((size_t)n * sizeof(DevOptics)); }

size_t partials_bytes(const wo_optics* o, int32_t n) {
  const Sampling sm = sampling_of(o);
  const int W = tf_tile_width(sm);
  return align_up((size_t)n * ((o->nx + W - 1) / W) * sizeof(double));
}

// Field sets the TF synthesis generates per patch: one per illumination aperture.
int field_sets(const wo_optics* o) { return o->model == WO_MODEL_SECTORS9_3D ? 9 : 1; }

// Lateral support of the fields and transfer functions of n patches
// (Methods, pupils): the detection pupil P is zero for |p| > NA_det/lambda0,
// the source S outside its tilted disc of radius NA_ill/lambda0, each widened
// by the soft edge.  The label-free fields A = S P e^{..} and B = P g e^{..}
// therefore vanish outside the columns and rows of P's support, and the
// transfer function, their correlation, outside the sum of the supports of A
// and B; the fluorescence OTF, the autocorrelation of P's field, outside
// twice P's support.  No wrap-around: the aliasing check keeps these sums
// below Nyquist.  Each bound keeps one spare column or row; compact widths
// are multiples of 16.
DevOptics dev_optics(const wo_optics& o);

LatSupport lateral_support(const wo_optics* o, int32_t n) {
  const Sampling sm = sampling_of(o);
  LatSupport ls = full_support(sm);
  const int X = o->nx, Y = o->ny, Xh = X / 2 + 1;
  const double fx1 = 1.0 / (X * o->dx), fy1 = 1.0 / (Y * o->dy);
  const double dnu = fmin(fx1, fy1);
  int px = 0, py = 0, ax = 0, ay = 0;
  for (int i = 0; i < n; ++i) {
    const double hw = o[i].edge_width * dnu;
    const double rd = det_radius(dev_optics(o[i])) + hw;   // the detection pupil's extent
    const double ri = o[i].na_ill / o[i].wavelength + hw;
    const double r = o[i].n_medium * sin(o[i].tilt_zenith) / o[i].wavelength;
    const double cy = fabs(r * sin(o[i].tilt_azimuth)), cx = fabs(r * cos(o[i].tilt_azimuth));
    // optics the library would reject (or a pupil wider than the grid) keep
    // the full layout
    const double qx = rd / fx1, qy = rd / fy1, sx = (cx + ri) / fx1, sy = (cy + ri) / fy1;
    if (!(qx >= 0.0 && qx < X && qy >= 0.0 && qy < Y && sx >= 0.0 && sy >= 0.0)) return ls;
    const int bx = (int)floor(qx) + 1, by = (int)floor(qy) + 1;
    px = std::max(px, bx);
    py = std::max(py, by);
    if (o->model == WO_MODEL_FLUOR_3D) {
      ax = px;
      ay = py;
    } else {
      ax = std::max(ax, std::min(bx, sx < X ? (int)floor(sx) + 1 : bx));
      ay = std::max(ay, std::min(by, sy < Y ? (int)floor(sy) + 1 : by));
    }
  }
  const int xc = (2 * px + 1 + 15) / 16 * 16;
  if (xc < X) {
    ls.xc = xc;
    ls.kp = px;
  }
  ls.xa = ls.xc;
  ls.kpa = ls.kp;
  const int xa = (2 * ax + 1 + 15) / 16 * 16;
  if (o->model != WO_MODEL_FLUOR_3D && xa < ls.xc && ax <= ls.kp && xa - ax <= ls.xc - ls.kp) {
    ls.xa = xa;   // A's columns: a subset of B's
    ls.kpa = ax;
  }
  const int kt = (px + ax + 1 + 15) / 16 * 16;
  if (kt < Xh) ls.kt = kt;
  if (2 * (py + ay) + 1 < Y) ls.ky = py + ay;
  // Shortest transform lengths with compiled stages that hold the
  // correlation without wrap-around (at least 2 (p + a) + 1 points), the kept
  // columns of the fields and, along X, the kept columns of the result as
  // non-negative frequencies.
  auto length_for = [](int need, int full) {
    static const int sizes[] = {64, 128, 160, 192, 240, 256, 320, 384, 480, 512, 1024};
    for (int n : sizes)
      if (n >= need && n < full) return n;
    return full;
  };
  ls.lx = length_for(std::max(std::max(2 * (px + ax) + 1, 2 * (ls.kt - 1)), ls.xc), X);
  ls.ly = ls.ky < Y ? length_for(2 * ls.ky + 1, Y) : Y;
  return ls;
}

// Complex values of the compact fields of nv field sets, rounded up to 256 bytes.
long compact_fields_elems(int nv, int nf, const Shape& s, const LatSupport& sup) {
  return ((long)nv * s.Z * sup.ly * (nf == 2 ? sup.xa + sup.xc : sup.xc) + 31) / 32 * 32;
}

// The support the transfer-function synthesis works on.  The label-free 3D
// models (one or nine apertures) keep the bank in its support until the Z
// pass, in a compact copy behind the compact fields (*compact_out) when both
// fit the field buffer; the others write their bank in place on the grid's
// own transform lengths.
LatSupport tf_support(const wo_optics* o, int32_t n, const Shape& s, bool* compact_out) {
  const Sampling sm = sampling_of(o);
  LatSupport sup = o->model == WO_MODEL_FLUOR_3D ? full_support(sm) : lateral_support(o, n);
  const int nf = o->model == WO_MODEL_FLUOR_3D ? 1 : 2;
  const int nv = n * field_sets(o);
  const int P3 = o->model == WO_MODEL_SECTORS9_3D ? 1 : 2;
  const long cplane = (long)sup.ly * sup.kt;
  *compact_out = (o->model == WO_MODEL_LABELFREE_3D || o->model == WO_MODEL_SECTORS9_3D ||
                  o->model == WO_MODEL_POL5_3D) &&
                 (sup.kt < s.Xh || sup.ky < s.Y) &&
                 compact_fields_elems(nv, nf, s, sup) + (long)nv * P3 * s.Z * cplane <=
                     (long)nv * nf * s.Z * s.Y * s.X;
  if (!*compact_out) {
    sup.ly = (int)s.Y;
    sup.lx = (int)s.X;
  }
  return sup;
}

// Vector model: the optics, the per-patch constants, the field spectra on the
// detection pupil's columns (later the bank's columns k < kt before its Z
// pass), the fields on the grid (6 + 3 per illumination state each) and the
// real channel responses.
// Transform lengths of the vector synthesis: with a compiled row length the
// fused X pass runs on the support's shortened transforms LY x LX (they hold
// the responses' band without wrap-around, as for the label-free bank);
// otherwise the grid's own, through the separate X pass and products.
struct VecLengths {
  bool fused;
  int LY, LX;
};
VecLengths vec_lengths(const Shape& s, const LatSupport& sup) {
  if (vec_rows_fused(sup.lx)) return VecLengths{true, sup.ly, sup.lx};
  return VecLengths{false, (int)s.Y, (int)s.X};
}

size_t vec_compact_elems(const wo_optics* o, int32_t n, const Shape& s, const LatSupport& sup, int LY) {
  const long F = 6 + 3 * (o->vec_channels == 0 ? 1 : 5);
  return (size_t)n * s.Z * LY * std::max(F * sup.xc, (long)s.C * s.P * sup.kt);
}

size_t vec_ws(const wo_optics* o, int32_t n, const Shape& s) {
  const int F = 6 + 3 * (o->vec_channels == 0 ? 1 : 5);
  const LatSupport sup = lateral_support(o, n);
  const VecLengths L = vec_lengths(s, sup);
  const size_t vox = (size_t)s.Z * L.LY * L.LX;
  const size_t full_fields = L.fused ? 0 : align_up((size_t)n * F * vox * sizeof(float2));
  return params_bytes(n) + align_up((size_t)n * sizeof(VecRec)) +
         align_up(vec_compact_elems(o, n, s, sup, L.LY) * sizeof(float2)) + full_fields +
         align_up((size_t)n * s.C * s.P * vox * sizeof(float));
}

size_t tf_ws(const wo_optics* o, int32_t n, const Shape& s) {
  if (o->model == WO_MODEL_VECTOR_3D) return vec_ws(o, n, s);
  const int nf = o->model == WO_MODEL_FLUOR_3D ? 1 : 2;
  const int nv = n * field_sets(o);
  size_t b = params_bytes(nv) + partials_bytes(o, nv);
  b += align_up((size_t)nv * nf * s.Z * s.Y * s.X * sizeof(float2));
  // the polarisation bank's label-free pair and the coupling records
  if (o->model == WO_MODEL_POL5_3D)
    b += align_up((size_t)n * 2 * s.Z * s.Y * s.Xh * sizeof(float2)) + align_up((size_t)n * sizeof(Coupling));
  return b;
}

// Spectra of the linear calls: max(C, P) channel slots per patch.
size_t linear_spec_bytes(int32_t n, const Shape& s) {
  const int CH = s.C > s.P ? s.C : s.P;
  const long zd = s.thin ? 1 : s.Z;
  return align_up((size_t)n * CH * zd * s.Y * s.Xh * sizeof(float2));
}

// The spectra, then (polarisation model) the coupling records of the reduced bank.
size_t linear_ws(int32_t n, const Shape& s) {
  return linear_spec_bytes(n, s) + (is_pol5(s) ? align_up((size_t)n * sizeof(Coupling)) : 0);
}

#define WO_TRY(expr)                         \
  do {                                       \
    hipError_t _e = (expr);                  \
    if (_e != hipSuccess) return WO_EHIP;    \
  } while (0)

// The FFT / operator / inverse-FFT sequence shared by forward, reconstruct and
// adjoint, in two halves: linear_in transforms the input into the spectrum
// (along X and Y), linear_out applies the per-frequency operator with the Z
// transforms and transforms back.  The bank vanishes outside the transfer
// function's lateral support, and so do the forward model's spectrum (but for
// its DC background term), the Tikhonov solution and the adjoint: for the 3D
// models the spectra are kept as the columns k < kt of every row (stored for
// the band rows only) and the Z pass covers the band.
struct LinearPlan {
  int cin, cout, CH;
  long zd;
  bool banded;
  int kt, ky;
};

LinearPlan linear_plan(const wo_optics* o, int32_t n, const Shape& s, int mode) {
  LinearPlan p;
  p.cin = mode == kModeForward ? s.P : s.C;
  p.cout = mode == kModeForward ? s.C : s.P;
  p.CH = p.cin > p.cout ? p.cin : p.cout;
  p.zd = s.thin ? 1 : s.Z;
  const LatSupport sup = s.thin ? full_support(sampling_of(o)) : lateral_support(o, n);
  p.banded = !s.thin && (sup.kt < s.Xh || sup.ky < s.Y);
  p.kt = p.banded ? sup.kt : (int)s.Xh;
  p.ky = p.banded ? sup.ky : (int)s.Y;
  return p;
}

int linear_in(const wo_optics* o, int32_t n, const Shape& s, const float* in, int mode, void* ws,
              hipStream_t st) {
  const LinearPlan p = linear_plan(o, n, s, mode);
  float2* spec = (float2*)ws;
  RowGroups gin{p.cin * p.zd * s.Y, p.cin * p.zd * s.Y, p.CH * p.zd * s.Y, n};
  if (p.banded) {
    WO_TRY(launch_rows_r2c(in, spec, (int)s.X, gin, st, p.kt, p.kt));
    WO_TRY(launch_cols(spec, (int)s.Y, p.kt, p.cin * p.zd, p.CH * p.zd, n, -1.f, st, "k_cols_y_fwd", 1,
                       p.ky));
  } else {
    WO_TRY(launch_rows_r2c(in, spec, (int)s.X, gin, st));
    WO_TRY(launch_cols(spec, (int)s.Y, s.Xh, p.cin * p.zd, p.CH * p.zd, n, -1.f, st, "k_cols_y_fwd"));
  }
  return WO_OK;
}

// bank_band: tf holds the band layout ([C][P][Z][band rows][kt], see
// wo_transfer_function_band) instead of [C][P][Z][Y][Xh]; the two coincide
// where the support fills the grid.
int linear_out(const wo_optics* o, int32_t n, const Shape& s, const float2* tf, float* out,
               const float* bg, int mode, float eta, void* ws, hipStream_t st, bool bank_band = false,
               const Coupling* cpl = nullptr) {
  const LinearPlan p = linear_plan(o, n, s, mode);
  float2* spec = (float2*)ws;
  const long M = s.Y * s.Xh;
  const double nfull = s.thin ? (double)s.Y * s.X : (double)s.Z * s.Y * s.X;
  const float inv_n = (float)(1.0 / nfull);
  RowGroups gout{p.cout * p.zd * s.Y, p.CH * p.zd * s.Y, p.cout * p.zd * s.Y, n};
  if (p.banded) {
    const SpecBand band{(int)s.Y, p.kt, p.ky, bank_band ? 1 : 0};
    WO_TRY(launch_zop(spec, tf, s.C, s.P, (int)s.Z, M, p.CH, n, mode, eta, bg, inv_n, nfull, st, &band, cpl));
    WO_TRY(launch_cols(spec, (int)s.Y, p.kt, p.cout * p.zd, p.CH * p.zd, n, 1.f, st, "k_cols_y_inv", 2,
                       p.ky));
    WO_TRY(launch_rows_c2r(spec, out, (int)s.X, gout, 1.f, st, p.kt, p.kt));
    return WO_OK;
  }
  if (s.thin) {
    WO_TRY(launch_op2d(spec, tf, s.C, s.P, M, p.CH, n, mode, eta, bg, inv_n, nfull, st));
  } else {
    WO_TRY(launch_zop(spec, tf, s.C, s.P, (int)s.Z, M, p.CH, n, mode, eta, bg, inv_n, nfull, st, nullptr,
                      cpl));
  }
  WO_TRY(launch_cols(spec, (int)s.Y, s.Xh, p.cout * p.zd, p.CH * p.zd, n, 1.f, st, "k_cols_y_inv"));
  WO_TRY(launch_rows_c2r(spec, out, (int)s.X, gout, 1.f, st));
  return WO_OK;
}

// reduced: tf is the polarisation bank in reduced form (the label-free pair);
// the coupling records go into the workspace behind the spectra.
int run_linear(const wo_optics* o, int32_t n, const Shape& s, const float2* tf, const float* in,
               float* out, const float* bg, int mode, float eta, void* ws, hipStream_t st,
               bool bank_band = false, bool reduced = false) {
  Coupling* cpl = nullptr;
  if (reduced) {
    cpl = (Coupling*)((char*)ws + linear_spec_bytes(n, s));
    std::vector<Coupling> h(n);
    for (int i = 0; i < n; ++i) h[i] = coupling_of(o[i].swing);
    WO_TRY(launch_set_coupling(cpl, h.data(), n, st));
  }
  int r = linear_in(o, n, s, in, mode, ws, st);
  if (r) return r;
  return linear_out(o, n, s, tf, out, bg, mode, eta, ws, st, bank_band, cpl);
}

// ---------------------------------------------------------------- auto-tune

// Workspace of one group of equally sampled patches, np patches x starts
// virtual patches (byte offsets from the group's base).
struct TuneLayout {
  int np, nv;
  long tiles, lbpp, dwpp;
  size_t off_opt, off_st, off_D, off_bank, off_ab, off_pp, off_lp, off_dp, off_gp, off_ip,
      off_ropt, off_reta, total;
};

TuneLayout tune_layout(const wo_optics* o, int32_t n, int32_t starts) {
  TuneLayout L;
  const Sampling sm = sampling_of(o);
  const long Z = o->nz, Y = o->ny, X = o->nx, Xh = X / 2 + 1;
  L.np = n;
  L.nv = n * starts;
  const int W = tf_tile_width(sm);
  L.tiles = (X + W - 1) / W;
  L.lbpp = loss_blocks(sm);
  L.dwpp = bwd_wg_per_patch(sm);
  size_t b = 0;
  auto take = [&](size_t bytes) { size_t o0 = b; b += align_up(bytes); return o0; };
  L.off_opt = take((size_t)L.nv * sizeof(DevOptics));
  L.off_st = take((size_t)L.nv * sizeof(TuneState));
  L.off_D = take((size_t)n * Z * Y * Xh * sizeof(float2));
  L.off_bank = take((size_t)L.nv * 2 * Z * Y * Xh * sizeof(float2));
  L.off_ab = take((size_t)L.nv * 2 * Z * Y * X * sizeof(float2));
  L.off_pp = take((size_t)L.nv * L.tiles * sizeof(double));
  L.off_lp = take((size_t)L.nv * L.lbpp * sizeof(double));
  L.off_dp = take((size_t)L.nv * L.dwpp * sizeof(double));
  const long gt = grad_tiles(sm);
  L.off_gp = take((size_t)L.nv * Z * gt * kGradAll * sizeof(double));
  L.off_ip = take((size_t)L.nv * gt * kThetaAll * sizeof(double));
  L.off_ropt = take((size_t)n * sizeof(DevOptics));
  L.off_reta = take((size_t)n * sizeof(float));
  L.total = b;
  return L;
}

// Patches that share a sampling are tuned by the same launches; a batch of
// uneven tiles forms one group per distinct shape, each with its own
// workspace slice.  `work` (voxels x starts) balances the graph branches.
struct TuneGroup {
  const wo_optics* rep;
  std::vector<int> idx;  // patch indices in the call, ascending
  TuneLayout L;
  size_t base;
  double work;
  int ab = 0;            // aberration-aware kernels (an aberrated patch, or dL/dc wanted)
  LatSupport sup;        // the fields' columns for every theta the tune may reach
};

// Lateral support of the auto-tune's fields: whatever NA and tilt the tune
// reaches, the detection pupil (and the source, within it) stays inside the
// shell |p| <= n/lambda0, so the shell's columns widened by the soft edge
// bound the fields, their gradients and the pupils' derivatives in every
// iteration.  The thin bank is written on the grid's own transforms and
// columns.
LatSupport tune_support(const wo_optics* o, const std::vector<int>& idx) {
  const Sampling sm = sampling_of(&o[idx[0]]);
  LatSupport ls = full_support(sm);
  const int X = sm.nx;
  const double fx1 = 1.0 / (X * sm.dx), dnu = fmin(fx1, 1.0 / (sm.ny * sm.dy));
  int px = 0;
  for (int i : idx) {
    const double q = (o[i].n_medium / o[i].wavelength + o[i].edge_width * dnu) / fx1;
    if (!(q >= 0.0 && q < X)) return ls;
    px = std::max(px, (int)floor(q) + 1);
  }
  const int xc = (2 * px + 1 + 15) / 16 * 16;
  if (xc < X) {
    ls.xc = ls.xa = xc;
    ls.kp = ls.kpa = px;
  }
  return ls;
}

std::vector<TuneGroup> tune_groups(const wo_optics* o, int32_t n, int32_t starts, size_t* total) {
  std::vector<TuneGroup> g;
  for (int i = 0; i < n; ++i) {
    size_t k = 0;
    while (k < g.size() && !same_sampling(g[k].rep, &o[i])) ++k;
    if (k == g.size()) g.push_back(TuneGroup{&o[i], {}, TuneLayout{}, 0, 0.0, 0, LatSupport{}});
    g[k].idx.push_back(i);
    if (aberrated(o[i])) g[k].ab = 1;
  }
  size_t b = 0;
  for (auto& t : g) {
    t.sup = tune_support(o, t.idx);
    t.L = tune_layout(t.rep, (int)t.idx.size(), starts);
    t.base = b;
    b += t.L.total;
    t.work = (double)t.idx.size() * starts * t.rep->nz * t.rep->ny * t.rep->nx;
  }
  if (total) *total = b;
  return g;
}

// Runs of consecutive patch indices inside a group: (first local index, length).
std::vector<std::pair<int, int>> index_runs(const std::vector<int>& idx) {
  std::vector<std::pair<int, int>> r;
  for (int j = 0; j < (int)idx.size();) {
    int k = j + 1;
    while (k < (int)idx.size() && idx[k] == idx[k - 1] + 1) ++k;
    r.push_back({j, k - j});
    j = k;
  }
  return r;
}

// Element offsets of packed per-patch arrays: stacks (nz ny nx) or thin
// reconstructions (2 ny nx).
std::vector<size_t> packed_offsets(const wo_optics* o, int32_t n, bool stacks) {
  std::vector<size_t> off(n + 1, 0);
  for (int i = 0; i < n; ++i)
    off[i + 1] = off[i] + (size_t)(stacks ? o[i].nz : 2) * o[i].ny * o[i].nx;
  return off;
}

// Number of lateral frequencies (full spectrum) with nu_c/8 <= |nu| <= nu_c/4,
// evaluated with the same expression as the loss kernel; rows and columns
// beyond nu_c/4 (plus one sample of margin) cannot be in the band.
double band_count(const wo_optics* o, double nu_c) {
  long cnt = 0;
  const double vy = 1.0 / ((double)o->ny * o->dy), vx = 1.0 / ((double)o->nx * o->dx);
  const double rmax = nu_c / 4.0;
  const long my = (long)(rmax / vy) + 1, mx = (long)(rmax / vx) + 1;
  std::vector<int> sxs;   // the signed columns within the band's reach
  for (int kx = 0; kx < o->nx; ++kx) {
    const int sx = kx < (o->nx + 1) / 2 ? kx : kx - o->nx;
    if (labs((long)sx) <= mx) sxs.push_back(sx);
  }
  for (int ky = 0; ky < o->ny; ++ky) {
    const int sy = ky < (o->ny + 1) / 2 ? ky : ky - o->ny;
    if (labs((long)sy) > my) continue;
    const double fy = sy * vy;
    for (int sx : sxs) {
      const double fx = sx * vx;
      const double r = sqrt(fy * fy + fx * fx);
      if (r >= nu_c / 8.0 && r <= nu_c / 4.0) ++cnt;
    }
  }
  return (double)cnt;
}

DevOptics dev_optics(const wo_optics& o) {
  DevOptics d;
  memset(&d, 0, sizeof(d));
  d.sector = -1;
  d.wavelength = o.wavelength;
  d.na_ill = o.na_ill;
  d.na_det = o.na_det;
  d.n_medium = o.n_medium;
  d.defocus = o.defocus;
  d.tilt_zenith = o.tilt_zenith;
  d.tilt_azimuth = o.tilt_azimuth;
  d.edge_width = o.edge_width;
  for (int j = 0; j < 7; ++j) d.zern[j] = (float)o.zernike[j];
  d.det_tilt = o.det_tilt;
  d.det_azimuth = o.det_azimuth;
  return d;
}

// One auto-tune iteration of every virtual patch of a group (update = 0: loss
// and gradient only).
int tune_iteration(const TuneGroup& g, char* ws, int starts, int update, hipStream_t hs) {
  const TuneLayout& L = g.L;
  char* w = ws + g.base;
  Sampling sm = sampling_of(g.rep);
  sm.aberrated = g.ab;
  const long Z = sm.nz, Y = sm.ny, Xh = sm.nx / 2 + 1;
  const long plane = Y * Xh;
  DevOptics* dopt = (DevOptics*)(w + L.off_opt);
  TuneState* st = (TuneState*)(w + L.off_st);
  float2* D = (float2*)(w + L.off_D);
  float2* bank = (float2*)(w + L.off_bank);
  float2* ab = (float2*)(w + L.off_ab);
  double* pp = (double*)(w + L.off_pp);
  double* lp = (double*)(w + L.off_lp);
  double* dp = (double*)(w + L.off_dp);
  double* gp = (double*)(w + L.off_gp);
  double* ip = (double*)(w + L.off_ip);
  const int nv = L.nv;
  WO_TRY(launch_tf_fields_y(dopt, sm, nv, ab, pp, hs, &g.sup));
  WO_TRY(launch_tf_rows_labelfree(pp, sm, nv, ab, bank, 2 * Z * plane, plane, 2 * plane, hs, &g.sup));
  WO_TRY(launch_cols(bank, (int)Y, Xh, 2 * Z, 2 * Z, nv, -1.f, hs, "k_cols_y_tf"));
  WO_TRY(launch_loss_grad(dopt, st, sm, nv, D, bank, lp, starts, hs));
  WO_TRY(launch_cols(bank, (int)Y, Xh, 2 * Z, 2 * Z, nv, 1.f, hs, "k_cols_y_grad"));
  WO_TRY(launch_tf_rows_bwd(pp, sm, nv, ab, bank, dp, hs, &g.sup));
  WO_TRY(launch_tf_grad_y(dopt, sm, nv, ab, gp, ip, hs, &g.sup));
  WO_TRY(launch_adam(dopt, st, sm, nv, pp, lp, dp, gp, ip, update, hs, &g.sup));
  return WO_OK;
}

// Thin-model reconstruction of every patch of a group at its best start's
// final theta: transfer function at that theta, per-frequency Tikhonov solve
// of the Z x 2 system with the patch's eta, inverse 2D transform into the
// packed output [2][ny][nx] of each patch.  Consumes the data spectra.
int tune_restore(const TuneGroup& g, char* ws, int starts, float* f_out, const size_t* foff,
                 hipStream_t hs) {
  const TuneLayout& L = g.L;
  char* w = ws + g.base;
  Sampling sm = sampling_of(g.rep);
  sm.aberrated = g.ab;
  const long Z = sm.nz, Y = sm.ny, X = sm.nx, Xh = X / 2 + 1;
  const long plane = Y * Xh;
  const int np = L.np;
  DevOptics* ropt = (DevOptics*)(w + L.off_ropt);
  float* reta = (float*)(w + L.off_reta);
  float2* D = (float2*)(w + L.off_D);
  float2* bank = (float2*)(w + L.off_bank);
  float2* ab = (float2*)(w + L.off_ab);
  double* pp = (double*)(w + L.off_pp);
  WO_TRY(launch_pick_best((const DevOptics*)(w + L.off_opt), (const TuneState*)(w + L.off_st), starts,
                          np, ropt, reta, hs));
  WO_TRY(launch_tf_fields_y(ropt, sm, np, ab, pp, hs, &g.sup));
  WO_TRY(launch_tf_rows_labelfree(pp, sm, np, ab, bank, 2 * Z * plane, plane, 2 * plane, hs, &g.sup));
  WO_TRY(launch_cols(bank, (int)Y, Xh, 2 * Z, 2 * Z, np, -1.f, hs, "k_cols_y_tf"));
  const double nfull = (double)Y * X;
  WO_TRY(launch_op2d(D, bank, (int)Z, 2, plane, (int)Z, np, kModeSolve, 0.f, nullptr,
                     (float)(1.0 / nfull), nfull, hs, reta));
  WO_TRY(launch_cols(D, (int)Y, Xh, 2, Z, np, 1.f, hs, "k_cols_y_inv"));
  for (auto r : index_runs(g.idx)) {
    RowGroups rg{2 * Y, Z * Y, 2 * Y, r.second};
    WO_TRY(launch_rows_c2r(D + (size_t)r.first * Z * plane, f_out + foff[g.idx[r.first]], (int)X, rg,
                           1.f, hs));
  }
  return WO_OK;
}

int validate_thin(const wo_optics* o, int32_t n) {
  if (!o || n < 1) return WO_EINVAL;
  for (int i = 0; i < n; ++i) {
    int st = check_sampling(&o[i]);
    if (st) return st;
    if (o[i].model != WO_MODEL_LABELFREE_THIN || o[i].nz < 2 || o[i].ny > 2048 || o[i].nx > 2048)
      return WO_EUNSUPPORTED;
    st = check_optics(&o[i]);
    if (st) return st;
  }
  return WO_OK;
}

// Largest theta box that keeps the detection pupil strictly inside the shell,
// intersected with the caller's box.
void clamp_box(const wo_optics* o, double lo[4], double hi[4]) {
  const double km = o->n_medium / o->wavelength;
  const double dnu = fmin(1.0 / (o->nx * o->dx), 1.0 / (o->ny * o->dy));
  const double hw = o->edge_width * dnu;
  const double na_max = (km - hw) * o->wavelength * (1.0 - 1e-9);
  if (hi[1] > na_max) hi[1] = na_max;
  if (lo[1] < 0.0) lo[1] = 0.0;
}

// Set-up of one group: per-virtual-patch optics and tune state, and the 2D
// spectra of the group's data stacks (read from the packed input `d`).
int tune_setup(const wo_optics* o, const TuneGroup& g, int starts, const double* theta0,
               const float* d, const size_t* doff, const double* eta, const double* nu_c,
               const double* lr, const double* lo, const double* hi, int mask, char* ws,
               hipStream_t hs, double lr_ab = 0.0, double bound_ab = 0.0) {
  const TuneLayout& L = g.L;
  char* w = ws + g.base;
  const int np = L.np, nv = L.nv;
  std::vector<DevOptics> hopt(nv);
  std::vector<TuneState> hst(nv);
  for (int j = 0; j < np; ++j) {
    const int i = g.idx[j];
    double blo[4], bhi[4];
    for (int k = 0; k < 4; ++k) {
      blo[k] = lo ? lo[k] : -1e300;
      bhi[k] = hi ? hi[k] : 1e300;
    }
    if (lo && hi) clamp_box(&o[i], blo, bhi);
    const double nuc = (nu_c && nu_c[i] > 0) ? nu_c[i] : (o[i].na_det + o[i].na_ill) / o[i].wavelength;
    const double bc = band_count(&o[i], nuc);
    if (bc < 1) return WO_EINVAL;
    for (int s = 0; s < starts; ++s) {
      const int v = j * starts + s;
      const long gv = (long)i * starts + s;
      hopt[v] = dev_optics(o[i]);
      if (theta0) {
        hopt[v].defocus = theta0[4 * gv + 0];
        hopt[v].na_det = theta0[4 * gv + 1];
        hopt[v].tilt_zenith = theta0[4 * gv + 2];
        hopt[v].tilt_azimuth = theta0[4 * gv + 3];
      }
      TuneState& t = hst[v];
      memset(&t, 0, sizeof(t));
      for (int k = 0; k < 4; ++k) {
        t.lr[k] = lr ? lr[k] : 0.0;
        t.lo[k] = blo[k];
        t.hi[k] = bhi[k];
      }
      t.lr_ab = lr_ab;
      t.bound_ab = bound_ab > 0.0 ? bound_ab : 1.0;
      t.eta = eta[i];
      t.nu_c = nuc;
      t.band_count = bc;
      t.mask = mask;
      // every virtual patch must describe valid optics at its start
      wo_optics ov = o[i];
      ov.defocus = hopt[v].defocus;
      ov.na_det = hopt[v].na_det;
      ov.tilt_zenith = hopt[v].tilt_zenith;
      ov.tilt_azimuth = hopt[v].tilt_azimuth;
      const int stt = check_optics(&ov);
      if (stt) return stt;
    }
  }
  WO_TRY(launch_set_params((DevOptics*)(w + L.off_opt), hopt.data(), nv, hs));
  WO_TRY(launch_set_tune((TuneState*)(w + L.off_st), hst.data(), nv, hs));
  const long Z = g.rep->nz, Y = g.rep->ny, Xh = g.rep->nx / 2 + 1;
  float2* D = (float2*)(w + L.off_D);
  for (auto r : index_runs(g.idx)) {
    RowGroups rg{Z * Y, Z * Y, Z * Y, r.second};
    WO_TRY(launch_rows_r2c(d + doff[g.idx[r.first]], D + (size_t)r.first * Z * Y * Xh, g.rep->nx, rg,
                           hs));
  }
  WO_TRY(launch_cols(D, (int)Y, Xh, Z, Z, np, -1.f, hs, "k_cols_y_data"));
  return WO_OK;
}

// Library streams for graph capture: one origin stream and up to kMaxBranches
// branch streams, default priority, created on first use and kept.
constexpr int kMaxBranches = 8;
struct CaptureStreams {
  hipStream_t cap = nullptr;
  hipStream_t br[kMaxBranches] = {};
  hipEvent_t fork = nullptr, join[kMaxBranches] = {}, ready = nullptr, done = nullptr;
};
std::mutex g_tune_mu;

int capture_streams(CaptureStreams** out) {
  static CaptureStreams cs;
  static bool made = false;
  if (!made) {
    WO_TRY(hipStreamCreateWithFlags(&cs.cap, hipStreamNonBlocking));
    for (int b = 0; b < kMaxBranches; ++b) {
      WO_TRY(hipStreamCreateWithFlags(&cs.br[b], hipStreamNonBlocking));
      WO_TRY(hipEventCreateWithFlags(&cs.join[b], hipEventDisableTiming));
    }
    WO_TRY(hipEventCreateWithFlags(&cs.fork, hipEventDisableTiming));
    WO_TRY(hipEventCreateWithFlags(&cs.ready, hipEventDisableTiming));
    WO_TRY(hipEventCreateWithFlags(&cs.done, hipEventDisableTiming));
    made = true;
  }
  *out = &cs;
  return WO_OK;
}

// Instantiated graphs of recent calls (a few; oldest evicted).  Used under
// g_tune_mu.
constexpr size_t kGraphCache = 8;
std::vector<std::pair<std::string, hipGraphExec_t>> g_graphs;

hipGraphExec_t graph_cache_find(const std::string& key) {
  for (auto& kv : g_graphs)
    if (kv.first == key) return kv.second;
  return nullptr;
}

void graph_cache_insert(const std::string& key, hipGraphExec_t exec) {
  if (g_graphs.size() >= kGraphCache) {
    (void)hipGraphExecDestroy(g_graphs.front().second);
    g_graphs.erase(g_graphs.begin());
  }
  g_graphs.push_back({key, exec});
}

std::string graph_key(const wo_optics* o, int32_t n, const wo_autotune_opts* opts, int starts,
                      int B, const void* ws, size_t ws_bytes, const float* d, const float* f_out) {
  std::string k;
  char b[256];
  snprintf(b, sizeof(b), "%d %d %d %d %d %p %zu %p %p %llu|", n, opts->use_graph, opts->iters, starts,
           B, ws, ws_bytes, (const void*)d, (const void*)f_out, fft_table_version());
  k += b;
  for (int i = 0; i < n; ++i) {
    // the aberration-aware kernel variants are part of the graph
    // and so are the fields' compact columns (tune_support)
    snprintf(b, sizeof(b), "%d %d %d %a %a %a %d %a %a %a;", o[i].nz, o[i].ny, o[i].nx, o[i].dz, o[i].dy,
             o[i].dx, aberrated(o[i]) || ((opts->tune_mask >> 4) & 0x7f) ? 1 : 0, o[i].wavelength,
             o[i].n_medium, o[i].edge_width);
    k += b;
  }
  return k;
}

// Longest-processing-time assignment of groups to branches: groups sorted by
// work, each placed on the least loaded branch.
std::vector<std::vector<int>> assign_branches(const std::vector<TuneGroup>& g, int B) {
  std::vector<int> order(g.size());
  for (size_t k = 0; k < g.size(); ++k) order[k] = (int)k;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return g[a].work > g[b].work; });
  std::vector<std::vector<int>> br(B);
  std::vector<double> load(B, 0.0);
  for (int k : order) {
    int best = 0;
    for (int b = 1; b < B; ++b)
      if (load[b] < load[best]) best = b;
    br[best].push_back(k);
    load[best] += g[k].work;
  }
  return br;
}

// The auto-tune of every patch (and, with f_out, the restoration), shared by
// wo_autotune and wo_restore_tiles.
int run_tune(wo_optics* o, int32_t n, const float* d, const double* eta,
             const wo_autotune_opts* opts, double* loss_out, float* f_out, void* ws,
             size_t ws_bytes, void* stream) {
  int st = validate_thin(o, n);
  if (st) return st;
  if (!d || !eta || !opts || !ws) return WO_EINVAL;
  const int starts = opts->multistart < 1 ? 1 : opts->multistart;
  if (opts->iters < 0 || opts->use_graph < 0 || opts->use_graph > 2) return WO_EINVAL;
  if (opts->branches < 0 || opts->branches > kMaxBranches) return WO_EINVAL;
  for (int i = 0; i < n; ++i)
    if (!(eta[i] > 0.0)) return WO_EINVAL;
  if ((opts->tune_mask >> 4) & 0x7f) {
    if (!(opts->lr_zernike >= 0.0) || !isfinite(opts->lr_zernike) || !isfinite(opts->zernike_bound))
      return WO_EINVAL;
  }
  size_t need = 0;
  std::vector<TuneGroup> groups = tune_groups(o, n, starts, &need);
  if (ws_bytes < need) return WO_ENOMEM;
  if ((opts->tune_mask >> 4) & 0x7f)
    for (auto& g : groups) g.ab = 1;   // tuned coefficients need the aberration-aware kernels
  const std::vector<size_t> doff = packed_offsets(o, n, true);
  const std::vector<size_t> foff = packed_offsets(o, n, false);
  hipStream_t hs = (hipStream_t)stream;
  char* w = (char*)ws;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& g : groups) {
    st = tune_setup(o, g, starts, opts->theta0, d, doff.data(), eta, opts->nu_c, opts->lr, opts->lo,
                    opts->hi, opts->tune_mask, w, hs, opts->lr_zernike, opts->zernike_bound);
    if (st) return st;
  }
  const int iters = opts->iters;
  // everything after the iterations: final loss, restoration
  auto tail = [&](const TuneGroup& g, hipStream_t s) -> int {
    int r = tune_iteration(g, w, starts, 0, s);
    if (!r && f_out) r = tune_restore(g, w, starts, f_out, foff.data(), s);
    return r;
  };
  if (opts->use_graph == 0 || (opts->use_graph == 1 && iters == 0)) {
    for (int it = 0; it < iters; ++it)
      for (auto& g : groups) {
        st = tune_iteration(g, w, starts, 1, hs);
        if (st) return st;
      }
    for (auto& g : groups) {
      st = tail(g, hs);
      if (st) return st;
    }
  } else {
    // use_graph 1: one iteration of every group captured and replayed `iters`
    // times; 2: the whole call (iterations, final loss, restoration) captured
    // and launched once.  Groups run on parallel branches of the graph.
    CaptureStreams* cs = nullptr;
    st = capture_streams(&cs);
    if (st) return st;
    int B = opts->branches > 0 ? opts->branches : 4;
    if (B > (int)groups.size()) B = (int)groups.size();
    const std::vector<std::vector<int>> br = assign_branches(groups, B);
    WO_TRY(hipEventRecord(cs->ready, hs));
    WO_TRY(hipStreamWaitEvent(cs->cap, cs->ready, 0));
    // A graph depends only on the shapes and samplings, the buffers, the counts
    // and the FFT schedules (parameters live in the workspace): reuse it when a
    // call repeats them.
    const std::string key = graph_key(o, n, opts, starts, B, ws, ws_bytes, d, f_out);
    hipGraphExec_t exec = graph_cache_find(key);
    if (!exec) {
      const bool was_timing = timing_enabled();
      if (was_timing) wo_timing_enable(0);
      hipGraph_t graph = nullptr;
      hipError_t ce = hipStreamBeginCapture(cs->cap, hipStreamCaptureModeThreadLocal);
      if (ce != hipSuccess) {
        if (was_timing) wo_timing_enable(1);
        return WO_EHIP;
      }
      int ist = WO_OK;
      hipError_t fe = hipEventRecord(cs->fork, cs->cap);
      for (int b = 0; b < B && fe == hipSuccess; ++b) fe = hipStreamWaitEvent(cs->br[b], cs->fork, 0);
      for (int b = 0; b < B && fe == hipSuccess && !ist; ++b) {
        for (int k : br[b]) {
          if (opts->use_graph == 1) {
            ist = tune_iteration(groups[k], w, starts, 1, cs->br[b]);
          } else {
            for (int it = 0; it < iters && !ist; ++it)
              ist = tune_iteration(groups[k], w, starts, 1, cs->br[b]);
            if (!ist) ist = tail(groups[k], cs->br[b]);
          }
          if (ist) break;
        }
      }
      for (int b = 0; b < B && fe == hipSuccess; ++b) {
        hipError_t e1 = hipEventRecord(cs->join[b], cs->br[b]);
        hipError_t e2 = hipStreamWaitEvent(cs->cap, cs->join[b], 0);
        if (e1 != hipSuccess) fe = e1;
        else if (e2 != hipSuccess) fe = e2;
      }
      ce = hipStreamEndCapture(cs->cap, &graph);
      if (was_timing) wo_timing_enable(1);
      if (ist || fe != hipSuccess || ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return ist ? ist : WO_EHIP;
      }
      const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (ie != hipSuccess) return WO_EHIP;
      graph_cache_insert(key, exec);
    }
    const int launches = opts->use_graph == 1 ? iters : 1;
    hipError_t le = hipSuccess;
    for (int it = 0; it < launches && le == hipSuccess; ++it) le = hipGraphLaunch(exec, cs->cap);
    hipError_t re = hipEventRecord(cs->done, cs->cap);
    if (re == hipSuccess) re = hipStreamWaitEvent(hs, cs->done, 0);
    hipError_t se = hipStreamSynchronize(cs->cap);
    if (le != hipSuccess || re != hipSuccess || se != hipSuccess) return WO_EHIP;
    if (opts->use_graph == 1)
      for (auto& g : groups) {
        st = tail(g, hs);
        if (st) return st;
      }
  }
  // read back the final state of every start; report the best one per patch
  for (auto& g : groups) {
    const TuneLayout& L = g.L;
    std::vector<TuneState> h(L.nv);
    std::vector<DevOptics> ho(L.nv);
    WO_TRY(hipMemcpyAsync(h.data(), w + g.base + L.off_st, L.nv * sizeof(TuneState),
                          hipMemcpyDeviceToHost, hs));
    WO_TRY(hipMemcpyAsync(ho.data(), w + g.base + L.off_opt, L.nv * sizeof(DevOptics),
                          hipMemcpyDeviceToHost, hs));
    WO_TRY(hipStreamSynchronize(hs));
    auto finite = [&](int v) {
      bool ok = isfinite(h[v].loss) && isfinite(ho[v].defocus) && isfinite(ho[v].na_det) &&
                isfinite(ho[v].tilt_zenith) && isfinite(ho[v].tilt_azimuth);
      for (int k = 0; k < 7; ++k) ok = ok && isfinite(ho[v].zern[k]);
      return ok;
    };
    for (int j = 0; j < L.np; ++j) {
      const int i = g.idx[j];
      int best = -1;   // the lowest final loss among the starts that ended finite
      for (int s2 = 0; s2 < starts; ++s2) {
        const int v = j * starts + s2;
        if (finite(v) && (best < 0 || h[v].loss < h[best].loss)) best = v;
      }
      if (opts->status_out) opts->status_out[i] = best < 0 ? WO_DIVERGED : WO_OK;
      if (best >= 0) {
        o[i].defocus = ho[best].defocus;
        o[i].na_det = ho[best].na_det;
        o[i].tilt_zenith = ho[best].tilt_zenith;
        o[i].tilt_azimuth = ho[best].tilt_azimuth;
        if ((opts->tune_mask >> 4) & 0x7f)
          for (int k = 0; k < 7; ++k) o[i].zernike[k] = ho[best].zern[k];
      }
      if (loss_out) loss_out[i] = best >= 0 ? h[best].loss : NAN;
      if (opts->all_theta_out)
        for (int s2 = 0; s2 < starts; ++s2) {
          const int v = j * starts + s2;
          const long gv = (long)i * starts + s2;
          opts->all_theta_out[4 * gv + 0] = ho[v].defocus;
          opts->all_theta_out[4 * gv + 1] = ho[v].na_det;
          opts->all_theta_out[4 * gv + 2] = ho[v].tilt_zenith;
          opts->all_theta_out[4 * gv + 3] = ho[v].tilt_azimuth;
          if (opts->all_loss_out) opts->all_loss_out[gv] = h[v].loss;
        }
    }
  }
  return WO_OK;
}

}  // namespace

extern "C" {

int wo_version(void) { return 200; }

int wo_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(wo::g_tmu);
  wo::g_timing = on != 0;
  return WO_OK;
}

int wo_timing_select(const char* name) {
  std::lock_guard<std::mutex> lk(wo::g_tmu);
  wo::g_tsel = name ? name : "";
  return WO_OK;
}

int wo_timing_report(char* buf, size_t len) {
  std::vector<wo::TimingRec> recs;
  {
    std::lock_guard<std::mutex> lk(wo::g_tmu);
    recs.swap(wo::g_recs);
  }
  std::map<std::string, std::pair<long, double>> agg;
  int status = WO_OK;
  for (auto& r : recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) != hipSuccess || hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess)
      status = WO_EHIP;
    auto& a = agg[r.name];
    a.first += 1;
    a.second += ms;
  }
  {
    std::lock_guard<std::mutex> lk(wo::g_tmu);
    for (auto& r : recs) {
      wo::g_pool.push_back(r.a);
      wo::g_pool.push_back(r.b);
    }
  }
  std::string out;
  for (auto& kv : agg) {
    char line[256];
    snprintf(line, sizeof(line), "%s %ld %.6f\n", kv.first.c_str(), kv.second.first, kv.second.second);
    out += line;
  }
  if (buf && len) {
    size_t n = out.size() < len - 1 ? out.size() : len - 1;
    memcpy(buf, out.data(), n);
    buf[n] = 0;
  }
  return status;
}

const char* wo_strerror(int status) {
  switch (status) {
    case WO_OK: return "ok";
    case WO_EINVAL: return "invalid argument or optics outside the model's validity";
    case WO_EUNSUPPORTED: return "unsupported size or mode";
    case WO_ENOMEM:
      return "workspace too small (below wo_workspace_size(), or beyond the static scratch of "
             "wo_reconstruct_noalloc)";
    case WO_EHIP: return "HIP runtime error";
    case WO_EALIAS: return "transfer-function support exceeds the sampled band";
    case WO_DIVERGED: return "no start of the patch ended with a finite loss and parameters";
    default: return "unknown status";
  }
}

int wo_bank_shape(const wo_optics* o, int32_t* C, int32_t* P, int32_t* dims, int64_t* elems) {
  Shape s;
  if (!o || !bank_shape(o, &s)) return WO_EINVAL;
  if (C) *C = s.C;
  if (P) *P = s.P;
  if (dims) *dims = s.dims;
  if (elems) *elems = bank_elems(s);
  return WO_OK;
}

size_t wo_workspace_size(const wo_optics* o, int32_t n, int32_t op) {
  Shape s;
  if (!o || n < 1 || !bank_shape(o, &s)) return 0;
  if (op == WO_OP_TRANSFER_FUNCTION) return tf_ws(o, n, s);
  if (op == WO_OP_FORWARD || op == WO_OP_RECONSTRUCT || op == WO_OP_ADJOINT) return linear_ws(n, s);
  return 0;
}

int wo_lateral_support(const wo_optics* o, int32_t n, wo_support* out) {
  int st = validate(o, n);
  if (st) return st;
  if (!out) return WO_EINVAL;
  Shape s;
  if (!bank_shape(o, &s)) return WO_EINVAL;
  const LatSupport ls = lateral_support(o, n);
  bool compact_out = false;
  const LatSupport ts = tf_support(o, n, s, &compact_out);
  const bool one_field = o->model == WO_MODEL_FLUOR_3D;
  out->field_cols[0] = one_field ? ts.xc : ts.xa;
  out->field_cols[1] = one_field ? 0 : ts.xc;
  out->tf_cols = ls.kt;
  out->band_rows = ls.ky >= o->ny ? o->ny : 2 * ls.ky + 1;
  out->tf_lengths[0] = ts.ly;
  out->tf_lengths[1] = ts.lx;
  if (o->model == WO_MODEL_VECTOR_3D) {   // every field on the detection pupil's columns
    const VecLengths L = vec_lengths(s, ls);
    out->field_cols[0] = out->field_cols[1] = ls.xc;
    out->tf_lengths[0] = L.LY;
    out->tf_lengths[1] = L.LX;
  }
  return WO_OK;
}

// The vector bank: field spectra, their inverse lateral transforms (Y by the
// column passes, X by complex row passes), the per-voxel channel responses,
// and the forward 3D transform of each response into tf [patch][C][P][Z][Y][Xh].
static int run_vector_tf(const wo_optics* o, int32_t n, const Shape& s, float2* tf, void* ws, hipStream_t hs,
                         bool band_out) {
  const int NS = o->vec_channels == 0 ? 1 : 5;
  const int F = 6 + 3 * NS;
  const LatSupport sup = lateral_support(o, n);   // the detection pupils' columns: sup.xc, sup.kp
  const VecLengths L = vec_lengths(s, sup);
  std::vector<DevOptics> h(n);
  std::vector<VecRec> vr(n);
  for (int i = 0; i < n; ++i) {
    h[i] = dev_optics(o[i]);
    if (!vec_rec(o[i], &vr[i], L.LY, L.LX)) return WO_EINVAL;
  }
  const long vox = s.Z * (long)L.LY * L.LX;
  char* w = (char*)ws;
  DevOptics* dopt = (DevOptics*)w;
  w += params_bytes(n);
  VecRec* drec = (VecRec*)w;
  w += align_up((size_t)n * sizeof(VecRec));
  float2* spec = (float2*)w;
  w += align_up(vec_compact_elems(o, n, s, sup, L.LY) * sizeof(float2));
  float2* fields = (float2*)w;
  if (!L.fused) w += align_up((size_t)n * F * vox * sizeof(float2));
  float* resp = (float*)w;
  WO_TRY(launch_set_params(dopt, h.data(), n, hs));
  WO_TRY(launch_set_vec(drec, vr.data(), n, hs));
  const Sampling sm = sampling_of(o);
  WO_TRY(launch_vec_spectra(dopt, drec, sm, n, NS, spec, sup.xc, sup.kp, L.LY, hs));
  WO_TRY(launch_cols(spec, L.LY, sup.xc, (long)F * s.Z, (long)F * s.Z, n, 1.f, hs, "k_cols_vec"));
  if (L.fused) {
    WO_TRY(launch_vec_rows_resp(drec, spec, resp, L.LX, sup.xc, sup.kp, s.Z * (long)L.LY, NS, n, hs));
  } else {
    WO_TRY(launch_rows_c2c(spec, fields, L.LX, sup.xc, sup.kp, (long)n * F * s.Z * L.LY, 1.f, hs));
    WO_TRY(launch_vec_products(drec, fields, resp, vox, F, n, hs));
  }
  // the bank vanishes outside the columns k < kt and the band rows: the X and
  // Y transforms keep those (in the spectra's buffer), the Z pass writes the
  // full bank with zeros elsewhere, or the band layout (band_out)
  const long rows = (long)s.C * s.P * s.Z * L.LY;
  const RowGroups g{rows, rows, rows, n};
  WO_TRY(launch_rows_r2c(resp, spec, L.LX, g, hs, sup.kt, sup.kt, "k_rows_r2c_tf"));
  const long planes = (long)s.C * s.P * s.Z;
  WO_TRY(launch_cols(spec, L.LY, sup.kt, planes, planes, n, -1.f, hs, "k_cols_y_tf", 1, sup.ky));
  WO_TRY(launch_cols_expand(spec, tf, (int)s.Z, L.LY, (int)s.Y, (int)s.Xh, sup.kt, sup.ky,
                            (long)n * s.C * s.P, -1.f, hs, band_out));
  return WO_OK;
}

// Transfer-function synthesis of validated optics into tf_out (workspace
// tf_ws bytes at ws).
static int run_tf(const wo_optics* o, int32_t n, const Shape& s, void* tf_out, void* ws, hipStream_t hs,
                  bool band_out = false) {
  if (o->model == WO_MODEL_VECTOR_3D) return run_vector_tf(o, n, s, (float2*)tf_out, ws, hs, band_out);
  const int fs = field_sets(o);
  const int nv = n * fs;          // field sets: patch i, aperture c at i * fs + c
  std::vector<DevOptics> h(nv);
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < fs; ++c) {
      DevOptics& d = h[i * fs + c];
      d = dev_optics(o[i]);
      if (fs == 9) d.sector = c < 8 ? c : -1;
    }
  char* w = (char*)ws;
  DevOptics* dopt = (DevOptics*)w;
  w += params_bytes(nv);
  double* partials = (double*)w;
  w += partials_bytes(o, nv);
  const int nf = o->model == WO_MODEL_FLUOR_3D ? 1 : 2;
  float2* ab = (float2*)w;
  w += align_up((size_t)nv * nf * s.Z * s.Y * s.X * sizeof(float2));
  WO_TRY(launch_set_params(dopt, h.data(), nv, hs));
  Sampling sm = sampling_of(o);
  for (int i = 0; i < n; ++i) sm.aberrated |= aberrated(o[i]) ? 1 : 0;
  // The label-free models compute and store only the columns of the
  // detection pupil's support; the 3D ones also keep the transfer function
  // in its support (columns kx < kt, band rows) until the Z pass, which
  // writes the full bank (zeros outside), when that compact copy fits the
  // field buffer behind the compact fields.
  bool compact_out = false;
  LatSupport sup = tf_support(o, n, s, &compact_out);
  float2* tf = (float2*)tf_out;
  const long M = s.Y * s.Xh;
  const long plane = s.Y * s.Xh;
  const long cplane = (long)sup.ly * sup.kt;   // a compact plane: ly rows of kt columns
  float2* cb = ab + compact_fields_elems(nv, nf, s, sup);
  WO_TRY(launch_tf_fields_y(dopt, sm, nv, ab, partials, hs, &sup));
  LatSupport full_out = sup;
  full_out.kt = (int)s.Xh;
  switch (o->model) {
    case WO_MODEL_FLUOR_3D:
      WO_TRY(launch_tf_rows_fluor(partials, sm, n, ab, tf, hs));
      WO_TRY(launch_cols(tf, (int)s.Y, s.Xh, s.Z, s.Z, n, -1.f, hs, "k_cols_y_tf"));
      WO_TRY(launch_cols(tf, (int)s.Z, M, 1, 1, n, -1.f, hs, "k_cols_z_tf"));
      break;
    case WO_MODEL_LABELFREE_3D:
      if (compact_out) {
        WO_TRY(launch_tf_rows_labelfree(partials, sm, n, ab, cb, 2 * s.Z * cplane, s.Z * cplane, cplane,
                                        hs, &sup, sup.kt));
        WO_TRY(launch_cols(cb, sup.ly, sup.kt, 2 * s.Z, 2 * s.Z, n, -1.f, hs, "k_cols_y_tf", 1, sup.ky));
        WO_TRY(launch_cols_expand(cb, tf, (int)s.Z, sup.ly, (int)s.Y, (int)s.Xh, sup.kt, sup.ky, 2L * n,
                                  -1.f, hs, band_out));
      } else {
        WO_TRY(launch_tf_rows_labelfree(partials, sm, n, ab, tf, 2 * s.Z * plane, s.Z * plane, plane, hs,
                                        &full_out));
        WO_TRY(launch_cols(tf, (int)s.Y, s.Xh, 2 * s.Z, 2 * s.Z, n, -1.f, hs, "k_cols_y_tf"));
        WO_TRY(launch_cols(tf, (int)s.Z, M, 2, 2, n, -1.f, hs, "k_cols_z_tf"));
      }
      break;
    case WO_MODEL_LABELFREE_THIN:
      WO_TRY(launch_tf_rows_labelfree(partials, sm, n, ab, tf, 2 * s.Z * plane, plane, 2 * plane, hs,
                                      &full_out));
      WO_TRY(launch_cols(tf, (int)s.Y, s.Xh, 2 * s.Z, 2 * s.Z, n, -1.f, hs, "k_cols_y_tf"));
      break;
    case WO_MODEL_SECTORS9_3D:
      // phase TF of every aperture: [patch][aperture][1][Z][Y][Xh]
      if (compact_out) {
        WO_TRY(launch_tf_rows_labelfree(partials, sm, nv, ab, cb, s.Z * cplane, -1, cplane, hs, &sup,
                                        sup.kt));
        WO_TRY(launch_cols(cb, sup.ly, sup.kt, s.Z, s.Z, nv, -1.f, hs, "k_cols_y_tf", 1, sup.ky));
        WO_TRY(launch_cols_expand(cb, tf, (int)s.Z, sup.ly, (int)s.Y, (int)s.Xh, sup.kt, sup.ky, nv, -1.f,
                                  hs, band_out));
      } else {
        WO_TRY(launch_tf_rows_labelfree(partials, sm, nv, ab, tf, s.Z * plane, -1, plane, hs, &full_out));
        WO_TRY(launch_cols(tf, (int)s.Y, s.Xh, s.Z, s.Z, nv, -1.f, hs, "k_cols_y_tf"));
        WO_TRY(launch_cols(tf, (int)s.Z, M, 1, 1, nv, -1.f, hs, "k_cols_z_tf"));
      }
      break;
    case WO_MODEL_POL5_3D: {
      // The 5 x 4 bank is the label-free pair mixed by a constant coupling:
      // the pair in the band layout [2][Z][band rows][kt] (the full layout
      // where the support fills the grid) is the reduced bank, written to
      // tf_out (band_out) or to the workspace and expanded into the full bank.
      float2* red = band_out ? tf : (float2*)w;
      int kt = (int)s.Xh, ky = (int)s.Y;
      if (compact_out) {
        WO_TRY(launch_tf_rows_labelfree(partials, sm, n, ab, cb, 2 * s.Z * cplane, s.Z * cplane, cplane,
                                        hs, &sup, sup.kt));
        WO_TRY(launch_cols(cb, sup.ly, sup.kt, 2 * s.Z, 2 * s.Z, n, -1.f, hs, "k_cols_y_tf", 1, sup.ky));
        WO_TRY(launch_cols_expand(cb, red, (int)s.Z, sup.ly, (int)s.Y, (int)s.Xh, sup.kt, sup.ky, 2L * n,
                                  -1.f, hs, true));
        kt = sup.kt;
        ky = sup.ky;
      } else {
        WO_TRY(launch_tf_rows_labelfree(partials, sm, n, ab, red, 2 * s.Z * plane, s.Z * plane, plane, hs,
                                        &full_out));
        WO_TRY(launch_cols(red, (int)s.Y, s.Xh, 2 * s.Z, 2 * s.Z, n, -1.f, hs, "k_cols_y_tf"));
        WO_TRY(launch_cols(red, (int)s.Z, M, 2, 2, n, -1.f, hs, "k_cols_z_tf"));
      }
      if (!band_out) {
        Coupling* cp = (Coupling*)((char*)w + align_up((size_t)n * 2 * s.Z * s.Y * s.Xh * sizeof(float2)));
        std::vector<Coupling> hc(n);
        for (int i = 0; i < n; ++i) hc[i] = coupling_of(o[i].swing);
        WO_TRY(launch_set_coupling(cp, hc.data(), n, hs));
        WO_TRY(launch_pol5_mix(cp, red, tf, (int)s.Z, (int)s.Y, (int)s.Xh, kt, ky, n, hs));
      }
      break;
    }
    default:
      return WO_EINVAL;
  }
  return WO_OK;
}

int wo_transfer_function(const wo_optics* o, int32_t n, void* tf_out, void* ws, size_t ws_bytes,
                         void* stream) {
  int st = validate(o, n);
  if (st) return st;
  if (!tf_out || !ws) return WO_EINVAL;
  Shape s;
  bank_shape(o, &s);
  if (ws_bytes < tf_ws(o, n, s)) return WO_ENOMEM;
  return run_tf(o, n, s, tf_out, ws, (hipStream_t)stream);
}

int wo_transfer_function_band(const wo_optics* o, int32_t n, void* tf_out, void* ws, size_t ws_bytes,
                              void* stream) {
  int st = validate(o, n);
  if (st) return st;
  if (!tf_out || !ws) return WO_EINVAL;
  Shape s;
  bank_shape(o, &s);
  // the band layout is the full one where the support fills the grid; else it
  // comes from the compact Z pass of the label-free 3D models
  bool compact_out = false;
  const LatSupport sup = tf_support(o, n, s, &compact_out);
  if (o->model != WO_MODEL_VECTOR_3D && !compact_out && (s.thin || sup.kt < s.Xh || sup.ky < s.Y))
    return WO_EUNSUPPORTED;
  if (ws_bytes < tf_ws(o, n, s)) return WO_ENOMEM;
  return run_tf(o, n, s, tf_out, ws, (hipStream_t)stream, true);
}

int wo_pol5_coupling(double swing, float* kappa_out) {
  if (!kappa_out || !isfinite(swing)) return WO_EINVAL;
  const Coupling c = coupling_of(swing);
  memcpy(kappa_out, &c.k[0][0][0], sizeof(c.k));
  return WO_OK;
}

int wo_linear_band(int32_t op, const wo_optics* o, int32_t n, const void* tf, const float* in,
                   const float* b, double eta, float* out, void* ws, size_t ws_bytes, void* stream) {
  if (!o || n < 1) return WO_EINVAL;
  if (op != WO_OP_FORWARD && op != WO_OP_RECONSTRUCT && op != WO_OP_ADJOINT) return WO_EINVAL;
  int st = check_sampling(o);
  if (st) return st;
  for (int i = 1; i < n; ++i)
    if (!same_sampling(&o[0], &o[i])) return WO_EINVAL;
  if (!tf || !in || !out || !ws) return WO_EINVAL;
  Shape s;
  bank_shape(o, &s);
  if (s.thin) return WO_EUNSUPPORTED;
  if (s.P != 1 && s.P != 2 && s.P != 4) return WO_EUNSUPPORTED;
  if (!zop_fits((int)s.Z, std::max(s.C, s.P))) return WO_EUNSUPPORTED;
  const int mode = op == WO_OP_FORWARD ? kModeForward : (op == WO_OP_RECONSTRUCT ? kModeSolve : kModeAdjoint);
  if (mode == kModeSolve) {
    if (!(eta >= 0.0) || !isfinite(eta)) return WO_EINVAL;
    if (eta == 0.0 && s.P != 1) return WO_EUNSUPPORTED;
  }
  if (ws_bytes < linear_ws(n, s)) return WO_ENOMEM;
  return run_linear(o, n, s, (const float2*)tf, in, out, mode == kModeAdjoint ? nullptr : b, mode,
                    mode == kModeSolve ? (float)eta : 0.f, ws, (hipStream_t)stream, true, is_pol5(s));
}

int wo_forward(const wo_optics* o, int32_t n, const void* tf, const float* f, const float* b,
               float* d_out, void* ws, size_t ws_bytes, void* stream) {
  if (!o || n < 1) return WO_EINVAL;
  int st = check_sampling(o);
  if (st) return st;
  for (int i = 1; i < n; ++i)
    if (!same_sampling(&o[0], &o[i])) return WO_EINVAL;
  if (!tf || !f || !d_out || !ws) return WO_EINVAL;
  Shape s;
  bank_shape(o, &s);
  if (s.P != 1 && s.P != 2 && s.P != 4) return WO_EUNSUPPORTED;
  if (!s.thin && !zop_fits((int)s.Z, std::max(s.C, s.P))) return WO_EUNSUPPORTED;
  if (ws_bytes < linear_ws(n, s)) return WO_ENOMEM;
  return run_linear(o, n, s, (const float2*)tf, f, d_out, b, kModeForward, 0.f, ws,
                    (hipStream_t)stream);
}

int wo_reconstruct(const wo_optics* o, int32_t n, const void* tf, const float* d, const float* b,
                   double eta, float* f_out, void* ws, size_t ws_bytes, void* stream) {
  if (!o || n < 1) return WO_EINVAL;
  int st = check_sampling(o);
  if (st) return st;
  for (int i = 1; i < n; ++i)
    if (!same_sampling(&o[0], &o[i])) return WO_EINVAL;
  if (!tf || !d || !f_out || !ws) return WO_EINVAL;
  if (!(eta >= 0.0) || !isfinite(eta)) return WO_EINVAL;
  Shape s;
  bank_shape(o, &s);
  if (s.P != 1 && s.P != 2 && s.P != 4) return WO_EUNSUPPORTED;
  if (!s.thin && !zop_fits((int)s.Z, std::max(s.C, s.P))) return WO_EUNSUPPORTED;
  if (eta == 0.0 && s.P != 1) return WO_EUNSUPPORTED;
  if (ws_bytes < linear_ws(n, s)) return WO_ENOMEM;
  return run_linear(o, n, s, (const float2*)tf, d, f_out, b, kModeSolve, (float)eta, ws,
                    (hipStream_t)stream);
}

int wo_adjoint(const wo_optics* o, int32_t n, const void* tf, const float* r, float* g_out,
               void* ws, size_t ws_bytes, void* stream) {
  if (!o || n < 1) return WO_EINVAL;
  int st = check_sampling(o);
  if (st) return st;
  for (int i = 1; i < n; ++i)
    if (!same_sampling(&o[0], &o[i])) return WO_EINVAL;
  if (!tf || !r || !g_out || !ws) return WO_EINVAL;
  Shape s;
  bank_shape(o, &s);
  if (s.P != 1 && s.P != 2 && s.P != 4) return WO_EUNSUPPORTED;
  if (!s.thin && !zop_fits((int)s.Z, std::max(s.C, s.P))) return WO_EUNSUPPORTED;
  if (ws_bytes < linear_ws(n, s)) return WO_ENOMEM;
  return run_linear(o, n, s, (const float2*)tf, r, g_out, nullptr, kModeAdjoint, 0.f, ws,
                    (hipStream_t)stream);
}

}  // extern "C"

// ---------------------------------------------------------------- gradient of a loss of the 3D reconstruction

namespace {

// Columns the gradient of the 3D reconstruction keeps of both fields: the
// detection pupil's lateral support (the source's lies within it), which holds
// the pupils' derivatives too (the soft edge is inside the bound); transforms
// on the grid's own lengths.
LatSupport grad3_support(const wo_optics* o, int32_t n) {
  const Sampling sm = sampling_of(o);
  LatSupport ls = full_support(sm);
  const LatSupport lat = lateral_support(o, n);
  ls.xc = ls.xa = lat.xc;
  ls.kp = ls.kpa = lat.kp;
  return ls;
}

struct Grad3Layout {
  size_t opt, st, pp, lp, dp, gp, ip, ab, bank, D, G, cpl, total;
};

Grad3Layout grad3_layout(const wo_optics* o, int32_t n, const Shape& s, const LatSupport& sup) {
  const Sampling sm = sampling_of(o);
  const long plane = s.Y * s.Xh;
  Grad3Layout L;
  size_t b = 0;
  auto take = [&](size_t bytes) { size_t o0 = b; b += align_up(bytes); return o0; };
  L.opt = take((size_t)n * sizeof(DevOptics));
  L.st = take((size_t)n * sizeof(TuneState));
  L.pp = take((size_t)n * ((s.X + tf_tile_width(sm) - 1) / tf_tile_width(sm)) * sizeof(double));
  L.lp = take((size_t)n * loss_blocks(sm) * sizeof(double));
  L.dp = take((size_t)n * bwd_wg_per_patch(sm) * sizeof(double));
  L.gp = take((size_t)n * s.Z * grad_tiles(sm) * kGradAll * sizeof(double));
  L.ip = take((size_t)n * grad_tiles(sm) * kThetaAll * sizeof(double));
  L.ab = take((size_t)n * 2 * s.Z * s.Y * sup.xc * sizeof(float2));
  L.bank = take((size_t)n * s.Z * 2 * plane * sizeof(float2));
  L.D = take((size_t)n * s.C * s.Z * plane * sizeof(float2));
  L.G = take((size_t)n * s.P * s.Z * plane * sizeof(float2));
  L.cpl = take((size_t)n * sizeof(Coupling));
  L.total = b;
  return L;
}

bool grad3_model(const wo_optics* o) {
  return o->model == WO_MODEL_LABELFREE_3D || o->model == WO_MODEL_POL5_3D;
}

}  // namespace

extern "C" size_t wo_reconstruct_grad_workspace_size(const wo_optics* o, int32_t n) {
  Shape s;
  if (!o || n < 1 || !bank_shape(o, &s) || !grad3_model(o)) return 0;
  return grad3_layout(o, n, s, grad3_support(o, n)).total;
}

extern "C" int wo_reconstruct_grad(const wo_optics* o, int32_t n, const float* d, const float* b,
                                   double eta, const float* dL_df, double* dL_dtheta_out, float* dL_dd_out,
                                   void* ws, size_t ws_bytes, void* stream) {
  int st = validate(o, n);
  if (st) return st;
  if (!grad3_model(o)) return WO_EUNSUPPORTED;
  if (!d || !dL_df || !ws || (!dL_dtheta_out && !dL_dd_out)) return WO_EINVAL;
  if (!(eta > 0.0) || !isfinite(eta)) return WO_EINVAL;
  Shape s;
  bank_shape(o, &s);
  const LatSupport sup = grad3_support(o, n);
  const Grad3Layout L = grad3_layout(o, n, s, sup);
  if (ws_bytes < L.total) return WO_ENOMEM;
  if (n > 65535) return WO_EUNSUPPORTED;
  hipStream_t hs = (hipStream_t)stream;
  char* w = (char*)ws;
  DevOptics* dopt = (DevOptics*)(w + L.opt);
  TuneState* tst = (TuneState*)(w + L.st);
  double* pp = (double*)(w + L.pp);
  double* lp = (double*)(w + L.lp);
  double* dp = (double*)(w + L.dp);
  double* gp = (double*)(w + L.gp);
  double* ip = (double*)(w + L.ip);
  float2* ab = (float2*)(w + L.ab);
  float2* bank = (float2*)(w + L.bank);
  float2* D = (float2*)(w + L.D);
  float2* G = (float2*)(w + L.G);
  Coupling* cpl = is_pol5(s) ? (Coupling*)(w + L.cpl) : nullptr;
  {
    std::vector<DevOptics> h(n);
    std::vector<TuneState> t(n);
    std::vector<Coupling> hc(n);
    for (int i = 0; i < n; ++i) {
      h[i] = dev_optics(o[i]);
      memset(&t[i], 0, sizeof(TuneState));
      t[i].band_count = 1.0;   // no loss of its own: the loss partials are zero
      t[i].eta = eta;
      if (cpl) hc[i] = coupling_of(o[i].swing);
    }
    WO_TRY(launch_set_params(dopt, h.data(), n, hs));
    WO_TRY(launch_set_tune(tst, t.data(), n, hs));
    if (cpl) WO_TRY(launch_set_coupling(cpl, hc.data(), n, hs));
  }
  Sampling sm = sampling_of(o);
  for (int i = 0; i < n; ++i) sm.aberrated |= aberrated(o[i]) ? 1 : 0;
  sm.det_grad = 1;   // also d/d(det_tilt, det_azimuth)
  const long Z = s.Z, Y = s.Y, X = s.X, Xh = s.Xh, plane = Y * Xh;
  const int C = s.C, P = s.P;
  const double nfull = (double)Z * Y * X;
  WO_TRY(hipMemsetAsync(lp, 0, (size_t)n * loss_blocks(sm) * sizeof(double), hs));
  // the label-free pair at these optics, per plane then along Z: [v][Z][2][Y][Xh]
  WO_TRY(launch_tf_fields_y(dopt, sm, n, ab, pp, hs, &sup));
  WO_TRY(launch_tf_rows_labelfree(pp, sm, n, ab, bank, 2 * Z * plane, plane, 2 * plane, hs, &sup));
  WO_TRY(launch_cols(bank, (int)Y, Xh, 2 * Z, 2 * Z, n, -1.f, hs, "k_cols_y_tf"));
  WO_TRY(launch_cols(bank, (int)Z, 2 * plane, 1, 1, n, -1.f, hs, "k_cols_z_tf"));
  // spectra of the data and of dL/df
  WO_TRY(launch_rows_r2c(d, D, (int)X, RowGroups{C * Z * Y, C * Z * Y, C * Z * Y, n}, hs));
  WO_TRY(launch_cols(D, (int)Y, Xh, C * Z, C * Z, n, -1.f, hs, "k_cols_y_fwd"));
  WO_TRY(launch_cols(D, (int)Z, plane, C, C, n, -1.f, hs, "k_cols_z_fwd"));
  WO_TRY(launch_rows_r2c(dL_df, G, (int)X, RowGroups{P * Z * Y, P * Z * Y, P * Z * Y, n}, hs));
  WO_TRY(launch_cols(G, (int)Y, Xh, P * Z, P * Z, n, -1.f, hs, "k_cols_y_fwd"));
  WO_TRY(launch_cols(G, (int)Z, plane, P, P, n, -1.f, hs, "k_cols_z_fwd"));
  // dL/dH* of the pair per frequency (and H Y, the spectrum of dL/dd)
  WO_TRY(launch_recon_grad(bank, D, G, b, cpl, sm, n, (float)eta, nfull, dL_dd_out ? 1 : 0, hs));
  if (dL_dtheta_out) {
    // per-plane 2D gradients (the adjoint of the Z transform), then the
    // per-plane reverse mode through the synthesis shared with the thin model
    WO_TRY(launch_cols(bank, (int)Z, 2 * plane, 1, 1, n, 1.f, hs, "k_cols_z_grad"));
    WO_TRY(launch_cols(bank, (int)Y, Xh, 2 * Z, 2 * Z, n, 1.f, hs, "k_cols_y_grad"));
    WO_TRY(launch_tf_rows_bwd(pp, sm, n, ab, bank, dp, hs, &sup));
    WO_TRY(launch_tf_grad_y(dopt, sm, n, ab, gp, ip, hs, &sup));
    WO_TRY(launch_adam(dopt, tst, sm, n, pp, lp, dp, gp, ip, 0, hs, &sup));
  }
  if (dL_dd_out) {
    WO_TRY(launch_cols(D, (int)Z, plane, C, C, n, 1.f, hs, "k_cols_z_inv"));
    WO_TRY(launch_cols(D, (int)Y, Xh, C * Z, C * Z, n, 1.f, hs, "k_cols_y_inv"));
    WO_TRY(launch_rows_c2r(D, dL_dd_out, (int)X, RowGroups{C * Z * Y, C * Z * Y, C * Z * Y, n},
                           (float)(1.0 / nfull), hs));
  }
  if (dL_dtheta_out) {
    std::vector<TuneState> t(n);
    WO_TRY(hipMemcpyAsync(t.data(), tst, n * sizeof(TuneState), hipMemcpyDeviceToHost, hs));
    WO_TRY(hipStreamSynchronize(hs));
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < kThetaAll; ++j) dL_dtheta_out[kThetaAll * i + j] = t[i].grad[j];
  }
  return WO_OK;
}

// ---------------------------------------------------------------- reconstruction without allocation
//
// Scratch of wo_reconstruct_noalloc: one copy of this array per GPU, held until
// the process ends.  In host code `scratch` names a host-side stand-in, not a
// device address; the device address comes from hipGetSymbolAddress, taken
// once per device with that device current, and only that address is used.
static __device__ __align__(256) unsigned char scratch[WO_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of the current device's scratch (resolved on its first use).
int scratch_address(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return WO_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return WO_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return WO_EHIP;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return WO_OK;
}
}  // namespace

extern "C" int wo_reconstruct_noalloc(const wo_optics* o, int32_t n, const void* tf, const float* d,
                                      const float* b, double eta, float* f_out, void* stream) {
  if (!o || n < 1) return WO_EINVAL;
  int st = check_sampling(o);
  if (st) return st;
  for (int i = 1; i < n; ++i)
    if (!same_sampling(&o[0], &o[i])) return WO_EINVAL;
  if (!tf || !d || !f_out) return WO_EINVAL;
  if (!(eta >= 0.0) || !isfinite(eta)) return WO_EINVAL;
  Shape s;
  bank_shape(o, &s);
  if (s.P != 1 && s.P != 2 && s.P != 4) return WO_EUNSUPPORTED;
  if (!s.thin && !zop_fits((int)s.Z, std::max(s.C, s.P))) return WO_EUNSUPPORTED;
  if (eta == 0.0 && s.P != 1) return WO_EUNSUPPORTED;
  if (linear_ws(n, s) > (size_t)WO_NOALLOC_SCRATCH_BYTES) return WO_ENOMEM;
  // the stream must run on the current device, whose scratch is used
  hipStream_t hs = (hipStream_t)stream;
  if (hs) {
    int cur = 0;
    hipDevice_t sdev = 0;
    if (hipGetDevice(&cur) != hipSuccess || hipStreamGetDevice(hs, &sdev) != hipSuccess) return WO_EHIP;
    if ((int)sdev != cur) return WO_EINVAL;
  }
  void* ws = nullptr;
  st = scratch_address(&ws);
  if (st) return st;
  // the linear pipeline writes every scratch value it reads: nothing to clear
  return run_linear(o, n, s, (const float2*)tf, d, f_out, b, kModeSolve, (float)eta, ws, hs);
}

extern "C" {

size_t wo_tune_workspace_size(const wo_optics* o, int32_t n, int32_t starts) {
  if (!o || n < 1 || starts < 1) return 0;
  for (int i = 0; i < n; ++i)
    if (o[i].model != WO_MODEL_LABELFREE_THIN) return 0;
  size_t total = 0;
  tune_groups(o, n, starts, &total);
  return total;
}

static int midband(const wo_optics* o, int32_t n, const float* d, const double* eta, const double* nu_c,
                   double* loss_out, double* grad_out, int with_aberration, void* ws, size_t ws_bytes,
                   void* stream) {
  int st = validate_thin(o, n);
  if (st) return st;
  if (!d || !eta || !ws || !loss_out) return WO_EINVAL;
  for (int i = 0; i < n; ++i)
    if (!(eta[i] > 0.0)) return WO_EINVAL;
  size_t need = 0;
  std::vector<TuneGroup> groups = tune_groups(o, n, 1, &need);
  if (ws_bytes < need) return WO_ENOMEM;
  if (with_aberration)
    for (auto& g : groups) g.ab = 1;
  const std::vector<size_t> doff = packed_offsets(o, n, true);
  hipStream_t hs = (hipStream_t)stream;
  char* w = (char*)ws;
  for (auto& g : groups) {
    st = tune_setup(o, g, 1, nullptr, d, doff.data(), eta, nu_c, nullptr, nullptr, nullptr, 0, w, hs);
    if (st) return st;
    st = tune_iteration(g, w, 1, 0, hs);
    if (st) return st;
  }
  for (auto& g : groups) {
    std::vector<TuneState> h(g.L.np);
    WO_TRY(hipMemcpyAsync(h.data(), w + g.base + g.L.off_st, g.L.np * sizeof(TuneState),
                          hipMemcpyDeviceToHost, hs));
    WO_TRY(hipStreamSynchronize(hs));
    for (int j = 0; j < g.L.np; ++j) {
      const int i = g.idx[j];
      loss_out[i] = h[j].loss;
      if (grad_out && with_aberration) {
        for (int k = 0; k < 4; ++k) grad_out[11 * i + k] = h[j].grad[k];
        for (int k = 0; k < 7; ++k) grad_out[11 * i + 4 + k] = h[j].gab[k];
      } else if (grad_out) {
        for (int k = 0; k < 4; ++k) grad_out[4 * i + k] = h[j].grad[k];
      }
    }
  }
  return WO_OK;
}

int wo_midband_loss_grad(const wo_optics* o, int32_t n, const float* d, const double* eta,
                         const double* nu_c, double* loss_out, double* grad_out, void* ws,
                         size_t ws_bytes, void* stream) {
  return midband(o, n, d, eta, nu_c, loss_out, grad_out, 0, ws, ws_bytes, stream);
}

int wo_midband_loss_grad_aberration(const wo_optics* o, int32_t n, const float* d, const double* eta,
                                    const double* nu_c, double* loss_out, double* grad_out, void* ws,
                                    size_t ws_bytes, void* stream) {
  return midband(o, n, d, eta, nu_c, loss_out, grad_out, 1, ws, ws_bytes, stream);
}

int wo_autotune(wo_optics* o, int32_t n, const float* d, const double* eta,
                const wo_autotune_opts* opts, double* loss_out, void* ws, size_t ws_bytes,
                void* stream) {
  return run_tune(o, n, d, eta, opts, loss_out, nullptr, ws, ws_bytes, stream);
}

int wo_restore_tiles(wo_optics* o, int32_t n, const float* d, const double* eta,
                     const wo_autotune_opts* opts, double* loss_out, float* f_out, void* ws,
                     size_t ws_bytes, void* stream) {
  if (!f_out) return WO_EINVAL;
  return run_tune(o, n, d, eta, opts, loss_out, f_out, ws, ws_bytes, stream);
}

}  // extern "C"
