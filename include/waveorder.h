/*
 * waveorder.h -- C ABI of the MI355X (gfx950) WaveOrder hot path.
 *
 * WaveOrder (arXiv 2412.09775) models an imaging system as d = H f + b
 * (Methods, "Imaging and reconstruction as linear operators", Eq. fwd) with a
 * bank of shift-invariant transfer functions H_cp, one per data channel c and
 * object property p (Methods, "Linear contrast-separable shift-invariant
 * imaging systems"), built from an illumination pupil S, a scattering model G
 * and a detection pupil P (Methods, "Summary of transfer functions"; Table 1),
 * and reconstructs f by a Tikhonov-regularised least-squares solve
 * (Methods, "Reconstructing object properties" and "Reconstruction
 * algorithm", Eq. tls_solution).
 *
 * Conventions shared by every call
 * --------------------------------
 *  * All array pointers are DEVICE pointers owned by the caller.  The library
 *    never allocates device memory: scratch space comes from `ws`, whose size
 *    wo_workspace_size() gives.  Nothing is freed by the library.
 *  * Calls are asynchronous on `stream` (a hipStream_t, NULL = default
 *    stream); arguments are validated synchronously before anything is
 *    enqueued, and an error leaves the outputs untouched.  The optics array
 *    `o` is host memory and is read (and copied into `ws`) during the call.
 *  * A call processes `n` patches that share the sampling (model, nz, ny, nx,
 *    dz, dy, dx) but may differ in every optical parameter.  Patch i of an
 *    array argument follows patch i-1 contiguously.
 *  * Volumes are float32, C-contiguous [Z][Y][X] with X fastest.  Channel and
 *    property maps of one patch are stacked in front: [C][Z][Y][X].
 *  * Spectra and transfer functions are complex64 (interleaved re, im) on the
 *    half spectrum along X: kx = 0..X/2, so Xh = X/2 + 1 values per row; ky
 *    and kz are in FFT order (DC first).  The full spectrum is the Hermitian
 *    extension H(-nu) = conj(H(nu)) (transfer functions of real data are
 *    Hermitian, Methods "Summary of transfer functions").
 *  * Sizes nz, ny, nx must factor into 2, 3 and 5 and lie in [1, 4096] (ny, nx
 *    even); otherwise WO_EUNSUPPORTED.  wo_forward, wo_reconstruct and
 *    wo_adjoint of a 3D model also need max(C, P) * nz <= 8192 (one Z line of
 *    every channel and property in one workgroup), else WO_EUNSUPPORTED.
 *  * Units: lengths in micrometres, angles in radians.  Label-free properties
 *    are radians per voxel (phase 2 pi dn dz / lambda0, absorption
 *    2 pi dkappa dz / lambda0); label-free data are the relative contrast
 *    I / I_bg - 1.
 *
 * Models (WO_MODEL_*), bank shape C x P and spatial dimensions:
 *   FLUOR_3D        1 x 1, 3D  scalar fluorescence OTF [P * P], H(0) = 1
 *   LABELFREE_3D    1 x 2, 3D  scalar label-free [phase, absorption]
 *   LABELFREE_THIN  nz x 2, 2D phase from a defocus stack: channel k is the
 *                   plane at z_k = dz (k - (nz-1)/2); properties are a thin
 *                   object [phase, absorption] of shape [Y][X]
 *   POL5_3D         5 x 4, 3D  five polarisation states (swing) through a
 *                   circular analyser; properties [phase, rho cos 2w,
 *                   rho sin 2w, absorption]
 *   SECTORS9_3D     9 x 1, 3D  multi-aperture phase: channels 0-7 illuminate
 *                   through the azimuthal sectors [c pi/4, (c+1) pi/4) of the
 *                   source disc (about its centre; the centre point in sector
 *                   0), channel 8 through the full disc; each channel's data
 *                   are relative to its own background (Results,
 *                   cardiomyocytes; Methods "Cardiomyocyte reconstructions";
 *                   Fig. 4c's 9 x 1 column)
 *   VECTOR_3D       C x P, 3D  vector (non-paraxial) label-free bank (Table 1,
 *                   vector column): C = 4 Stokes channels or the 5 swing
 *                   states, P = vec_nprops spherical-harmonic coefficients
 *                   (see the vec_* fields of wo_optics)
 */
#ifndef WAVEORDER_H
#define WAVEORDER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  WO_OK = 0,
  WO_EINVAL = -1,        /* bad argument or optics outside the model's validity */
  WO_EUNSUPPORTED = -2,  /* size or mode the kernels do not implement */
  WO_ENOMEM = -3,        /* workspace smaller than wo_workspace_size() */
  WO_EHIP = -4,          /* the HIP runtime reported an error */
  WO_EALIAS = -5,        /* transfer-function support exceeds the sampled band */
  WO_DIVERGED = -6       /* per patch (wo_autotune status_out): no start ended with a
                            finite loss and finite parameters */
};

enum {
  WO_MODEL_FLUOR_3D = 0,
  WO_MODEL_LABELFREE_3D = 1,
  WO_MODEL_LABELFREE_THIN = 2,
  WO_MODEL_POL5_3D = 3,
  WO_MODEL_SECTORS9_3D = 4,
  WO_MODEL_VECTOR_3D = 5
};

enum {
  WO_OP_TRANSFER_FUNCTION = 0,
  WO_OP_FORWARD = 1,
  WO_OP_RECONSTRUCT = 2,
  WO_OP_ADJOINT = 3
};

/* Optics and sampling of one patch (Ext. Data Fig. 3: calc_ill_pupil takes
 * NA_ill and the tilt; calc_det_pupil takes NA_det and the defocus offset). */
typedef struct wo_optics {
  int32_t model;           /* WO_MODEL_* */
  int32_t nz, ny, nx;      /* volume shape */
  double dz, dy, dx;       /* voxel size, um */
  double wavelength;       /* vacuum wavelength lambda0, um (emission for fluorescence) */
  double na_ill;           /* illumination NA (ignored for fluorescence) */
  double na_det;           /* detection NA */
  double n_medium;         /* refractive index of the medium; the pupils live on the
                              shell of radius n / lambda0 */
  double defocus;          /* focal-plane offset dz0, um: every plane z -> z - dz0 */
  double tilt_zenith;      /* illumination tilt: source disc centred at */
  double tilt_azimuth;     /*   (n sin(zenith)/lambda0)(cos az, sin az) in (x, y) */
  double edge_width;       /* pupil edge: 0 = hard disc (boundary included); w > 0 =
                              C1 smoothstep of half-width w lateral frequency pixels */
  double swing;            /* POL5_3D only: retarder swing in waves */
  double zernike[7];       /* detection aberration, waves, on Zernike polynomials
                              Noll j = 5..11 (astigmatism 5, 6; coma 7, 8; trefoil
                              9, 10; primary spherical 11), unit-RMS (Noll)
                              normalisation over the pupil radius NA_det/lambda0:
                              the detection pupil becomes P(p) exp(i 2 pi W(p)),
                              W = sum_j zernike[j-5] Z_j(rho, phi), rho = |p| /
                              (NA_det/lambda0), phi = atan2(p_y, p_x) (Methods,
                              detection-parameter branch: Zernike coefficients in
                              calc_det_pupil).  Zero: no aberration. */
  /* Oblique detection (the light-path figure's oblique detection path;
     neuromasts imaged with oblique and straight detection): the detection
     axis is tilted by det_tilt (zenith, rad) in the azimuth det_azimuth,
     a = (sin t sin az, sin t cos az, cos t) in (y, x, z), and the detection
     pupil is the cap of the shell within NA_det about it:
     P = edge(NA_det/lambda0 - |p'|), |p'|^2 = (n/lambda0)^2 - (k . a)^2,
     k = (p, kz(p)), k . a > 0 (the disc at det_tilt = 0).  The cap must stay
     inside the shell (WO_EINVAL); not combined with zernike
     (WO_EUNSUPPORTED).  The data stay on the sample grid. */
  double det_tilt;
  double det_azimuth;
  /* Vector label-free model (WO_MODEL_VECTOR_3D; Table 1, vector column,
     label-free row; Methods "Physically interpretable basis functions").  The
     source point q of the disc illuminates with the plane wave of
     polarisation e(q) = Q(q) J, J the Jones vector in the condenser pupil and
     Q(q) = t^ r^T + f^ f^_t^T the aplanatic map of the pupil's radial and
     azimuthal directions onto the wave's polar and azimuthal unit vectors;
     the detection pupil tensor is P E Q^T and the Green's tensor spectrum
     (I - k^ k^T) g.  Channels (vec_channels): 0 the four Stokes parameters
     S0..S3 of the detected field (analysers I, diag(1, -1), [[0, 1], [1, 0]],
     [[0, -i], [i, 0]]) under the Jones state ill_jones; 1 the five swing
     states of POL5_3D through its circular analyser.  Properties: vec_nprops
     (1..8) real coefficients, property k of the tensor Y_b (vec_props[k] =
     2 b) or i Y_b (2 b + 1) with the spherical-harmonic tensors b = 0 the
     identity (phase; its imaginary coefficient absorption), 1..3 the
     antisymmetric (yz - zy)/2, (zx - xz)/2, (xy - yx)/2, 4..8 the symmetric
     traceless (xy + yx)/2, (yz + zy)/2, (2zz - xx - yy)/(2 sqrt 3),
     (xz + zx)/2, (xx - yy)/2.  Data are E^H M_c E / I_bg with the channel
     background J^H M_c J.  Every patch of a call has the same channels and
     properties.  Not combined with det_tilt (WO_EUNSUPPORTED).  The linear
     calls take vec_nprops 1, 2 or 4.  Other models ignore these fields. */
  int32_t vec_channels;
  int32_t vec_nprops;
  int32_t vec_props[8];
  double ill_jones[4];     /* re Jx, im Jx, re Jy, im Jy */
} wo_optics;

/* Bank shape of the model: *C channels, *P properties, *dims spatial
 * dimensions (3 or 2); *bank_elems complex64 values per patch
 * (C*P*nz*ny*Xh for 3D models, C*P*ny*Xh for the thin model). */
int wo_bank_shape(const wo_optics* o, int32_t* C, int32_t* P, int32_t* dims, int64_t* bank_elems);

/* Workspace bytes an operation (WO_OP_*) needs for n patches of this sampling. */
size_t wo_workspace_size(const wo_optics* o, int32_t n, int32_t op);

/* Transfer-function bank (Table 1, scalar column; the polarisation bank is
 * the paraxial Jones reduction H_cp = Re(kappa_cp) H_phase + Im(kappa_cp) H_abs;
 * WO_MODEL_VECTOR_3D the vector column: H_cp = FFT3(2 Re R_cp) with the
 * first-order channel response R_cp = 1/(Y X I_bg) sum M_c^{ii'} conj(v_ik)
 * u_i'n T_p^{nk} of the detected scattered fields u = IFFT2[P_i'j G_jn prop]
 * and the detected direct fields times the conjugate incident field
 * v = IFFT2[S P_ik' e_k' conj(e_k) prop], computed on the full lateral grid).
 * tf_out: complex64 [n][C][P][nz][ny][Xh] (3D) or [n][nz][2][ny][Xh] (thin).
 * WO_EINVAL if a pupil reaches the evanescent boundary n/lambda0 or an NA,
 * size or wavelength is not positive; WO_EALIAS if the lateral support
 * exceeds the lateral Nyquist frequency or the axial support the axial one. */
int wo_transfer_function(const wo_optics* o, int32_t n, void* tf_out, void* ws, size_t ws_bytes,
                         void* stream);

/* Lateral support of the model's fields and transfer-function bank for n
 * patches (Methods, pupils): the detection pupil is zero beyond NA_det/lambda0
 * and the source beyond its tilted disc of radius NA_ill/lambda0 (each widened
 * by the soft edge), so the label-free field B = P g e^{..} vanishes outside
 * the detection pupil's columns, A = S P e^{..} also outside the source's, and
 * the bank outside the sum of the two supports (twice the detection pupil's
 * for fluorescence).  Bounds keep one spare column or row and are rounded up
 * to multiples of 16.  The 3D linear calls (wo_forward, wo_reconstruct,
 * wo_adjoint) read the bank only within the support and take it as zero
 * elsewhere, as wo_transfer_function writes it. */
typedef struct wo_support {
  int32_t field_cols[2];  /* lateral columns the synthesis keeps of field A (or the
                             fluorescence field) and of B (0: no second field); the
                             vector model keeps every field on B's columns */
  int32_t tf_cols;        /* the bank's half-spectrum columns k < tf_cols can be nonzero */
  int32_t band_rows;      /* and its rows y <= ky or y >= ny - ky: 2 ky + 1 (ny: all) */
  int32_t tf_lengths[2];  /* (y, x) transform lengths of the synthesis: the bank is a
                             correlation of the fields' spectra, so lengths beyond its
                             extent give it exactly; the label-free 3D models, and the
                             vector model where that x length is compiled, use the
                             shortest compiled lengths that hold it, the others (ny, nx) */
} wo_support;
int wo_lateral_support(const wo_optics* o, int32_t n, wo_support* out);

/* Forward model D_c = sum_p H_cp F_p + N b_c delta(nu), d_c = IFFT(D_c)
 * (Methods, "Linear contrast-separable shift-invariant imaging systems").
 * tf: bank from wo_transfer_function, or any Hermitian bank of that layout
 * that vanishes outside the model's lateral support (wo_lateral_support; the
 * 3D models do not read it there);
 * f: [n][P][vol], b: [n][C] or NULL, d_out: [n][C][vol]; vol = nz*ny*nx
 * (3D) or ny*nx for the thin model's object. */
int wo_forward(const wo_optics* o, int32_t n, const void* tf, const float* f, const float* b,
               float* d_out, void* ws, size_t ws_bytes, void* stream);

/* Tikhonov reconstruction f = argmin ||d - b - H f||^2 + eta ||f||^2, solved
 * per spatial frequency as F = (H^H H + eta I)^-1 H^H (D - N b delta)
 * (Eq. recon and Eq. tls_solution).  d: [n][C][vol], b: [n][C] or NULL,
 * f_out: [n][P][vol] (thin: [n][2][ny][nx]).  eta >= 0 (absolute); eta == 0
 * is supported for P == 1 only (F = 0 where H = 0), else WO_EUNSUPPORTED. */
int wo_reconstruct(const wo_optics* o, int32_t n, const void* tf, const float* d, const float* b,
                   double eta, float* f_out, void* ws, size_t ws_bytes, void* stream);

/* The bank on its lateral support (see wo_lateral_support): [n][C][P][nz][band_rows][tf_cols] complex64, row b of a
 * plane the bank's row y = b (b <= ky) or ny - band_rows + b, columns
 * k < tf_cols of the half spectrum; every other value of the full bank is zero
 * and implied, as the Hermitian half is.  The values are those
 * wo_transfer_function writes there, bit for bit.  Label-free 3D models
 * (one or nine apertures), the polarisation model, the vector model, or any
 * 3D model whose support fills the grid (then the layout is the full one);
 * others: WO_EUNSUPPORTED.  Workspace as for wo_transfer_function.
 *
 * POL5_3D is stored in reduced form: its 5 x 4 bank is a constant mix of the
 * label-free pair, H_cp = Re(kappa_cp) H_phase + Im(kappa_cp) H_abs (the
 * paraxial Jones reduction of Table 1's vector row; kappa from
 * wo_pol5_coupling), so the band layout holds only that pair,
 * [n][2][nz][band_rows][tf_cols] (H_phase, H_abs), a tenth of the entries.
 * wo_transfer_function's full bank is exactly its expansion: on the support
 * each entry is Re(kappa) * H_phase + Im(kappa) * H_abs evaluated in FP32 with
 * every product and the sum rounded on their own (no fused multiply-add),
 * zero elsewhere. */
int wo_transfer_function_band(const wo_optics* o, int32_t n, void* tf_out, void* ws, size_t ws_bytes,
                              void* stream);
/* wo_forward (op WO_OP_FORWARD: in = f, out = d, eta ignored), wo_reconstruct
 * (WO_OP_RECONSTRUCT: in = d, out = f) or wo_adjoint (WO_OP_ADJOINT: in = r,
 * out = g, b ignored) with the bank in the band layout of
 * wo_transfer_function_band; results bit for bit those of the full-layout
 * call.  POL5_3D takes the reduced form: the forward model and the adjoint
 * form the entries per frequency from the pair and each patch's coupling (bit
 * for bit as above); the reconstruction forms H^H H and H^H x from the pair and
 * constants of the coupling without the entries (the same solve up to FP32
 * rounding order).  3D models only (thin: WO_EUNSUPPORTED); workspace as for
 * those calls. */
int wo_linear_band(int32_t op, const wo_optics* o, int32_t n, const void* tf, const float* in,
                   const float* b, double eta, float* out, void* ws, size_t ws_bytes, void* stream);

/* Polarisation coupling of the POL5_3D model for a swing (host only, no GPU
 * work): kappa_cp = conj(a^H e_c) (a^H B_p e_c) for the five illumination
 * states e_c (the extinction state e_0 = (1, i)/sqrt2 and four retarder
 * settings of that swing), the circular analyser a = (1, -i)/sqrt2 and the
 * property matrices B_p (phase I, rho cos 2w diag(1, -1)/2,
 * rho sin 2w [[0, 1], [1, 0]]/2, absorption i I), computed in FP64 and
 * rounded once to the FP32 values the kernels use:
 * kappa_out[(c * 4 + p) * 2 + {0, 1}] = (re, im).  WO_EINVAL if swing is not
 * finite or kappa_out is NULL. */
int wo_pol5_coupling(double swing, float* kappa_out);

/* Adjoint g_p = IFFT(sum_c conj(H_cp) R_c): r [n][C][vol] -> g_out [n][P][vol]. */
int wo_adjoint(const wo_optics* o, int32_t n, const void* tf, const float* r, float* g_out,
               void* ws, size_t ws_bytes, void* stream);

/* Gradient of a scalar loss of the Tikhonov reconstruction with respect to
 * the optics and the data (Ext. Data Fig. 3: backpropagation through the
 * Tikhonov inverse into the transfer-function synthesis; Results,
 * "Physics-guided ML auto-tunes multi-contrast blind deconvolution").  Given
 * dL/df of the reconstruction f = wo_reconstruct(transfer function of o, d, b,
 * eta), returns dL/dtheta for theta = (defocus, na_det, tilt_zenith,
 * tilt_azimuth, det_tilt, det_azimuth) of each patch and dL/dd.  The transfer function is recomputed
 * from o (not stored), the same bank wo_transfer_function writes.  Per 3D
 * frequency, with x = D - N b delta, M = H^H H + eta I, F = M^-1 H^H x:
 * dL/dF* = FFT3(dL/df) / (2N), Y = M^-1 dL/dF*, dL/dH* = (x - H F) Y^H - H Y F^H,
 * dL/dd = Re IFFT3(2N H Y); dL/dH* then goes back through the 3D transform of
 * the per-plane label-free pair (whose adjoint along z is the unnormalised
 * inverse DFT), the correlation of the two arms and the pupils (analytic
 * derivatives of the soft edge; hard edges give no NA or tilt gradient; the
 * detection axis enters through the tilted detection pupil).
 * Aberrated optics are accepted (dL/dNA includes the aberration's NA
 * dependence).  Models LABELFREE_3D and POL5_3D (whose 5 x 4 bank is the
 * coupling's mix of the pair); others WO_EUNSUPPORTED.
 * d: device [n][C][vol]; b: device [n][C] or NULL; eta > 0; dL_df: device
 * [n][P][vol]; dL_dtheta_out: host [n][6] or NULL; dL_dd_out: device
 * [n][C][vol] or NULL (not both NULL).  Workspace of
 * wo_reconstruct_grad_workspace_size bytes (0: unsupported model).
 * Synchronises `stream` when dL_dtheta_out is not NULL. */
size_t wo_reconstruct_grad_workspace_size(const wo_optics* o, int32_t n);
int wo_reconstruct_grad(const wo_optics* o, int32_t n, const float* d, const float* b, double eta,
                        const float* dL_df, double* dL_dtheta_out, float* dL_dd_out, void* ws,
                        size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * wo_reconstruct without a workspace argument.  Its scratch is a static
 * device array of WO_NOALLOC_SCRATCH_BYTES inside the library, one per GPU,
 * held until the process ends; the call allocates and frees nothing.  The
 * caller still passes tf, d, b and f_out as for wo_reconstruct, and the
 * results are those of wo_reconstruct bit for bit (same kernels and
 * schedules).  WO_ENOMEM if wo_workspace_size(o, n, WO_OP_RECONSTRUCT)
 * exceeds WO_NOALLOC_SCRATCH_BYTES; WO_EINVAL if `stream` belongs to another
 * device than the current one (whose scratch is used).  Every call on one GPU
 * shares that GPU's array, so calls that overlap in time on one GPU (other
 * streams, other host threads) race and give undefined results; calls in
 * order on one stream are safe.  Nothing in the array needs to start at zero:
 * each call writes every scratch value it reads. */
#define WO_NOALLOC_SCRATCH_BYTES (64u << 20)
int wo_reconstruct_noalloc(const wo_optics* o, int32_t n, const void* tf, const float* d,
                           const float* b, double eta, float* f_out, void* stream);

/* ---------------------------------------------------------------- auto-tune
 * Thin phase-from-defocus model only (WO_MODEL_LABELFREE_THIN).  Parameters
 * theta = (defocus, na_det, tilt_zenith, tilt_azimuth) are tuned per patch to
 * maximise the power of the reconstructed phase in a mid-band of lateral
 * frequencies (Results, "Physics-guided ML auto-tunes multi-contrast blind
 * deconvolution"; Methods, "Cell-scale optical pooled screen data";
 * Ext. Data Fig. 3).  The band is nu_c/8 <= |nu| <= nu_c/4 with nu_c the
 * transverse cutoff, by default (na_det + na_ill)/wavelength of the patch's
 * given optics, held fixed while theta moves; the loss is
 * L = -(1/|band|) sum_band |F_phase(nu)|^2 on the unnormalised 2D DFT of the
 * Tikhonov phase reconstruction.  Gradients are hand-written reverse mode
 * through the solve and the transfer-function synthesis; the transfer
 * function is recomputed every iteration.  Soft pupil edges (edge_width > 0)
 * are needed for non-zero NA and tilt gradients.  Aberrated optics are
 * accepted (their aberration stays fixed while theta moves; dL/dNA includes
 * the NA dependence of the aberration through rho); the gradient with respect
 * to the aberration coefficients themselves comes from
 * wo_midband_loss_grad_aberration. */

/* Unlike the calls above, the calls of this section accept patches of uneven
 * shapes (each o[i] its own nz >= 2, ny and nx <= 2048, dz, dy, dx): the stacks are
 * packed, patch i's [nz_i][ny_i][nx_i] floats following patch i-1's, and the
 * patches that share a sampling are processed by the same launches
 * (shift-variant processing of overlapping tiles, Methods "Cell-scale optical
 * pooled screen data" and "Organelle-scale optical pooled screen data").  */

/* Workspace bytes for wo_midband_loss_grad (starts = 1), wo_autotune or
 * wo_restore_tiles (0 if any patch is not WO_MODEL_LABELFREE_THIN). */
size_t wo_tune_workspace_size(const wo_optics* o, int32_t n, int32_t starts);

/* Loss and dL/dtheta at each patch's optics.  d: device, packed stacks;
 * eta, nu_c: host [n] (nu_c may be NULL or <= 0 for the default);
 * loss_out: host [n]; grad_out: host [n][4] or NULL.  Synchronises `stream`
 * before returning. */
int wo_midband_loss_grad(const wo_optics* o, int32_t n, const float* d, const double* eta,
                         const double* nu_c, double* loss_out, double* grad_out, void* ws,
                         size_t ws_bytes, void* stream);

/* As wo_midband_loss_grad, with grad_out host [n][11]: dL/d(defocus, na_det,
 * tilt_zenith, tilt_azimuth) then dL/d zernike[0..6] (Noll 5..11, per wave).
 * The aberration phase 2 pi W multiplies both arms of the transfer function,
 * so dA/dc_j = i 2 pi Z_j A and dB/dc_j = i 2 pi Z_j B (Table 1 with the
 * aberrated detection pupil); the terms are summed with the same reverse-mode
 * factors as the defocus gradient.  Valid at zero coefficients too. */
int wo_midband_loss_grad_aberration(const wo_optics* o, int32_t n, const float* d, const double* eta,
                                    const double* nu_c, double* loss_out, double* grad_out, void* ws,
                                    size_t ws_bytes, void* stream);

typedef struct wo_autotune_opts {
  int32_t iters;           /* Adam iterations (the paper uses 100) */
  int32_t multistart;      /* starts per patch, M >= 1; the lowest final loss wins */
  int32_t use_graph;       /* 0: plain launches; 1: one iteration of every patch
                              captured in a HIP graph and replayed `iters` times;
                              2: the whole call (iterations, final loss and, for
                              wo_restore_tiles, the reconstruction) captured in
                              one HIP graph and launched once.  The library keeps
                              the graphs of its last 8 distinct calls and reuses
                              one when a call repeats the shapes and samplings,
                              the buffers (d, ws, f_out), the counts and the FFT
                              schedule table; parameters may differ */
  int32_t tune_mask;       /* bit j set: theta_j is tuned */
  double lr[4];            /* Adam learning rates per parameter */
  double lo[4], hi[4];     /* box for theta (NA is further capped inside the shell) */
  const double* theta0;    /* host [n][M][4] starting theta, or NULL: each patch's optics */
  const double* nu_c;      /* host [n] band cutoffs, or NULL for the default */
  double* all_theta_out;   /* host [n][M][4] final theta of every start, or NULL */
  double* all_loss_out;    /* host [n][M] final loss of every start, or NULL */
  int32_t branches;        /* graph modes: concurrent branches the shape groups
                              are spread over (0: 4; at most 8), balanced by
                              voxels x starts */
  double lr_zernike;       /* Adam rate of the aberration coefficients: tune_mask
                              bit 4 + j tunes zernike[j] (Noll 5 + j), starting from
                              each patch's optics (also for every multistart start) */
  double zernike_bound;    /* box [-bound, bound] waves for them (<= 0: 1 wave) */
  int32_t* status_out;     /* host [n] per-patch status, or NULL: WO_OK, or WO_DIVERGED
                              when no start of the patch ended with a finite loss and
                              finite parameters (the patch's optics are then left as
                              they were passed and its loss_out is NaN; the call itself
                              still returns WO_OK) */
} wo_autotune_opts;

/* Adam (beta 0.9, 0.999, eps 1e-8) on theta for opts->iters iterations, every
 * patch and start in one batched launch sequence; theta is clipped to the box
 * after each step.  On return o[i] holds the best start's theta (and tuned
 * aberration coefficients): the lowest final loss among the starts that ended
 * finite; loss_out[i] (host, may be NULL) its loss at that theta.  A patch
 * none of whose starts ended finite (for instance non-finite data) is
 * reported in opts->status_out and does not fail the batch.  d: device, packed
 * stacks; eta: host [n].  Not reentrant across host threads (calls
 * serialise on a library lock).  Synchronises `stream` before returning. */
int wo_autotune(wo_optics* o, int32_t n, const float* d, const double* eta,
                const wo_autotune_opts* opts, double* loss_out, void* ws, size_t ws_bytes,
                void* stream);

/* Shift-variant restoration of uneven tiles: wo_autotune, then the thin-model
 * Tikhonov reconstruction (Eq. tls_solution, one Z x 2 system per lateral
 * frequency, eta[i]) of every tile at its best start's final theta, written
 * to f_out (device, packed [2][ny_i][nx_i] per tile: phase, absorption; the
 * same values as wo_transfer_function + wo_reconstruct at that theta).  With
 * opts->use_graph = 2 the whole call is one graph launch.  The workspace size
 * is wo_tune_workspace_size(o, n, multistart).  f_out NULL: WO_EINVAL. */
int wo_restore_tiles(wo_optics* o, int32_t n, const float* d, const double* eta,
                     const wo_autotune_opts* opts, double* loss_out, float* f_out, void* ws,
                     size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- field of view
 * Shift-variant restoration of a large field of view tiles it, restores every
 * tile with its own parameters (wo_restore_tiles) and blends the tiles back
 * (Methods, "Cell-scale optical pooled screen data": a grid of tiles with 20 %
 * overlap; "Organelle-scale optical pooled screen data": a 5 x 5 grid with 25
 * pixels of overlap, stitched with linearly weighted Euclidean-distance-
 * transform blending). */

/* Tile size and starts along one axis of `length` pixels: `count` (1..32)
 * evenly spaced tiles, the first at 0 and the last flush with the far edge
 * (one tile: centred), of the smallest even {2,3,5}-smooth size that gives at
 * least `overlap` pixels between neighbours.  tile: host int32; starts: host
 * int32[count].  WO_EINVAL if the tiles would not fit. */
int wo_tile_grid(int32_t length, int32_t count, int32_t overlap, int32_t* tile, int32_t* starts);

/* Blends tiles into a field: out[p][y][x] = sum_t w_t f_t[p][y - y0_t][x - x0_t]
 * / sum_t w_t over the tiles t covering (y, x), with w_t the tile's distance
 * transform min(u + 1, ty - u, v + 1, tx - v) at tile pixel (u, v) (0 where no
 * tile covers).  tiles: device [ny_t * nx_t][P][ty][tx], row-major over the
 * grid; ys, xs: host int32 starts (ascending, inside the field; grid up to
 * 32 x 32); out: device [P][H][W]. */
int wo_stitch_tiles(const float* tiles, int32_t ny_t, int32_t nx_t, int32_t P, int32_t ty, int32_t tx,
                    const int32_t* ys, const int32_t* xs, int32_t H, int32_t W, float* out,
                    void* stream);

/* ---------------------------------------------------------------- FFT schedule tuner
 * Not in the paper (its transforms are library calls).  Every FFT pass of the
 * library -- rows along X (real <-> half spectrum), strided columns along Y
 * (and Z for the transfer functions), the Z pass fused with the
 * per-frequency operator, and the row pass of the label-free transfer
 * functions (inverse X transforms of both fields, their product, forward X
 * transform) -- is launched with a schedule: the lines, rows or columns
 * one workgroup transforms, the workgroup size, and the radix plan (compiled
 * stages for the compiled lengths, else a runtime plan in one of three radix
 * orders; plan 4, for the column passes at a compiled length and width, is a
 * resident grid whose workgroups loop over the tiles).  Without tuning each pass takes a fixed heuristic schedule; a
 * process-wide table keyed by (pass, length, columns, batch[, P, C, mode])
 * overrides it.  Tuning or importing changes launch schedules only: results
 * are the same transform up to FP32 rounding.  The table is guarded by a
 * mutex; tuning while other threads launch work on the same device distorts
 * its timings. */

/* Runs one call -- op WO_OP_TRANSFER_FUNCTION (writes `out` as tf_out),
 * WO_OP_FORWARD (in = f, out = d), WO_OP_RECONSTRUCT (in = d, out = f, eta)
 * or WO_OP_ADJOINT (in = r, out = g), arguments as for that call, b = NULL --
 * while recording its tunable passes; then, pass by pass, times the whole
 * call `reps` times with every candidate schedule of that pass (the other
 * passes keeping their current schedules) and stores the one with the
 * fastest single call.  op | WO_FFT_TUNE_BAND runs the band-layout variant of
 * the call instead (wo_transfer_function_band, or wo_linear_band with `tf` a
 * band-layout bank).
 * On return `out` and `ws` hold unspecified values (run the call again);
 * tf and in are only read.  Synchronises `stream`. */
#define WO_FFT_TUNE_BAND 16
int wo_fft_tune(int32_t op, const wo_optics* o, int32_t n, const void* tf, const float* in, float* out,
                double eta, int32_t reps, void* ws, size_t ws_bytes, void* stream);
/* The table as text, one line "kind n m batch extra w threads plan" per entry
 * (kind: rows_r2c, rows_c2r, cols, zop, tf_rows, tf_fields -- the field kernel's
 * planes per workgroup in w); NUL-terminated, truncated to len;
 * *needed (may be NULL) receives the full size including the NUL. */
int wo_fft_plans_export(char* buf, size_t len, size_t* needed);
/* Adds entries in the export format; all or none: WO_EINVAL if a line is
 * malformed or names a schedule the pass does not accept on this device. */
int wo_fft_plans_import(const char* text);
int wo_fft_plans_clear(void);
/* Every schedule the pass "kind n m batch extra" accepts on this device, in
 * the export format (the first line is the default schedule). */
int wo_fft_candidates(const char* key_line, char* buf, size_t len, size_t* needed);

/* ---------------------------------------------------------------- learned initialiser
 * Not in the paper: a small 3D CNN that regresses normalised (defocus, NA_det,
 * tilt_zenith) from a defocus stack, used to start the auto-tune.  4 blocks of
 * [3x3x3 convolution, stride 2, padding 1, bias, GELU] with channels
 * 1 -> 32 -> 64 -> 128 -> 256, global average pooling, linear head to 3
 * outputs; loss mean((y - t)^2); AdamW.  Convolutions run as implicit GEMMs on
 * BF16 MFMA with FP32 accumulation; activations are BF16, parameters FP32
 * (a BF16 copy of the weights feeds the MFMA).
 * Parameter layout (flat FP32): for each block, weights [Cout][3][3][3][Cin]
 * then bias [Cout]; then head weights [3][256] and bias [3].
 * Inputs x: device [batch][nz][ny][nx] FP32 stacks; each sample is scaled by
 * its RMS before the first convolution.  batch * nz * ny * nx must stay below
 * 2^31 (else WO_EINVAL, and a workspace size of 0). */
int64_t wo_cnn_param_count(void);
size_t wo_cnn_workspace_size(int32_t batch, int32_t nz, int32_t ny, int32_t nx);
/* y_out: device [batch][3]. */
int wo_cnn_forward(const float* params, const float* x, int32_t batch, int32_t nz, int32_t ny,
                   int32_t nx, float* y_out, void* ws, size_t ws_bytes, void* stream);
/* Forward, loss (device scalar) and gradient (device flat FP32, or NULL to keep
 * it in the workspace) for targets [batch][3]. */
int wo_cnn_gradient(const float* params, const float* x, const float* target, int32_t batch,
                    int32_t nz, int32_t ny, int32_t nx, float* y_out, float* loss_out,
                    float* grad_out, void* ws, size_t ws_bytes, void* stream);
/* One AdamW step (step t >= 1, beta 0.9/0.999, eps 1e-8, decoupled weight decay)
 * on params with moments adam_m, adam_v (device, param_count floats each). */
int wo_cnn_train_step(float* params, float* adam_m, float* adam_v, int32_t t, double lr,
                      double weight_decay, const float* x, const float* target, int32_t batch,
                      int32_t nz, int32_t ny, int32_t nx, float* y_out, float* loss_out, void* ws,
                      size_t ws_bytes, void* stream);
/* The prior box the network's outputs are normalised over: output j in
 * [-1, 1] maps to lo[j] + (y + 1) (hi[j] - lo[j]) / 2 for (defocus um, NA_det,
 * tilt_zenith rad): lo = (-2, 1.0, 0), hi = (2, 1.3, 30 degrees). */
void wo_cnn_prior(double lo[3], double hi[3]);
/* Workspace bytes of wo_cnn_init_theta for n patches (0 if n < 1 or too many). */
size_t wo_cnn_init_workspace_size(int32_t n);
/* The learned initialiser as the start of wo_autotune / wo_restore_tiles:
 * patches packed as for those calls (o[i] their shapes, any nz, ny, nx; d
 * device), the centred 32 x 64 x 64 window of each (first voxel at
 * floor((n - 32) / 2), floor((n - 64) / 2) per axis: central planes and
 * pixels of larger patches, symmetric zero padding of smaller ones) through
 * the network with parameters params (device, wo_cnn_param_count floats),
 * denormalised over wo_cnn_prior into theta_out (host [n][4]: defocus, NA_det,
 * tilt_zenith, and o[i].tilt_azimuth, which the network does not predict) --
 * the theta0 of a start.  Synchronises `stream` before returning. */
int wo_cnn_init_theta(const float* params, const wo_optics* o, int32_t n, const float* d, double* theta_out,
                      void* ws, size_t ws_bytes, void* stream);
/* Single strided (2) 3x3x3 convolutions with padding 1 on BF16 operands (raw
 * 16-bit storage), channels-last x [N][D][H][W][Cin], weights [Cout][27][Cin]:
 * forward out [N][Do][Ho][Wo][Cout] (no bias), input gradient from
 * gz [N][Do][Ho][Wo][Cout] to out [N][D][H][W][Cin], weight gradient
 * out [Cout][27][Cin] (ws: FP32 split-K partials).  Do = (D - 1)/2 + 1;
 * N * D * H * W below 2^31 (else WO_EINVAL). */
int wo_conv3d_forward(const uint16_t* x, const uint16_t* w, int32_t N, int32_t D, int32_t H,
                      int32_t W, int32_t Cin, int32_t Cout, float* out, void* stream);
int wo_conv3d_input_grad(const uint16_t* gz, const uint16_t* w, int32_t N, int32_t D, int32_t H,
                         int32_t W, int32_t Cin, int32_t Cout, float* out, void* stream);
int wo_conv3d_weight_grad(const uint16_t* x, const uint16_t* gz, int32_t N, int32_t D, int32_t H,
                          int32_t W, int32_t Cin, int32_t Cout, float* out, void* ws,
                          size_t ws_bytes, void* stream);
/* Training data for the learned initialiser (counter-based hashing, so the
 * same seed gives the same data): thin cells out [n][2][ny][nx] (phase,
 * absorption) with semi-axes U(0.8, 2.5) um, phase U(0.1, 0.5), absorption
 * U(0, 0.02); and in-place additive Gaussian noise. */
int wo_synth_thin_cells(float* out, int32_t n, int32_t ny, int32_t nx, double pixel, int32_t ncells,
                        uint64_t seed, void* stream);
int wo_add_gaussian_noise(float* x, int64_t n, double sigma, uint64_t seed, void* stream);

/* Fixed-size network input from a stack of any size: out[i][z][y][x] =
 * in[i][z + z0][y + y0][x + x0] where that voxel exists and, if keep_z (device
 * [n]) is not NULL, |2 z - (oz - 1)| < keep_z[i] (only the central keep_z[i]
 * planes); 0 elsewhere.  Offsets may be negative (zero padding).  A thin stack
 * with fewer planes than the network input is, zero-padded symmetrically,
 * the same as a full stack with its outer planes cleared (the planes share
 * z_k = dz (k - (nz-1)/2)); keep_z produces that case for training.  in: device
 * [n][nz][ny][nx]; out: device [n][oz][oy][ox]; in == out only with equal
 * shapes and zero offsets (else WO_EALIAS). */
int wo_crop_stacks(const float* in, int32_t n, int32_t nz, int32_t ny, int32_t nx, float* out,
                   int32_t oz, int32_t oy, int32_t ox, int32_t z0, int32_t y0, int32_t x0,
                   const int32_t* keep_z, void* stream);

/* Instrumentation (not part of the method): while enabled, every kernel the
 * library launches is bracketed by HIP events on the stream it runs on.
 * wo_timing_report() waits for the recorded events, writes one line
 * "<kernel> <launches> <total_ms>" per kernel name into buf (NUL-terminated,
 * truncated to len), and clears the records.  Returns WO_EHIP if an event
 * failed. */
int wo_timing_enable(int on);
int wo_timing_report(char* buf, size_t len);
/* Restricts the events to launches of one kernel name (as reported); NULL or
 * "" selects every kernel again.  The name is copied. */
int wo_timing_select(const char* name);

/* Human-readable message for a status code. */
const char* wo_strerror(int status);

/* ABI version of this header (major * 100 + minor). */
int wo_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WAVEORDER_H */
