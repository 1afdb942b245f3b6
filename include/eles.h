/*
 * eles.h - C ABI of the MI355X explicit-filter library.
 *
 * The library computes, on one gfx950 GPU, the explicit filter of eq. (2)
 * of Bae & Lozano-Duran, "DNS-aided explicitly filtered LES of channel
 * flow" (Sec. 2.1), with a kernel of constant width in all three
 * directions, periodic in x and z and applied in y to the flow extended
 * across both walls as in eq. (7) (Sec. 2.2); and the exact subgrid stress
 * of the four-step procedure of Sec. 2.1,
 *     tau_ij = F(u_i u_j) - F(u_i) F(u_j),
 * with the filtered DNS velocity standing in for the discretised LES
 * velocity (LES grid = DNS grid).
 *
 * Filter. The kernel is the separable Gaussian g_D(r) =
 * sqrt(6/(pi D^2)) exp(-6 r^2 / D^2) per direction; its variance D^2/12 is
 * the second moment of a top hat of width D (the equal-second-moment rule
 * of Sec. 3). Eq. (2) is discretised by quadrature on the grid nodes:
 * rectangle rule in x and z (with periodic images), trapezoid rule on the
 * wall-normal nodes of the reflected, period-4 extended line; every output
 * node's weights are normalised to sum to one. Kernel values below
 * max(tail_tol, 1e-17) times the peak are dropped before normalisation.
 * Fields of odd parity (u2, u1u2, u2u3) are reflected with a sign change
 * and are treated as zero at the walls (eqs. (8) and (11)).
 *
 * Data layout. Every field is FP32, [nx][ny][nz] row-major (z fastest),
 * with grid nodes x_i = i lx/nx, y_j = y[j], z_k = k lz/nz. A stack of
 * fields is [nfields][nx][ny][nz]. Velocity stacks are (u1, u2, u3) =
 * (streamwise, wall-normal, spanwise); stress stacks hold
 * (tau11, tau12, tau13, tau22, tau23, tau33).
 *
 * Ownership. The caller allocates every device buffer (state, workspace,
 * inputs, outputs) and keeps it alive while work that uses it is queued.
 * The library never allocates device memory. Handles are host objects;
 * *_destroy frees host memory only.
 *
 * Execution. Every call enqueues work on the given stream and returns
 * without waiting for it, except the ones that read device results on the
 * host, which wait for their stream: the setup calls (filter_setup reads
 * the operators' band structure back to plan the y pass), closure_create,
 * closure_get_params / closure_set_params, and closure_infer in its
 * checked modes. One handle must not be used from two streams or threads
 * at once (a call keeps per-call data, such as the shift profile of the
 * stress, in the handle's state). Separate handles of the same
 * configuration share nothing: snapshots alternating between two streams,
 * each with its own handle and output buffers, give results bitwise equal
 * to one handle on one stream, and let one call's later passes overlap the
 * next call's first ones. All device pointers must be 16-byte aligned.
 *
 * Errors. Arguments are validated before anything is enqueued; a failing
 * validation returns a non-zero eles_status and enqueues nothing. A HIP
 * error at launch returns ELES_EHIP. No exception crosses the ABI.
 */
#ifndef ELES_H
#define ELES_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ELES_OK = 0,
  ELES_EINVAL = 1,    /* invalid argument: sizes, grid, widths, pointers   */
  ELES_ENOSPACE = 2,  /* state or workspace smaller than required          */
  ELES_EHIP = 3,      /* a HIP call or kernel launch failed                 */
  ELES_ENUMERIC = 4,  /* a normalisation would underflow or overflow        */
  ELES_ENOTSUP = 5    /* valid but outside what the kernels support         */
} eles_status;

/* Arithmetic of the wall-normal operator product (the y-pass). */
typedef enum {
  ELES_YGEMM_FP32 = 0,   /* FP32 operands on the matrix cores, FP32 sums      */
  ELES_YGEMM_BF16 = 1,   /* operator and field rounded to BF16, FP32 sums     */
  ELES_YGEMM_BF16X3 = 2  /* hi/lo BF16 split of both, three products, FP32    */
} eles_ygemm;

typedef struct {
  int32_t nx, ny, nz;     /* nx, nz >= 1; ny >= 3                               */
  double lx, lz;          /* periodic lengths, > 0                              */
  const double *y;        /* host, ny values, strictly increasing,
                             y[0] = -1 and y[ny-1] = +1 exactly (the walls)     */
  double delta_x, delta_y, delta_z;   /* filter widths D, > 0                   */
  double tail_tol;        /* in [0, 1e-2]; 0 keeps the kernel down to 1e-17     */
  int32_t ygemm;          /* eles_ygemm                                         */
} eles_filter_desc;

typedef struct eles_filter_s *eles_filter;

/* Byte offsets of the operators inside the device state (for inspection). */
typedef struct {
  int32_t mx, mz;          /* half-widths of the x and z stencils             */
  int32_t ny_pad_m;        /* rows of the padded y operators (multiple of 16) */
  int32_t ny_pad_k;        /* columns of the padded y operators (mult. of 32) */
  size_t off_wp64, off_wm64;   /* FP64 [ny][ny] W^+ and W^-                   */
  size_t off_wx64, off_wz64;   /* FP64 [2m+1] taps for offsets -m..m          */
  size_t off_y64;              /* FP64 [ny] copy of y                          */
  size_t off_shift;            /* FP64 [3][ny]: m, M = W^+ m, W^+ m^2 - M^2
                                  of the last sgs_stress call                  */
  size_t state_bytes;
  int32_t y_groups;            /* row groups of the LDS-staged FP32 stress y
                                  pass; 0 when this grid uses the direct
                                  y pass instead                              */
  int32_t y_blocks;            /* persistent blocks of the staged y pass      */
  int32_t xz_waves;            /* waves of the matrix-core stress x/z pass;
                                  0 when this grid uses the vector-unit
                                  x/z pass instead                            */
  int32_t xz_wide;             /* 1 when that pass is the wide-stencil kernel
                                  (three of the nine fields per wave: x or z
                                  half-width above 16)                        */
} eles_state_layout;

/* Human-readable name of a status code. Never NULL. */
const char *eles_status_string(int32_t status);

/* Device bytes the state of this descriptor needs; 0 if the descriptor is
 * invalid. */
size_t filter_state_bytes(const eles_filter_desc *desc);

/* Build the filter operators (Sec. 2.1 eq. (2) with the Sec. 2.2 wall
 * extension) on the device, in FP64, into the caller's state buffer.
 * desc->y is copied; the descriptor may be freed after the call. On success
 * *out receives a new handle. Errors: EINVAL (descriptor, null pointers),
 * ENOSPACE (state_bytes too small), ENUMERIC (width underflow), ENOTSUP
 * (stencil half-width above the kernels' limit), EHIP. */
int32_t filter_setup(const eles_filter_desc *desc, void *state, size_t state_bytes,
                     hipStream_t stream, eles_filter *out);

/* Choose the y-pass arithmetic (eles_ygemm) for later calls. */
int32_t filter_set_ygemm(eles_filter f, int32_t ygemm);

/* Choose how later sgs_stress calls evaluate the periodic x and z parts of
 * the filter (Sec. 2.1, eq. (2)) on the nine fields: 1 = on the matrix cores
 * (the default wherever those kernels cover the grid: nx >= 4 and either x
 * and z stencil half-widths up to 16, or half-widths up to 44 in x and 48
 * in z with nz % 4 == 0), 0 = on the vector units. Both give the
 * same result up to FP32 rounding order. Errors: EINVAL (null handle, value
 * other than 0 or 1), ENOTSUP (1 asked for a grid the matrix-core kernel
 * does not cover; the setting is left unchanged). */
int32_t filter_set_xz(eles_filter f, int32_t matrix_cores);

/* Operator layout of the handle's state. */
int32_t filter_state_layout(eles_filter f, eles_state_layout *out);

/* Workspace bytes of filter_fields with nfields fields. */
size_t filter_workspace_bytes(eles_filter f, int32_t nfields);

/* Workspace bytes of sgs_stress. */
size_t sgs_workspace_bytes(eles_filter f);

/* out[k] = F^(s_k)(in[k]) for k < nfields: eq. (2) with parity
 * s_k = parity[k] in {+1, -1} under the eq. (7) reflection (host array).
 * in, out: device [nfields][nx][ny][nz]; they must not overlap. Errors:
 * EINVAL, ENOSPACE, EHIP. */
int32_t filter_fields(eles_filter f, const float *in, int32_t nfields,
                      const int8_t *parity, float *out, void *ws, size_t ws_bytes,
                      hipStream_t stream);

/* Filtered velocity and exact subgrid stress (Sec. 2.1, four steps).
 * u: device [3][nx][ny][nz]; ubar: device [3][...] = F(u_i) with parities
 * (+, -, +); tau: device [6][...] = F(u_i u_j) - F(u_i) F(u_j), product
 * parities s_i s_j. stats: device FP64 [9][ny] plane averages over x and z
 * (Sec. 4.1) of ubar_1..3 then tau_11..33, or NULL. Internally u1 is
 * shifted by a y-profile sampled from u1 before the products are formed,
 * which leaves the exact result unchanged and removes most cancellation.
 * u must not overlap ubar or tau. Errors: EINVAL, ENOSPACE, EHIP. */
int32_t sgs_stress(eles_filter f, const float *u, float *ubar, float *tau,
                   double *stats, void *ws, size_t ws_bytes, hipStream_t stream);

/* Per-pass GPU timing of later sgs_stress / filter_fields calls on this
 * handle, with HIP events recorded on the call's stream around the kernels
 * of the passes selected by pass_mask (bit p times pass p). Passes: 0 shift
 * profile and correction operators, 1 x/z pass, 2 y pass, 3 plane
 * statistics. Each event pair adds a few microseconds between kernels, so
 * a throughput measurement times only the passes it needs.
 * filter_profile_begin creates events for up to max_calls calls (host-side
 * HIP events; no device memory). After the timed calls, filter_profile_end
 * waits for the last event and returns, per pass, the summed milliseconds
 * and the number of launches timed (zero for passes not selected), then
 * releases the events. Errors: EINVAL (pass_mask zero or naming a pass
 * past ELES_NPASS - 1), EHIP. */
#define ELES_NPASS 4
int32_t filter_profile_begin(eles_filter f, int32_t max_calls, uint32_t pass_mask);
int32_t filter_profile_end(eles_filter f, double *ms /* [ELES_NPASS] */,
                           int32_t *launches /* [ELES_NPASS] */);

void filter_destroy(eles_filter f);

/* ======================================================================
 * The paper's own filter: Germano's differential filter (Sec. 3,
 * eq. (12)), the kernel exp(-|r|/a) / (4 pi a^2 |r|) of parameter a. It is
 * the free-space Green's function of (1 - a^2 lap), so the filtered field
 * solves (1 - a^2 lap) ubar = u. Discretisation (the paper states none):
 * spectral second derivatives in the periodic x and z directions (symbol
 * -k^2 on the grid wavenumbers), and in y the three-point second
 * difference on the non-uniform nodes of the flow reflected across each
 * wall as in eq. (7): an even field takes the mirrored value at the mirror
 * node, an odd field is zero at the wall nodes (eqs. (8), (11)). Layouts,
 * ownership, streams and errors as for the Gaussian filter above.
 * ====================================================================== */
typedef struct {
  int32_t nx, ny, nz;     /* nx, nz >= 8; 4 <= ny <= 8192; nx ny nz < 2^29      */
  double lx, lz;          /* periodic lengths, > 0                              */
  const double *y;        /* host, ny values, strictly increasing,
                             y[0] = -1 and y[ny-1] = +1 exactly (the walls)     */
  double a;               /* filter parameter, > 0 (the paper: 0.1)            */
} eles_dfilter_desc;

typedef struct eles_dfilter_s *eles_dfilter;

/* Device bytes of the state of this descriptor; 0 if it is invalid. */
size_t dfilter_state_bytes(const eles_dfilter_desc *desc);

/* Build the operators on the device in FP64 (rounded to FP32 where the
 * kernels read them): the real Fourier transforms of x and z, and the
 * factors of the wall-normal tridiagonal system of every wavenumber pair
 * and parity. Waits for the stream. Errors: EINVAL, ENOSPACE, ENOTSUP
 * (grid too large for 32-bit offsets), EHIP. */
int32_t dfilter_setup(const eles_dfilter_desc *desc, void *state, size_t state_bytes, hipStream_t stream,
                      eles_dfilter *out);

/* Workspace bytes of dfilter_fields with nfields fields, and of
 * dfilter_sgs_stress. */
size_t dfilter_workspace_bytes(eles_dfilter f, int32_t nfields);
size_t dfilter_sgs_workspace_bytes(eles_dfilter f);

/* out[k] = F^(s_k)(in[k]), the differential filter of a field of parity
 * s_k = parity[k] in {+1, -1} (host array). in, out: device
 * [nfields][nx][ny][nz], not overlapping; 1 <= nfields <= 32. An odd
 * field's input values on the wall planes are not read into the solve and
 * its output there is exactly 0. Errors: EINVAL (also a parity other than
 * +-1), ENOSPACE, EHIP. */
int32_t dfilter_fields(eles_dfilter f, const float *in, int32_t nfields, const int8_t *parity, float *out,
                       void *ws, size_t ws_bytes, hipStream_t stream);

/* Filtered velocity and exact subgrid stress with the differential filter
 * (Sec. 2.1, four steps); arguments as for sgs_stress. u1 is shifted by
 * its plane-mean profile m(y) before the products are formed; the terms
 * the shift leaves (F(m u_j) - F(m) F(u_j), F(m^2) - F(m)^2) are filtered
 * with the rest, so the result is the exact stress of the unshifted
 * field. Errors: EINVAL, ENOSPACE, EHIP. */
int32_t dfilter_sgs_stress(eles_dfilter f, const float *u, float *ubar, float *tau, double *stats, void *ws,
                           size_t ws_bytes, hipStream_t stream);

/* The inverse filter, u = (1 - a^2 lap) ubar with the same discretisation
 * (the operator the filter inverts; Sec. 4.2 compares unfiltered LES and
 * DNS velocities through it). Arguments, parities, layouts, workspace size
 * (dfilter_workspace_bytes) and errors as for dfilter_fields; odd outputs
 * are exactly 0 on the wall planes. */
int32_t dfilter_inverse(eles_dfilter f, const float *in, int32_t nfields, const int8_t *parity, float *out,
                        void *ws, size_t ws_bytes, hipStream_t stream);

/* Errors of an LES velocity against a DNS velocity on this grid, the forms
 * of eqs. (13)-(15). les, dns: device [3][nx][ny][nz] (u1, u2, u3), each
 * scaled by its friction velocity (utau_les, utau_dns > 0, finite). out:
 * device FP64 [5]:
 *   out[0] eq. (13): volume relative L2 error of u1, over the channel;
 *   out[1] eq. (14): relative L2 error of the <u1>(y) profile;
 *   out[2 + i] eq. (15): relative L2 error of the rms profile of u_{i+1};
 * <.> is the average over x and z, rms = sqrt(<u^2> - <u>^2), and the
 * profile integrals run from the lower wall to the centreline (nodes with
 * y <= 0). Integrals in y use the bounded trapezoid rule on the nodes
 * used; sums in FP64. Workspace: dfilter_errors_workspace_bytes. Errors:
 * EINVAL, ENOSPACE, EHIP. */
size_t dfilter_errors_workspace_bytes(eles_dfilter f);
int32_t dfilter_errors(eles_dfilter f, const float *les, const float *dns, double utau_les, double utau_dns,
                       double *out, void *ws, size_t ws_bytes, hipStream_t stream);

/* Per-pass GPU timing of later dfilter_sgs_stress / dfilter_fields /
 * dfilter_inverse calls on this handle, with HIP events recorded on the
 * call's stream around the passes selected by pass_mask (bit p times pass
 * p; EINVAL when zero or naming a pass past ELES_DNPASS - 1): 0 shift profile, 1 x forward transform (with the products), 2 z
 * forward transform, 3 y solves (dfilter_inverse: the y operator), 4 z
 * inverse transform, 5 x inverse transform, 6 stress epilogue and plane
 * statistics (dfilter_fields and dfilter_inverse time passes 1 .. 5). dfilter_profile_begin creates events for up to max_calls
 * calls (host-side HIP events; no device memory); dfilter_profile_end waits
 * for the device and returns, per pass, the summed milliseconds and the
 * number of timed launches, then releases the events. Errors: EINVAL,
 * EHIP. */
#define ELES_DNPASS 7
int32_t dfilter_profile_begin(eles_dfilter f, int32_t max_calls, uint32_t pass_mask);
int32_t dfilter_profile_end(eles_dfilter f, double *ms /* [ELES_DNPASS] */,
                            int32_t *launches /* [ELES_DNPASS] */);

void dfilter_destroy(eles_dfilter f);

/* ======================================================================
 * The stress on an LES grid (Sec. 2, the discrete filtered equations):
 * T_ij = I(F(u_i u_j)) - I(F(u_i)) I(F(u_j)), with I the discretization
 * operator, second-order linear interpolation from the DNS grid to the LES
 * grid (Sec. 4; the LES2 / LES4 grids are coarser by 2 and 4), and the
 * commutation error of I with second-order differentiation, which the
 * paper notes for stretched meshes (Sec. 4).
 *
 * Interpolation: separable, periodic in x and z (LES node k at k L/n_les,
 * DNS node i at i L/n), in y between the bracketing DNS nodes. It works
 * from the DNS-grid outputs of either filter: with F(u_i u_j) = tau_ij +
 * ubar_i ubar_j and weights summing to one, T_ij is I(tau_ij) plus the
 * weighted covariance of the eight corner values of ubar.
 * ====================================================================== */
typedef struct {
  int32_t nx, ny, nz;          /* DNS grid; ny >= 3                              */
  const double *y;             /* host, ny nodes, increasing, y[0] = -1, y[ny-1] = 1 */
  int32_t nx_les, ny_les, nz_les; /* LES grid; ny_les >= 3                       */
  const double *y_les;         /* host, ny_les nodes, increasing, within [-1, 1] */
} eles_les_desc;

typedef struct eles_les_s *eles_les;

/* Device bytes of the state (weights, indices, derivative stencils); 0 if
 * the descriptor is invalid. */
size_t les_state_bytes(const eles_les_desc *desc);

/* Build the interpolation and stencils (FP64 on the host; weights stored in
 * FP32, stencils in FP64) and copy them into state; waits for the stream.
 * Errors: EINVAL, ENOSPACE, EHIP. */
int32_t les_setup(const eles_les_desc *desc, void *state, size_t state_bytes, hipStream_t stream, eles_les *out);

/* ubar_les [3] = I(ubar_i) and T [6] (order 11, 12, 13, 22, 23, 33) on the
 * LES grid [nx_les][ny_les][nz_les], from ubar [3] and tau [6] on the DNS
 * grid (the outputs of sgs_stress or dfilter_sgs_stress). FP32. Outputs
 * must not overlap the inputs or each other. Errors: EINVAL, EHIP. */
int32_t les_stress(eles_les h, const float *ubar, const float *tau, float *ubar_les, float *T, hipStream_t stream);

/* Commutation error of one DNS field g [nx][ny][nz] (FP64, device out[1]):
 * ||d_y^LES(I g) - I(d_y^DNS g)|| / ||I(d_y^DNS g)|| over the LES volume
 * (uniform in x and z, trapezoid in y), d_y the three-point second-order
 * first derivative on each mesh (one-sided three-point at the walls).
 * Workspace: les_commutation_workspace_bytes. Errors: EINVAL, ENOSPACE,
 * EHIP. */
size_t les_commutation_workspace_bytes(eles_les h);
int32_t les_commutation(eles_les h, const float *g, double *out, void *ws, size_t ws_bytes, hipStream_t stream);

void les_destroy(eles_les h);

/* ======================================================================
 * Learned closure of the exact stress.
 *
 * The paper proposes using the exact stress computed from DNS data to
 * inform subgrid models, naming machine learning as one route (Sec. 2.1,
 * last paragraph; Sec. 5). This closure is a perceptron 10 -> 64 -> 64 ->
 * 64 -> 6 with GELU hidden layers and a linear output. GELU(x) = x Phi(x),
 * Phi the standard normal CDF; the kernels evaluate it as max(x, 0) -
 * h(min(|x|, 4)) with h a degree-7 polynomial fitted to s Phi(-s), within
 * 2.4e-4 of x Phi(x) in exact arithmetic (training: in s, FP32, derivative
 * within 5e-3; inference: in s/2 - 1, packed FP16, within 1.3e-3 as
 * rounded). Its
 * inputs at every grid point are the nine components d ubar_i / d x_k
 * (i, k = 1..3, row-major) of the filtered velocity gradient and the wall
 * distance 1 - |y|; its outputs are tau_11, tau_12, tau_13, tau_22, tau_23,
 * tau_33. Inputs and outputs are standardised with training-set means and
 * standard deviations. Training runs BF16 weights and activations on the
 * matrix cores with FP32 accumulation, master weights and Adam moments in
 * FP32; inference runs FP16 weights (rounded from the FP32 masters) and
 * activations with FP32 accumulation.
 * Parameters are packed W1 (64x10, row-major), b1, W2 (64x64), b2, W3, b3,
 * W4 (6x64), b4: ELES_CLOSURE_NPARAM floats.
 * ====================================================================== */
#define ELES_CLOSURE_NPARAM 9414

typedef struct eles_closure_s *eles_closure;

typedef struct {
  int32_t batch;      /* minibatch size, a multiple of 32                     */
  int32_t steps;      /* Adam steps of this call                              */
  uint64_t seed;      /* minibatch stream: draw n = step * batch + slot of
                         SplitMix64(seed), index = ((r >> 32) * count) >> 32  */
  float lr, beta1, beta2, eps;
} eles_train_desc;

/* Device bytes of a closure state. */
size_t closure_state_bytes(void);

/* Create a closure in the caller's state buffer. params: host
 * [ELES_CLOSURE_NPARAM] initial weights; norms: host FP64 [32] = feature
 * means [10], feature standard deviations [10], target means [6], target
 * standard deviations [6]. gm_coef: host FP64 [3] or NULL. With c =
 * gm_coef the closure adds the gradient model, the leading term of the
 * small-width expansion of the filtered stress (cf. the invertible filters
 * of Sec. 2.1), G_ij = sum_k c_k (d ubar_i/dx_k)(d ubar_j/dx_k), to the
 * network: tau = G + mu + sd N(x'), and training fits N to the
 * standardised remainder (tau - G - mu) / sd. For a filter of widths D_k,
 * c_k = D_k^2 / 12; NULL (or zeros) is the plain network. Waits for its
 * copies. Errors: EINVAL, ENOSPACE, ENUMERIC (non-finite values,
 * non-positive deviations, negative coefficients), EHIP. */
int32_t closure_create(void *state, size_t state_bytes, const float *params, const double *norms,
                       const double *gm_coef, hipStream_t stream, eles_closure *out);

/* Adam steps taken so far (-1 for a null handle). */
int64_t closure_step(eles_closure c);

/* Checkpoint blob: FP32 weights, Adam m and v, FP64 norms, int64 step,
 * FP64 gradient-model coefficients [3].
 * closure_get_params copies the state into the host blob on the stream
 * (after the work already queued there) and waits for the stream.
 * closure_set_params validates the blob on the host (ENUMERIC: non-finite
 * values or non-positive deviations; EINVAL: negative step), then copies
 * it on the stream and waits for the stream. Errors: EINVAL (null handle
 * or blob, bytes < closure_blob_bytes()), ENUMERIC, EHIP. */
size_t closure_blob_bytes(void);
int32_t closure_get_params(eles_closure c, void *blob, size_t bytes, hipStream_t stream);
int32_t closure_set_params(eles_closure c, const void *blob, size_t bytes, hipStream_t stream);

/* Features of a filtered velocity ubar (device [3][nx][ny][nz]) on the
 * filter's grid: feat (device [10][nx][ny][nz]) = d ubar_i/dx (spectral,
 * dense differentiation matrix), d/dy (three-point difference, wall rows
 * through the mirror node with the eq. (7) parities), d/dz (spectral), in
 * (i, k) row-major order, then 1 - |y|. Errors: EINVAL, EHIP. */
int32_t closure_features(eles_filter f, const float *ubar, float *feat, hipStream_t stream);

/* FP64 mean and standard deviation of every channel of data (device
 * [nsnap][nchan][npts]) into out (device [2][nchan]). */
size_t closure_moments_workspace_bytes(int32_t nchan);
int32_t closure_moments(const float *data, int32_t nchan, int32_t nsnap, int64_t npts, double *out, void *ws,
                        size_t ws_bytes, hipStream_t stream);

/* closure_moments for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid
 * allocation): no workspace argument. Its partial sums live in a static
 * device array of ELES_MOMENTS_NOALLOC_MAX_CHAN x 1024 doubles (512 KiB)
 * that each GPU the library runs on holds until the process ends; the
 * call allocates nothing. The stream must belong to the current device.
 * Results are bit for bit those of closure_moments. Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (from two streams
 * or threads) race and must be serialised by the caller. Errors: EINVAL
 * (null pointers, nchan, nsnap or npts < 1), ENOSPACE (nchan above
 * ELES_MOMENTS_NOALLOC_MAX_CHAN: beyond the static array), EHIP. */
#define ELES_MOMENTS_NOALLOC_MAX_CHAN 64
int32_t closure_moments_noalloc(const float *data, int32_t nchan, int32_t nsnap, int64_t npts, double *out,
                                hipStream_t stream);

/* Adam training on minibatches drawn from nsnap snapshots of features
 * (device [nsnap][10][npts]) and exact stresses (device [nsnap][6][npts]);
 * loss = mean squared error of the standardised outputs. loss_hist:
 * device FP32 [steps] or NULL. A later call continues the same minibatch
 * stream and Adam state. Errors: EINVAL, ENOSPACE, ENOTSUP, EHIP. */
size_t closure_train_workspace_bytes(int32_t batch);
int32_t closure_train(eles_closure c, const float *feat, const float *tau, int32_t nsnap, int64_t npts,
                      const eles_train_desc *d, float *loss_hist, void *ws, size_t ws_bytes, hipStream_t stream);

/* Predicted stress from a filtered velocity: features, then the network,
 * with the exact filtered stress of Sec. 2.1 as the fallback. tau_pred:
 * device [6][nx][ny][nz]; stats: device FP64 [6][ny] plane averages of
 * tau_pred (the returned one, network or exact), or NULL.
 *
 * fallback selects what happens to a non-finite prediction (a NaN or an
 * infinity anywhere in tau_pred, detected through the FP64 plane sums of
 * tau_pred, which carry any of them):
 *   ELES_INFER_UNCHECKED: no test; the call only enqueues work.
 *   ELES_INFER_CHECK:     the call waits for the stream and returns
 *                         ENUMERIC, tau_pred holding the network's output.
 *   ELES_INFER_FALLBACK:  the call waits for the stream and, on a
 *                         non-finite prediction, computes the exact stress
 *                         of u_or_null (device [3][nx][ny][nz], the
 *                         unfiltered velocity ubar was filtered from) into
 *                         tau_pred with sgs_stress on the same handle and
 *                         stream, bit for bit what sgs_stress returns.
 * *fell_back (host, may be NULL) is set to 1 when the exact stress
 * replaced the prediction, else 0. u_or_null is read only on fallback and
 * must not overlap tau_pred or ws. Workspace:
 * closure_infer_workspace_bytes(f, fallback == ELES_INFER_FALLBACK).
 * Errors: EINVAL (also fallback out of range, or ELES_INFER_FALLBACK with
 * u_or_null NULL or misaligned), ENOSPACE, ENUMERIC (ELES_INFER_CHECK
 * only), EHIP; on fallback, the errors of sgs_stress. */
#define ELES_INFER_UNCHECKED (-1)
#define ELES_INFER_CHECK 0
#define ELES_INFER_FALLBACK 1
size_t closure_infer_workspace_bytes(eles_filter f, int32_t with_fallback);
int32_t closure_infer(eles_closure c, eles_filter f, const float *ubar, float *tau_pred, double *stats,
                      int32_t fallback, const float *u_or_null, int32_t *fell_back, void *ws, size_t ws_bytes,
                      hipStream_t stream);

/* The minibatch indices the trainer draws at `step` (device int64 [batch]). */
int32_t closure_sample_indices(uint64_t seed, int64_t step, int32_t batch, uint64_t count, int64_t *out,
                               hipStream_t stream);

void closure_destroy(eles_closure c);

#ifdef __cplusplus
}
#endif

#endif /* ELES_H */
