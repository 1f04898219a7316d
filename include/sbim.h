/*
 * sbim.h -- C ABI of the MI355X spectral boundary integral (SBIM) library.
 *
 * One handle advances the exterior half-spaces of one or two boundary planes
 * of a regular n1 x n3 grid through time.  Per time step the caller pushes
 * the boundary displacement (hybrid step item 2, Sec. 2.4) and then asks for
 * the boundary tractions of that same step (item 3, Sec. 2.4), which follow
 * the boundary relation of Sec. 2.3 (Eq. SBI):
 *
 *     tau_i = tau_inf_i - eta_ij (mu / c_s) du_j/dt + s_i ,
 *
 * with eta = diag(1, c_p/c_s, 1) (the paper prints eta_22 = c_s/c_p; the
 * exact half-space impedance of a normally incident P wave is c_p/c_s, which
 * is what is used) and s_i the nonlocal term: a 2-D Fourier transform in space
 * and, per Fourier mode, a truncated time convolution of the displacement
 * history with the elastodynamic half-space kernels (the paragraph after
 * Eq. SBI; truncation as cited in Sec. 1).
 *
 * Conventions shared by every entry point
 *   Fields are contiguous device arrays [P][3][n1][n3] (P = nplanes,
 *   component index 0,1,2 = x1, x2 (plane normal), x3; x3 fastest), in the
 *   handle's working precision: double for SBIM_FP64, float otherwise.
 *   Tractions are sigma_i2 on the plane.  Plane p with side = +1 bounds a
 *   half-space lying on its +x2 side (top boundary of the strip), side = -1
 *   one lying on its -x2 side.
 *   Fourier convention: forward exp(-i k.x) over the stored half spectrum
 *   (i1 = 0..n1-1, i3 = 0..n3/2); k1 = 2 pi m1 / (n1 dx1) with
 *   m1 = i1 for i1 < n1/2 and i1 - n1 otherwise; k3 = 2 pi i3 / (n3 dx3);
 *   q = sqrt(k1*k1 + k3*k3).  The inverse takes the real part of the inverse
 *   transform of the Hermitian extension of the stored half, divided by
 *   n1*n3 (imaginary parts of the i3 = 0 and i3 = n3/2 columns are dropped).
 *   History: the displacement is piecewise constant over each step and the
 *   kernels are integrated exactly over each step; the history before the
 *   first push is zero.  Mode k keeps W(q) past steps (lag 0 = the step just
 *   pushed): W = window_cap for SBIM_W_FIXED, or
 *   W = min(window_cap, ceil(2 pi eta_w / (q c_s dt))) for SBIM_W_PER_MODE.
 *
 * Streams and ownership
 *   Every call enqueues work on the handle's HIP stream (config.stream,
 *   0 = the null stream) and returns without synchronising, except where a
 *   comment says otherwise.  The caller owns all field buffers passed in and
 *   must keep them alive until the stream reaches the call.  The handle owns
 *   the history ring, kernel tables, running state and scratch; it allocates
 *   them in sbim_init (the adjoint ring at the first sbim_backward) and frees
 *   them in sbim_destroy.
 *
 * Errors
 *   Every int-returning call returns SBIM_OK (0) or a negative code and never
 *   aborts or throws; sbim_last_error gives a message for the last failure on
 *   that handle.  On an error nothing has been enqueued and the handle's state
 *   is unchanged.  HIP runtime failures map to SBIM_E_DEVICE.
 */
#ifndef SBIM_H
#define SBIM_H

#ifdef __cplusplus
extern "C" {
#endif

#define SBIM_OK 0
#define SBIM_E_INVALID (-1) /* bad argument or configuration */
#define SBIM_E_OOM (-2)     /* device memory for the requested sizes not available */
#define SBIM_E_STATE (-3)   /* call out of order (e.g. tractions before any push) */
#define SBIM_E_DEVICE (-4)  /* HIP runtime error */

/* precision */
#define SBIM_FP64 0       /* double fields, FFTs, history, kernels, sums */
#define SBIM_FP32 1       /* float fields, FFTs, history, kernels; plain float sums */
#define SBIM_FP32_COMP 2  /* as SBIM_FP32 with compensated (Kahan) history sums */
/* window_mode */
#define SBIM_W_FIXED 0
#define SBIM_W_PER_MODE 1
/* quasi-dynamic limit (Sec. 7 pairs it with the dynamic relation for cycle
 * simulations): each mode keeps only the step just pushed and the kernels act
 * through their static integrals G_ab(infinity), i.e. the half-space's static
 * surface stiffness; the damping term is kept.  window_cap is ignored and dt
 * may change between pushes (sbim_set_dt). */
#define SBIM_W_STATIC 2
/* input_kind */
#define SBIM_ABSOLUTE 0   /* push receives u^n - u^0 */
#define SBIM_INCREMENT 1  /* push receives u^n - u^{n-1} */

#define SBIM_MAX_PLANES 2

typedef struct {
  int side;      /* +1 or -1, see above */
  double mu;     /* shear modulus, > 0 */
  double cs;     /* shear wave speed, > 0 */
  double cp;     /* pressure wave speed, cp > cs * sqrt(4/3) */
} sbim_plane;

typedef struct {
  int n1, n3;            /* grid, powers of two in [4, 4096] */
  double dx1, dx3;       /* grid spacing, > 0 */
  double dt;             /* time step, > 0 */
  int nplanes;           /* 1 or 2 */
  sbim_plane plane[SBIM_MAX_PLANES];
  int window_cap;        /* >= 1: longest history kept per mode */
  int window_mode;       /* SBIM_W_FIXED, SBIM_W_PER_MODE or SBIM_W_STATIC */
  double eta_w;          /* > 0, used by SBIM_W_PER_MODE */
  int precision;         /* SBIM_FP64, SBIM_FP32 or SBIM_FP32_COMP */
  int input_kind;        /* SBIM_ABSOLUTE or SBIM_INCREMENT */
  void *stream;          /* hipStream_t for all work of this handle (0 = null stream) */
} sbim_config;

typedef struct sbim_handle sbim_handle;

/* Sizes and derived quantities of a handle (host struct filled by sbim_get_info). */
typedef struct {
  long long modes_per_plane;   /* n1 * (n3/2 + 1) */
  long long kernel_classes;    /* distinct (q, W) rows of the kernel tables, all groups */
  long long ring_bytes;        /* forward history ring */
  long long table_bytes;       /* kernel tables */
  long long state_bytes;       /* float64 running state */
  long long step;              /* pushes since init / reset */
  long long backward_step;     /* sbim_backward calls since the last reset */
  int material_groups;         /* planes sharing (c_s, c_p) share one table and one pass */
  int sweep_depth;             /* steps served by one pass over a block's history: 32 on
                                  the matrix cores (below); otherwise 6 when the mean
                                  window is under 64 lags, else 12 (float64, compensated,
                                  and float32 from a mean window of 1500 lags) or 8
                                  (float32 below that); the environment variable
                                  SBIM_SWEEP_DEPTH (1, 2, 4, 6, 8, 12 or 16; 16 or 32 on
                                  the matrix cores) overrides it at sbim_init, for tuning */
  int sweep_matrix_cores;      /* 1: the history sweep runs as 16x16x4 float32 matrix-core
                                  products (float32 forms, one window for every mode, two
                                  planes of one material, mean window of 64 lags or more);
                                  SBIM_SWEEP_KIND=valu or mfma overrides it, for tuning */
  int sweep_lag_chunks;        /* matrix-core sweep: wavefronts per group of four modes,
                                  each summing a range of lags (1, 2 or 4; 0 otherwise);
                                  SBIM_SWEEP_CHUNKS overrides it, for tuning */
  int sweep_quads;             /* matrix-core sweep: groups of four modes per work-group
                                  (1, 2 or 4, at most 4 / sweep_lag_chunks; 0 otherwise):
                                  2 for the compensated form (two lag ranges), 1 for
                                  plain float32 (four); SBIM_SWEEP_QUADS overrides it,
                                  for tuning */
} sbim_info;

/*
 * sbim_init: validate *cfg, allocate the ring, tables and state on the
 * current HIP device, and tabulate the kernels (float64 quadrature of the
 * half-space kernels' branch-cut integrals, rounded to the working precision).
 * Synchronises the stream before returning.  On success *out is a new handle
 * (step 0); on failure *out is set to NULL and a message can be fetched with
 * sbim_last_error(NULL).  SBIM_E_OOM is returned before any allocation when
 * the sizes exceed the free device memory.
 */
int sbim_init(const sbim_config *cfg, sbim_handle **out);

/*
 * sbim_push_displacement: advance the history by one step.
 *   u          device [P][3][n1][n3]: u^n - u^0 (SBIM_ABSOLUTE) or
 *              u^n - u^{n-1} (SBIM_INCREMENT)
 *   v_or_null  device [P][3][n1][n3] velocity prediction for the damping term
 *              of this step, or NULL to use (u^n - u^{n-1}) / dt
 * Exactly one push precedes each sbim_tractions call.  The push computes
 * the traction spectrum of this step (the inverse transform is left to
 * sbim_tractions) and, in the same launch, the history sweep for the coming
 * steps: the 64-mode blocks whose turn it is (one in sweep_depth of them, in
 * rotation) read their history window up to the previous step once and store
 * the part of each of the next sweep_depth steps' history sums that this
 * history already fixes; every step thus reads each history entry
 * 1/sweep_depth times on average.
 */
int sbim_push_displacement(sbim_handle *h, const void *u, const void *v_or_null);

/*
 * sbim_tractions: tau^n of the last pushed step into device [P][3][n1][n3].
 *   tau_inf_or_null  device [P][3][n1][n3] far-field traction added to the
 *                    result, or NULL for zero.
 * It applies the inverse transform to the traction spectrum that the last
 * push completed and changes no state: calling it again before the next push
 * returns the same tractions.
 * SBIM_E_STATE if no step was pushed since init/reset.
 */
int sbim_tractions(sbim_handle *h, const void *tau_inf_or_null, void *tau);

/*
 * sbim_backward: one step of the exact transpose of the map from the pushed
 * inputs to the tractions.  After N forward steps call it for n = N-1, ..., 0
 * with g = dL/dtau^n (device [P][3][n1][n3]); it writes dL/du^n (with respect
 * to what push received: u^n - u^0 or the increment) into dL_du, and, when
 * velocities were pushed explicitly, dL/dv^n into dL_dv (pass NULL when they
 * were not).  The transpose is the same operator run as a time-reversed
 * correlation (the per-mode operators are Hermitian), so it needs no forward
 * state; it keeps its own history of g.  sbim_backward_reset restarts it.
 */
int sbim_backward(sbim_handle *h, const void *dL_dtau, void *dL_du, void *dL_dv_or_null);
int sbim_backward_reset(sbim_handle *h);

/* sbim_reset: zero the history, running state and step counters (forward and backward). */
int sbim_reset(sbim_handle *h);

/* sbim_destroy: synchronise the stream and free everything; NULL is accepted. */
int sbim_destroy(sbim_handle *h);

/* Message of the last failure on h (or of the last failed sbim_init when h is NULL). */
const char *sbim_last_error(const sbim_handle *h);

/*
 * Use another HIP stream for subsequent calls.  Work queued on the new stream
 * is ordered after everything already queued on the old one (an event recorded
 * there and waited on by the new stream); the host is not synchronised.
 * SBIM_E_DEVICE if that ordering cannot be set up (the stream is then unchanged).
 */
int sbim_set_stream(sbim_handle *h, void *stream);

/*
 * sbim_set_dt: the time step of the following pushes (the velocity of the
 * damping term when none is pushed, and the updates of a fault or strip on
 * this handle).  Only for SBIM_W_STATIC handles, whose boundary relation does
 * not depend on dt (variable time stepping); SBIM_E_STATE otherwise, since the
 * dynamic kernels are integrated over the step of sbim_init.
 */
int sbim_set_dt(sbim_handle *h, double dt);

/*
 * sbim_traction_spectrum: copy the traction spectrum of the last push (the
 * nonlocal, instantaneous and damping terms of Sec. 2.3, Eq. SBI, in the
 * (x1, x2, x3) frame, before tau^infinity and the inverse transform) into dst:
 * device memory of [P][3][n3/2+1][n1] complex values of the handle's precision
 * (interleaved re, im; bin (i1, i3) at i3 * n1 + i1; forward transform
 * exp(-i k.x), no 1/(n1 n3) factor).  Asynchronous on the handle's stream; a
 * diagnostic for checking the step before the inverse transform.
 * SBIM_E_STATE before the first push.
 */
int sbim_traction_spectrum(sbim_handle *h, void *dst);

/* Fill *out (host memory). */
int sbim_get_info(const sbim_handle *h, sbim_info *out);

/*
 * sbim_count_nonfinite: the number of infinities and NaNs in a device field
 * [P][3][n1][n3] of the handle's precision (a displacement or velocity before it
 * is pushed, or a traction output) into *count (host).  Synchronises the
 * stream.  A diagnostic beside the step: the step itself does not check values.
 */
int sbim_count_nonfinite(sbim_handle *h, const void *field, long long *count);

/*
 * sbim_count_nonfinite_noalloc: the same count, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  It calls no hipMalloc, hipFree or other
 * allocating routine: the per-work-group partial counts go to a static device
 * array of the library (1024 counts, 8 KiB; each GPU the library runs on holds
 * its own copy until the process ends, its address looked up once per device
 * by sbim_init), and a second one-work-group kernel writes their sum to
 * *count_dev, a caller-owned device int64.  Asynchronous on the handle's
 * stream (no host synchronisation); the count is there once the stream has
 * passed this call.  The scratch size does not depend on the field size, so
 * every field the handle accepts fits.  Calls that overlap on one GPU (other
 * streams, other handles, other threads) share the array and race: order them.
 * Errors: SBIM_E_INVALID for a NULL handle, field or count_dev; SBIM_E_STATE
 * when the current device is not the handle's; SBIM_E_DEVICE for a launch
 * failure.
 */
int sbim_count_nonfinite_noalloc(sbim_handle *h, const void *field, long long *count_dev);

/*
 * Snapshots for checkpointing: the full forward state (ring, running state,
 * pending history sums of the coming steps, traction spectrum of the last
 * step, step counter) is sbim_state_bytes() bytes.  save/load
 * copy it to/from a caller-owned device buffer of at least that size,
 * asynchronously on the handle's stream.
 */
long long sbim_state_bytes(const sbim_handle *h);
int sbim_save_state(sbim_handle *h, void *dst_device);
int sbim_load_state(sbim_handle *h, const void *src_device);

/*
 * Light snapshots for checkpointing long runs: only the float64 running state
 * (the accumulated displacement spectrum of every mode) and the step counter,
 * sbim_running_state_bytes() bytes, copied to/from a caller-owned device buffer
 * asynchronously on the handle's stream.  Loading one also empties the history
 * ring and the pending sums.  The truncated convolution reads only the last
 * W + sweep_depth + 1 pushes, so after loading the running state of step n0 and
 * pushing steps n0 .. a-1 again with a - n0 >= W_cap + sweep_depth + 2, the
 * handle is in the state of the original run at step a (bit for bit: the same
 * history entries, summed by the same launches); tractions of the replayed
 * steps before that are not the original ones.  SBIM_E_INVALID for NULL
 * arguments or a corrupt header.
 */
long long sbim_running_state_bytes(const sbim_handle *h);
int sbim_save_running_state(sbim_handle *h, void *dst_device);
int sbim_load_running_state(sbim_handle *h, const void *src_device);

/*
 * Work of the step with index n (0-based): *mode_lags = the number of
 * (plane, mode, lag) products of that step's history sums, i.e. min(W(q), n+1)
 * summed over planes and modes; *conv_bytes = the bytes that the one launch
 * of that step's push must move: the history sweep (the history up to step
 * n-1 of the modes whose block sweeps for steps n+1 .. n+sweep_depth, phase
 * (n+1) mod sweep_depth; the kernel rows of each distinct row class in those
 * blocks; their row/window indices and block descriptors; the sweep_depth
 * pending sums written per mode and plane) and the mode items (spectrum
 * gathered, float64 state read and written, ring slot written, pending sum
 * read, newest lags and their kernel rows read, traction spectrum written,
 * per-mode indices and geometry).
 */
int sbim_step_work(const sbim_handle *h, long long n, double *mode_lags, double *conv_bytes);

/*
 * Diagnostics (synchronising): the kernel row the handle uses for half-spectrum
 * bin (i1, i3) of plane p: returns W(q) for that bin (>= 0) or a negative
 * error, and copies min(W, max_lags) lags of (w11, w12, w22, w33) as float64
 * into host_out[4][max_lags] (row-major by kernel).
 */
int sbim_mode_kernel(sbim_handle *h, int p, int i1, int i3, double *host_out, int max_lags);

/*
 * Timing of the push / history sweep launch (the dominant kernel of a step):
 * with every = n >= 1, HIP events on the handle's stream bracket every n-th of
 * its launches made by sbim_push_displacement (the first, the (n+1)-th, ...,
 * counted from this call); every = 0 turns the timing off.  A bracketed launch
 * also pays for its two event records (a few microseconds at the start and end
 * of the launch), so sampling with n > 1 keeps that cost off most steps.
 * sbim_conv_timing synchronises and returns the summed device time (ms) and
 * the number of bracketed launches since the last sbim_profile_conv.
 * Synchronises the handle's stream.  Errors: SBIM_E_INVALID for a NULL handle
 * or every < 0.
 */
int sbim_profile_conv(sbim_handle *h, int every);
int sbim_conv_timing(sbim_handle *h, double *total_ms, long long *launches);

/*
 * ---------------------------------------------------------------------------
 * Frictional fault between two half-spaces (stand-alone boundary-integral
 * dynamic rupture).
 *
 * The fault is the plane x2 = 0 of the grid.  Above it lies the half-space of
 * plane 0 (side +1); below it the half-space of plane 1 (side -1) when the
 * handle has two planes, otherwise the mirror image of plane 0 (same
 * material, u-(x) = (-u1+, u2+, -u3+)): the fault is then a symmetry plane
 * and its normal traction stays at tau0_2 (Sec. 3.1 uses this symmetry).
 * Each side obeys its own boundary relation (Eq. SBI, two independent
 * half-spaces).  The interface conditions are those of Sec. 2.2: the
 * traction is continuous across the fault; per cell either stick (Eq. stick,
 * zero slip rate, shear traction within the strength) or slip (Eq. slip,
 * shear traction at the strength, slip rate along it), chosen as in
 * Eq. stickslip; strength = normal stress x mu(delta), mu the linear
 * slip-weakening coefficient of Eq. slipweak and delta the amplitude of the
 * slip vector (Sec. 2.2).  The fault does not open: the normal velocity is
 * continuous.
 *
 * One sbim_fault_step is the explicit step n (displacements u+ = u- = 0 and
 * slip D = 0 before step 0):
 *   1. push each side's displacement u^n (u^n - u^{n-1} for an SBIM_INCREMENT
 *      handle) with the damping term left out, and take that push's
 *      tractions: s = the nonlocal and instantaneous parts of Eq. SBI;
 *   2. f = tau0 + s per side; with Z_i = eta_ii mu / c_s per side (the
 *      damping coefficients of Eq. SBI, eta_22 = c_p / c_s):
 *        tau_2 = (Z2- f2+ + Z2+ f2-) / (Z2+ + Z2-)
 *        t~    = (Z1- f+  + Z1+ f- ) / (Z1+ + Z1-)   for the shear pair (1, 3)
 *        S     = max(-tau_2, 0) mu(|D^n|)            (compression positive)
 *        |t~| <= S: tau = t~, V = 0;  else tau = S t~ / |t~|,
 *                   V = (t~ - tau)(1/Z1+ + 1/Z1-)
 *   3. v+ = (f+ - tau) / Z+, v- = (tau - f-) / Z-; u^{n+1} = u^n + dt v;
 *      slip D^{n+1} = D^n + dt V.
 * The fault's arithmetic and state are float64 for every precision; the
 * traction functional s and the pushed displacement have the handle's
 * precision.  Fault fields are device arrays [rows][n1][n3] of double
 * (x3 fastest): traction rows (x1, x2, x3), slip and slip-rate rows (x1, x3).
 *
 * Ownership: the fault keeps copies of the parameters, its state, and two
 * field buffers of the handle's precision.  It drives its handle: between
 * sbim_fault_create and sbim_fault_destroy the handle must not be pushed,
 * reset or destroyed by other calls (SBIM_E_STATE is returned when the step
 * counts disagree).  Destroy the fault before its handle.
 */
typedef struct sbim_fault sbim_fault;

typedef struct {
  const double *tau0;  /* device [3][n1][n3]: background traction sigma_2i (i = 2: normal, tension > 0) */
  const double *mu_s;  /* device [n1][n3]: static friction coefficient, >= mu_k */
  const double *mu_k;  /* device [n1][n3]: kinetic friction coefficient, >= 0 */
  const double *d_c;   /* device [n1][n3]: slip-weakening distance, > 0 */
} sbim_fault_params;

/* fields of sbim_fault_read */
#define SBIM_FAULT_TRACTION 0     /* [3][n1][n3] tau of the last step */
#define SBIM_FAULT_SLIP_RATE 1    /* [2][n1][n3] V of the last step (x1, x3) */
#define SBIM_FAULT_SLIP 2         /* [2][n1][n3] D after the last step */
#define SBIM_FAULT_DISPLACEMENT 3 /* [2][3][n1][n3] u+ then u- after the last step */
#define SBIM_FAULT_VELOCITY 4     /* [2][3][n1][n3] v+ then v- of the last step */

/*
 * sbim_fault_create: a fault on handle h (planes as described above, handle at
 * step 0).  The parameter arrays are copied (the caller may free them
 * afterwards) and checked on the device; synchronises the stream.
 * SBIM_E_INVALID names the first offending cell (non-finite value, d_c <= 0,
 * mu_k < 0 or mu_s < mu_k).  A cell can be locked (a bonded interface) by a
 * static coefficient that no traction reaches.
 */
int sbim_fault_create(sbim_handle *h, const sbim_fault_params *prm, sbim_fault **out);

/*
 * sbim_fault_step: one explicit step (push, inverse transform, interface solve
 * on the handle's stream).  tau_or_null / slip_rate_or_null: optional device
 * [3][n1][n3] / [2][n1][n3] doubles that also receive the step's traction and
 * slip rate.
 */
int sbim_fault_step(sbim_fault *f, double *tau_or_null, double *slip_rate_or_null);

/* Copy one fault field (SBIM_FAULT_*) into device memory dst (asynchronous). */
int sbim_fault_read(const sbim_fault *f, int field, double *dst);

/* Zero the fault state and reset its handle (sbim_reset). */
int sbim_fault_reset(sbim_fault *f);

/* Synchronise the stream and free the fault (not its handle); NULL is accepted. */
int sbim_fault_destroy(sbim_fault *f);

/*
 * ---------------------------------------------------------------------------
 * Hybrid finite-element / boundary-integral rupture (Sec. 2.4).
 *
 * A strip of 8-node hexahedral finite elements (Sec. 2.2, FEM) of side
 * h = dx1 = dx3 lies on the fault: `layers` element layers between the fault
 * (node layer 0) and the virtual boundary S+ (node layer `layers`), periodic
 * in x1 and x3 on the handle's n1 x n3 grid.  The handle has one plane (side
 * +1): the half-space above S+, whose boundary relation (Eq. SBI) closes the
 * strip.  The fault plane is a symmetry plane (Sec. 3.1): the lower half of
 * the strip is the mirror image, the slip is twice the tangential
 * displacement of the fault nodes, and the fault normal traction keeps its
 * background value.  Elements: trilinear shape functions, 2x2x2 Gauss points,
 * isotropic elasticity per element layer (Eq. linelasticity), lumped mass
 * rho h^3/8 per element corner.
 *
 * One sbim_strip_step advances t -> t+1 (Sec. 2.2 predictor-corrector,
 * Sec. 2.4 items 1-7; dt = the handle's dt):
 *   1. v_{t+1/2} = v_t + dt/2 a_t, u_{t+1} = u_t + dt v_{t+1/2},
 *      v^pred = v_t + dt a_t (Eq. fepred; the displacement advances with the
 *      half-step velocity, the form under which the stick condition after
 *      Eq. freeslip keeps the slip fixed);
 *   2. push the S+ layer's u_{t+1} (or its increment) with v^pred as the
 *      velocity of the damping term; the tractions of that push act on the S+
 *      nodes with area h^2;
 *   3. r = -K u_{t+1} + S+ forces; at a fault node the stick traction is
 *      tau~ = tau0 + M v* / (dt h^2) with v* = v_{t+1/2} + dt r / M the next
 *      half-step velocity without fault traction (Eqs. freeslip,
 *      sticktraction for two mirrored sides); strength S = max(-tau0_2, 0)
 *      mu(|slip|) (Eq. slipweak); tau = tau~ if |tau~| <= S, else
 *      S tau~/|tau~| (Eq. stickslip); the fault adds -h^2 (tau - tau0);
 *   4. a_{t+1} = r / M, v_{t+1} = v_{t+1/2} + dt/2 a_{t+1} (Eqs. tintf, fecorr).
 *
 * Two-sided strip (layers_below > 0; the handle has two planes, sides +1 and
 * -1 in that order): elements on both sides of a split-node fault, each block
 * closed by its own boundary relation (S+ above, S- below, whose tractions act
 * on the S- nodes with outward normal -e2).  The fault nodes have an upper and
 * a lower copy.  In step 3 the stick traction closes the jump of their next
 * half-step velocities, tau~ = tau0 + (v*+ - v*-) / (dt h^2 (1/M+ + 1/M-))
 * (Eqs. freeslip, sticktraction with two sides), its normal component is
 * applied as it is (no opening), the shear pair is limited by
 * S = max(-tau_2, 0) mu(|u+ - u-|) (Eqs. stickslip, slipweak), and the upper
 * and lower copies receive -h^2 (tau - tau0) and +h^2 (tau - tau0).  Slip and
 * slip rate are then the upper minus the lower copy.
 *
 * On a quasi-dynamic handle (SBIM_W_STATIC) the step size may change between
 * strip steps (sbim_set_dt): each step then runs with the handle's current dt
 * (the library evaluates item 1 of a step at the end of the previous one, and
 * evaluates it again with the new size when the size has changed).
 *
 * All strip arithmetic is float64; the S+/S- push has the handle's precision.
 * Fault fields are device [rows][n1][n3] doubles; node fields
 * [3][L][n1][n3] over the storage node layers: L = layers + 1 one-sided
 * (0 = fault, layers = S+); two-sided L = layers_below + layers + 2, layers
 * 0 .. layers_below the lower block (0 = S-, layers_below = lower fault
 * copy), then the upper block from its fault copy to S+.  Ownership rules as
 * for sbim_fault.  The scheme is
 * explicit: dt must satisfy the elements' CFL limit (the highest frequency of
 * the lumped-mass hexahedra is 2 c_p / h, so c_p dt / h < 1).
 */
typedef struct sbim_strip sbim_strip;

typedef struct {
  int layers;           /* element layers between the fault and S+, 1..4096 */
  const double *rho;    /* host [layers]: density of each element layer (fault side first) */
  const double *cp;     /* host [layers]: pressure wave speed, > cs sqrt(4/3) */
  const double *cs;     /* host [layers]: shear wave speed, > 0 */
  int layers_below;     /* element layers between the fault and S-, 0 (one-sided) .. 4096 */
  const double *rho_below;  /* host [layers_below], fault side first; NULL when one-sided */
  const double *cp_below;
  const double *cs_below;
} sbim_strip_config;

/* fields of sbim_strip_read */
#define SBIM_STRIP_TRACTION 0     /* [3][n1][n3] fault traction of the last step */
#define SBIM_STRIP_SLIP_RATE 1    /* [2][n1][n3] slip rate v_{t+1} jump (x1, x3): 2 v one-sided */
#define SBIM_STRIP_SLIP 2         /* [2][n1][n3] slip u_{t+1} jump: 2 u one-sided */
#define SBIM_STRIP_SLIDING 3      /* [n1][n3] 1 where the slip branch was taken, else 0 */
#define SBIM_STRIP_DISPLACEMENT 4 /* [3][L][n1][n3], L storage node layers */
#define SBIM_STRIP_VELOCITY 5     /* [3][L][n1][n3] */

/*
 * sbim_strip_create: a strip on handle h (one plane of side +1, or planes of
 * sides +1, -1 when layers_below > 0; dx1 == dx3; at step 0) with the fault parameters of sbim_fault_params (copied and
 * checked on the device; synchronises the stream).
 */
int sbim_strip_create(sbim_handle *h, const sbim_strip_config *cfg, const sbim_fault_params *prm,
                      sbim_strip **out);
/* One step; tau_or_null / slip_rate_or_null as in sbim_fault_step. */
int sbim_strip_step(sbim_strip *s, double *tau_or_null, double *slip_rate_or_null);
/* Copy one strip field (SBIM_STRIP_*) into device memory dst (asynchronous). */
int sbim_strip_read(const sbim_strip *s, int field, double *dst);
/* Zero the strip state and reset its handle. */
int sbim_strip_reset(sbim_strip *s);
/* Synchronise the stream and free the strip (not its handle); NULL is accepted. */
int sbim_strip_destroy(sbim_strip *s);

#ifdef __cplusplus
}
#endif

#endif /* SBIM_H */
