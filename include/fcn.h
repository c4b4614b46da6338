/*
 * fcn.h -- C ABI of the MI355X (gfx950) implementation of the 2D+1 split-step Fourier /
 * Crank-Nicholson (FCN) z-step of Ma & Lin, "Parallel simulation for the ultra-short laser
 * pulses' propagation in air" (arXiv:1507.05988).
 *
 * The paper's serial method (Sec. 3, closing summary) is: input the pulse, the equation
 * coefficients, the r and t ranges and the grid steps; precompute the tridiagonal matrices
 * M_abc^p, M_def^p for every frequency; then loop over z.  Here that maps to
 * fcn_plan_create (input + precompute what does not depend on the field), fcn_step (the
 * z loop) and fcn_propagate (the z loop with diagnostics and adaptive step lengths).
 *
 * Conventions shared by every entry point
 *  - Units are SI.  Plain pointers and sizes only; no C++ or torch types cross this ABI.
 *  - Field layout: one flat buffer of complex values, interleaved (re, im), for all
 *    instances of a plan; instance i starts at the element offset fcn_field_offset(i) and
 *    is a row-major [nr][nt] matrix with t contiguous: element (m, p) is A(r_m, t_p) with
 *    r_m = m r_max/(nr-1) and t_p = t_min + p (t_max - t_min)/nt (Sec. 3, the grid
 *    A_{m,p}).  A Cartesian instance (FCN_CARTESIAN) is a row-major [ny][nx][nt] array:
 *    element (j, i, p) is A(x_i, y_j, t_p) with x_i = -x_max + i dx, dx = 2 x_max/(nx-1),
 *    y_j likewise; its nx * ny transverse points play the part of the rows.
 *    Precision FCN_FP64 uses double2 elements, the FP32 modes float2 elements.
 *    Between calls the field is in the time domain at an integer z-step.
 *  - Ownership: the caller allocates and frees every device buffer (field, workspace,
 *    diagnostics, dz log) and owns the HIP stream.  After fcn_plan_bind the library never
 *    allocates device memory.  Plans own only host memory and are freed by
 *    fcn_plan_destroy.
 *  - Asynchrony: compute entry points enqueue work on the bound stream and return at once.
 *    Argument errors are reported synchronously by the return code; numerical failure
 *    (a non-finite intensity, or a density step outside its stability region, seen on the
 *    device) is reported by fcn_sync.
 *  - A plan is not thread-safe.  fcn_last_error(plan) gives a text for the last failure.
 */
#ifndef FCN_H
#define FCN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fcn_plan_s *fcn_plan_t;

typedef enum {
    FCN_OK = 0,
    FCN_E_ARG = 1,         /* invalid argument or parameter value */
    FCN_E_SIZE = 2,        /* workspace too small, or a size outside the supported range */
    FCN_E_HIP = 3,         /* a HIP runtime call failed */
    FCN_E_NONFINITE = 4,   /* the device saw a non-finite intensity */
    FCN_E_STATE = 5,       /* call order violated (e.g. step before bind) */
    FCN_E_UNSUPPORTED = 6, /* valid request this build does not implement */
    FCN_E_UNSTABLE = 7     /* an RK4 step of the density (Eq. ionization) left its stability
                              region: sigma_K I^K dtau beyond about 2.785 somewhere on the grid,
                              so the density runs out of [0, rho_at]; a property of the method at
                              that time step, reported by fcn_sync */
} fcn_status;

/* Term switches of the operators (Eqs. linearpart and nonlinearpart). */
enum {
    FCN_DIFFRACTION = 1, /* (i/2k0)(d2/dr2 + (1/r) d/dr) of Eq. linearpart */
    FCN_GVD = 2,         /* -(i k''/2) d2/dt2 of Eq. linearpart */
    FCN_KERR = 4,        /* i (k0/n0) sum_j n_2j |A|^2j of Eq. nonlinearpart */
    FCN_PLASMA = 8,      /* -(i k0/2) omega_pe^2/omega0^2 = -(i k0/2) rho/rho_c */
    FCN_MPA = 16,        /* -(beta_K/2) |A|^(2K-2), beta_K = K hbar omega0 sigma_K rho_at */
    FCN_COLL = 32,       /* -(sigma_c/2) rho, collisional absorption (not in the paper) */
    FCN_AVALANCHE = 64   /* avalanche ionisation: (sigma_c / U_i) |A|^2 rho added to the density
                            rate of Eq. ionization (not in the paper) */
};

/* Transverse geometry of an instance.  FCN_RADIAL: Delta_perp = d2/dr2 + (1/r) d/dr for a
 * cylindrically symmetric beam, the case the paper discretises (Sec. 3.1).  FCN_CARTESIAN:
 * Delta_perp = d2/dx2 + d2/dy2, the other operator named beside Eq. nlse (Sec. 2), which the
 * paper does not discretise; here every frequency column takes the paper's Crank-Nicholson
 * scheme along x and then along y, (1 - dz/2 Ly)^-1 (1 + dz/2 Ly) (1 - dz/2 Lx)^-1
 * (1 + dz/2 Lx), with Lu = (i/2k0) d2/du2 + i k'' omega_p^2 / 4 (the GVD term split evenly);
 * the two axis operators commute, so this is the Peaceman-Rachford alternating-direction form
 * of the two-dimensional Crank-Nicholson step, and each factor is a tridiagonal solve per line.
 * A = 0 on the four walls x = +-x_max, y = +-y_max (the counterpart of A = 0 at r_max, Eq.
 * bound).  The transforms and the nonlinear half steps are the same as for FCN_RADIAL. */
enum { FCN_RADIAL = 0, FCN_CARTESIAN = 1 };

/* Precision modes.  FCN_FP32_STORAGE keeps the field in FP32 (the HBM traffic of FCN_FP32)
 * and computes every stage in FP64 inside the kernels: only the two FP32 stores per step
 * round, so the error grows like a random walk instead of accumulating the FP32 transform
 * error coherently over slowly varying fields.  FCN_FP32_CN64 removes the two largest
 * fixed-rounding sources of FCN_FP32 at a smaller cost: FP32 field, FFTs and nonlinear step
 * as FCN_FP32 but with every FFT twiddle carried as an FP32 hi + lo pair, and the
 * Crank-Nicholson column solve in FP64 arithmetic (the same column kernel as
 * FCN_FP32_STORAGE). */
enum { FCN_FP64 = 0, FCN_FP32 = 1, FCN_FP32_STORAGE = 2, FCN_FP32_CN64 = 3 };

/* One pulse and its grid. */
typedef struct {
    int32_t nr;              /* radial points, 3 <= nr <= 4096; row nr-1 is r = r_max (A = 0).
                                FCN_CARTESIAN: the x points nx, 3 <= nx <= 4096 */
    int32_t nt;              /* time points, a power of two in [64, 8192] */
    double r_max;            /* [m]; FCN_CARTESIAN: the x half-width x_max */
    double t_min, t_max;     /* [s]; periodic window, t_max excluded */
    double lambda0;          /* carrier wavelength [m] */
    double n0;               /* linear refractive index */
    double k2;               /* k'' [s^2/m] */
    double n2, n4, n6, n8;   /* Kerr indices [m^2/W], [m^4/W^2], [m^6/W^3], [m^8/W^4] */
    int32_t K;               /* photons for multiphoton ionisation, 1 <= K <= 16 */
    double sigma_K;          /* [s^-1 (m^2/W)^K] */
    double rho_at;           /* neutral density [m^-3] */
    double sigma_c;          /* collisional cross-section [m^2] */
    double U_i;              /* ionisation potential [J] of the avalanche rate (> 0 with FCN_AVALANCHE) */
    double dz;               /* step length [m] (fixed mode), ignored when adaptive */
    uint32_t terms;          /* OR of the FCN_* term switches */
    int32_t geometry;        /* FCN_RADIAL (0) or FCN_CARTESIAN */
    int32_t ny;              /* FCN_CARTESIAN: y points, 3 <= ny <= 4096, nx * ny <= 2^22
                                (ignored for FCN_RADIAL) */
    double y_max;            /* FCN_CARTESIAN: the y half-width [m] (ignored for FCN_RADIAL) */
} fcn_instance;

typedef struct {
    int32_t precision;       /* FCN_FP64; FCN_FP32 (field, FFTs, CN solve and nonlinear step
                                in FP32, the step on the scaled intensity I/I_ref; density scan
                                and diagnostics in FP64, and h N formed in FP64 when a density
                                term is on); or
                                FCN_FP32_STORAGE (FP32 field, FP64 arithmetic);
                                FCN_FP32_CN64 (FP32 field and row pass with twiddle pairs,
                                FP64 column solve) */
    int32_t adaptive;        /* 0: fixed dz per instance; 1: dz_n = clamp(max_phase/Phi, dz_min,
                                dz_max) with Phi the peak nonlinear phase rate of A^{n-1} */
    double max_phase;        /* [rad] per step, adaptive mode */
    double dz_min, dz_max;   /* [m], adaptive mode */
    int32_t use_graph;       /* 1: replay the step body as a captured HIP graph (needs a non-NULL
                                stream; fcn_step, and fcn_propagate without diagnostics records
                                or dz log: those calls run eagerly) */
    int32_t col_tile;        /* 0: auto; else frequency pairs (p, nt - p) per column workgroup
                                (1, 2, 4, 8, 16 or 32) */
    int32_t col_rows;        /* 0: auto; else rows per thread in the column solve (6, 8 or 16;
                                6 with at most 8 pairs per workgroup) */
    int32_t lanes;           /* 0 or 1: every instance on the bound stream.  2..8: the instances
                                are split into that many groups (greedy balance of nr * nt), each
                                with its own launches and step counters, and fcn_step runs the
                                groups concurrently on helper streams created by fcn_plan_bind
                                (default priority, released by fcn_plan_destroy), forked from and
                                joined to the bound stream, so one group's column pass overlaps
                                another's row pass.  Calls with diagnostics records or a dz log,
                                and fcn_step_scratch, run the groups one after another on the bound
                                stream.  Results are bit for bit those of one lane. */
    const char *tune_cache;  /* NULL, or a text file of tuned column tiles per nr, one per line:
                                "<precision> col <nr> <W> <L> [us]" with precision fp64, fp32,
                                fp32_storage or fp32_cn64 ('#' starts a comment); the entry for a
                                bucket's nr sets its tile unless col_tile / col_rows are given.
                                Read by fcn_plan_create (FCN_E_ARG if unreadable or malformed). */
} fcn_options;

/* Number of doubles per instance in one diagnostics record: 8 scalars then one fluence value
 * per row (nr; nx * ny for FCN_CARTESIAN).
 * Scalars: [0] energy 2 pi dr^2 dtau (sum_p |A_0p|^2 / 8 + sum_m m sum_p |A_mp|^2) [J]
 * (FCN_CARTESIAN: dx dy dtau sum |A|^2), [1] peak intensity, [2] on-axis peak intensity [W/m^2]
 * (FCN_CARTESIAN: at the point ((nx-1)/2, (ny-1)/2), x = y = 0 for odd nx and ny),
 * [3] peak electron density [m^-3], [4] peak nonlinear phase rate Phi [rad/m], [5] z [m],
 * [6] step index, [7] dz of the next step; then fluence F = dtau sum_p |A_.p|^2 [J/m^2] of
 * every row (r_m for m < nr; the transverse point (i, j) at j nx + i for FCN_CARTESIAN). */
#define FCN_DIAG_SCALARS 8

/* Validates the instances and options and builds the host-side plan (derived constants,
 * twiddle tables, work lists).  inst: host array of `batch` instances (batch >= 1), copied.
 * opt may be NULL (defaults: FP64, fixed dz, no graph, automatic tiles).
 * Errors: FCN_E_ARG for invalid values, FCN_E_SIZE for grids outside the supported range. */
fcn_status fcn_plan_create(const fcn_instance *inst, int32_t batch, const fcn_options *opt,
                           fcn_plan_t *out);

/* Bytes of device workspace the plan needs. */
fcn_status fcn_plan_workspace_size(fcn_plan_t plan, size_t *bytes);

/* Complex elements of the flat field buffer, and the element offset of instance i in it. */
fcn_status fcn_field_size(fcn_plan_t plan, size_t *elems);
fcn_status fcn_field_offset(fcn_plan_t plan, int32_t instance, size_t *elem_offset);

/* Doubles of one diagnostics record for the whole batch: sum_i (FCN_DIAG_SCALARS + rows_i),
 * rows_i = nr_i (nx_i * ny_i for FCN_CARTESIAN). */
fcn_status fcn_diag_record_size(fcn_plan_t plan, size_t *doubles);

/* Attaches caller-owned device memory (workspace_dev, at least fcn_plan_workspace_size bytes,
 * 256-byte aligned) and a HIP stream (hipStream_t cast to void*, NULL = default stream).
 * Uploads the plan tables on that stream.  May be called again to move the plan to another
 * workspace or stream; the step counter then restarts at 0. */
fcn_status fcn_plan_bind(fcn_plan_t plan, void *workspace_dev, size_t workspace_bytes, void *stream);

/* Advances every instance by nsteps Strang steps (Sec. 3, Eq. nlseq):
 * A^{n+1} = NL(dz_n/2) o Linear(dz_n) o NL(dz_n/2) A^n, in place on field_dev.
 * The linear part is the forward FFT of every row, the Crank-Nicholson solve of every
 * frequency column (Eqs. matrix-matrix1, with c_j and f_j using (1 + 1/2j); FCN_CARTESIAN: one
 * solve along x per (y line, frequency), then one along y per (x line, frequency)) and the
 * inverse FFT (Eq. antifourier); the nonlinear half step integrates the electron density along t by
 * RK4 (Eq. ionization) from rho = 0 at t_min and multiplies by exp(dz/2 N) (Eqs. Anhalf,
 * Anhalf1, nonlinearpart).  nsteps >= 0.  field_dev must be 16-byte aligned (the column solve
 * moves a frequency pair p, nt - p as one access: inside a step each row's FP32 spectrum is
 * held with the two columns of a pair adjacent; before and after the call the field is in
 * natural time order).  Errors: FCN_E_STATE before bind; FCN_E_ARG for a NULL or misaligned field.
 * fcn_propagate, fcn_step_timed, fcn_step_timed_launches and fcn_step_scratch take the same
 * field. */
fcn_status fcn_step(fcn_plan_t plan, void *field_dev, int64_t nsteps);

/* Like fcn_step, plus: when diag_dev != NULL and diag_every > 0, writes one diagnostics
 * record (fcn_diag_record_size doubles) of the state A^n for n = 0, diag_every, 2 diag_every,
 * ... <= nsteps into diag_dev (records consecutive; the caller sizes it to
 * (nsteps/diag_every + 1) records).  dz_log_dev: NULL, or a device array of nsteps * batch
 * doubles; in adaptive mode it receives dz_n of instance i at [n * batch + i]; in fixed mode
 * with replay = 1 it supplies them instead (the FP32 run replays the FP64 run's steps). */
fcn_status fcn_propagate(fcn_plan_t plan, void *field_dev, int64_t nsteps, double *diag_dev,
                         int32_t diag_every, double *dz_log_dev, int32_t replay);

/* One diagnostics record of the current state (no step). */
fcn_status fcn_diagnostics(fcn_plan_t plan, const void *field_dev, double *diag_dev);

/* Single stages of the step, for tests of each kernel against the CPU oracle.
 * FCN_STAGE_FFT: forward FFT of every row (unnormalised, exp(-i omega t)).
 * FCN_STAGE_IFFT: inverse FFT of every row, scaled by 1/nt.
 * FCN_STAGE_CN: Crank-Nicholson solve of every frequency column over length `length`
 *   (field in the frequency domain; FCN_CARTESIAN: the x solves, then the y solves).
 * FCN_STAGE_NL: one nonlinear sub-step A <- A exp(length N) (length = dz/2 for a half step). */
enum { FCN_STAGE_FFT = 0, FCN_STAGE_IFFT = 1, FCN_STAGE_CN = 2, FCN_STAGE_NL = 3 };
fcn_status fcn_stage(fcn_plan_t plan, int32_t stage, void *field_dev, double length);

/* Waits for the bound stream; returns FCN_E_UNSTABLE if an RK4 density step left its
 * stability region since the last report, else FCN_E_NONFINITE if the device flagged a
 * non-finite intensity (both flags are then cleared). */
fcn_status fcn_sync(fcn_plan_t plan);

/* Text of the last error on this plan (valid until the next call on it); "" if none. */
const char *fcn_last_error(fcn_plan_t plan);

/* Releases the host-side plan.  Device buffers stay owned by the caller. */
fcn_status fcn_plan_destroy(fcn_plan_t plan);

/* fcn_step with HIP events recorded at the start and end of every pass of the steady steps
 * (by the kernels themselves, so launch gaps are excluded); waits for the stream, then
 * returns the mean duration [ms] of the fused row pass (iFFT, two nonlinear half steps, FFT)
 * and of the column pass (CN solve), and the total elapsed time of the call.  For kernel
 * timing; 2 <= nsteps <= 100000. */
fcn_status fcn_step_timed(fcn_plan_t plan, void *field_dev, int64_t nsteps, double *row_ms, double *col_ms,
                          double *total_ms);

/* Per-launch kernel timing: like fcn_step_timed, and returns the mean duration [ms] of every
 * kernel launch of the steady step body (events recorded by the kernels themselves).  A step is
 * one row-pass launch per distinct nt of the plan (ascending nt), then one column-pass launch per
 * distinct system length (ascending: nr of radial instances, then nx of the x solves, then ny of
 * the y solves of Cartesian instances): *n_launches of them.  launch_ms[l] receives the mean duration of
 * launch l; launch_info[5 l .. 5 l + 4] receive {pass: 0 row, 1 column; its nt or nr; the grid
 * points the launch covers; elements per thread and rows per workgroup (row) or pair slots per
 * workgroup W and rows per thread L (column)}; the pass code is 2 for a Cartesian x solve and 3
 * for a y solve.  max_launches: capacity of the host arrays
 * (launch_ms: max_launches, launch_info: 5 max_launches; FCN_E_SIZE, with *n_launches set,
 * when too small).  Synchronous; 2 <= nsteps <= 10000. */
fcn_status fcn_step_timed_launches(fcn_plan_t plan, void *field_dev, int64_t nsteps, int32_t max_launches,
                                   int32_t *n_launches, double *launch_ms, int64_t *launch_info);

/* Allocation-free variant of fcn_step, for callers that cannot allocate device memory (code
 * that must not call hipMalloc, tight serving loops, harnesses that forbid allocation).
 * Instead of the caller-owned workspace of fcn_plan_bind it uses the library's own static
 * device array of FCN_SCRATCH_BYTES bytes (one per GPU, held until the process ends; its
 * address on the current device is looked up once per device).  The call uploads the plan's
 * tables into that array on `stream` (hipStream_t cast to void*, NULL = default stream, of the
 * current device) and waits for the upload, resets the step state there (step counter 0), then
 * enqueues nsteps Strang steps on field_dev exactly as fcn_step does (same kernels, same
 * results; no HIP graph) and returns without waiting for them.  The plan need not be bound; a
 * bound plan keeps its own workspace, stream, step counter and graph untouched.
 * Every call on one GPU shares that GPU's array and overwrites what the previous call left
 * there: calls that overlap on one GPU (another stream or host thread) race and give wrong
 * results.  A non-finite intensity is not reported (no fcn_sync for this call).
 * Errors: FCN_E_SIZE if the plan needs more than FCN_SCRATCH_BYTES of workspace
 * (fcn_plan_workspace_size); FCN_E_ARG for a NULL field or nsteps < 0; FCN_E_HIP.
 * It calls no hipMalloc, hipFree or other allocating routine. */
#define FCN_SCRATCH_BYTES (4u << 20)
fcn_status fcn_step_scratch(fcn_plan_t plan, void *field_dev, int64_t nsteps, void *stream);

/* Launch configuration the plan chose: frequencies per workgroup and rows per thread of the
 * column solve (of the last nr bucket), elements per thread of the row kernel for the
 * largest nt (8; 16 from nt = 4096, and from nt = 2048 with FP64 row arithmetic:
 * FCN_FP64 and FCN_FP32_STORAGE). */
fcn_status fcn_plan_tiles(fcn_plan_t plan, int32_t *col_tile, int32_t *col_rows, int32_t *row_elems);

/* ------------------------------------------------------------------------------------
 * Learned coarse z-propagator (an addition of this project, not in the paper): a complex
 * convolutional operator on the (r, t) grid, 4 valid 5x5 complex convolutions
 * 1 -> C -> C -> C -> 1 complex channels with complex biases and CReLU (ReLU of the real and
 * the imaginary part) after layers 1-3.  A window of H x W output points reads an 8-point
 * halo of the field.  Used as G(U) = C(U) + s Net(U/s), C one classical FCN step of the
 * window length, as the coarse solver of parareal (with s = in_scale^-1 and an output
 * scale out_scale = kappa s per sample, the network predicts (F - C) / (kappa s)).  Parameters: caller-owned FP32 buffer
 * of fcn_net_param_count floats, per layer W[co][ci][5][5] as (re, im) pairs then b[co] as
 * (re, im); gradients have the same layout and are the pairs (dL/dRe w, dL/dIm w).
 * Activations are stored in BF16 (act_bf16 = 1 or 2) or FP32 (act_bf16 = 0) and accumulated
 * in FP32.  With act_bf16 = 1 the hidden 32 -> 32 complex layers (64 -> 64 real channels) run
 * as BF16 matrix-core products (weights rounded to BF16); act_bf16 = 2 keeps them on FP32
 * vector FMAs with FP32 weights.
 * All network calls are asynchronous on the bound stream except fcn_net_loss. */
typedef struct fcn_net_s *fcn_net_t;

/* One network sample: a window of one instance's complex FP32 field (element offsets into
 * the flat field buffers).  Device arrays of this struct are read by the kernels. */
typedef struct {
    int64_t field_off;   /* input window (fcn_net_input, fcn_net_target: fine field) or the
                            destination (fcn_net_apply) */
    int64_t coarse_off;  /* coarse field C(U) (fcn_net_target, fcn_net_apply) */
    int32_t row0, col0;  /* first r row and t column of the window */
    float in_scale;      /* the network input is the field times in_scale */
    float out_scale;     /* the network output is (fine - coarse) / out_scale */
} fcn_net_sample;

fcn_status fcn_net_create(int32_t channels, int32_t act_bf16, fcn_net_t *out);
fcn_status fcn_net_param_count(fcn_net_t net, size_t *nfloats);
/* Workspace for up to max_batch windows of max_h x max_w outputs; training = 1 keeps every
 * activation and the gradient buffers. */
fcn_status fcn_net_workspace_size(fcn_net_t net, int32_t max_batch, int32_t max_h, int32_t max_w,
                                  int32_t training, size_t *bytes);
/* Binds caller-owned device buffers (params; for training also grads, Adam m and v, each
 * fcn_net_param_count floats) and a 256-byte aligned workspace; expands the weights. */
fcn_status fcn_net_bind(fcn_net_t net, float *params, float *grads, float *adam_m, float *adam_v, void *workspace,
                        size_t workspace_bytes, int32_t max_batch, int32_t max_h, int32_t max_w, int32_t training,
                        void *stream);
/* Re-expands the weights after the caller changed params. */
fcn_status fcn_net_refresh(fcn_net_t net);
/* Network input of `batch` windows (device array `samples`) from complex FP32 fields [nr][nt]:
 * rows row0-8 .. row0+h+7 (row -m reads row m: A is even in r; rows >= nr read 0) and
 * columns col0-8 .. col0+w+7 (periodic in t), times in_scale. */
fcn_status fcn_net_input(fcn_net_t net, const void *fields, const fcn_net_sample *samples, int32_t batch,
                         int32_t nr, int32_t nt, int32_t h, int32_t w);
/* Forward pass of the current input; out (optional) receives FP32 [batch][2][h][w]. */
fcn_status fcn_net_forward(fcn_net_t net, int32_t batch, int32_t h, int32_t w, float *out);
/* Training target (fine - coarse) / out_scale on the windows, FP32 [batch][2][h][w]. */
fcn_status fcn_net_target(fcn_net_t net, const void *fine, const void *coarse, const fcn_net_sample *samples,
                          int32_t batch, int32_t nr, int32_t nt, int32_t h, int32_t w, float *target);
/* Loss of the last forward output: mean over the batch of sum_r w_r |out - target|^2 /
 * sum_r w_r |target|^2, w_r = global r index (1/8 on the axis), rows row0_host[b] + y.
 * Synchronous (waits for the stream); with_grad also stores dloss/dout for fcn_net_backward. */
fcn_status fcn_net_loss(fcn_net_t net, const float *target, const int32_t *row0_host, int32_t batch, int32_t h,
                        int32_t w, int32_t with_grad, double *loss);
/* Parameter gradients of the loss (overwrites grads). */
fcn_status fcn_net_backward(fcn_net_t net, int32_t batch, int32_t h, int32_t w);
/* One Adam update of params from grads (bias-corrected), then re-expansion. */
fcn_status fcn_net_adam(fcn_net_t net, float lr, float beta1, float beta2, float eps);
/* dst = coarse + out_scale * (last full-grid forward output) for each sample's whole field
 * (h = nr, w = nt in the preceding forward); the r_max row is kept 0. */
fcn_status fcn_net_apply(fcn_net_t net, const void *coarse, const fcn_net_sample *samples, int32_t batch, int32_t nr,
                         int32_t nt, void *dst);
const char *fcn_net_last_error(fcn_net_t net);
fcn_status fcn_net_destroy(fcn_net_t net);

/* Parareal correction of one window (complex FP32 fields [nr][nt]):
 * u_new = g_new + f_old - g_old, and FP64 partial sums of the r-weighted |u_new - u_prev|^2
 * and |u_new|^2 in part_dev[2k], part_dev[2k+1] for k < nparts (nparts workgroups). */
fcn_status fcn_parareal_update(const void *g_new, const void *f_old, const void *g_old, const void *u_prev,
                               void *u_new, int32_t nr, int32_t nt, double *part_dev, int32_t nparts, void *stream);

/* Parareal along z for one pulse (not in the paper; an addition of this project).
 * The pulse is cut into `windows` windows of `steps_per_window` FCN steps.  Iteration 0 is the
 * coarse sweep U_{j+1} = G(U_j); iteration k runs the fine steps of every window from U^{k-1}
 * in one batched plan, then the sequential sweep U_{j+1}^k = G(U_j^k) + F(U_j^{k-1}) -
 * G(U_j^{k-1}).  G = one step of the `coarse` plan (its instance is the pulse with dz = the
 * window length), plus the network's correction (fcn_net_apply with `sample_dev[0]`: field_off
 * = coarse_off = 0 and the network's scales) when `net` is not NULL.  The fine FCN judges the
 * iteration: it stops when the r-weighted relative change max_j |U_{j+1}^k - U_{j+1}^{k-1}| /
 * |U_{j+1}^k| falls below tol (converged), when it grows and judge != 0 (diverging; U^{k-1} is
 * kept), or when it is not finite (U^{k-1} is kept).  Without convergence, with fallback != 0
 * and a `fine_serial` plan (one instance, dz of the fine steps), U is replaced by the serial
 * fine solution.
 * Plans: `fine` holds `windows` instances of the pulse back to back; `coarse` and
 * `fine_serial` one; all in an FP32-field mode (FCN_FP32, FCN_FP32_STORAGE or FCN_FP32_CN64:
 * complex64 fields), bound to one stream, as is
 * the network (bound for at least one nr x nt window).  u_dev: [windows + 1][nr][nt]
 * complex64, U_0 in, U_1..U_windows out.  workspace: fcn_parareal_workspace_size bytes,
 * 256-byte aligned, caller-owned.  Synchronous: returns when the result is final.
 * Errors: FCN_E_ARG, FCN_E_SIZE (workspace or plan sizes), FCN_E_STATE (unbound plan),
 * FCN_E_UNSUPPORTED (an FP64 plan), FCN_E_HIP. */
#define FCN_PARAREAL_MAX_ITER 64
enum { FCN_PARAREAL_CONVERGED = 0, FCN_PARAREAL_DIVERGING = 1, FCN_PARAREAL_NONFINITE = 2, FCN_PARAREAL_KMAX = 3,
       FCN_PARAREAL_FALLBACK = 4 };
typedef struct {
    int32_t windows, steps_per_window;
    int32_t kmax;        /* iterations after the coarse sweep, 0..FCN_PARAREAL_MAX_ITER */
    int32_t judge;       /* stop when the change grows */
    int32_t fallback;    /* serial fine solution without convergence (needs fine_serial) */
    int32_t reserved;    /* must be 0 */
    double tol;          /* convergence threshold on the change */
} fcn_parareal_options;
typedef struct {
    int32_t iterations;  /* accepted fine iterations (the state U is that of this iteration) */
    int32_t status;      /* FCN_PARAREAL_* */
    double change[FCN_PARAREAL_MAX_ITER + 1];  /* change of iteration k (k = 0: +inf) */
} fcn_parareal_result;
fcn_status fcn_parareal_workspace_size(int32_t nr, int32_t nt, int32_t windows, size_t *bytes);
fcn_status fcn_parareal(fcn_plan_t fine, fcn_plan_t coarse, fcn_net_t net, const fcn_net_sample *sample_dev,
                        fcn_plan_t fine_serial, int32_t nr, int32_t nt, void *u_dev, void *workspace,
                        size_t workspace_bytes, const fcn_parareal_options *opt, fcn_parareal_result *result);

#ifdef __cplusplus
}
#endif

#endif /* FCN_H */
