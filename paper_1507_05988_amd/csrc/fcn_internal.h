// fcn_internal.h -- device-side plan layout shared by the kernels and the host runtime of
// the FCN library.  Not part of the public ABI (include/fcn.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fcn {

// Scalars at the head of each instance's diagnostics record (FCN_DIAG_SCALARS in fcn.h).
constexpr int DIAG_SCALARS = 8;

// Per-instance constants, computed once on the host in FP64 and uploaded with the plan.
// The operator coefficients are pre-multiplied so a kernel needs no division:
//   s_n     = dz_n * diff_unit          the CN off-diagonal scale dz/(4 k0 dr^2)
//                                       (Cartesian: dz/(4 k0 dx^2); diff_unit_y for y)
//   gamma_p = q_p^2 * dz_n * gvd_unit   the CN GVD term k'' omega_p^2 dz / 4
//                                       (Cartesian: k'' omega_p^2 dz / 8 in each axis solve)
//   Im N    = I (ck1 + I (ck2 + I (ck3 + I ck4))) + c_plasma rho
//   Re N    = c_mpa I^(K-1) + c_coll rho
struct DevInst {
    int32_t nr, nt;         // rows (nx * ny for a Cartesian instance) and time points
    int32_t geom;           // 0: radial; 1: Cartesian, field [ny][nx][nt]
    int32_t nx, ny;         // Cartesian grid (nx = nr, ny = 1 for a radial instance)
    int32_t axis_row;       // row of the on-axis diagnostics (0; Cartesian ((ny-1)/2, (nx-1)/2))
    int64_t field_off;      // complex elements from the start of the field buffer
    int32_t row_base;       // first global row index (row diagnostics partials)
    int32_t diag_off;       // double offset of this instance in a diagnostics record
    int32_t rowcoef_off;    // offset (in rows) of this instance's (1 -+ 1/2m) table
    int32_t tw_off;         // complex offset of the twiddle table for nt
    uint32_t terms;
    int32_t K;
    double dz_fixed;
    double diff_unit;       // 1/(4 k0 dr^2) (Cartesian 1/(4 k0 dx^2)), 0 when diffraction is off
    double diff_unit_y;     // Cartesian 1/(4 k0 dy^2), 0 when diffraction is off
    double e_unit;          // energy per unit of the weighted sum: 2 pi dr^2 dtau, or dx dy dtau
    double gvd_unit;        // k'' (2 pi/(nt dtau))^2 / 4 (Cartesian: / 8), 0 when GVD is off
    double dtau, dr;
    double ck1, ck2, ck3, ck4;  // (k0/n0) n_2j, 0 when Kerr is off
    double c_plasma;        // -k0/(2 rho_c), 0 when the plasma term is off
    double c_mpa;           // -beta_K/2, 0 when MPA is off
    double c_coll;          // -sigma_c/2, 0 when collisional absorption is off
    double sigma_K, rho_at; // density source sigma_K I^K (rho_at - rho)
    double need_rho;        // 1 if the density enters N (plasma or collisional)
    double phi_kerr;        // 1 if the Kerr rate enters Phi
    double phi_plasma;      // k0/(2 rho_c) if the plasma rate enters Phi, else 0
    double need_ik1;        // 1 if I^(K-1) is used (MPA on, or the density scan)
    double c_aval;          // sigma_c / U_i, the avalanche rate per intensity (0 when off)
    // FP32 nonlinear step on the scaled intensity u = I / I_ref, I_ref = (sigma_K dtau)^(-1/K)
    // when the density is on (so sigma_K I^K dtau = u^K), else 1/|ck1| (or 1):
    float f_inv_iref;       // 1 / I_ref
    float fk1, fk2, fk3, fk4;  // ck_j I_ref^j
    float f_mpa;            // c_mpa I_ref^(K-1)
    float f_aval;           // c_aval I_ref dtau: the avalanche rate in units of the scaled intensity
    float f_pad;
};

// Mutable device state, one per lane of a plan (independent instance groups), in the workspace.
struct DevState {
    int64_t cnt_col;        // step index read by the column kernels
    int64_t cnt_row;        // step index read by the row kernels
    int32_t nonfinite;      // set to 1 when a non-finite intensity is seen
    int32_t unstable;       // set to 1 when an RK4 density step leaves [0, 1] (see the row kernel)
    double z_pad[5];
};

// Work item of the row pass: one (instance, row).
struct RowItem {
    int32_t inst;
    int32_t m;
};

// Work item of the column pass: W pair slots [p0, p0+W) of one instance, slot s standing for
// the frequency columns s and nt - s (slots beyond nt/2 are empty); for a Cartesian axis solve
// also the line: the y index of an x solve, the x index of a y solve (0 for radial items).
struct ColItem {
    int32_t inst;
    int32_t p0;
    int32_t line;
    int32_t pad;
};

// Systems of a column-pass launch: radial columns, or the x or y lines of Cartesian instances.
enum : int { COL_RADIAL = 0, COL_X = 1, COL_Y = 2 };

// Row-kernel stage flags (compile-time).
enum : int {
    RK_IFFT_IN = 1,     // input is a spectrum: inverse FFT (with 1/nt) first
    RK_NL_A = 2,        // nonlinear half step with dz_{n-1}
    RK_DIAG = 4,        // diagnostics of the state after RK_NL_A (A^n)
    RK_NL_B = 8,        // nonlinear half step with dz_n
    RK_FFT_OUT = 16,    // forward FFT, write the spectrum.  With RK_NL_A or RK_NL_B (a z-step's
                        // launches) an FP32 spectrum read by RK_IFFT_IN and written by RK_FFT_OUT
                        // is in pair order: entry 2s holds column s and entry 2s + 1 column
                        // nt - s (0 < s < nt/2), entries 0 and 1 columns 0 and nt/2 (the column
                        // pass then moves a frequency pair with one 16-byte access); an FP64
                        // spectrum (16-byte values, already 64 contiguous bytes per 4-column
                        // run) and the stand-alone transform stages use natural order
    RK_STORE = 32,      // write the row back (time domain unless RK_FFT_OUT)
    RK_STAGE_LEN = 64,  // stage test: NL_B uses the explicit length argument as its exponent
    RK_SCAN = 128,      // some instance of the launch has a density term: contiguous-chunk
                        // layout and the density scan (otherwise pointwise, strided layout)
    RK_TW_PAIR = 256,   // FP32 transforms with twiddles carried as hi + lo pairs
    RK_NOABS = 512,     // no instance of the launch has a density or absorption term (MPA,
                        // collisions): the nonlinear step is the Kerr phase rotation alone
    RK_AVAL = 1024,     // with RK_SCAN: some instance has the avalanche rate in its density equation
};

// Step-length source of a row kernel.
enum : int { DZ_FIXED = 0, DZ_ADAPTIVE = 1, DZ_REPLAY = 2 };

// Arguments common to the row-kernel launches.
struct RowArgs {
    const DevInst *inst;
    const RowItem *items;
    int32_t nitems;
    int32_t batch;
    void *field;
    const void *twiddle;      // complex table base (precision of the kernel)
    double *row_diag;         // [global row][4]: sum I, max I, max rho, max Phi
    unsigned long long *phi_slot;  // [2][batch] bit patterns of non-negative doubles
    double *dz_ring;          // [2][batch]
    double *dz_log;           // [n][batch] or null
    DevState *state;
    int32_t dz_mode;
    int32_t log_dz;           // adaptive: write dz_n to dz_log
    int32_t seed_slots;       // also write Phi into the lagged slot (first pass after reset)
    int32_t pad;
    int64_t log_base;         // step index of dz_log[0]
    double max_phase, dz_min, dz_max;
    double stage_len;         // RK_STAGE_LEN
};

struct ColArgs {
    const DevInst *inst;
    const ColItem *items;
    int32_t nitems;
    int32_t batch;
    void *field;
    const double *rowcoef;    // [row][2]: 1 - 1/(2m), 1 + 1/(2m)
    double *dz_ring;
    unsigned long long *phi_slot;
    double *zpos;
    DevState *state;
    int32_t use_stage_len;
    int32_t dir;              // COL_RADIAL, COL_X or COL_Y (the launch's systems)
    int32_t pair_order;       // 1: the spectrum is in pair order (FP32, within a z-step; see RK_FFT_OUT)
    int32_t pad;
    double stage_len;
};

// Launchers (defined in the kernel translation units).
// e0/e1: optional events recorded at the kernel's start and end (nullptr: none).
hipError_t launch_row(int precision, int nt, int elems, int flags, const RowArgs &a, int grid,
                      hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// nr: the length of the launch's systems (nr, nx or ny after a.dir).
hipError_t launch_col(int precision, int w, int l, int nr, const ColArgs &a, int grid, hipStream_t s,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
int row_rows_per_group(int nt, int elems);
// Elements per thread of the row kernel.  16 from nt = 4096: at nt = 8192 a row stays within
// 512 threads and so within the 256-VGPR budget (1024 threads would cap every thread at 128
// VGPRs and spill); at nt = 4096 a 256-thread row lets two rows share a CU where a 512-thread
// one at 163 VGPRs fits alone (436 against 531 us for the 4096-point rows of the batched
// sweep).  With FP64 arithmetic also 16 at nt = 2048 (three radix-16 passes: 39.5 against
// 44.2 us for the full-model row pass); FP32 keeps 8 there (25.8 against 19.4 us with 16).
constexpr int row_elems_for(int nt, bool fp64_arith) { return nt >= 4096 || (fp64_arith && nt >= 2048) ? 16 : 8; }
// Precision codes of include/fcn.h as seen by the two passes: FP64 arithmetic in the row pass
// (FCN_FP64, FCN_FP32_STORAGE) and in the column pass (also FCN_FP32_CN64).
constexpr bool row_fp64_arith(int precision) { return precision == 0 || precision == 2; }
constexpr bool col_fp64_arith(int precision) { return precision != 1; }
hipError_t launch_finalize(const DevInst *inst, int batch, const double *row_diag, const double *zpos,
                           const double *dz_ring, const DevState *state, double *out, hipStream_t s);
hipError_t launch_init_state(DevState *state, int nstates, unsigned long long *phi_slot, double *dz_ring,
                             double *zpos, int batch, int64_t n0, hipStream_t s);
hipError_t launch_clear_flag(DevState *state, int nstates, hipStream_t s);

}  // namespace fcn
