// runtime.cpp -- host side of the FCN library: plan construction, workspace layout, the
// step schedule and the C ABI declared in include/fcn.h.
//
// Step schedule (Sec. 3 summary, re-organised as in Sec. 4): a call advancing nsteps runs
//   row pass  [NL(dz_n0/2), diagnostics of A^n0, FFT]
//   nsteps x ( column pass [CN solve with dz_n]
//              row pass    [iFFT, NL(dz_n/2) -> A^{n+1}, diagnostics, NL(dz_{n+1}/2), FFT] )
// where the last row pass stops after the diagnostics and writes the time-domain field.
// Row passes are launched once per distinct nt (templated FFT), column passes once per
// distinct nr (workgroup size W * ceil(nr/L)); in a batch every launch covers all
// instances of its bucket.  The step index, the dz ring and the phase-rate slots live in
// device memory, so the step body is identical from step to step and can be replayed
// from a captured HIP graph.  With lanes > 1 the instances are split into independent groups
// (greedy balance of the grid points), each with its own buckets and step counters, stepped on
// its own stream between a fork from and a join to the bound stream: one group's column pass
// (latency-bound) can then overlap another group's row pass (arithmetic-bound).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fcn.h"
#include "fcn_internal.h"

using namespace fcn;

namespace {

constexpr double kC = 299792458.0;
constexpr double kHbar = 1.054571817e-34;
constexpr double kMe = 9.1093837015e-31;
constexpr double kQe = 1.602176634e-19;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kPi = 3.14159265358979323846;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Workgroups of a row-kernel launch at most: 1024 (4 per CU of the 256), and 512 from nt = 4096,
// where a workgroup's twiddle table (nt entries, twice with twiddle pairs) is worth staging for
// more rows (the batched sweep's 4096-point rows: 50.8 against 54.1 us per launch; 1024 stays
// faster for the shorter rows, and measured faster than 2048, 4096 and one workgroup per row group).
constexpr int row_groups_for(int nt) { return nt >= 4096 ? 512 : 1024; }

struct RowBucket {
    int lane;
    int nt;
    int scan;  // RK_SCAN when an instance of the bucket has a density term (| RK_AVAL when one
               // also has the avalanche rate), RK_NOABS when none has a density or absorption
               // term, else 0
    int item_off, nitems;
    int grid;
    int64_t points;  // grid points of the launch
};
struct ColBucket {
    int lane;
    int dir;   // COL_RADIAL, COL_X or COL_Y
    int nr;    // system length: nr, nx or ny
    int w, l;
    int item_off, nitems;
    int64_t points;
};

// Rows of an instance as the row pass sees them: nr radii, or nx * ny transverse points.
int rows_of(const fcn_instance &in) { return in.geometry == FCN_CARTESIAN ? in.nr * in.ny : in.nr; }

}  // namespace

struct fcn_plan_s {
    std::vector<fcn_instance> insts;
    fcn_options opt{};
    int batch = 0;
    int precision = 0;
    size_t csize = 16;  // bytes per complex element of the arithmetic (twiddle tables)

    std::vector<DevInst> dinst;
    size_t field_elems = 0;
    size_t diag_doubles = 0;
    int total_rows = 0;
    std::vector<RowItem> row_items;
    std::vector<ColItem> col_items;
    std::vector<RowBucket> row_buckets;
    std::vector<ColBucket> col_buckets;
    std::vector<double> rowcoef;        // [row][2]
    std::vector<unsigned char> twiddles;  // complex tables, precision of the plan
    int col_w = 0, col_l = 0;

    // workspace layout (byte offsets)
    size_t off_inst = 0, off_rowitems = 0, off_colitems = 0, off_rowcoef = 0, off_tw = 0;
    size_t off_rowdiag = 0, off_slots = 0, off_ring = 0, off_zpos = 0, off_state = 0, ws_bytes = 0;
    size_t const_bytes = 0;  // bytes [0, const_bytes) are the uploaded read-only tables
    std::vector<unsigned char> image;

    unsigned char *ws = nullptr;
    hipStream_t stream = nullptr;
    bool bound = false;
    int64_t n_host = 0;     // step index of the field as seen by the host
    bool seeded = false;    // phase-rate slots hold Phi of the current state's predecessor

    int nlanes = 1;                       // independent instance groups
    std::vector<int> lane_of;             // lane of each instance
    std::vector<hipStream_t> lane_streams;  // one per lane when nlanes > 1 (created at bind)
    std::vector<hipEvent_t> lane_events;
    hipEvent_t fork_event = nullptr;
    bool serial = false;                  // run every lane on the bound stream (scratch calls)

    std::vector<hipGraphExec_t> graph_exec;  // per lane (one entry with a single lane)
    int graph_steps = 0;
    void *graph_field = nullptr;

    std::string err;
    std::string tune_cache_path;

    DevInst *d_inst() const { return reinterpret_cast<DevInst *>(ws + off_inst); }
    RowItem *d_rowitems() const { return reinterpret_cast<RowItem *>(ws + off_rowitems); }
    ColItem *d_colitems() const { return reinterpret_cast<ColItem *>(ws + off_colitems); }
    double *d_rowcoef() const { return reinterpret_cast<double *>(ws + off_rowcoef); }
    void *d_tw() const { return ws + off_tw; }
    double *d_rowdiag() const { return reinterpret_cast<double *>(ws + off_rowdiag); }
    unsigned long long *d_slots() const { return reinterpret_cast<unsigned long long *>(ws + off_slots); }
    double *d_ring() const { return reinterpret_cast<double *>(ws + off_ring); }
    double *d_zpos() const { return reinterpret_cast<double *>(ws + off_zpos); }
    DevState *d_state(int lane = 0) const { return reinterpret_cast<DevState *>(ws + off_state) + lane; }
};

namespace {

fcn_status fail(fcn_plan_t p, fcn_status st, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
fcn_status fail(fcn_plan_t p, fcn_status st, const char *fmt, ...) {
    if (p) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        p->err = buf;
    }
    return st;
}

fcn_status hip_fail(fcn_plan_t p, hipError_t e, const char *what) {
    return fail(p, FCN_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

const char *check_instance(const fcn_instance &in) {
    if (in.geometry != FCN_RADIAL && in.geometry != FCN_CARTESIAN) return "unknown geometry";
    if (in.nr < 3 || in.nr > 4096) return "nr (nx) must be in [3, 4096]";
    if (in.geometry == FCN_CARTESIAN) {
        if (in.ny < 3 || in.ny > 4096) return "ny must be in [3, 4096]";
        if ((int64_t)in.nr * in.ny > (int64_t)1 << 22) return "nx * ny must be at most 2^22";
        if (!(in.y_max > 0.0) || !std::isfinite(in.y_max)) return "y_max must be positive";
    }
    if (!is_pow2(in.nt) || in.nt < 64 || in.nt > 8192) return "nt must be a power of two in [64, 8192]";
    if (!(in.r_max > 0.0) || !std::isfinite(in.r_max)) return "r_max must be positive";
    if (!(in.t_max > in.t_min) || !std::isfinite(in.t_max) || !std::isfinite(in.t_min)) return "t_max must exceed t_min";
    if (!(in.lambda0 > 0.0) || !(in.n0 > 0.0)) return "lambda0 and n0 must be positive";
    if (!std::isfinite(in.k2) || !std::isfinite(in.n2) || !std::isfinite(in.n4) || !std::isfinite(in.n6) ||
        !std::isfinite(in.n8))
        return "non-finite dispersion or Kerr coefficient";
    if (in.K < 1 || in.K > 16) return "K must be in [1, 16]";
    if (!(in.sigma_K >= 0.0) || !(in.rho_at >= 0.0) || !(in.sigma_c >= 0.0)) return "negative density coefficient";
    if ((in.terms & ~127u) != 0) return "unknown term bit";
    if ((in.terms & FCN_AVALANCHE) && !(in.U_i > 0.0 && std::isfinite(in.U_i)))
        return "the avalanche term needs a positive ionisation potential U_i";
    if (!(in.dz >= 0.0) || !std::isfinite(in.dz)) return "dz must be finite and non-negative";
    return nullptr;
}

// Twiddles W_nt^k = exp(-2 pi i k / nt), k < nt: cos/sin of the reduced angle in FP64,
// using the octant symmetries so each entry is a correctly reduced evaluation.
void twiddle_table(int nt, std::vector<double> &re, std::vector<double> &im) {
    re.resize(nt);
    im.resize(nt);
    for (int k = 0; k < nt; k++) {
        // angle = 2 pi k / nt in [0, 2 pi): reduce to u = k mod (nt/8) style via exact integers
        const long q8 = (long)k * 8;
        const int oct = (int)(q8 / nt);          // octant 0..7
        const long rem = q8 - (long)oct * nt;    // 0 <= rem < nt
        // theta = (oct + rem/nt) * pi/4
        double c, s;
        const double x = (double)rem / (double)nt * (kPi / 4.0);  // in [0, pi/4)
        const double cx = std::cos(x), sx = std::sin(x);
        const double cy = std::cos(kPi / 4.0 - x), sy = std::sin(kPi / 4.0 - x);
        switch (oct) {
            case 0: c = cx; s = sx; break;
            case 1: c = sy; s = cy; break;
            case 2: c = -sx; s = cx; break;
            case 3: c = -cy; s = sy; break;
            case 4: c = -cx; s = -sx; break;
            case 5: c = -sy; s = -cy; break;
            case 6: c = sx; s = -cx; break;
            default: c = cy; s = -sy; break;
        }
        re[k] = c;
        im[k] = -s;  // exp(-i theta)
    }
}

// FP32 twiddle from FP64 (c, s): among the float pairs within one ulp of each component,
// the one whose modulus is closest to 1 (ties: closest to the FP64 value).  Plain
// rounding leaves |w|^2 - 1 ~ 1e-7 at fixed entries, which makes the forward/inverse
// transform pair scale some components the same way at every step.
void round_unit_f32(double c, double s, float out[2]) {
    const float c0 = (float)c, s0 = (float)s;
    float best_c = c0, best_s = s0;
    double best_m = 1e300, best_d = 1e300;
    for (int i = -1; i <= 1; i++) {
        float cc = c0;
        if (i < 0) cc = std::nextafter(c0, -2.0f);
        if (i > 0) cc = std::nextafter(c0, 2.0f);
        for (int j = -1; j <= 1; j++) {
            float ss = s0;
            if (j < 0) ss = std::nextafter(s0, -2.0f);
            if (j > 0) ss = std::nextafter(s0, 2.0f);
            const double m = std::fabs((double)cc * cc + (double)ss * ss - 1.0);
            const double d = std::fabs((double)cc - c) + std::fabs((double)ss - s);
            if (m < best_m || (m == best_m && d < best_d)) {
                best_m = m;
                best_d = d;
                best_c = cc;
                best_s = ss;
            }
        }
    }
    out[0] = best_c;
    out[1] = best_s;
}

bool col_tiles_supported(int w, int l) {
    return ((w == 1 || w == 2 || w == 4 || w == 8 || w == 16) && (l == 8 || l == 16)) || (w == 32 && l == 8) ||
           ((w == 1 || w == 2 || w == 4 || w == 8) && (l == 4 || l == 6));
}

// Column tile choice: frequencies per workgroup W and rows per thread L.
void choose_col_tiles(int precision, int nr, const fcn_options &opt, int &w, int &l) {
    l = opt.col_rows ? opt.col_rows : (precision == FCN_FP32 ? 16 : 8);
    w = opt.col_tile ? opt.col_tile : 4;
    // keep the workgroup within 512 threads: fewer frequencies per workgroup first (down to 4,
    // which keeps 32-byte row segments), then 16 rows per thread, then 2 and 1 frequencies
    // (tall columns, nr > 2048 with 16 rows or nr > 1024 with 8)
    while (w * ((nr + l - 1) / l) > 512 && w > 4) w /= 2;
    while (w * ((nr + l - 1) / l) > 512 && l < 16 && opt.col_rows == 0 && precision == FCN_FP32) l *= 2;
    while (w * ((nr + l - 1) / l) > 512 && w > 1) w /= 2;
}

const char *precision_name(int precision) {
    switch (precision) {
        case FCN_FP64: return "fp64";
        case FCN_FP32: return "fp32";
        case FCN_FP32_STORAGE: return "fp32_storage";
        default: return "fp32_cn64";
    }
}

// Column tiles per nr from a tune cache file: lines "<precision> col <nr> <W> <L> [us]"
// ('#' starts a comment; other passes and precisions are skipped).  Returns false if the
// file cannot be read or a line of this plan's precision is malformed.
bool read_tune_cache(const char *path, int precision, std::map<int, std::pair<int, int>> &col) {
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool ok = true;
    const std::string prec = precision_name(precision);
    while (std::fgets(line, sizeof line, f)) {
        char *hash = std::strchr(line, '#');
        if (hash) *hash = 0;
        char pname[64] = {0}, pass[16] = {0};
        int size = 0, a = 0, b = 0;
        const int n = std::sscanf(line, "%63s %15s %d %d %d", pname, pass, &size, &a, &b);
        if (n <= 0) continue;  // blank or comment
        if (prec != pname || std::strcmp(pass, "col") != 0) continue;
        if (n < 5 || size < 3 || a < 1 || b < 1) {
            ok = false;
            break;
        }
        col[size] = std::make_pair(a, b);
    }
    std::fclose(f);
    return ok;
}

fcn_status build_plan(fcn_plan_t p) {
    const int B = p->batch;
    const bool row64 = row_fp64_arith(p->precision);
    const bool pair = p->precision == FCN_FP32_CN64;
    p->csize = row64 ? 16 : 8;
    p->dinst.resize(B);

    // twiddle tables per distinct nt (with twiddle pairs: nt high parts, then nt low parts)
    std::map<int, int> tw_off;
    size_t tw_elems = 0;
    for (const auto &in : p->insts)
        if (!tw_off.count(in.nt)) {
            tw_off[in.nt] = (int)tw_elems;
            tw_elems += pair ? 2 * (size_t)in.nt : in.nt;
        }
    p->twiddles.assign(tw_elems * p->csize, 0);
    for (auto &kv : tw_off) {
        std::vector<double> re, im;
        twiddle_table(kv.first, re, im);
        for (int k = 0; k < kv.first; k++) {
            const size_t e = (size_t)kv.second + k;
            if (row64) {
                double v[2] = {re[k], im[k]};
                memcpy(&p->twiddles[e * 16], v, 16);
            } else if (pair) {
                // W = hi + lo to about 2^-48: hi the nearest float pair, lo the rounded rest
                const float hi[2] = {(float)re[k], (float)im[k]};
                const float lo[2] = {(float)(re[k] - (double)hi[0]), (float)(im[k] - (double)hi[1])};
                memcpy(&p->twiddles[e * 8], hi, 8);
                memcpy(&p->twiddles[(e + kv.first) * 8], lo, 8);
            } else {
                float v[2];
                round_unit_f32(re[k], im[k], v);
                memcpy(&p->twiddles[e * 8], v, 8);
            }
        }
    }

    // row-coefficient tables per distinct nr
    std::map<int, int> rc_off;
    int rc_rows = 0;
    for (const auto &in : p->insts)
        if (in.geometry == FCN_RADIAL && !rc_off.count(in.nr)) {
            rc_off[in.nr] = rc_rows;
            rc_rows += in.nr;
        }
    p->rowcoef.assign(2 * (size_t)rc_rows, 0.0);
    for (auto &kv : rc_off)
        for (int m = 1; m < kv.first; m++) {
            p->rowcoef[2 * ((size_t)kv.second + m)] = 1.0 - 1.0 / (2.0 * m);
            p->rowcoef[2 * ((size_t)kv.second + m) + 1] = 1.0 + 1.0 / (2.0 * m);
        }

    // per-instance constants and offsets
    size_t off = 0;
    int row = 0;
    size_t doff = 0;
    for (int i = 0; i < B; i++) {
        const fcn_instance &in = p->insts[i];
        const bool cart = in.geometry == FCN_CARTESIAN;
        const int rows = rows_of(in);
        DevInst d{};
        d.nr = rows;
        d.nt = in.nt;
        d.geom = cart ? 1 : 0;
        d.nx = in.nr;
        d.ny = cart ? in.ny : 1;
        d.axis_row = cart ? (in.ny - 1) / 2 * in.nr + (in.nr - 1) / 2 : 0;
        d.field_off = (int64_t)off;
        d.row_base = row;
        d.diag_off = (int)doff;
        d.rowcoef_off = cart ? 0 : rc_off[in.nr];
        d.tw_off = tw_off[in.nt];
        d.terms = in.terms;
        d.K = in.K;
        d.dz_fixed = in.dz;
        const double k0 = 2.0 * kPi * in.n0 / in.lambda0;
        const double w0 = 2.0 * kPi * kC / in.lambda0;
        const double rho_c = kEps0 * kMe * w0 * w0 / (kQe * kQe);
        const double beta = (double)in.K * kHbar * w0 * in.sigma_K * in.rho_at;
        // radial: dr = r_max/(nr-1); Cartesian: dx = 2 x_max/(nx-1), dy = 2 y_max/(ny-1)
        d.dr = (cart ? 2.0 : 1.0) * in.r_max / (double)(in.nr - 1);
        const double dy = cart ? 2.0 * in.y_max / (double)(in.ny - 1) : 0.0;
        d.dtau = (in.t_max - in.t_min) / (double)in.nt;
        const bool diff = (in.terms & FCN_DIFFRACTION) != 0;
        d.diff_unit = diff ? 1.0 / (4.0 * k0 * d.dr * d.dr) : 0.0;
        d.diff_unit_y = diff && cart ? 1.0 / (4.0 * k0 * dy * dy) : 0.0;
        d.e_unit = cart ? d.dr * dy * d.dtau : 2.0 * kPi * d.dr * d.dr * d.dtau;
        const double wu = 2.0 * kPi / ((double)in.nt * d.dtau);
        // the Cartesian step splits the GVD term evenly between its x and y solves
        d.gvd_unit = (in.terms & FCN_GVD) ? in.k2 * wu * wu / (cart ? 8.0 : 4.0) : 0.0;
        const bool kerr = (in.terms & FCN_KERR) != 0;
        d.ck1 = kerr ? k0 / in.n0 * in.n2 : 0.0;
        d.ck2 = kerr ? k0 / in.n0 * in.n4 : 0.0;
        d.ck3 = kerr ? k0 / in.n0 * in.n6 : 0.0;
        d.ck4 = kerr ? k0 / in.n0 * in.n8 : 0.0;
        d.c_plasma = (in.terms & FCN_PLASMA) ? -k0 / (2.0 * rho_c) : 0.0;
        d.c_mpa = (in.terms & FCN_MPA) ? -beta / 2.0 : 0.0;
        d.c_coll = (in.terms & FCN_COLL) ? -in.sigma_c / 2.0 : 0.0;
        d.sigma_K = in.sigma_K;
        d.rho_at = in.rho_at;
        d.need_rho = ((in.terms & (FCN_PLASMA | FCN_COLL)) != 0 && in.rho_at > 0.0 && in.sigma_K > 0.0) ? 1.0 : 0.0;
        d.phi_kerr = kerr ? 1.0 : 0.0;
        d.phi_plasma = (in.terms & FCN_PLASMA) ? k0 / (2.0 * rho_c) : 0.0;
        d.need_ik1 = (d.need_rho != 0.0 || d.c_mpa != 0.0) ? 1.0 : 0.0;
        d.c_aval = (in.terms & FCN_AVALANCHE) ? in.sigma_c / in.U_i : 0.0;
        double iref = 1.0;
        if (d.need_rho != 0.0)
            iref = std::pow(in.sigma_K * d.dtau, -1.0 / (double)in.K);
        else if (d.ck1 != 0.0)
            iref = 1.0 / std::fabs(d.ck1);
        else if (d.c_mpa != 0.0)
            iref = std::pow(std::fabs(d.c_mpa), -1.0 / (double)std::max(in.K - 1, 1));
        d.f_inv_iref = (float)(1.0 / iref);
        d.fk1 = (float)(d.ck1 * iref);
        d.fk2 = (float)(d.ck2 * iref * iref);
        d.fk3 = (float)(d.ck3 * iref * iref * iref);
        d.fk4 = (float)(d.ck4 * iref * iref * iref * iref);
        d.f_mpa = (float)(d.c_mpa * std::pow(iref, (double)(in.K - 1)));
        d.f_aval = (float)(d.c_aval * iref * d.dtau);
        p->dinst[i] = d;
        off += (size_t)rows * in.nt;
        row += rows;
        doff += DIAG_SCALARS + rows;
    }
    p->field_elems = off;
    p->total_rows = row;
    p->diag_doubles = doff;

    // lanes: greedy balance of the grid points (largest instances first)
    p->nlanes = std::max(1, std::min(p->opt.lanes, B));
    p->lane_of.assign(B, 0);
    {
        std::vector<int> order(B);
        for (int i = 0; i < B; i++) order[i] = i;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return (int64_t)rows_of(p->insts[a]) * p->insts[a].nt > (int64_t)rows_of(p->insts[b]) * p->insts[b].nt;
        });
        std::vector<int64_t> load(p->nlanes, 0);
        for (int i : order) {
            const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            p->lane_of[i] = l;
            load[l] += (int64_t)rows_of(p->insts[i]) * p->insts[i].nt;
        }
    }

    // row work lists, one bucket per (lane, nt)
    std::map<std::pair<int, int>, std::vector<int>> by_nt;
    for (int i = 0; i < B; i++) by_nt[{p->lane_of[i], p->insts[i].nt}].push_back(i);
    for (auto &kv : by_nt) {
        RowBucket b{};
        b.lane = kv.first.first;
        b.nt = kv.first.second;
        b.item_off = (int)p->row_items.size();
        b.points = 0;
        for (int i : kv.second) {
            for (int m = 0; m < rows_of(p->insts[i]); m++) p->row_items.push_back(RowItem{i, m});
            b.points += (int64_t)rows_of(p->insts[i]) * p->insts[i].nt;
        }
        b.nitems = (int)p->row_items.size() - b.item_off;
        // the density scan if any instance has a density term; otherwise the phase-only step
        // if no instance has an absorption term either
        b.scan = RK_NOABS;
        for (int i : kv.second) {
            if (p->dinst[i].need_rho != 0.0) b.scan |= RK_SCAN;
            if (p->dinst[i].need_rho != 0.0 && p->dinst[i].c_aval != 0.0) b.scan |= RK_AVAL;
            if (p->dinst[i].c_mpa != 0.0 || p->dinst[i].c_coll != 0.0 || p->dinst[i].need_rho != 0.0)
                b.scan &= ~RK_NOABS;
        }
        // the row kernel steps through row groups (blockIdx.x, + gridDim.x, ...), so a workgroup
        // stages its twiddle table once for several rows: at most row_groups_for(nt) workgroups
        const int rpw = row_rows_per_group(b.nt, row_elems_for(b.nt, row_fp64_arith(p->precision)));
        b.grid = std::min((b.nitems + rpw - 1) / rpw, row_groups_for(b.nt));
        p->row_buckets.push_back(b);
    }
    // column work lists, one bucket per nr; tiles from the options, else the tune cache, else
    // the default rule
    std::map<int, std::pair<int, int>> cached;
    if (p->opt.tune_cache && !read_tune_cache(p->opt.tune_cache, p->precision, cached))
        return fail(p, FCN_E_ARG, "tune cache %s unreadable or malformed", p->opt.tune_cache);
    // buckets keyed (lane, direction, system length): within a lane the radial solves, then the
    // Cartesian x solves, then the y solves, which need the x solves' output
    std::map<std::tuple<int, int, int>, std::vector<int>> by_nr;
    for (int i = 0; i < B; i++) {
        const fcn_instance &in = p->insts[i];
        if (in.geometry == FCN_CARTESIAN) {
            by_nr[{p->lane_of[i], (int)COL_X, in.nr}].push_back(i);
            by_nr[{p->lane_of[i], (int)COL_Y, in.ny}].push_back(i);
        } else {
            by_nr[{p->lane_of[i], (int)COL_RADIAL, in.nr}].push_back(i);
        }
    }
    for (auto &kv : by_nr) {
        ColBucket b{};
        b.lane = std::get<0>(kv.first);
        b.dir = std::get<1>(kv.first);
        b.nr = std::get<2>(kv.first);
        fcn_options o = p->opt;
        const auto hit = cached.find(b.nr);
        if (hit != cached.end()) {
            if (o.col_tile == 0) o.col_tile = hit->second.first;
            if (o.col_rows == 0) o.col_rows = hit->second.second;
        }
        choose_col_tiles(p->precision, b.nr, o, b.w, b.l);
        if (b.w * ((b.nr + b.l - 1) / b.l) > 512) return fail(p, FCN_E_SIZE, "nr=%d too large for the column solve", b.nr);
        if (!col_tiles_supported(b.w, b.l)) return fail(p, FCN_E_ARG, "column tile %dx%d not built", b.w, b.l);
        b.item_off = (int)p->col_items.size();
        // pair slots s = 0 .. nt/2 (columns s and nt - s share their matrices), W per workgroup;
        // Cartesian: for every line of the other axis (y lines for the x solves, x for the y)
        b.points = 0;
        for (int i : kv.second) {
            const fcn_instance &in = p->insts[i];
            const int lines = b.dir == COL_X ? in.ny : (b.dir == COL_Y ? in.nr : 1);
            for (int line = 0; line < lines; line++)
                for (int s0 = 0; s0 <= in.nt / 2; s0 += b.w) p->col_items.push_back(ColItem{i, s0, line, 0});
            b.points += (int64_t)rows_of(in) * in.nt;
        }
        b.nitems = (int)p->col_items.size() - b.item_off;
        p->col_buckets.push_back(b);
        p->col_w = b.w;
        p->col_l = b.l;
    }

    // workspace layout
    size_t o = 0;
    p->off_inst = o;
    o = align_up(o + sizeof(DevInst) * B, 256);
    p->off_rowitems = o;
    o = align_up(o + sizeof(RowItem) * p->row_items.size(), 256);
    p->off_colitems = o;
    o = align_up(o + sizeof(ColItem) * p->col_items.size(), 256);
    p->off_rowcoef = o;
    o = align_up(o + sizeof(double) * p->rowcoef.size(), 256);
    p->off_tw = o;
    o = align_up(o + p->twiddles.size(), 256);
    p->const_bytes = o;
    p->off_rowdiag = o;
    o = align_up(o + sizeof(double) * 4 * (size_t)p->total_rows, 256);
    p->off_slots = o;
    o = align_up(o + sizeof(unsigned long long) * 2 * B, 256);
    p->off_ring = o;
    o = align_up(o + sizeof(double) * 2 * B, 256);
    p->off_zpos = o;
    o = align_up(o + sizeof(double) * B, 256);
    p->off_state = o;
    o = align_up(o + sizeof(DevState) * (size_t)p->nlanes, 256);
    p->ws_bytes = o;

    p->image.assign(p->const_bytes, 0);
    memcpy(&p->image[p->off_inst], p->dinst.data(), sizeof(DevInst) * B);
    memcpy(&p->image[p->off_rowitems], p->row_items.data(), sizeof(RowItem) * p->row_items.size());
    memcpy(&p->image[p->off_colitems], p->col_items.data(), sizeof(ColItem) * p->col_items.size());
    memcpy(&p->image[p->off_rowcoef], p->rowcoef.data(), sizeof(double) * p->rowcoef.size());
    memcpy(&p->image[p->off_tw], p->twiddles.data(), p->twiddles.size());
    return FCN_OK;
}

RowArgs row_args(fcn_plan_t p, void *field, const RowBucket &b) {
    RowArgs a{};
    a.inst = p->d_inst();
    a.items = p->d_rowitems() + b.item_off;
    a.nitems = b.nitems;
    a.batch = p->batch;
    a.field = field;
    a.twiddle = p->d_tw();
    a.row_diag = p->d_rowdiag();
    a.phi_slot = p->d_slots();
    a.dz_ring = p->d_ring();
    a.dz_log = nullptr;
    a.dz_mode = p->opt.adaptive ? DZ_ADAPTIVE : DZ_FIXED;
    a.state = p->d_state(b.lane);
    a.max_phase = p->opt.max_phase;
    a.dz_min = p->opt.dz_min;
    a.dz_max = p->opt.dz_max;
    return a;
}

ColArgs col_args(fcn_plan_t p, void *field, const ColBucket &b) {
    ColArgs a{};
    a.inst = p->d_inst();
    a.items = p->d_colitems() + b.item_off;
    a.nitems = b.nitems;
    a.batch = p->batch;
    a.field = field;
    a.rowcoef = p->d_rowcoef();
    a.dz_ring = p->d_ring();
    a.phi_slot = p->d_slots();
    a.zpos = p->d_zpos();
    a.state = p->d_state(b.lane);
    return a;
}

struct StepCtx {
    double *dz_log = nullptr;
    int64_t log_base = 0;
    int replay = 0;
};

// e0 / e1: optional events recorded at the start of the pass's first kernel and the end of
// its last kernel.
// Stream of a lane (lane < 0: every bucket, on the bound stream).
hipStream_t lane_stream(fcn_plan_t p, int lane) { return lane < 0 ? p->stream : p->lane_streams[lane]; }

// lev: optional events, two per launch (start, end), recorded by each launch itself.
// lane >= 0: only that lane's buckets, on its stream; lane < 0: all buckets on the bound stream.
hipError_t row_pass(fcn_plan_t p, void *field, int flags, const StepCtx &ctx, int seed, double stage_len = 0.0,
                    hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr, const hipEvent_t *lev = nullptr,
                    int lane = -1) {
    const size_t nb = p->row_buckets.size();
    for (size_t bi = 0; bi < nb; bi++) {
        const auto &b = p->row_buckets[bi];
        if (lane >= 0 && b.lane != lane) continue;
        RowArgs a = row_args(p, field, b);
        a.dz_log = ctx.dz_log;
        a.log_base = ctx.log_base;
        if (ctx.replay && !p->opt.adaptive) a.dz_mode = DZ_REPLAY;
        a.seed_slots = seed;
        a.stage_len = stage_len;
        const bool nl = (flags & (RK_NL_A | RK_NL_B | RK_DIAG)) != 0;
        hipError_t e = launch_row(p->precision, b.nt, row_elems_for(b.nt, row_fp64_arith(p->precision)),
                                  nl ? (flags | b.scan) : flags, a, b.grid, lane_stream(p, lane),
                                  lev ? lev[2 * bi] : (bi == 0 ? e0 : nullptr),
                                  lev ? lev[2 * bi + 1] : (bi + 1 == nb ? e1 : nullptr));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t col_pass(fcn_plan_t p, void *field, int stage, double stage_len = 0.0, hipEvent_t e0 = nullptr,
                    hipEvent_t e1 = nullptr, const hipEvent_t *lev = nullptr, int lane = -1) {
    const size_t nb = p->col_buckets.size();
    for (size_t bi = 0; bi < nb; bi++) {
        const auto &b = p->col_buckets[bi];
        if (lane >= 0 && b.lane != lane) continue;
        ColArgs a = col_args(p, field, b);
        a.dir = b.dir;
        a.use_stage_len = stage;
        // a z-step's FP32 spectrum is in pair order; an FP64 one and the CN stage's natural
        a.pair_order = stage == 0 && p->precision != FCN_FP64 ? 1 : 0;
        a.stage_len = stage_len;
        hipError_t e = launch_col(p->precision, b.w, b.l, b.nr, a, b.nitems, lane_stream(p, lane),
                                  lev ? lev[2 * bi] : (bi == 0 ? e0 : nullptr),
                                  lev ? lev[2 * bi + 1] : (bi + 1 == nb ? e1 : nullptr));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

constexpr int F_FIRST = RK_NL_B | RK_DIAG | RK_FFT_OUT | RK_STORE;
constexpr int F_MIDDLE = RK_IFFT_IN | RK_NL_A | RK_DIAG | RK_NL_B | RK_FFT_OUT | RK_STORE;
constexpr int F_LAST = RK_IFFT_IN | RK_NL_A | RK_DIAG | RK_STORE;
constexpr int F_DIAG = RK_DIAG;

hipError_t finalize(fcn_plan_t p, double *out) {
    return launch_finalize(p->d_inst(), p->batch, p->d_rowdiag(), p->d_zpos(), p->d_ring(), p->d_state(0), out,
                           p->stream);
}

void destroy_graphs(fcn_plan_t p) {
    for (auto &g : p->graph_exec)
        if (g) (void)hipGraphExecDestroy(g);
    p->graph_exec.clear();
    p->graph_steps = 0;
    p->graph_field = nullptr;
}

// Captures `steps` step bodies (column pass + middle row pass) of one lane (lane < 0: all
// buckets on the bound stream) into an executable graph.
fcn_status ensure_graph(fcn_plan_t p, void *field, int steps, int lane) {
    const size_t slot = (size_t)(lane + 1);  // slot 0: every bucket on the bound stream
    if (p->graph_exec.size() <= slot) p->graph_exec.resize(slot + 1, nullptr);
    if (p->graph_exec[slot] && p->graph_steps == steps) return FCN_OK;
    if (p->graph_exec[slot]) {
        (void)hipGraphExecDestroy(p->graph_exec[slot]);
        p->graph_exec[slot] = nullptr;
    }
    const hipStream_t s = lane_stream(p, lane);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(p, e, "hipStreamBeginCapture");
    StepCtx ctx;
    for (int k = 0; k < steps && e == hipSuccess; k++) {
        e = col_pass(p, field, 0, 0.0, nullptr, nullptr, nullptr, lane);
        if (e == hipSuccess) e = row_pass(p, field, F_MIDDLE, ctx, 0, 0.0, nullptr, nullptr, nullptr, lane);
    }
    hipError_t e2 = hipStreamEndCapture(s, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(p, e, "kernel launch during capture");
    }
    if (e2 != hipSuccess) return hip_fail(p, e2, "hipStreamEndCapture");
    e = hipGraphInstantiate(&p->graph_exec[slot], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(p, e, "hipGraphInstantiate");
    p->graph_steps = steps;
    p->graph_field = field;
    return FCN_OK;
}

// The step sequence of one lane (lane < 0: every bucket on the bound stream, with the optional
// diagnostics records): first row pass, nsteps - 1 fused steps (graph chunks when allowed), last
// row pass.  Does not advance the host step index.
fcn_status run_sequence(fcn_plan_t p, void *field, int64_t nsteps, double *diag, int diag_every,
                        const StepCtx &ctx, bool graph_ok, int lane) {
    const bool want_diag = diag != nullptr && diag_every > 0;
    int64_t rec = 0;
    hipError_t e = row_pass(p, field, F_FIRST, ctx, 0, 0.0, nullptr, nullptr, nullptr, lane);
    if (e != hipSuccess) return hip_fail(p, e, "row pass");
    if (want_diag) {
        e = finalize(p, diag + (rec++) * p->diag_doubles);
        if (e != hipSuccess) return hip_fail(p, e, "finalize");
    }
    const hipStream_t s = lane_stream(p, lane);
    int64_t k = 0;
    // middle steps: k = 0 .. nsteps-2 end with a middle row pass (state A^{n0+k+1})
    while (k < nsteps - 1) {
        if (graph_ok) {
            const int gs = 16;
            if (nsteps - 1 - k >= gs) {
                fcn_status st = ensure_graph(p, field, gs, lane);
                if (st != FCN_OK) return st;
                e = hipGraphLaunch(p->graph_exec[(size_t)(lane + 1)], s);
                if (e != hipSuccess) return hip_fail(p, e, "hipGraphLaunch");
                k += gs;
                continue;
            }
        }
        e = col_pass(p, field, 0, 0.0, nullptr, nullptr, nullptr, lane);
        if (e == hipSuccess) e = row_pass(p, field, F_MIDDLE, ctx, 0, 0.0, nullptr, nullptr, nullptr, lane);
        if (e != hipSuccess) return hip_fail(p, e, "step");
        k += 1;
        if (want_diag && k % diag_every == 0) {
            e = finalize(p, diag + (rec++) * p->diag_doubles);
            if (e != hipSuccess) return hip_fail(p, e, "finalize");
        }
    }
    e = col_pass(p, field, 0, 0.0, nullptr, nullptr, nullptr, lane);
    if (e == hipSuccess) e = row_pass(p, field, F_LAST, ctx, 0, 0.0, nullptr, nullptr, nullptr, lane);
    if (e != hipSuccess) return hip_fail(p, e, "last step");
    if (want_diag && nsteps % diag_every == 0) {
        e = finalize(p, diag + (rec++) * p->diag_doubles);
        if (e != hipSuccess) return hip_fail(p, e, "finalize");
    }
    return FCN_OK;
}

// The column pass moves a frequency pair of the pair-order spectrum with 16-byte accesses.
bool field_aligned(const void *field) { return ((uintptr_t)field & 15) == 0; }

fcn_status run_steps(fcn_plan_t p, void *field, int64_t nsteps, double *diag, int diag_every, double *dz_log,
                     int replay) {
    if (!p->bound) return fail(p, FCN_E_STATE, "plan is not bound to a workspace");
    if (!field) return fail(p, FCN_E_ARG, "field is NULL");
    if (!field_aligned(field)) return fail(p, FCN_E_ARG, "field is not 16-byte aligned");
    if (nsteps < 0) return fail(p, FCN_E_ARG, "nsteps < 0");
    if (replay && (!dz_log || p->opt.adaptive)) return fail(p, FCN_E_ARG, "replay needs a dz log and fixed mode");
    if (nsteps == 0 && !diag) return FCN_OK;
    StepCtx ctx{dz_log, p->n_host, replay};
    const bool want_diag = diag != nullptr && diag_every > 0;
    hipError_t e = hipSuccess;
    // Adaptive mode: Phi of the state before the first step seeds both slots (dz_0 from A^0).
    if (p->opt.adaptive && !p->seeded) {
        e = row_pass(p, field, F_DIAG, ctx, 1);
        if (e != hipSuccess) return hip_fail(p, e, "diagnostics pass");
        p->seeded = true;
    }
    if (nsteps == 0) {
        e = row_pass(p, field, F_DIAG, ctx, 0);
        if (e == hipSuccess && want_diag) e = finalize(p, diag);
        return e == hipSuccess ? FCN_OK : hip_fail(p, e, "diagnostics");
    }
    // Lanes run concurrently only without diagnostics records or a dz log (both need every
    // instance at the same step between launches) and outside allocation-free calls.
    const bool lanes = p->nlanes > 1 && !p->serial && !want_diag && dz_log == nullptr &&
                       (int)p->lane_streams.size() == p->nlanes;
    // graphs need a capturable (non-default) stream; they hold the field pointer and their
    // kernels' arguments, so calls with a dz log (adaptive logging or replay) run eagerly
    const bool graph_ok = p->opt.use_graph && !p->serial && !want_diag && dz_log == nullptr &&
                          (lanes || p->stream != nullptr);
    if (graph_ok && p->graph_field != nullptr && p->graph_field != field) destroy_graphs(p);
    fcn_status st = FCN_OK;
    if (!lanes) {
        st = run_sequence(p, field, nsteps, diag, diag_every, ctx, graph_ok, -1);
    } else {
        e = hipEventRecord(p->fork_event, p->stream);
        for (int l = 0; l < p->nlanes && e == hipSuccess; l++) e = hipStreamWaitEvent(p->lane_streams[l], p->fork_event, 0);
        if (e != hipSuccess) return hip_fail(p, e, "fork to the lane streams");
        for (int l = 0; l < p->nlanes && st == FCN_OK; l++)
            st = run_sequence(p, field, nsteps, nullptr, 0, ctx, graph_ok, l);
        // join even after a failed launch, so the bound stream never runs ahead of the lanes
        for (int l = 0; l < p->nlanes && e == hipSuccess; l++) {
            e = hipEventRecord(p->lane_events[l], p->lane_streams[l]);
            if (e == hipSuccess) e = hipStreamWaitEvent(p->stream, p->lane_events[l], 0);
        }
        if (st == FCN_OK && e != hipSuccess) st = hip_fail(p, e, "join of the lane streams");
    }
    if (st == FCN_OK) p->n_host += nsteps;
    return st;
}

}  // namespace

namespace {

// Device memory of fcn_step_scratch: one array per GPU, living until the process ends.  In
// host code `scratch` is only a host-side handle of the symbol; its device address is looked
// up per device with hipGetSymbolAddress and only that address is ever passed to kernels or
// copies.
static __device__ __align__(256) unsigned char scratch[FCN_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// Address of the static scratch on the current device, looked up once per device.
fcn_status scratch_on_current_device(fcn_plan_t p, unsigned char **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(p, e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(p, FCN_E_HIP, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(p, e, "hipGetSymbolAddress(scratch)");
        if (!ptr || ((uintptr_t)ptr & 255) != 0) return fail(p, FCN_E_HIP, "static scratch is not 256-byte aligned");
        g_scratch_ptr[dev] = static_cast<unsigned char *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return FCN_OK;
}

}  // namespace

namespace fcn {
// accessors for the library's other translation units (parareal driver)
int plan_precision(fcn_plan_t p) { return p->precision; }
hipStream_t plan_stream(fcn_plan_t p) { return p->stream; }
bool plan_bound(fcn_plan_t p) { return p->bound; }
}  // namespace fcn

extern "C" {

fcn_status fcn_plan_create(const fcn_instance *inst, int32_t batch, const fcn_options *opt, fcn_plan_t *out) {
    if (!out) return FCN_E_ARG;
    *out = nullptr;
    if (!inst || batch < 1) return FCN_E_ARG;
    fcn_plan_t p = new fcn_plan_s();
    p->batch = batch;
    p->insts.assign(inst, inst + batch);
    if (opt) p->opt = *opt;
    if (p->opt.tune_cache) {  // the plan keeps its own copy of the path
        p->tune_cache_path = p->opt.tune_cache;
        p->opt.tune_cache = p->tune_cache_path.c_str();
    }
    p->precision = p->opt.precision;
    if (p->precision != FCN_FP64 && p->precision != FCN_FP32 && p->precision != FCN_FP32_STORAGE &&
        p->precision != FCN_FP32_CN64) {
        delete p;
        return FCN_E_ARG;
    }
    if (p->opt.adaptive) {
        if (!(p->opt.max_phase > 0.0) || !(p->opt.dz_min > 0.0) || !(p->opt.dz_max >= p->opt.dz_min)) {
            delete p;
            return FCN_E_ARG;
        }
    }
    if (p->opt.col_tile && p->opt.col_tile != 1 && p->opt.col_tile != 2 && p->opt.col_tile != 4 &&
        p->opt.col_tile != 8 && p->opt.col_tile != 16 && p->opt.col_tile != 32) {
        delete p;
        return FCN_E_ARG;
    }
    if (p->opt.col_rows && p->opt.col_rows != 4 && p->opt.col_rows != 6 && p->opt.col_rows != 8 &&
        p->opt.col_rows != 16) {
        delete p;
        return FCN_E_ARG;
    }
    if (p->opt.lanes < 0 || p->opt.lanes > 8) {
        delete p;
        return FCN_E_ARG;
    }
    for (int i = 0; i < batch; i++) {
        const char *why = check_instance(inst[i]);
        if (why) {
            delete p;
            const bool big = inst[i].nr > 4096 || inst[i].nt > 8192 ||
                             (inst[i].geometry == FCN_CARTESIAN &&
                              (inst[i].ny > 4096 || (int64_t)inst[i].nr * inst[i].ny > (int64_t)1 << 22));
            return big ? FCN_E_SIZE : FCN_E_ARG;
        }
        if (!p->opt.adaptive && !(inst[i].dz > 0.0)) {
            delete p;
            return FCN_E_ARG;
        }
    }
    fcn_status st = build_plan(p);
    if (st != FCN_OK) {
        delete p;
        return st;
    }
    *out = p;
    return FCN_OK;
}

fcn_status fcn_plan_workspace_size(fcn_plan_t p, size_t *bytes) {
    if (!p || !bytes) return FCN_E_ARG;
    *bytes = p->ws_bytes;
    return FCN_OK;
}

fcn_status fcn_field_size(fcn_plan_t p, size_t *elems) {
    if (!p || !elems) return FCN_E_ARG;
    *elems = p->field_elems;
    return FCN_OK;
}

fcn_status fcn_field_offset(fcn_plan_t p, int32_t instance, size_t *elem_offset) {
    if (!p || !elem_offset) return FCN_E_ARG;
    if (instance < 0 || instance >= p->batch) return fail(p, FCN_E_ARG, "instance %d out of range", instance);
    *elem_offset = (size_t)p->dinst[instance].field_off;
    return FCN_OK;
}

fcn_status fcn_diag_record_size(fcn_plan_t p, size_t *doubles) {
    if (!p || !doubles) return FCN_E_ARG;
    *doubles = p->diag_doubles;
    return FCN_OK;
}

fcn_status fcn_plan_tiles(fcn_plan_t p, int32_t *col_tile, int32_t *col_rows, int32_t *row_elems) {
    if (!p) return FCN_E_ARG;
    if (col_tile) *col_tile = p->col_w;
    if (col_rows) *col_rows = p->col_l;
    if (row_elems) {
        int nt_max = 0;
        for (const auto &in : p->insts) nt_max = std::max(nt_max, (int)in.nt);
        *row_elems = row_elems_for(nt_max, row_fp64_arith(p->precision));
    }
    return FCN_OK;
}

fcn_status fcn_plan_bind(fcn_plan_t p, void *workspace_dev, size_t workspace_bytes, void *stream) {
    if (!p) return FCN_E_ARG;
    p->err.clear();
    if (!workspace_dev) return fail(p, FCN_E_ARG, "workspace is NULL");
    if (((uintptr_t)workspace_dev & 255) != 0) return fail(p, FCN_E_ARG, "workspace must be 256-byte aligned");
    if (workspace_bytes < p->ws_bytes)
        return fail(p, FCN_E_SIZE, "workspace has %zu bytes, plan needs %zu", workspace_bytes, p->ws_bytes);
    destroy_graphs(p);
    p->ws = static_cast<unsigned char *>(workspace_dev);
    p->stream = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(p->ws, p->image.data(), p->const_bytes, hipMemcpyHostToDevice, p->stream);
    if (e != hipSuccess) return hip_fail(p, e, "upload plan tables");
    e = launch_init_state(p->d_state(0), p->nlanes, p->d_slots(), p->d_ring(), p->d_zpos(), p->batch, 0, p->stream);
    if (e != hipSuccess) return hip_fail(p, e, "init state");
    // helper streams of the lanes (default priority; kept across binds, released by destroy)
    if (p->nlanes > 1 && p->lane_streams.empty()) {
        e = hipEventCreateWithFlags(&p->fork_event, hipEventDisableTiming);
        for (int l = 0; l < p->nlanes && e == hipSuccess; l++) {
            hipStream_t ls = nullptr;
            hipEvent_t le = nullptr;
            e = hipStreamCreateWithFlags(&ls, hipStreamNonBlocking);
            if (e == hipSuccess) p->lane_streams.push_back(ls);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&le, hipEventDisableTiming);
            if (e == hipSuccess) p->lane_events.push_back(le);
        }
        if (e != hipSuccess) return hip_fail(p, e, "lane streams");
    }
    // the host image must stay alive until the copy has run
    e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(p, e, "hipStreamSynchronize");
    p->bound = true;
    p->n_host = 0;
    p->seeded = false;
    return FCN_OK;
}

fcn_status fcn_step(fcn_plan_t p, void *field_dev, int64_t nsteps) {
    if (!p) return FCN_E_ARG;
    p->err.clear();
    return run_steps(p, field_dev, nsteps, nullptr, 0, nullptr, 0);
}

fcn_status fcn_propagate(fcn_plan_t p, void *field_dev, int64_t nsteps, double *diag_dev, int32_t diag_every,
                         double *dz_log_dev, int32_t replay) {
    if (!p) return FCN_E_ARG;
    p->err.clear();
    if (diag_dev && diag_every <= 0) return fail(p, FCN_E_ARG, "diag_every must be positive with a diag buffer");
    return run_steps(p, field_dev, nsteps, diag_dev, diag_every, dz_log_dev, replay);
}

fcn_status fcn_diagnostics(fcn_plan_t p, const void *field_dev, double *diag_dev) {
    if (!p) return FCN_E_ARG;
    p->err.clear();
    if (!p->bound) return fail(p, FCN_E_STATE, "plan is not bound to a workspace");
    if (!field_dev || !diag_dev) return fail(p, FCN_E_ARG, "NULL buffer");
    StepCtx ctx;
    hipError_t e = row_pass(p, const_cast<void *>(field_dev), F_DIAG, ctx, 0);
    if (e == hipSuccess) e = finalize(p, diag_dev);
    return e == hipSuccess ? FCN_OK : hip_fail(p, e, "diagnostics");
}

fcn_status fcn_stage(fcn_plan_t p, int32_t stage, void *field_dev, double length) {
    if (!p) return FCN_E_ARG;
    p->err.clear();
    if (!p->bound) return fail(p, FCN_E_STATE, "plan is not bound to a workspace");
    if (!field_dev) return fail(p, FCN_E_ARG, "field is NULL");
    if (!std::isfinite(length)) return fail(p, FCN_E_ARG, "length must be finite");
    StepCtx ctx;
    hipError_t e;
    switch (stage) {
        case FCN_STAGE_FFT: e = row_pass(p, field_dev, RK_FFT_OUT | RK_STORE, ctx, 0); break;
        case FCN_STAGE_IFFT: e = row_pass(p, field_dev, RK_IFFT_IN | RK_STORE, ctx, 0); break;
        case FCN_STAGE_NL: e = row_pass(p, field_dev, RK_NL_B | RK_STORE | RK_STAGE_LEN, ctx, 0, length); break;
        case FCN_STAGE_CN: e = col_pass(p, field_dev, 1, length); break;
        default: return fail(p, FCN_E_ARG, "unknown stage %d", stage);
    }
    return e == hipSuccess ? FCN_OK : hip_fail(p, e, "stage");
}

fcn_status fcn_sync(fcn_plan_t p) {
    if (!p) return FCN_E_ARG;
    if (!p->bound) return fail(p, FCN_E_STATE, "plan is not bound to a workspace");
    hipError_t e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return hip_fail(p, e, "hipStreamSynchronize");
    std::vector<DevState> states((size_t)p->nlanes);
    e = hipMemcpy(states.data(), p->d_state(0), sizeof(DevState) * states.size(), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(p, e, "read flags");
    int32_t flags[2] = {0, 0};  // any lane's nonfinite, unstable
    for (const auto &x : states) {
        flags[0] |= x.nonfinite;
        flags[1] |= x.unstable;
    }
    if (flags[0] || flags[1]) {
        e = launch_clear_flag(p->d_state(0), p->nlanes, p->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
        if (flags[1])
            return fail(p, FCN_E_UNSTABLE,
                        "an RK4 density step left its stability region (sigma_K I^K dtau beyond about 2.785)%s",
                        flags[0] ? "; the field then became non-finite" : "");
        return fail(p, FCN_E_NONFINITE, "non-finite intensity in the field");
    }
    return FCN_OK;
}

fcn_status fcn_step_scratch(fcn_plan_t p, void *field_dev, int64_t nsteps, void *stream) {
    if (!p) return FCN_E_ARG;
    p->err.clear();
    if (!field_dev) return fail(p, FCN_E_ARG, "field is NULL");
    if (!field_aligned(field_dev)) return fail(p, FCN_E_ARG, "field is not 16-byte aligned");
    if (nsteps < 0) return fail(p, FCN_E_ARG, "nsteps < 0");
    if (p->ws_bytes > FCN_SCRATCH_BYTES)
        return fail(p, FCN_E_SIZE, "plan needs %zu bytes of workspace, the static scratch holds %u", p->ws_bytes,
                    (unsigned)FCN_SCRATCH_BYTES);
    unsigned char *scr = nullptr;
    fcn_status st = scratch_on_current_device(p, &scr);
    if (st != FCN_OK) return st;
    // run on the scratch with a temporary binding; the plan's own binding is restored after
    unsigned char *const ws0 = p->ws;
    const hipStream_t stream0 = p->stream;
    const bool bound0 = p->bound, seeded0 = p->seeded;
    const int64_t n0 = p->n_host;
    const int32_t graph0 = p->opt.use_graph;
    p->ws = scr;
    p->stream = static_cast<hipStream_t>(stream);
    hipError_t e = hipMemcpyAsync(p->ws, p->image.data(), p->const_bytes, hipMemcpyHostToDevice, p->stream);
    if (e == hipSuccess)
        e = launch_init_state(p->d_state(0), p->nlanes, p->d_slots(), p->d_ring(), p->d_zpos(), p->batch, 0, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);  // the host image is read by the copy
    if (e != hipSuccess) {
        st = hip_fail(p, e, "upload plan tables to the static scratch");
    } else {
        p->bound = true;
        p->n_host = 0;
        p->seeded = false;
        p->opt.use_graph = 0;  // a graph would hold this call's addresses
        p->serial = true;      // every lane on the given stream: no helper streams, no events
        st = run_steps(p, field_dev, nsteps, nullptr, 0, nullptr, 0);
        p->serial = false;
    }
    p->ws = ws0;
    p->stream = stream0;
    p->bound = bound0;
    p->seeded = seeded0;
    p->n_host = n0;
    p->opt.use_graph = graph0;
    return st;
}

fcn_status fcn_step_timed(fcn_plan_t p, void *field_dev, int64_t nsteps, double *row_ms, double *col_ms,
                          double *total_ms) {
    if (!p) return FCN_E_ARG;
    p->err.clear();
    if (!p->bound) return fail(p, FCN_E_STATE, "plan is not bound to a workspace");
    if (!field_dev || !row_ms || !col_ms || !total_ms) return fail(p, FCN_E_ARG, "NULL argument");
    if (!field_aligned(field_dev)) return fail(p, FCN_E_ARG, "field is not 16-byte aligned");
    if (nsteps < 2 || nsteps > 100000) return fail(p, FCN_E_ARG, "nsteps must be in [2, 100000]");
    // Steady steps s = 0 .. mid-1 each run a column pass then a fused row pass; each pass is
    // bracketed by events recorded at its kernels' own start and end.
    const int64_t mid = nsteps - 1;
    std::vector<hipEvent_t> ev((size_t)(4 * mid + 2), nullptr);
    hipError_t e = hipSuccess;
    for (auto &x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    StepCtx ctx;
    if (e == hipSuccess && p->opt.adaptive && !p->seeded) {
        e = row_pass(p, field_dev, F_DIAG, ctx, 1);
        p->seeded = true;
    }
    hipEvent_t t0 = ev[4 * mid], t1 = ev[4 * mid + 1];
    if (e == hipSuccess) e = row_pass(p, field_dev, F_FIRST, ctx, 0, 0.0, t0, nullptr);
    for (int64_t s = 0; s < mid && e == hipSuccess; s++) {
        e = col_pass(p, field_dev, 0, 0.0, ev[4 * s], ev[4 * s + 1]);
        if (e == hipSuccess) e = row_pass(p, field_dev, F_MIDDLE, ctx, 0, 0.0, ev[4 * s + 2], ev[4 * s + 3]);
    }
    if (e == hipSuccess) e = col_pass(p, field_dev, 0);
    if (e == hipSuccess) e = row_pass(p, field_dev, F_LAST, ctx, 0, 0.0, nullptr, t1);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    double rsum = 0.0, csum = 0.0;
    float tot = 0.f;
    for (int64_t s = 0; s < mid && e == hipSuccess; s++) {
        float c = 0.f, r = 0.f;
        e = hipEventElapsedTime(&c, ev[4 * s], ev[4 * s + 1]);
        if (e == hipSuccess) e = hipEventElapsedTime(&r, ev[4 * s + 2], ev[4 * s + 3]);
        csum += c;
        rsum += r;
    }
    if (e == hipSuccess) e = hipEventElapsedTime(&tot, t0, t1);
    for (auto &x : ev)
        if (x) hipEventDestroy(x);
    if (e != hipSuccess) return hip_fail(p, e, "timed step");
    p->n_host += nsteps;
    *col_ms = csum / (double)mid;
    *row_ms = rsum / (double)mid;
    *total_ms = tot;
    return FCN_OK;
}

fcn_status fcn_step_timed_launches(fcn_plan_t p, void *field_dev, int64_t nsteps, int32_t max_launches,
                                   int32_t *n_launches, double *launch_ms, int64_t *launch_info) {
    if (!p) return FCN_E_ARG;
    p->err.clear();
    if (!p->bound) return fail(p, FCN_E_STATE, "plan is not bound to a workspace");
    if (!field_dev || !n_launches) return fail(p, FCN_E_ARG, "NULL argument");
    if (!field_aligned(field_dev)) return fail(p, FCN_E_ARG, "field is not 16-byte aligned");
    if (nsteps < 2 || nsteps > 10000) return fail(p, FCN_E_ARG, "nsteps must be in [2, 10000]");
    const int nrow = (int)p->row_buckets.size(), ncol = (int)p->col_buckets.size(), nl = nrow + ncol;
    *n_launches = nl;
    if (max_launches < nl || !launch_ms || !launch_info)
        return fail(p, FCN_E_SIZE, "the plan's step has %d launches; buffers hold %d", nl, max_launches);
    // per steady step: column launches then row launches, two events each
    const int64_t mid = nsteps - 1;
    std::vector<hipEvent_t> ev((size_t)(2 * nl * mid), nullptr);
    hipError_t e = hipSuccess;
    for (auto &x : ev)
        if (e == hipSuccess) e = hipEventCreate(&x);
    StepCtx ctx;
    if (e == hipSuccess && p->opt.adaptive && !p->seeded) {
        e = row_pass(p, field_dev, F_DIAG, ctx, 1);
        p->seeded = true;
    }
    if (e == hipSuccess) e = row_pass(p, field_dev, F_FIRST, ctx, 0);
    for (int64_t s = 0; s < mid && e == hipSuccess; s++) {
        const hipEvent_t *base = ev.data() + (size_t)(2 * nl * s);
        e = col_pass(p, field_dev, 0, 0.0, nullptr, nullptr, base + 2 * nrow);
        if (e == hipSuccess) e = row_pass(p, field_dev, F_MIDDLE, ctx, 0, 0.0, nullptr, nullptr, base);
    }
    if (e == hipSuccess) e = col_pass(p, field_dev, 0);
    if (e == hipSuccess) e = row_pass(p, field_dev, F_LAST, ctx, 0);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    std::vector<double> sum((size_t)nl, 0.0);
    for (int64_t s = 0; s < mid && e == hipSuccess; s++)
        for (int l = 0; l < nl && e == hipSuccess; l++) {
            float ms = 0.f;
            e = hipEventElapsedTime(&ms, ev[(size_t)(2 * nl * s + 2 * l)], ev[(size_t)(2 * nl * s + 2 * l + 1)]);
            sum[l] += ms;
        }
    for (auto &x : ev)
        if (x) hipEventDestroy(x);
    if (e != hipSuccess) return hip_fail(p, e, "timed launches");
    p->n_host += nsteps;
    for (int l = 0; l < nl; l++) {
        launch_ms[l] = sum[l] / (double)mid;
        int64_t pts = 0;
        if (l < nrow) {
            const auto &b = p->row_buckets[l];
            pts = b.points;
            launch_info[5 * l] = 0;
            launch_info[5 * l + 1] = b.nt;
            launch_info[5 * l + 3] = row_elems_for(b.nt, row_fp64_arith(p->precision));
            launch_info[5 * l + 4] = row_rows_per_group(b.nt, (int)launch_info[5 * l + 3]);
        } else {
            const auto &b = p->col_buckets[l - nrow];
            pts = b.points;
            launch_info[5 * l] = 1 + b.dir;
            launch_info[5 * l + 1] = b.nr;
            launch_info[5 * l + 3] = b.w;
            launch_info[5 * l + 4] = b.l;
        }
        launch_info[5 * l + 2] = pts;
    }
    return FCN_OK;
}

const char *fcn_last_error(fcn_plan_t p) { return p ? p->err.c_str() : "NULL plan"; }

fcn_status fcn_plan_destroy(fcn_plan_t p) {
    if (!p) return FCN_E_ARG;
    destroy_graphs(p);
    for (auto ls : p->lane_streams) (void)hipStreamDestroy(ls);
    for (auto le : p->lane_events) (void)hipEventDestroy(le);
    if (p->fork_event) (void)hipEventDestroy(p->fork_event);
    delete p;
    return FCN_OK;
}

}  // extern "C"
