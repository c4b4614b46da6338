// parareal.cpp -- parareal along z driven inside the library (fcn_parareal in include/fcn.h).
//
// For one pulse cut into W windows of `steps_per_window` FCN steps (an addition of this project;
// the paper integrates z serially):
//   iteration 0:  U_{j+1} = G(U_j)                                   (coarse sweep)
//   iteration k:  F_j = F(U_j^{k-1}) for all j in one batched plan    (fine, parallel in z)
//                 U_{j+1}^k = G(U_j^k) + F_j - G(U_j^{k-1})           (sequential sweep)
// G is one classical FCN step of the whole window (the coarse plan), plus the learned
// network's correction when a network is given.  The fine FCN is the judge: the r-weighted
// change max_j |U_{j+1}^k - U_{j+1}^{k-1}| / |U_{j+1}^k| ends the iteration below tol; a
// growing or non-finite change stops it and keeps U^{k-1}; without convergence the serial
// fine solution is computed instead (fallback).  Every arithmetic step runs in the library's
// kernels; the host reads the W change partial sums once per iteration.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "../../include/fcn.h"
#include "net_internal.h"

namespace fcn {
int plan_precision(fcn_plan_t p);
hipStream_t plan_stream(fcn_plan_t p);
bool plan_bound(fcn_plan_t p);
hipStream_t net_stream(fcn_net_t n);
}  // namespace fcn

using namespace fcn;

namespace {

constexpr int kParts = 256;  // workgroups of the combination kernel (change partial sums)

size_t al(size_t x) { return (x + 255) / 256 * 256; }

struct Layout {
    size_t batch, gold, unew, gnew, tmp, parts, total;
};

Layout layout(int64_t n, int windows) {
    Layout L{};
    size_t o = 0;
    const size_t f = (size_t)n * 8;  // complex64
    L.batch = o;
    o = al(o + f * windows);
    L.gold = o;
    o = al(o + f * windows);
    L.unew = o;
    o = al(o + f * (windows + 1));
    L.gnew = o;
    o = al(o + f);
    L.tmp = o;
    o = al(o + f);
    L.parts = o;
    o = al(o + sizeof(double) * 2 * kParts * (size_t)windows);
    L.total = o;
    return L;
}

}  // namespace

extern "C" {

fcn_status fcn_parareal_workspace_size(int32_t nr, int32_t nt, int32_t windows, size_t *bytes) {
    if (!bytes || nr < 3 || nt < 1 || windows < 1) return FCN_E_ARG;
    *bytes = layout((int64_t)nr * nt, windows).total;
    return FCN_OK;
}

fcn_status fcn_parareal(fcn_plan_t fine, fcn_plan_t coarse, fcn_net_t net, const fcn_net_sample *sample_dev,
                        fcn_plan_t fine_serial, int32_t nr, int32_t nt, void *u_dev, void *workspace,
                        size_t workspace_bytes, const fcn_parareal_options *opt, fcn_parareal_result *result) {
    if (!fine || !coarse || !u_dev || !workspace || !opt || !result) return FCN_E_ARG;
    const int W = opt->windows, S = opt->steps_per_window, kmax = opt->kmax;
    if (W < 1 || S < 1 || kmax < 0 || kmax > FCN_PARAREAL_MAX_ITER || nr < 3 || nt < 1 || !(opt->tol >= 0.0))
        return FCN_E_ARG;
    if (((uintptr_t)workspace & 255) != 0) return FCN_E_ARG;
    const int64_t n = (int64_t)nr * nt;
    const Layout L = layout(n, W);
    if (workspace_bytes < L.total) return FCN_E_SIZE;
    if (!plan_bound(fine) || !plan_bound(coarse) || (fine_serial && !plan_bound(fine_serial))) return FCN_E_STATE;
    // complex64 fields only (FP32 or FP32 storage), one stream for everything
    auto c64 = [](fcn_plan_t p) { return plan_precision(p) != FCN_FP64; };
    if (!c64(fine) || !c64(coarse) || (fine_serial && !c64(fine_serial))) return FCN_E_UNSUPPORTED;
    hipStream_t st = plan_stream(fine);
    if (plan_stream(coarse) != st || (fine_serial && plan_stream(fine_serial) != st) || (net && net_stream(net) != st))
        return FCN_E_ARG;
    if (net && !sample_dev) return FCN_E_ARG;
    // the fine plan holds W instances of this grid back to back; the others one instance
    size_t sz = 0, off = 0;
    if (fcn_field_size(fine, &sz) != FCN_OK || sz != (size_t)n * W) return FCN_E_SIZE;
    for (int j = 0; j < W; j++)
        if (fcn_field_offset(fine, j, &off) != FCN_OK || off != (size_t)n * j) return FCN_E_SIZE;
    if (fcn_field_size(coarse, &sz) != FCN_OK || sz != (size_t)n) return FCN_E_SIZE;
    if (fine_serial && (fcn_field_size(fine_serial, &sz) != FCN_OK || sz != (size_t)n)) return FCN_E_SIZE;

    unsigned char *ws = (unsigned char *)workspace;
    float2 *U = (float2 *)u_dev;
    float2 *batch = (float2 *)(ws + L.batch), *gold = (float2 *)(ws + L.gold), *unew = (float2 *)(ws + L.unew);
    float2 *gnew = (float2 *)(ws + L.gnew), *tmp = (float2 *)(ws + L.tmp);
    double *parts = (double *)(ws + L.parts);
    const size_t fb = (size_t)n * sizeof(float2);
    hipError_t e = hipSuccess;
    fcn_status rc = FCN_OK;

    // out = G(u)
    auto G = [&](const float2 *u, float2 *out) -> fcn_status {
        if ((e = hipMemcpyAsync(tmp, u, fb, hipMemcpyDeviceToDevice, st)) != hipSuccess) return FCN_E_HIP;
        fcn_status r = fcn_step(coarse, tmp, 1);
        if (r != FCN_OK) return r;
        if (!net) return hipMemcpyAsync(out, tmp, fb, hipMemcpyDeviceToDevice, st) == hipSuccess ? FCN_OK : FCN_E_HIP;
        if ((r = fcn_net_input(net, u, sample_dev, 1, nr, nt, nr, nt)) != FCN_OK) return r;
        if ((r = fcn_net_forward(net, 1, nr, nt, nullptr)) != FCN_OK) return r;
        return fcn_net_apply(net, tmp, sample_dev, 1, nr, nt, out);
    };

    result->iterations = 0;
    result->status = FCN_PARAREAL_KMAX;
    for (int k = 0; k <= FCN_PARAREAL_MAX_ITER; k++) result->change[k] = 0.0;

    // iteration 0: coarse sweep
    for (int j = 0; j < W && rc == FCN_OK; j++) {
        rc = G(U + (size_t)j * n, gold + (size_t)j * n);
        if (rc == FCN_OK && (e = hipMemcpyAsync(U + (size_t)(j + 1) * n, gold + (size_t)j * n, fb,
                                                hipMemcpyDeviceToDevice, st)) != hipSuccess)
            rc = FCN_E_HIP;
    }
    if (rc == FCN_OK && (e = hipMemcpyAsync(unew, U, fb, hipMemcpyDeviceToDevice, st)) != hipSuccess) rc = FCN_E_HIP;
    result->change[0] = INFINITY;

    std::vector<double> hparts((size_t)2 * kParts * W);
    double prev = INFINITY;
    for (int k = 1; k <= kmax && rc == FCN_OK; k++) {
        // fine propagation of every window from U^{k-1}, batched
        if ((e = hipMemcpyAsync(batch, U, fb * W, hipMemcpyDeviceToDevice, st)) != hipSuccess) { rc = FCN_E_HIP; break; }
        if ((rc = fcn_step(fine, batch, S)) != FCN_OK) break;
        for (int j = 0; j < W && rc == FCN_OK; j++) {
            if ((rc = G(unew + (size_t)j * n, gnew)) != FCN_OK) break;
            if ((e = launch_parareal_update(gnew, batch + (size_t)j * n, gold + (size_t)j * n, U + (size_t)(j + 1) * n,
                                            unew + (size_t)(j + 1) * n, nr, nt, parts + (size_t)2 * kParts * j, kParts,
                                            st)) != hipSuccess ||
                (e = hipMemcpyAsync(gold + (size_t)j * n, gnew, fb, hipMemcpyDeviceToDevice, st)) != hipSuccess)
                rc = FCN_E_HIP;
        }
        if (rc != FCN_OK) break;
        if ((e = hipMemcpyAsync(hparts.data(), parts, hparts.size() * sizeof(double), hipMemcpyDeviceToHost, st)) !=
                hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess) {
            rc = FCN_E_HIP;
            break;
        }
        double change = 0.0;
        for (int j = 0; j < W; j++) {
            double d = 0.0, u = 0.0;
            for (int q = 0; q < kParts; q++) {
                d += hparts[(size_t)2 * kParts * j + 2 * q];
                u += hparts[(size_t)2 * kParts * j + 2 * q + 1];
            }
            const double c = std::sqrt(d / (u > 1e-300 ? u : 1e-300));
            change = (std::isnan(c) || std::isnan(change)) ? NAN : (c > change ? c : change);
        }
        result->change[k] = change;
        if (!std::isfinite(change)) {
            result->status = FCN_PARAREAL_NONFINITE;
            break;
        }
        if (opt->judge && change > prev) {
            result->status = FCN_PARAREAL_DIVERGING;
            break;
        }
        if ((e = hipMemcpyAsync(U + n, unew + n, fb * W, hipMemcpyDeviceToDevice, st)) != hipSuccess) { rc = FCN_E_HIP; break; }
        result->iterations = k;
        prev = change;
        if (change < opt->tol) {
            result->status = FCN_PARAREAL_CONVERGED;
            break;
        }
    }
    if (rc != FCN_OK) return rc;
    if (result->status != FCN_PARAREAL_CONVERGED && opt->fallback && fine_serial) {
        // serial fine solution, window by window
        for (int j = 0; j < W && rc == FCN_OK; j++) {
            if ((e = hipMemcpyAsync(U + (size_t)(j + 1) * n, U + (size_t)j * n, fb, hipMemcpyDeviceToDevice, st)) !=
                hipSuccess) {
                rc = FCN_E_HIP;
                break;
            }
            rc = fcn_step(fine_serial, U + (size_t)(j + 1) * n, S);
        }
        if (rc == FCN_OK) result->status = FCN_PARAREAL_FALLBACK;
    }
    if (rc == FCN_OK && (e = hipStreamSynchronize(st)) != hipSuccess) rc = FCN_E_HIP;
    return rc;
}

}  // extern "C"
