// Autotuner of the step kernels' launch shape (native part of the runtime).
//
// For a grid and parameter set it builds a scratch solver on the caller's
// workspace, times every candidate shape (kernel form x harmonics per wave x
// waves per block) with HIP events on the caller's stream, and returns the
// fastest.  The candidates are exactly the shapes bte_set_tuning accepts, so
// the result can be applied to any solver with the same grid and precision.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <vector>

#include "../../include/bte.h"
#include "bte_internal.h"

namespace {

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair()
    {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

// Time n steps of solver s with tuning t; returns microseconds per step or a
// negative value on failure.
double time_steps(bte_solver* s, const bte_tuning& t, int n, hipStream_t st, EventPair& ev)
{
    if (bte_set_tuning(s, &t) != BTE_OK) return -1.0;
    const int warm = std::max(2, t.graph_steps);
    if (bte_step(s, warm) != BTE_OK) return -1.0;
    if (hipEventRecord(ev.a, st) != hipSuccess) return -1.0;
    if (bte_step(s, n) != BTE_OK) return -1.0;
    if (hipEventRecord(ev.b, st) != hipSuccess) return -1.0;
    if (hipEventSynchronize(ev.b) != hipSuccess) return -1.0;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev.a, ev.b) != hipSuccess) return -1.0;
    return 1e3 * static_cast<double>(ms) / n;
}

}  // namespace

extern "C" bte_status bte_tune(const bte_grid* grid, const bte_params* params, void* workspace,
                               size_t workspace_bytes, void* hip_stream, int32_t kernel_form,
                               double target_ms, bte_tuning* best, double* best_us_per_step)
{
    if (!best) {
        bte::set_last_error("best must not be NULL");
        return BTE_EINVAL;
    }
    if (kernel_form < -1 || kernel_form > BTE_KERNEL_FUSED3) {
        bte::set_last_error("kernel_form must be -1 or a bte_kernel value");
        return BTE_EINVAL;
    }
    bte_solver* s = nullptr;
    bte_status rc = bte_create(grid, params, workspace, workspace_bytes, hip_stream, &s);
    if (rc != BTE_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    EventPair ev;
    if (hipEventCreate(&ev.a) != hipSuccess || hipEventCreate(&ev.b) != hipSuccess) {
        bte_destroy(s);
        bte::set_last_error("hipEventCreate failed");
        return BTE_EDEVICE;
    }
    if (!(target_ms > 0)) target_ms = 2.0;

    bte_tuning base{};
    (void)bte_get_tuning(s, &base);   // library default for this grid
    if (kernel_form >= 0) base.kernel = kernel_form;
    const int G = base.graph_steps;

    // steps per trial: about target_ms at the default shape, a multiple of G
    double us0 = time_steps(s, base, std::max(G, 8), st, ev);
    if (us0 <= 0) {
        bte_destroy(s);
        bte::set_last_error("timing the default shape failed");
        return BTE_EDEVICE;
    }
    int n = static_cast<int>(target_ms * 1e3 / us0);
    n = std::max(n, std::max(G, 8));
    if (G > 0) n = (n + G - 1) / G * G;

    // Harmonics per wave: for every chunk count c the smallest R that gives
    // c chunks (R = ceil(n_x / c), the most even split).  How many tiles a
    // launch has against how many waves the GPU holds at once decides how
    // much of the last round of waves idles, so the whole range is timed.
    std::vector<int> rows;
    for (int c = 1; c <= grid->n_x; ++c) {
        const int R = (grid->n_x + c - 1) / c;
        if (R > 62) continue;
        if (R < 2 && !rows.empty()) break;
        if (rows.empty() || rows.back() != R) rows.push_back(std::max(R, 1));
    }
    const int wpbs[] = {1, 2, 4, 8};
    bte_tuning win = base;
    double win_us = time_steps(s, base, n, st, ev);
    for (int kernel = BTE_KERNEL_FUSED; kernel <= BTE_KERNEL_FUSED3; ++kernel) {
        if (kernel_form >= 0 && kernel != kernel_form) continue;
        for (int R : rows) {
            for (int w : wpbs) {
                if (kernel == BTE_KERNEL_FUSED2 && (R > 58 || w > 4)) continue;
                if (kernel == BTE_KERNEL_FUSED3 && (R > 54 || w > 4)) continue;
                bte_tuning t{};
                t.kernel = kernel;
                t.rows_per_wave = R;
                t.waves_per_block = w;
                t.graph_steps = G;
                const double us = time_steps(s, t, n, st, ev);
                // a later candidate must win by more than the timing noise, so
                // repeated tuning of one problem tends to return one shape
                if (us > 0 && (win_us <= 0 || us < 0.995 * win_us)) {
                    win_us = us;
                    win = t;
                }
            }
        }
    }
    bte_destroy(s);
    if (win_us <= 0) {
        bte::set_last_error("no candidate shape could be timed");
        return BTE_EDEVICE;
    }
    *best = win;
    if (best_us_per_step) *best_us_per_step = win_us;
    return BTE_OK;
}
