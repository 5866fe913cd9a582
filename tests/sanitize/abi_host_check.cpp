// Host sanitizer run of the C ABI's argument validation (test
// infrastructure): every entry point is called with arguments its header
// rejects, before any device work, against a libbte built with host-side
// AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitizers.py.  No GPU is needed or touched.
#include <cstdio>
#include <cstring>

#include "bte.h"
#include "bte_mlp.h"

#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                                     \
        }                                                                 \
    } while (0)

int main()
{
    bte_grid g{64, 201, -8.0, 8.0};
    bte_params p{};
    p.E_dc = 1.0; p.E_w = 0.0; p.omega = 1.0; p.B = 0.0; p.mu = 1.0; p.alpha = 1.0;
    p.tau = 1.0; p.dt = 1e-3; p.precision = BTE_FP64; p.flags = 0;
    size_t bytes = 0;
    CHECK(bte_workspace_bytes(&g, &p, &bytes) == BTE_OK && bytes > 0);
    CHECK(bte_workspace_bytes(nullptr, &p, &bytes) == BTE_EINVAL);
    CHECK(bte_workspace_bytes(&g, nullptr, &bytes) == BTE_EINVAL);
    CHECK(bte_workspace_bytes(&g, &p, nullptr) == BTE_EINVAL);
    bte_grid bad = g;
    bad.n_x = 1;
    CHECK(bte_workspace_bytes(&bad, &p, &bytes) == BTE_EINVAL);
    bad = g; bad.n_y = 2;
    CHECK(bte_workspace_bytes(&bad, &p, &bytes) == BTE_EINVAL);
    bad = g; bad.phiy_max = bad.phiy_min;
    CHECK(bte_workspace_bytes(&bad, &p, &bytes) == BTE_EINVAL);
    bte_params q = p; q.tau = 2.0;
    CHECK(bte_workspace_bytes(&g, &q, &bytes) == BTE_EINVAL);
    q = p; q.dt = -1.0;
    CHECK(bte_workspace_bytes(&g, &q, &bytes) == BTE_EINVAL);
    q = p; q.B = 1e6;   // leap-frog bound dt |B| / (2 dphi) < 1 broken
    CHECK(bte_workspace_bytes(&g, &q, &bytes) == BTE_EINVAL);
    q = p; q.flags = 1;
    CHECK(bte_workspace_bytes(&g, &q, &bytes) == BTE_EINVAL);
    q = p; q.precision = 7;
    CHECK(bte_workspace_bytes(&g, &q, &bytes) == BTE_EINVAL);
    bte_solver* s = nullptr;
    CHECK(bte_create(&g, &p, nullptr, 0, nullptr, &s) != BTE_OK && s == nullptr);
    CHECK(bte_create(&g, &p, nullptr, bytes, nullptr, nullptr) == BTE_EINVAL);

    // handle-taking calls reject a NULL handle without touching the device
    bte_obs o;
    bte_tuning t{};
    CHECK(bte_step(nullptr, 1) == BTE_EINVAL);
    CHECK(bte_set_window(nullptr, 0, 1) == BTE_EINVAL);
    CHECK(bte_observables(nullptr, &o) == BTE_EINVAL);
    CHECK(bte_get_state(nullptr, nullptr, nullptr, nullptr, nullptr) == BTE_EINVAL);
    CHECK(bte_set_state(nullptr, nullptr, nullptr, nullptr, nullptr, 0) == BTE_EINVAL);
    CHECK(bte_set_tuning(nullptr, &t) == BTE_EINVAL);
    CHECK(bte_get_tuning(nullptr, &t) == BTE_EINVAL);
    CHECK(bte_reconstruct(nullptr, 4, nullptr) == BTE_EINVAL);
    bte_result rr;
    CHECK(bte_run_periods(nullptr, 1e-6, 2, 10, 1, &rr) == BTE_EINVAL);
    bte_destroy(nullptr);

    // state observables: sizes and pointers
    CHECK(bte_state_observables_bytes(1, &bytes) == BTE_EINVAL);
    CHECK(bte_state_observables_bytes(16385, &bytes) == BTE_EINVAL);
    CHECK(bte_state_observables_bytes(4, &bytes) == BTE_OK && bytes > 0);
    double fake[8];
    CHECK(bte_state_observables(nullptr, fake, 4, 10, 10, -1, 1, 1, nullptr, 0, nullptr, fake) ==
          BTE_EINVAL);
    CHECK(bte_state_observables(fake, fake, 4, 10, 9, -1, 1, 1, nullptr, 0, nullptr, fake) ==
          BTE_EINVAL);
    CHECK(bte_state_observables_noalloc(fake, fake, 16385, 3, 3, -1, 1, 1, nullptr, fake) ==
          BTE_EINVAL);
    CHECK(bte_state_observables_noalloc(fake, fake, 4, 10, 10, 1, -1, 1, nullptr, fake) ==
          BTE_EINVAL);
    CHECK(bte_reconstruct_coeffs(nullptr, fake, 4, 10, 10, 8, fake, nullptr) == BTE_EINVAL);

    // batched sweeps: configuration and instances
    bte_batch_config c{};
    c.n_x = 16; c.precision = BTE_FP32_BULK; c.phiy_min = -6; c.phiy_max = 6; c.dt = 1e-3;
    c.alpha = 1.0; c.tol = 1e-6; c.min_periods = 2; c.max_periods = 10; c.confirm = 1;
    bte_instance in[2]{};
    for (auto& x : in) { x.E_dc = 1; x.E_w = 0.1; x.omega = 2; x.B = 1; x.mu = 1; x.n_y = 33; }
    bte_batch_tuning bt{BTE_KERNEL_FUSED2, 20, 4, 0, BTE_BATCH_WIDE};
    CHECK(bte_batch_workspace_bytes(&c, 2, in, &bt, &bytes) == BTE_OK && bytes > 0);
    CHECK(bte_batch_workspace_bytes(&c, 0, in, &bt, &bytes) == BTE_EINVAL);
    CHECK(bte_batch_workspace_bytes(&c, 2, nullptr, &bt, &bytes) == BTE_EINVAL);
    bte_batch_config cb = c; cb.min_periods = 1;
    CHECK(bte_batch_workspace_bytes(&cb, 2, in, &bt, &bytes) == BTE_EINVAL);
    cb = c; cb.tol = 0.0;
    CHECK(bte_batch_workspace_bytes(&cb, 2, in, &bt, &bytes) == BTE_EINVAL);
    bte_instance ib[2] = {in[0], in[1]};
    ib[1].omega = 0.0;
    CHECK(bte_batch_workspace_bytes(&c, 2, ib, &bt, &bytes) == BTE_EINVAL);
    ib[1] = in[1]; ib[1].reserved = 3;
    CHECK(bte_batch_workspace_bytes(&c, 2, ib, &bt, &bytes) == BTE_EINVAL);
    bte_batch_tuning btb = bt; btb.waves_per_group = 3;
    CHECK(bte_batch_workspace_bytes(&c, 2, in, &btb, &bytes) == BTE_EINVAL);
    bte_batch_tuning tuned{};
    CHECK(bte_batch_tune(&cb, 2, in, nullptr, 1, &tuned, nullptr) == BTE_EINVAL);
    CHECK(bte_batch_tune(&c, 2, ib, nullptr, 1, &tuned, nullptr) == BTE_EINVAL);
    CHECK(bte_batch_tune(&c, 2, in, nullptr, 1, nullptr, nullptr) == BTE_EINVAL);
    CHECK(bte_batch_run(nullptr) == BTE_EINVAL);
    int32_t left = 0;
    CHECK(bte_batch_advance(nullptr, 1, &left) == BTE_EINVAL);
    CHECK(bte_batch_results(nullptr, &rr) == BTE_EINVAL);
    bte_batch_destroy(nullptr);

    // network: shapes
    CHECK(bte_mlp_workspace_bytes(0, 0) == 0);
    bte_mlp* m = nullptr;
    CHECK(bte_mlp_create(0, 0, nullptr, 0, nullptr, &m) != BTE_OK);
    CHECK(bte_stream_copy(nullptr, fake, 16, nullptr) == BTE_EINVAL);
    CHECK(bte_stream_copy(fake, fake + 1, 16, nullptr) == BTE_EINVAL);
    CHECK(std::strlen(bte_version()) > 0);
    CHECK(bte_last_error() != nullptr);
    std::printf("abi host sanitizer run ok\n");
    return 0;
}
