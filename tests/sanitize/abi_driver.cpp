// Runs the host paths of libpd's C ABI -- argument checks, workspace sizes,
// status strings, switches -- with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code, and no GPU work: every call
// below returns an error (or a size) before anything is enqueued, so the
// pointers handed in are never dereferenced.  Prints OK.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "pd.h"

static void *fake(uintptr_t k) { return reinterpret_cast<void *>(0x100000 + 0x1000 * k); }

#define EXPECT(cond)                                                        \
    do {                                                                    \
        if (!(cond)) {                                                      \
            std::printf("failed: %s (line %d)\n", #cond, __LINE__);         \
            return 1;                                                       \
        }                                                                   \
    } while (0)

int main()
{
    double h[12];
    EXPECT(pd_symmlet(6, h) == PD_OK);
    pd_wavelet wav{12, h};
    std::vector<double> lw(10, 0.1);
    pd_weights w{lw.data(), nullptr, 0};
    pd_params prm{0.5, 10, 0, 0};
    pd_operator id{PD_OP_IDENTITY, 0, nullptr, 0, nullptr};
    pd_operator blur{PD_OP_ROWBLUR, 2, fake(9), 0, nullptr};
    const pd_shape ok{64, 64, 1, 6};
    const pd_shape bad_shapes[] = {{100, 64, 1, 3}, {64, 64, 1, 7}, {64, 64, 0, 3}, {64, 64, 5, 3},
                                   {1, 64, 1, 1},   {64, 64, 1, 0}, {0, 0, 0, 0}};
    for (int dt = 0; dt < 2; ++dt) {
        EXPECT(pd_workspace_size(&ok, dt) > 0);
        for (const pd_shape &b : bad_shapes) {
            EXPECT(pd_workspace_size(&b, dt) == 0);
            EXPECT(pd_solve(&b, dt, &id, &wav, &w, &prm, fake(1), fake(2), fake(3), 1, nullptr, nullptr,
                            fake(4), 1u << 30, nullptr) != PD_OK);
        }
        const size_t need = pd_workspace_size(&ok, dt);
        // workspace one byte short, aliased state, bad step, bad iteration count, missing input
        EXPECT(pd_solve(&ok, dt, &blur, &wav, &w, &prm, fake(1), fake(2), fake(3), 1, nullptr, nullptr,
                        fake(4), need - 1, nullptr) == PD_ERR_WORKSPACE);
        EXPECT(pd_solve(&ok, dt, &blur, &wav, &w, &prm, fake(1), fake(2), fake(2), 1, nullptr, nullptr,
                        fake(4), need, nullptr) == PD_ERR_ARG);
        pd_params bad_tau{0.0, 10, 0, 0}, nan_tau{std::nan(""), 10, 0, 0}, bad_it{0.5, -1, 0, 0};
        EXPECT(pd_solve(&ok, dt, &blur, &wav, &w, &bad_tau, fake(1), fake(2), fake(3), 1, nullptr, nullptr,
                        fake(4), need, nullptr) == PD_ERR_TAU);
        EXPECT(pd_solve(&ok, dt, &blur, &wav, &w, &nan_tau, fake(1), fake(2), fake(3), 1, nullptr, nullptr,
                        fake(4), need, nullptr) == PD_ERR_TAU);
        EXPECT(pd_solve(&ok, dt, &blur, &wav, &w, &bad_it, fake(1), fake(2), fake(3), 1, nullptr, nullptr,
                        fake(4), need, nullptr) == PD_ERR_ARG);
        EXPECT(pd_solve(&ok, dt, &blur, &wav, &w, &prm, nullptr, fake(2), fake(3), 1, nullptr, nullptr,
                        fake(4), need, nullptr) == PD_ERR_ARG);
        EXPECT(pd_solve_noalloc(&ok, 7, &blur, &wav, &w, &prm, fake(1), fake(2), fake(3), 1, nullptr,
                                nullptr, nullptr) == PD_ERR_ARG);
        const pd_shape big{4096, 4096, 1, 12};
        EXPECT(pd_solve_noalloc(&big, dt, &blur, &wav, &w, &prm, fake(1), fake(2), fake(3), 1, nullptr,
                                nullptr, nullptr) == PD_ERR_WORKSPACE);
        // reverse mode, transforms, tuning, operator application
        EXPECT(pd_backward_workspace_size(&ok, dt, 100, 10) > need);
        EXPECT(pd_backward_workspace_size(&ok, dt, -1, 10) == 0);
        EXPECT(pd_backward(&ok, dt, &blur, &wav, &w, &prm, fake(1), fake(2), fake(3), nullptr, 10, fake(4), 16,
                           nullptr) == PD_ERR_WORKSPACE);
        EXPECT(pd_fwt(&ok, dt, &wav, 0, fake(1), fake(1), fake(4), need, nullptr) == PD_ERR_ARG);
        EXPECT(pd_fwt(&ok, dt, &wav, 0, fake(1), fake(2), fake(4), 16, nullptr) == PD_ERR_WORKSPACE);
        EXPECT(pd_tune(&ok, dt, &blur, nullptr, 0, nullptr, nullptr) == PD_ERR_ARG);
        EXPECT(pd_apply_op(&ok, dt, nullptr, 0, fake(1), fake(2), nullptr) == PD_ERR_ARG);
        // batched: sizes and argument errors
        pd_image_desc d[2];
        for (int b = 0; b < 2; ++b) d[b] = pd_image_desc{ok, (int64_t)b * 64 * 64, 0.5, blur, w};
        EXPECT(pd_batched_workspace_size(2, d, dt) > 0);
        EXPECT(pd_batched_workspace_size(0, d, dt) == 0);
        EXPECT(pd_solve_batched(2, d, dt, &wav, 10, fake(1), fake(2), nullptr, fake(4), 8, nullptr) ==
               PD_ERR_WORKSPACE);
        EXPECT(pd_solve_batched(-1, d, dt, &wav, 10, fake(1), fake(2), nullptr, fake(4), 8, nullptr) != PD_OK);
        // wavelet domain, ADMM, FFT, decomposition sizes and errors
        EXPECT(pd_csr_transpose_workspace_size(4096) > 0);
        EXPECT(pd_wsolve_workspace_size(&ok, dt) > 0);
        EXPECT(pd_admm_workspace_size(&ok, dt, 5) > 0);
        EXPECT(pd_admm_workspace_size(&ok, dt, 0) == 0);
        EXPECT(pd_fft2_workspace_size(64, 64, dt) > 0);
        EXPECT(pd_fft2(60, 64, 1, dt, 0, fake(1), fake(2), 1u << 20, nullptr) != PD_OK);
        EXPECT(pd_spmv(nullptr, dt, fake(1), fake(2), nullptr) == PD_ERR_ARG);
    }
    EXPECT(pd_decompose_workspace_size(&ok, 5) > 0);
    EXPECT(pd_decompose_workspace_size(&ok, 0) == 0);
    int64_t nnz = 0;
    EXPECT(pd_decompose(&ok, &blur, &wav, 1.0, 0, &nnz, nullptr, nullptr, nullptr, nullptr, 0, nullptr) != PD_OK);
    // switches and the timing record
    EXPECT(pd_graphs_enable(0) == PD_OK && pd_graphs_enable(1) == PD_OK);
    EXPECT(pd_fuse_enable(0) == PD_OK && pd_fuse_enable(1) == PD_OK);
    EXPECT(pd_timing_enable(1) == PD_OK);
    std::vector<int32_t> kc(8), lv(8), ns(8);
    std::vector<int64_t> la(8);
    std::vector<double> ms(8);
    int32_t rows = -1;
    (void)pd_timing_read(8, kc.data(), lv.data(), la.data(), ms.data(), &rows);
    EXPECT(pd_timing_enable(0) == PD_OK);
    for (int code = -12; code <= 2; ++code) EXPECT(pd_strerror(code) != nullptr);
    std::printf("OK\n");
    return 0;
}
