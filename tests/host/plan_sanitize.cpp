// Drives the host-side code of the library that runs without a GPU (the
// batch planner behind ssm_workspace_size, argument checks of every entry
// point, error reporting) over many problem shapes, so that a build with
// host AddressSanitizer + UndefinedBehaviorSanitizer reports any
// out-of-bounds access or undefined operation.  Compiled and run by
// tests/test_sanitize.py.  Prints OK.
#include "ssm.h"

#include <cstdio>
#include <cstring>
#include <vector>

static int fails = 0;
#define EXPECT(c)                                                      \
    do {                                                               \
        if (!(c)) { std::printf("FAILED %s line %d\n", #c, __LINE__); ++fails; } \
    } while (0)

int main()
{
    EXPECT(ssm_version() >= 1);
    for (int i = -1; i <= SSM_N_KERNELS; ++i) (void)ssm_kernel_name(i);
    // every lattice shape class: ragged, powers of two, 1..16 layers, limits
    const int dims[] = {1, 2, 3, 5, 16, 17, 33, 64, 100, 255, 256, 257, 511, 1000, 1024};
    const int zs[] = {1, 2, 3, 4, 7, 8, 9, 16};
    size_t bytes = 0;
    int ok = 0, unsupported = 0;
    for (int prec : {SSM_FP64, SSM_FP32_MIXED, SSM_FP32_MIXED | SSM_WITH_RK})
        for (int nx : dims)
            for (int ny : dims)
                for (int nz : zs) {
                    ssm_problem p = {nx, ny, nz, 3, 1.0, 0.3, 0.1, 0.02};
                    const ssm_status st = ssm_workspace_size(&p, 1, prec, &bytes);
                    if (st == SSM_OK) { ++ok; EXPECT(bytes > 0); }
                    else { ++unsupported; EXPECT(st == SSM_EUNSUPPORTED); EXPECT(std::strlen(ssm_last_error(nullptr)) > 0); }
                }
    EXPECT(ok > 0 && unsupported > 0);
    // batches of uneven problems (layers rounding to one power of two)
    std::vector<ssm_problem> batch;
    for (int i = 0; i < 256; ++i) batch.push_back({48 + i % 49, 48 + (7 * i) % 49, 1, 2 + i % 30, 1.0, 0.2, 0.1, 0.01});
    EXPECT(ssm_workspace_size(batch.data(), 256, SSM_FP32_MIXED, &bytes) == SSM_OK);
    batch.push_back(batch[0]);
    EXPECT(ssm_workspace_size(batch.data(), 257, SSM_FP32_MIXED, &bytes) == SSM_EUNSUPPORTED);
    ssm_problem mix[2] = {{8, 8, 2, 3, 1, 0, 0, 0}, {8, 8, 5, 3, 1, 0, 0, 0}};
    EXPECT(ssm_workspace_size(mix, 2, SSM_FP64, &bytes) == SSM_EUNSUPPORTED);
    // argument errors, detected before any GPU work
    ssm_problem p = {8, 8, 1, 4, 1.0, 0.3, 0.1, 0.02};
    ssm_problem bad[] = {{0, 8, 1, 4, 1, 0, 0, 0}, {8, 8, 1, 1, 1, 0, 0, 0}, {8, 8, 1, 4, 1.0 / 0.0 * 0.0, 0, 0, 0},
                         {2048, 8, 1, 4, 1, 0, 0, 0}, {8, 8, 17, 4, 1, 0, 0, 0}, {8, 8, 1, 2000, 1, 0, 0, 0}};
    for (const ssm_problem& b : bad) EXPECT(ssm_workspace_size(&b, 1, SSM_FP64, &bytes) != SSM_OK);
    EXPECT(ssm_workspace_size(&p, 1, 7, &bytes) == SSM_EINVAL);
    EXPECT(ssm_workspace_size(nullptr, 1, SSM_FP64, &bytes) == SSM_EINVAL);
    EXPECT(ssm_workspace_size(&p, 1, SSM_FP64, nullptr) == SSM_EINVAL);
    ssm_ctx* ctx = nullptr;
    EXPECT(ssm_create(&p, 1, SSM_FP64, nullptr, 0, nullptr, &ctx) == SSM_EINVAL && ctx == nullptr);
    EXPECT(ssm_create(&p, 1, SSM_FP64, reinterpret_cast<void*>(0x1001), 1 << 20, nullptr, &ctx) == SSM_EINVAL);
    EXPECT(ssm_create(&p, 1, SSM_FP64, reinterpret_cast<void*>(0x1000), 16, nullptr, &ctx) == SSM_EINVAL);
    EXPECT(ssm_create(&p, 1, SSM_FP64, reinterpret_cast<void*>(0x1000), 1 << 20, nullptr, nullptr) == SSM_EINVAL);
    EXPECT(ssm_destroy(nullptr) == SSM_OK);
    EXPECT(ssm_set_params(nullptr, 0, 1, 0, 0, 0) == SSM_EINVAL);
    EXPECT(ssm_iterate(nullptr, 1, 0.1, 0.0, nullptr) == SSM_EINVAL);
    EXPECT(ssm_eval(nullptr, nullptr, nullptr, nullptr, nullptr) == SSM_EINVAL);
    int32_t flags = 0;
    EXPECT(ssm_check(nullptr, &flags) == SSM_EINVAL);
    double e[4];
    EXPECT(ssm_eval_noalloc(nullptr, 1, SSM_FP64, e, nullptr, e, nullptr, nullptr) == SSM_EINVAL);
    EXPECT(ssm_eval_noalloc(&p, 0, SSM_FP64, e, nullptr, e, nullptr, nullptr) == SSM_EUNSUPPORTED);
    EXPECT(ssm_eval_noalloc(&p, 1, 9, e, nullptr, e, nullptr, nullptr) == SSM_EINVAL);
    std::printf("%d shapes planned, %d refused\n", ok, unsupported);
    if (fails) return 1;
    std::printf("OK\n");
    return 0;
}
