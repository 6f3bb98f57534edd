// Host-side checks of the C ABI, built with AddressSanitizer and
// UndefinedBehaviorSanitizer on the host code (tests/test_host_sanitizers.py):
// argument validation, workspace sizing, status strings and option checks --
// every path that runs before anything is launched, so no GPU is needed.
#include <stdio.h>
#include <stdint.h>
#include <string.h>

#include "msf.h"

static int failures = 0;
#define CHECK(cond)                                                     \
    do {                                                                \
        if (!(cond)) { fprintf(stderr, "FAILED: %s (line %d)\n", #cond, __LINE__); ++failures; } \
    } while (0)

int main() {
    const void* F = (const void*)0x1000;          // never dereferenced
    uint64_t total = 0;
    msf_options o;
    memset(&o, 0, sizeof o);
    // sizes and pointers
    CHECK(msf_compute((const int32_t*)F, (const int32_t*)F, (const uint32_t*)F, -1, 5,
                      (uint8_t*)F, &total, nullptr, 0, nullptr, nullptr, nullptr) == MSF_EINVAL);
    CHECK(msf_compute((const int32_t*)F, (const int32_t*)F, (const uint32_t*)F, 3, 0,
                      (uint8_t*)F, &total, nullptr, 0, nullptr, nullptr, nullptr) == MSF_EINVAL);
    CHECK(msf_compute(nullptr, (const int32_t*)F, (const uint32_t*)F, 3, 5, (uint8_t*)F, &total,
                      nullptr, 0, nullptr, nullptr, nullptr) == MSF_EINVAL);
    // options
    for (int k = 0; k < 7; ++k) {
        msf_options b = o;
        if (k == 0) b.algo = 7;
        if (k == 1) b.quantile = 2.f;
        if (k == 2) b.dedup_policy = 9;
        if (k == 3) b.split_retries = -1;
        if (k == 4) b.defer_edges = -5;
        if (k == 5) b.reserved[2] = 1;
        if (k == 6) b.tail_threshold = 2000;
        CHECK(msf_compute((const int32_t*)F, (const int32_t*)F, (const uint32_t*)F, 3, 5,
                          (uint8_t*)F, &total, nullptr, 0, nullptr, &b, nullptr) == MSF_EINVAL);
    }
    // workspace sizes: monotone, and every policy and algorithm sized
    for (int algo = 0; algo < 2; ++algo)
        for (int d = 0; d < 4; ++d) {
            msf_options b = o;
            b.algo = algo;
            b.dedup_policy = d;
            const size_t a = msf_workspace_bytes(1000, 100, &b);
            const size_t c = msf_workspace_bytes(1 << 22, 1 << 21, &b);
            CHECK(a > 0 && c > a);
        }
    // too small and misaligned workspaces
    const size_t need = msf_workspace_bytes(10, 5, nullptr);
    CHECK(msf_compute((const int32_t*)F, (const int32_t*)F, (const uint32_t*)F, 10, 5,
                      (uint8_t*)F, &total, (void*)F, need - 1, nullptr, nullptr, nullptr) ==
          MSF_EWORKSPACE);
    CHECK(msf_compute((const int32_t*)F, (const int32_t*)F, (const uint32_t*)F, 10, 5,
                      (uint8_t*)F, &total, (void*)((const char*)F + 16), need, nullptr, nullptr,
                      nullptr) == MSF_EINVAL);
    // the empty graph, with statistics
    msf_stats st;
    CHECK(msf_compute(nullptr, nullptr, nullptr, 0, 7, nullptr, &total, nullptr, 0, nullptr,
                      nullptr, &st) == MSF_OK && total == 0 && st.base_cases == 1);
    // no-allocation entry point: sizes beyond its scratch are rejected first
    CHECK(msf_compute_noalloc((const int32_t*)F, (const int32_t*)F, (const uint32_t*)F, 4 << 20,
                              1 << 20, (uint8_t*)F, &total, nullptr, nullptr, nullptr) ==
          MSF_EWORKSPACE);
    CHECK(strstr(msf_last_error(), "static scratch") != nullptr);
    // batched options
    msf_batch_options bo;
    memset(&bo, 0, sizeof bo);
    bo.block = 300;
    CHECK(msf_compute_batched((const int32_t*)F, (const int32_t*)F, (const uint32_t*)F,
                              (const int64_t*)F, (const int64_t*)F, 3, 10, nullptr, (uint8_t*)F,
                              (uint64_t*)F, nullptr, (void*)F, 1 << 30, nullptr, &bo) ==
          MSF_EINVAL);
    memset(&bo, 0, sizeof bo);
    bo.wave_min = 1;
    CHECK(msf_compute_batched((const int32_t*)F, (const int32_t*)F, (const uint32_t*)F,
                              (const int64_t*)F, (const int64_t*)F, 3, 10, nullptr, (uint8_t*)F,
                              (uint64_t*)F, nullptr, (void*)F, 1 << 30, nullptr, &bo) ==
          MSF_EINVAL);
    // pivot network blobs that must be refused before any device work
    unsigned char blob[64];
    memset(blob, 0, sizeof blob);
    CHECK(msf_pivot_model_load(blob, sizeof blob) == MSF_EINVAL);
    CHECK(msf_pivot_model_load(nullptr, 0) == MSF_EINVAL);
    // status strings
    for (int s = -7; s <= 1; ++s) CHECK(msf_status_string(s) != nullptr);
    CHECK(msf_mlp_param_count() == 64 * 16 + 64 + 64 * 64 + 64 + 64 + 1);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("host ABI checks passed\n");
    return 0;
}
