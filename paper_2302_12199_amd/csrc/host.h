// Host-side helpers shared by the drivers: error text, HIP error checks, the
// kernel-timing profiler and the per-round counter read-back.
#pragma once
#include <stdio.h>

#include "../../include/msf.h"
#include "common.h"

namespace msf {

void set_err(const char* what, hipError_t e);
void set_err_text(const char* text);
const char* last_err();

#define HIP_TRY(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) {                         \
            ::msf::set_err(#call, e_);                  \
            return MSF_EDEVICE;                         \
        }                                               \
    } while (0)

// Kernel families timed by the profiler.
enum KernelId { K_MINEDGE_R0, K_HOOK, K_JUMP, K_SCAN_ROOTS, K_LABEL, K_PASS, K_COMPACT,
                K_COMPOSE, K_FILL, K_PREP, K_SAMPLE, K_PARTITION, K_FILTER, K_PMAINT,
                K_MLP, K_BATCH, K_TAIL, K_PASS_R0, K_BK_INDEX, K_BK_SCATTER, K_BK_MIN,
                K_BK_LABEL, K_BK_PASS, K_DEDUP, K_COUNT };

bool prof_on();
int prof_begin(int kid, hipStream_t s);            // -1 when profiling is off
void prof_end(int h, hipStream_t s, double bytes);
void prof_add(int kid, double bytes);              // data-dependent bytes known later
void prof_resolve();                               // after a stream sync

// Copies the device control block to pinned host memory and waits.
int read_ctrl(const Ctrl* dctrl, Ctrl* host, hipStream_t s);
Ctrl* host_ctrl();                                 // pinned, one per process (guarded by caller)

}  // namespace msf
