// Batched solver: arguments shared by the kernel (batch.hip) and its C ABI
// (batch_api.hip).
#pragma once
#include "common.h"

namespace msf {

struct BatchArgs {
    const int32_t* u;
    const int32_t* v;
    const uint32_t* w;
    const int64_t* eoff;     // [G + 1] edge offsets
    const int64_t* voff;     // [G + 1] vertex offsets
    int64_t G;
    const int32_t* order;    // [G] processing order, or null
    uint8_t* mask;           // [eoff[G]]
    uint64_t* totals;        // [G]; ~0 for a graph with invalid input
    uint64_t* ticks;         // [G + 1] completion clock per graph, [G] = batch start; or null
    char* scratch;           // one slot per workgroup
    size_t slot_bytes;
    int64_t nmax;            // vertices per graph the slots are sized for
    uint32_t* queue;         // work counter, zeroed by the launch
    int lds_n;               // graphs with n <= lds_n keep their state in LDS
};

int launch_batch(const BatchArgs& A, int block, int workgroups, hipStream_t s);
size_t batch_slot_bytes(int64_t nmax);
bool batch_allow_lds(int block, size_t bytes);

}  // namespace msf
