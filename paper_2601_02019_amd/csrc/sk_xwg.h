// sk_xwg.h -- exchanges between the workgroups ("members") that share one
// problem in the multi-workgroup kernels (the tridiagonal reduction and
// CholeskyQR).
//
// A member publishes data with plain stores from one wavefront, one release
// fence at agent scope and a flag store; a reader polls the flag with
// relaxed loads, then one acquire fence, then plain loads.  A flag holds
// (epoch << 32) | stage: the epoch is taken once per launch from one
// process-wide counter shared by every kernel that uses a sketch's flags, and
// stages grow within a launch, so flags left by earlier launches (of any of
// these kernels) never satisfy a wait.  Waits are bounded: after XWG_POLLS
// polls they give up and the caller reports the failure (no wait can hang).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sk {

constexpr unsigned XWG_POLLS = 1u << 22;

// Next launch epoch (host).
uint64_t xwg_next_epoch();

__device__ __forceinline__ uint64_t xwg_flag(uint64_t epoch, unsigned stage) {
    return (epoch << 32) | (uint64_t)stage;
}

// Called by every lane of one wavefront after its stores: makes them visible
// at agent scope, then sets the flag.
__device__ __forceinline__ void xwg_publish(uint64_t* flag, uint64_t value) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if ((threadIdx.x & 63) == 0) __hip_atomic_store(flag, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Called by every lane of one wavefront: waits until flags[f0 + i] >= value
// for every i < count (count <= 64), then acquires.  Returns false on a
// timeout.
__device__ __forceinline__ bool xwg_wait(const uint64_t* flags, int count, uint64_t value) {
    const int lane = threadIdx.x & 63;
    unsigned polls = 0;
    bool ok = true;
    while (true) {
        const uint64_t f =
            lane < count ? __hip_atomic_load(flags + lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : value;
        if (__all(f >= value)) break;
        if (++polls > XWG_POLLS) {
            ok = false;
            break;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok;
}

}  // namespace sk
