// mr_probe.hip -- device atomic-rate probe of libmrecon (mr_probe_atomics in
// include/mr.h).
//
// The queue phase spends its time in device-scope atomics on scattered
// addresses: a load of a pixel's word, then a compare-and-swap whose result
// decides the next step, plus fetch-or and exchange on frontier bits and
// flags. MI355X's eight L2s are not coherent with one another, so every such
// atomic is executed beyond them, and no peak rate for it is published. This
// probe measures the ceiling the way the paper's atomic-throughput tables do
// (Table IV): many waves, each lane updating pseudo-random words of one
// buffer, with
//  - MR_PROBE_ADD: relaxed device-scope fetch-add of 1, result unused;
//  - MR_PROBE_CAS: relaxed device-scope load, then compare-and-swap of the
//    value read to that value + 1, retried with the returned value until it
//    lands (the queue's raise pattern: each lane waits for its result).
// Both add exactly one to some word per operation, so the buffer's sum grows
// by waves * 64 * per_lane and the caller can check that every operation
// happened. The probe is measurement support; no call of the reconstruction
// uses it.
#include "mr_internal.h"

using namespace mr;

namespace {

// MurmurHash3's 32-bit finalizer (Appleby): a bijective mixer, used here only
// to spread the addresses.
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

template <int KIND>
__global__ __launch_bounds__(64) void k_probe_atomics(uint32_t *__restrict__ words, uint32_t mask,
                                                      int32_t per_lane, uint32_t seed) {
    const uint32_t gid = blockIdx.x * 64u + threadIdx.x;
    const uint32_t base = fmix32(gid ^ seed);
    for (int32_t i = 0; i < per_lane; ++i) {
        uint32_t *p = words + (fmix32(base + (uint32_t)i * 0x9e3779b9u) & mask);
        if (KIND == MR_PROBE_ADD) {
            __hip_atomic_fetch_add(p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            uint32_t seen = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            while (!__hip_atomic_compare_exchange_strong(p, &seen, seen + 1u, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT)) {
            }
        }
    }
}

} // namespace

extern "C" int mr_probe_atomics(void *words, size_t n_words, int kind, int32_t per_lane,
                                int32_t waves, uint32_t seed, void *stream) {
    clear_error();
    if (!words || ((uintptr_t)words & 3) != 0 || n_words < 64 || (n_words & (n_words - 1)) != 0 ||
        n_words > (1ull << 32))
        return set_error(MR_EINVAL, "probe: words must be non-null and 4-byte aligned, n_words a "
                                    "power of two in [64, 2^32]");
    if (kind != MR_PROBE_ADD && kind != MR_PROBE_CAS)
        return set_error(MR_EINVAL, "probe: kind must be MR_PROBE_ADD or MR_PROBE_CAS");
    if (per_lane < 1 || per_lane > (1 << 16) || waves < 1 || waves > (1 << 20))
        return set_error(MR_EINVAL, "probe: per_lane must be in [1, 65536], waves in [1, 2^20]");
    const uint32_t mask = (uint32_t)(n_words - 1);
    hipStream_t s = (hipStream_t)stream;
    if (kind == MR_PROBE_ADD)
        hipLaunchKernelGGL((k_probe_atomics<MR_PROBE_ADD>), dim3((unsigned)waves), dim3(64), 0, s,
                           (uint32_t *)words, mask, per_lane, seed);
    else
        hipLaunchKernelGGL((k_probe_atomics<MR_PROBE_CAS>), dim3((unsigned)waves), dim3(64), 0, s,
                           (uint32_t *)words, mask, per_lane, seed);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(MR_EHIP, hipGetErrorString(e));
    return MR_OK;
}
