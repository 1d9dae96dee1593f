// mr_probe.hip -- device probes of libmrecon: the atomic-rate probe
// (mr_probe_atomics) and the random-access probe (mr_probe_random), both in
// include/mr.h.
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
// happened.
//
// The random-access probe follows the paper's micro-benchmark for irregular
// access (Sec. V-A, Table III): plain reads or writes of 32-bit words of a
// matrix at positions that a separate index vector holds, filled on the host.
// The index vector streams in order; only the matrix accesses scatter, as the
// queue phase's and the distance transform's plain loads of pixels do.
// Neither probe is used by any call of the reconstruction: they are
// measurement support.
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

// Lane g of the grid takes the operations g, g + S, g + 2S, ... (S = the
// grid's lane count), eight at a time while all eight exist so that eight
// index loads and then eight scattered accesses are in flight per lane.
// Reads add the words they fetch into the lane's 32-bit sum (wrapping), which
// the lane writes to sums[g]; writes store the operation's number i (the
// low 32 bits) at its position. Positions are the indices modulo the matrix
// size, a power of two, so every access stays inside the matrix.
template <int KIND>
__global__ __launch_bounds__(64) void k_probe_random(uint32_t *__restrict__ words, uint32_t mask,
                                                     const uint32_t *__restrict__ idx, uint64_t n,
                                                     uint32_t *__restrict__ sums) {
    constexpr int U = 8;
    const uint64_t g = (uint64_t)blockIdx.x * 64u + threadIdx.x;
    const uint64_t S = (uint64_t)gridDim.x * 64u;
    uint32_t acc = 0;
    uint64_t i = g;
    for (; i + (U - 1) * S < n; i += U * S) {
        uint32_t p[U];
#pragma unroll
        for (int u = 0; u < U; ++u) p[u] = idx[i + u * S] & mask;
        if (KIND == MR_RANDOM_READ) {
            uint32_t v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) v[u] = words[p[u]];
#pragma unroll
            for (int u = 0; u < U; ++u) acc += v[u];
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) words[p[u]] = (uint32_t)(i + u * S);
        }
    }
    for (; i < n; i += S) {
        const uint32_t p = idx[i] & mask;
        if (KIND == MR_RANDOM_READ)
            acc += words[p];
        else
            words[p] = (uint32_t)i;
    }
    if (KIND == MR_RANDOM_READ) sums[g] = acc;
}

} // namespace

extern "C" int mr_probe_random(void *words, size_t n_words, const void *indices, size_t n_ops,
                               int kind, int32_t waves, void *sums, void *stream) {
    clear_error();
    if (!words || ((uintptr_t)words & 3) != 0 || n_words < 64 || (n_words & (n_words - 1)) != 0 ||
        n_words > (1ull << 32))
        return set_error(MR_EINVAL, "probe: words must be non-null and 4-byte aligned, n_words a "
                                    "power of two in [64, 2^32]");
    if (kind != MR_RANDOM_READ && kind != MR_RANDOM_WRITE)
        return set_error(MR_EINVAL, "probe: kind must be MR_RANDOM_READ or MR_RANDOM_WRITE");
    if (!indices || ((uintptr_t)indices & 3) != 0 || n_ops < 1 || n_ops > (1ull << 34))
        return set_error(MR_EINVAL, "probe: indices must be non-null and 4-byte aligned, n_ops "
                                    "in [1, 2^34]");
    if (waves < 1 || waves > (1 << 20))
        return set_error(MR_EINVAL, "probe: waves must be in [1, 2^20]");
    if (kind == MR_RANDOM_READ && (!sums || ((uintptr_t)sums & 3) != 0))
        return set_error(MR_EINVAL, "probe: a read needs sums (4-byte aligned, waves * 64 words)");
    const uint32_t mask = (uint32_t)(n_words - 1);
    hipStream_t s = (hipStream_t)stream;
    if (kind == MR_RANDOM_READ)
        hipLaunchKernelGGL((k_probe_random<MR_RANDOM_READ>), dim3((unsigned)waves), dim3(64), 0, s,
                           (uint32_t *)words, mask, (const uint32_t *)indices, (uint64_t)n_ops,
                           (uint32_t *)sums);
    else
        hipLaunchKernelGGL((k_probe_random<MR_RANDOM_WRITE>), dim3((unsigned)waves), dim3(64), 0,
                           s, (uint32_t *)words, mask, (const uint32_t *)indices,
                           (uint64_t)n_ops, (uint32_t *)nullptr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(MR_EHIP, hipGetErrorString(e));
    return MR_OK;
}

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
