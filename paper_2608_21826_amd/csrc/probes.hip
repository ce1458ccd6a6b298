// Roofline probes for the resources the queue-driven solver uses: HBM
// bandwidth (a streaming copy, also the calibration kernel for the HBM byte
// counters), the device's 64-bit atomic rate (random atomicMin over a table,
// and atomicAdd on a single contended word) and its rate of random coherent
// 64-bit loads (the solver's key checks).
#include <hip/hip_runtime.h>
#include <limits.h>

#include "bq_device.hpp"
#include "host_common.hpp"

namespace {

__global__ void k_probe_copy(const uint4* __restrict__ src, uint4* __restrict__ dst,
                             unsigned long long n16) {
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
         i += stride)
        dst[i] = src[i];
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long x) {
    // SplitMix64 finalizer
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// ops_per_lane returning 64-bit atomicMins at uniformly random slots of a
// table of 2^log_slots words
__global__ void k_probe_atomic_min(long long* table, unsigned log_slots,
                                   unsigned long long ops_per_lane, unsigned long long seed,
                                   unsigned long long* sink) {
    const unsigned long long tid = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned long long mask = (1ull << log_slots) - 1ull;
    long long acc = 0;
    for (unsigned long long i = 0; i < ops_per_lane; i += 4) {
        long long o[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const unsigned long long h = mix64(seed ^ (tid * 0x100000001B3ull + i + r));
            o[r] = __hip_atomic_fetch_min(&table[h & mask], (long long)(h >> 20), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
        }
        acc += o[0] ^ o[1] ^ o[2] ^ o[3];
    }
    if (acc == 0x123456789ll) sink[0] = 1;  // keep the results live
}

// every lane: ops_per_lane atomicAdds on one word (fully contended)
__global__ void k_probe_atomic_add1(unsigned long long* word, unsigned long long ops_per_lane) {
    unsigned long long acc = 0;
    for (unsigned long long i = 0; i < ops_per_lane; ++i)
        acc += __hip_atomic_fetch_add(word, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (acc == 1ull) word[1] = acc;
}

// one lane per wave: ops_per_lane atomicAdds on one word (the pattern of a
// queue's control words, where a wave's leader lane does the atomic)
__global__ void k_probe_atomic_add1_leader(unsigned long long* word,
                                           unsigned long long ops_per_lane) {
    if ((threadIdx.x & 63u) != 0u) return;
    unsigned long long acc = 0;
    for (unsigned long long i = 0; i < ops_per_lane; ++i)
        acc += __hip_atomic_fetch_add(word, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (acc == 1ull) word[1] = acc;
}

// ops_per_lane agent-scope 64-bit loads at uniformly random words of a table
// of 2^log_slots words, 8 in flight per lane (the solver's check before the
// atomic: a coherent load of a random key)
__global__ void k_probe_load_rand(const long long* table, unsigned log_slots,
                                  unsigned long long ops_per_lane, unsigned long long seed,
                                  unsigned long long* sink) {
    const unsigned long long tid = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned long long mask = (1ull << log_slots) - 1ull;
    long long acc = 0;
    for (unsigned long long i = 0; i < ops_per_lane; i += 8) {
        long long o[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const unsigned long long h = mix64(seed ^ (tid * 0x100000001B3ull + i + r));
            o[r] = __hip_atomic_load(&table[h & mask], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) acc += o[r];
    }
    if (acc == 0x123456789ll) sink[0] = 1;  // keep the results live
}

// latency: each lane runs a dependent chain of ops_per_lane operations at
// random words of a table of 2^log_slots words (the next address depends on
// the last result); mode 0 agent-scope loads, mode 1 returning atomicMins
// whose value never changes the word (so the table stays as initialized)
__global__ void k_probe_chain(long long* table, unsigned log_slots,
                              unsigned long long ops_per_lane, unsigned mode,
                              unsigned long long* sink) {
    const unsigned long long tid = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned long long mask = (1ull << log_slots) - 1ull;
    unsigned long long x = mix64(tid);
    long long acc = 0;
    for (unsigned long long i = 0; i < ops_per_lane; ++i) {
        long long v;
        if (mode == 0)
            v = __hip_atomic_load(&table[x & mask], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        else
            v = __hip_atomic_fetch_min(&table[x & mask], LLONG_MAX, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        acc += v;
        x = mix64(x ^ (unsigned long long)v);
    }
    if (acc == 0x123456789ll) sink[0] = 1;  // keep the results live
}

// the wave primitives on n = grid * block inputs, over each wave's 64:
// out[4i] = inclusive sum scan, out[4i+1] = inclusive max scan (unsigned),
// out[4i+2] = the value of the lane below (0 for lane 0), out[4i+3] = the
// value of lane 63
__global__ void k_probe_wave_scan(const int* in, int* out) {
    const unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int x = in[i];
    out[4 * i] = bq::wave_incl_scan(x);
    out[4 * i + 1] = (int)bq::wave_incl_max((unsigned)x);
    out[4 * i + 2] = (int)bq::wave_shr1((unsigned)x);
    out[4 * i + 3] = bq::lane63(x);
}

// one lane per wave: ops_per_lane agent-scope loads of one word
__global__ void k_probe_load1_leader(unsigned long long* word, unsigned long long ops_per_lane) {
    if ((threadIdx.x & 63u) != 0u) return;
    unsigned long long acc = 0;
    for (unsigned long long i = 0; i < ops_per_lane; ++i)
        acc += __hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + i;
    if (acc == 1ull) word[1] = acc;
}

}  // namespace

extern "C" {

bq_status bq_probe(int32_t kind, void* d_a, void* d_b, uint64_t size, uint64_t ops_per_lane,
                   int32_t grid, int32_t block, double* h_ms, void* stream) {
    if (!d_a || !h_ms || grid < 1 || block < 64 || block > 1024) return BQ_EINVAL;
    hipStream_t s = bqh::as_stream(stream);
    hipEvent_t e0, e1;
    BQ_HIP_TRY(hipEventCreate(&e0));
    BQ_HIP_TRY(hipEventCreate(&e1));
    BQ_HIP_TRY(hipEventRecord(e0, s));
    switch (kind) {
        case 0:  // copy size bytes from d_a to d_b (size multiple of 16)
            if (!d_b || (size & 15ull)) return BQ_EINVAL;
            hipLaunchKernelGGL(k_probe_copy, dim3(grid), dim3(block), 0, s, (const uint4*)d_a,
                               (uint4*)d_b, (unsigned long long)(size / 16ull));
            break;
        case 1: {  // random atomicMin over a table of size (power of two) words
            if (!d_b || size < 2 || (size & (size - 1))) return BQ_EINVAL;
            unsigned lg = bqh::log2_exact(size);
            hipLaunchKernelGGL(k_probe_atomic_min, dim3(grid), dim3(block), 0, s, (long long*)d_a,
                               lg, (unsigned long long)ops_per_lane, 0x5EEDull,
                               (unsigned long long*)d_b);
            break;
        }
        case 2:  // single contended word (needs 2 words of space)
            hipLaunchKernelGGL(k_probe_atomic_add1, dim3(grid), dim3(block), 0, s,
                               (unsigned long long*)d_a, (unsigned long long)ops_per_lane);
            break;
        case 3:  // one lane per wave, atomicAdd on the single word d_a[0]
            hipLaunchKernelGGL(k_probe_atomic_add1_leader, dim3(grid), dim3(block), 0, s,
                               (unsigned long long*)d_a, (unsigned long long)ops_per_lane);
            break;
        case 4:  // one lane per wave, agent-scope loads of d_a[0]
            hipLaunchKernelGGL(k_probe_load1_leader, dim3(grid), dim3(block), 0, s,
                               (unsigned long long*)d_a, (unsigned long long)ops_per_lane);
            break;
        case 5: {  // random agent-scope loads over a table of size (power of two) words
            if (!d_b || size < 2 || (size & (size - 1)) || (ops_per_lane & 7ull)) return BQ_EINVAL;
            unsigned lg = bqh::log2_exact(size);
            hipLaunchKernelGGL(k_probe_load_rand, dim3(grid), dim3(block), 0, s,
                               (const long long*)d_a, lg, (unsigned long long)ops_per_lane,
                               0x5EEDull, (unsigned long long*)d_b);
            break;
        }
        case 8:  // wave primitives: d_a int32[size] in, d_b int32[4 * size] out
            if (!d_b || size != (uint64_t)grid * (uint64_t)block || (block & 63)) return BQ_EINVAL;
            hipLaunchKernelGGL(k_probe_wave_scan, dim3(grid), dim3(block), 0, s, (const int*)d_a,
                               (int*)d_b);
            break;
        case 6:    // latency chains of agent-scope loads (see k_probe_chain)
        case 7: {  // latency chains of returning atomicMins
            if (!d_b || size < 2 || (size & (size - 1))) return BQ_EINVAL;
            unsigned lg = bqh::log2_exact(size);
            hipLaunchKernelGGL(k_probe_chain, dim3(grid), dim3(block), 0, s, (long long*)d_a, lg,
                               (unsigned long long)ops_per_lane, (unsigned)(kind - 6),
                               (unsigned long long*)d_b);
            break;
        }
        default:
            return BQ_EINVAL;
    }
    BQ_HIP_TRY(hipGetLastError());
    BQ_HIP_TRY(hipEventRecord(e1, s));
    BQ_HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    BQ_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    *h_ms = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return BQ_OK;
}

}  // extern "C"
