// Host-side helpers shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bq.h"
#include "bq_device.hpp"

namespace bqh {

#define BQ_HIP_TRY(expr)                              \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) {                       \
            bqh::note_hip_error(e_, #expr, __LINE__); \
            return BQ_EHIP;                           \
        }                                             \
    } while (0)

void note_hip_error(hipError_t e, const char* what, int line);

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Resolved launch shape.
struct Launch {
    int wg_size;
    int wg_count;
    int batch;                 // ticket_batch b
    int row_chunk;             // solver row chunk (edges)
    int segments;              // solver queue segments (0 = default)
    int bucket_width;          // solver near / far buckets (0 = off)
    uint32_t flags;
    unsigned long long limit;  // watchdog, 100 MHz ticks
};

int device_cus();

// Fill defaults: wg_size 256, batch 1, watchdog 2 s; wg_count 0 -> default_wgs.
Launch resolve(const bq_launch* l, int default_wgs);

inline uint32_t log2_exact(unsigned long long x) {
    uint32_t r = 0;
    while ((1ull << r) < x) ++r;
    return r;
}

}  // namespace bqh
