// CSR checks shared by the solvers' BQ_F_VALIDATE paths.
#pragma once
#include <hip/hip_runtime.h>

#include "bq_device.hpp"

namespace {

// offsets[0] == 0, offsets[n] == m, offsets non-decreasing, every column in
// [0, n). `*bad` becomes non-zero on a defect (the caller clears it first).
__global__ void k_validate_csr(const long long* off, const int* col, int n, long long m,
                               unsigned long long* bad) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    bool b = false;
    if (tid == 0) b = off[0] != 0 || off[n] != m;
    for (long long v = tid; v < n; v += stride) b |= off[v + 1] < off[v];
    for (long long e = tid; e < m; e += stride) b |= (unsigned)col[e] >= (unsigned)n;
    if (__any(b) && bq::lane_id() == 0) bq::st_rlx(bad, 1ull);
}

}  // namespace
