// Caller atom order <-> stream order of the packed Hamiltonian.
//
// The builder stores atoms in the order that makes the H.x kernel's
// neighbour gathers contiguous (locality_order in builder.cpp); vectors
// crossing the C ABI are in the caller's order.  These kernels move whole
// atom rows (n_o scalars, complex interleaved) between the two orders with
// 4-byte words, one thread per word, grid-stride.
#include "tbh_internal.h"

namespace tbh {

namespace {

constexpr int TPB = 256;

int64_t grid_of(int64_t n) {
    const int64_t g = (n + TPB - 1) / TPB;
    return g < 1 ? 1 : (g > 65536 ? 65536 : g);
}

// dst[k][w] = src[perm[k]][w]
__global__ void k_rows_to_stream(int64_t n, const int64_t* __restrict__ perm, int64_t words,
                                 const uint32_t* __restrict__ src, uint32_t* __restrict__ dst) {
    const int64_t total = n * words;
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < total; i += int64_t(gridDim.x) * TPB) {
        const int64_t k = i / words, w = i - k * words;
        dst[i] = src[perm[k] * words + w];
    }
}

// dst[perm[k]][w] = src[k][w]
__global__ void k_rows_to_caller(int64_t n, const int64_t* __restrict__ perm, int64_t words,
                                 const uint32_t* __restrict__ src, uint32_t* __restrict__ dst) {
    const int64_t total = n * words;
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < total; i += int64_t(gridDim.x) * TPB) {
        const int64_t k = i / words, w = i - k * words;
        dst[perm[k] * words + w] = src[i];
    }
}

// dst[perm[k]][e] = scale * src[k][e] (FP64)
__global__ void k_rows_to_caller_f64(int64_t n, const int64_t* __restrict__ perm, int row, double scale,
                                     const double* __restrict__ src, double* __restrict__ dst) {
    const int64_t total = n * row;
    for (int64_t i = blockIdx.x * int64_t(TPB) + threadIdx.x; i < total; i += int64_t(gridDim.x) * TPB) {
        const int64_t k = i / row, e = i - k * row;
        dst[perm[k] * row + e] = scale * src[i];
    }
}

}  // namespace

void rows_to_stream(hipStream_t st, int64_t n, const int64_t* perm_d, size_t row_bytes, const void* src,
                    void* dst) {
    TBH_REQUIRE(row_bytes % 4 == 0, "row size must be a multiple of 4 bytes");
    const int64_t words = int64_t(row_bytes / 4);
    hipLaunchKernelGGL(k_rows_to_stream, dim3(grid_of(n * words)), dim3(TPB), 0, st, n, perm_d, words,
                       static_cast<const uint32_t*>(src), static_cast<uint32_t*>(dst));
    TBH_HIP(hipGetLastError());
}

void rows_to_caller(hipStream_t st, int64_t n, const int64_t* perm_d, size_t row_bytes, const void* src,
                    void* dst) {
    TBH_REQUIRE(row_bytes % 4 == 0, "row size must be a multiple of 4 bytes");
    const int64_t words = int64_t(row_bytes / 4);
    hipLaunchKernelGGL(k_rows_to_caller, dim3(grid_of(n * words)), dim3(TPB), 0, st, n, perm_d, words,
                       static_cast<const uint32_t*>(src), static_cast<uint32_t*>(dst));
    TBH_HIP(hipGetLastError());
}

void rows_to_caller_f64(hipStream_t st, int64_t n, const int64_t* perm_d, int row_doubles, double scale,
                        const double* src, double* dst) {
    hipLaunchKernelGGL(k_rows_to_caller_f64, dim3(grid_of(n * row_doubles)), dim3(TPB), 0, st, n, perm_d,
                       row_doubles, scale, src, dst);
    TBH_HIP(hipGetLastError());
}

}  // namespace tbh
