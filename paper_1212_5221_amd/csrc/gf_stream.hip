// gf_stream.hip -- plain streaming kernels that measure the memory ceiling
// the half-sweep is compared with: a copy that reads and writes every byte
// once (what one half-sweep does to the link planes) and a read-only pass,
// both with 16-byte vector accesses, UNROLL independent loads in flight per
// lane, and optional non-temporal loads or stores.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gf.h"

namespace {

// a native 4-float vector (the non-temporal builtins take vector types)
typedef float f4v __attribute__((ext_vector_type(4)));

constexpr int SBLOCK = 256;
constexpr int UNROLL = 4;

template <bool NTL, bool NTS>
__global__ __launch_bounds__(SBLOCK) void k_stream_copy(const f4v *src, f4v *dst, int64_t n) {
    const int64_t base = (int64_t)blockIdx.x * SBLOCK * UNROLL + threadIdx.x;
    f4v v[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
        const int64_t i = base + (int64_t)u * SBLOCK;
        if (i < n) {
            if constexpr (NTL)
                v[u] = __builtin_nontemporal_load(src + i);
            else
                v[u] = src[i];
        }
    }
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
        const int64_t i = base + (int64_t)u * SBLOCK;
        if (i < n) {
            if constexpr (NTS)
                __builtin_nontemporal_store(v[u], dst + i);
            else
                dst[i] = v[u];
        }
    }
}

// read-only: each block writes the sum of what it read to sink[blockIdx.x]
__global__ __launch_bounds__(SBLOCK) void k_stream_read(const f4v *src, float *sink, int64_t n) {
    __shared__ float sh[SBLOCK / 64];
    const int64_t base = (int64_t)blockIdx.x * SBLOCK * UNROLL + threadIdx.x;
    float acc = 0.0f;
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
        const int64_t i = base + (int64_t)u * SBLOCK;
        if (i < n) {
            const f4v v = src[i];
            acc += (v.x + v.y) + (v.z + v.w);
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) sink[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

}  // namespace

extern "C" {

int gf_stream_blocks(size_t bytes, int64_t *blocks) {
    if (!blocks || bytes % 16) return GF_E_INVALID;
    const int64_t n = (int64_t)(bytes / 16);
    *blocks = (n + (int64_t)SBLOCK * UNROLL - 1) / ((int64_t)SBLOCK * UNROLL);
    return GF_OK;
}

int gf_stream(void *hip_stream, int kind, void *dst, const void *src, size_t bytes) {
    if (!dst || !src || bytes == 0 || bytes % 16) return GF_E_INVALID;
    const int64_t n = (int64_t)(bytes / 16);
    const int64_t nb = (n + (int64_t)SBLOCK * UNROLL - 1) / ((int64_t)SBLOCK * UNROLL);
    if (nb > 0x7fffffff) return GF_E_INVALID;
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const f4v *a = static_cast<const f4v *>(src);
    f4v *b = static_cast<f4v *>(dst);
    switch (kind) {
        case GF_STREAM_COPY:
            k_stream_copy<false, false><<<(unsigned)nb, SBLOCK, 0, s>>>(a, b, n);
            break;
        case GF_STREAM_COPY_NT_LOAD:
            k_stream_copy<true, false><<<(unsigned)nb, SBLOCK, 0, s>>>(a, b, n);
            break;
        case GF_STREAM_COPY_NT_STORE:
            k_stream_copy<false, true><<<(unsigned)nb, SBLOCK, 0, s>>>(a, b, n);
            break;
        case GF_STREAM_COPY_NT:
            k_stream_copy<true, true><<<(unsigned)nb, SBLOCK, 0, s>>>(a, b, n);
            break;
        case GF_STREAM_READ:
            k_stream_read<<<(unsigned)nb, SBLOCK, 0, s>>>(a, static_cast<float *>(dst), n);
            break;
        default:
            return GF_E_INVALID;
    }
    return hipGetLastError() == hipSuccess ? GF_OK : GF_E_HIP;
}

}  // extern "C"
