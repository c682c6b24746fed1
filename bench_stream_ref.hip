// bench_stream_ref.hip -- a hand-written HBM streaming reference for bench.py
// (--stream-reference): how many bytes per second plain 16-byte buffer loads
// and stores move on this chip, with the default cache policy and with the
// non-temporal and coherence bits, for a read, a write and a copy.  It sets
// the ceiling against which the HBM-bound LW-ACM kernels are read: the
// single-step tile kernel moves the same 16-byte node records.  Measurement
// code only; not part of the LW-ACM library.
//
//     int stream_ref_run(int kind, int policy, void *dst, const void *src,
//                        unsigned bytes, int grid, int reps, float *ms)
//
// kind 0 copy (src -> dst), 1 read (src; dst takes a guard word that keeps
// the loads and is practically never written), 2 write (dst); policy: the cache-
// policy bits of the loads and stores (gfx950: bit 0 sc0, bit 1 nt, bit 4
// sc1; one of 0, 1, 2, 16, 17, 18); bytes a multiple of 16 below 2^32; grid
// workgroups of 256 threads.  Times `reps` launches (after two untimed ones)
// on the null stream with HIP events and writes the mean milliseconds per
// launch.  Returns 0, or -1 for an argument out of range, -2 for a HIP error.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void *p, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes,
                                             0x00020000);
}

// four independent 16-byte accesses per thread and pass, grid-strided
template <int P>
__global__ __launch_bounds__(256) void k_copy(const void *src, void *dst, unsigned bytes)
{
    const auto rs = rsrc(src, bytes), rd = rsrc(dst, bytes);
    const unsigned n16 = bytes / 16u, g = gridDim.x * 256u;
    for (unsigned i = blockIdx.x * 256u + threadIdx.x; i < n16; i += 4u * g) {
        u32x4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const unsigned j = i + (unsigned)k * g;
            v[k] = j < n16 ? __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(
                                                          rs, j * 16u, 0, P))
                           : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const unsigned j = i + (unsigned)k * g;
            if (j < n16) __builtin_amdgcn_raw_buffer_store_b128(v[k], rd, j * 16u, 0, P);
        }
    }
}

template <int P>
__global__ __launch_bounds__(256) void k_read(const void *src, unsigned bytes, unsigned *sink)
{
    const auto rs = rsrc(src, bytes);
    const unsigned n16 = bytes / 16u, g = gridDim.x * 256u;
    unsigned acc = 0u;
    for (unsigned i = blockIdx.x * 256u + threadIdx.x; i < n16; i += 4u * g) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const unsigned j = i + (unsigned)k * g;
            if (j < n16) {
                const u32x4 v = __builtin_bit_cast(
                    u32x4, __builtin_amdgcn_raw_buffer_load_b128(rs, j * 16u, 0, P));
                acc ^= v.x ^ v.y ^ v.z ^ v.w;
            }
        }
    }
    if (acc == 0x9e3779b9u) sink[0] = acc;  // keeps the loads; practically never taken
}

template <int P>
__global__ __launch_bounds__(256) void k_write(void *dst, unsigned bytes)
{
    const auto rd = rsrc(dst, bytes);
    const unsigned n16 = bytes / 16u, g = gridDim.x * 256u;
    const u32x4 v = {1u, 2u, 3u, 4u};
    for (unsigned i = blockIdx.x * 256u + threadIdx.x; i < n16; i += g)
        __builtin_amdgcn_raw_buffer_store_b128(v, rd, i * 16u, 0, P);
}

template <int P>
void launch(int kind, void *dst, const void *src, unsigned bytes, int grid, unsigned *sink)
{
    if (kind == 0)
        k_copy<P><<<grid, 256>>>(src, dst, bytes);
    else if (kind == 1)
        k_read<P><<<grid, 256>>>(src, bytes, sink);
    else
        k_write<P><<<grid, 256>>>(dst, bytes);
}

}  // namespace

extern "C" int stream_ref_run(int kind, int policy, void *dst, const void *src, unsigned bytes,
                              int grid, int reps, float *ms)
{
    if (kind < 0 || kind > 2 || bytes < 16u || bytes % 16u || grid < 1 || grid > (1 << 20) ||
        reps < 1 || !ms || !dst || (kind != 2 && !src))
        return -1;
    auto go = [&]() {
        unsigned *sink = static_cast<unsigned *>(dst);  // the read's guard word
        switch (policy) {
        case 0: launch<0>(kind, dst, src, bytes, grid, sink); break;
        case 1: launch<1>(kind, dst, src, bytes, grid, sink); break;
        case 2: launch<2>(kind, dst, src, bytes, grid, sink); break;
        case 16: launch<16>(kind, dst, src, bytes, grid, sink); break;
        case 17: launch<17>(kind, dst, src, bytes, grid, sink); break;
        case 18: launch<18>(kind, dst, src, bytes, grid, sink); break;
        default: return false;
        }
        return true;
    };
    if (!go() || !go()) return -1;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -2;
    hipError_t e = hipEventRecord(a, 0);
    for (int r = 0; r < reps; ++r) go();
    if (e == hipSuccess) e = hipEventRecord(b, 0);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (e != hipSuccess || hipGetLastError() != hipSuccess) return -2;
    *ms = t / (float)reps;
    return 0;
}
