// Measurement aid: the bandwidth a random gather of 64-byte chunks achieves on a working set
// of a given size, i.e. the peak of whichever level (L2, Infinity Cache, HBM) serves a working
// set that size.  It mirrors the replica kernel's access: a quad of lanes reads one chunk as
// four 16-byte loads, and chunk addresses are data-independent and scattered.
#include "gff_internal.hpp"

namespace gff {

// Quad q of the grid draws chunk indices from a xorshift32 sequence seeded by (q, seed); lane
// s of the quad reads the chunk's 16-byte word s.  Each lane XORs everything it read into
// sink[thread], which keeps every load live.
__global__ void __launch_bounds__(256) k_gather_probe(const uint4 *buf, unsigned n_chunks, int iters, unsigned seed,
                                                      unsigned *sink) {
    const unsigned gid = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned quad = gid >> 2, s = gid & 3;
    unsigned h = (quad * 0x9E3779B9u) ^ seed;
    if (h == 0u) h = 0x6D2B79F5u;                   // xorshift has no zero state
    unsigned acc0 = 0u, acc1 = 0u;
    int i = 0;
    for (; i + 1 < iters; i += 2) {                 // two gathers in flight per lane
        h ^= h << 13; h ^= h >> 17; h ^= h << 5;
        const unsigned c0 = __umulhi(h, n_chunks);
        h ^= h << 13; h ^= h >> 17; h ^= h << 5;
        const unsigned c1 = __umulhi(h, n_chunks);
        const uint4 v0 = buf[(size_t)c0 * 4 + s], v1 = buf[(size_t)c1 * 4 + s];
        acc0 ^= v0.x ^ v0.y ^ v0.z ^ v0.w;
        acc1 ^= v1.x ^ v1.y ^ v1.z ^ v1.w;
    }
    if (i < iters) {
        h ^= h << 13; h ^= h >> 17; h ^= h << 5;
        const uint4 v = buf[(size_t)__umulhi(h, n_chunks) * 4 + s];
        acc0 ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    sink[gid] = acc0 ^ acc1;
}

}  // namespace gff

using namespace gff;

extern "C" gff_status gff_gather_probe(const void *d_buf, size_t bytes, int n_threads, int iters, unsigned seed,
                                       unsigned *d_sink, void *stream) {
    if (!d_buf || !d_sink || bytes < 64 || bytes % 64 != 0 || ((uintptr_t)d_buf & 15) != 0) return GFF_EINVAL;
    if (n_threads < 256 || n_threads % 256 != 0 || iters < 1) return GFF_EINVAL;
    if (bytes / 64 > 0xffffffffull) return GFF_EINVAL;               // chunk indices are 32-bit
    hipLaunchKernelGGL(k_gather_probe, dim3(n_threads / 256), dim3(256), 0, (hipStream_t)stream,
                       (const uint4 *)d_buf, (unsigned)(bytes / 64), iters, seed, d_sink);
    return hip_status(hipGetLastError());
}
