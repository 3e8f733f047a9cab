// probe.hip -- bandwidth probes: the attainable HBM rate of the box for a
// plain copy and for the update's own access pattern, measured on a context's
// state buffer (a measurement aid beside the roofline of the update kernel).
#include "device.h"
#include "kernels.h"

namespace mts {

namespace {

// dst[i] = src[i], one float4 per thread and pass; the grid strides over
// copies of more than 2^31 float4 (a dispatch holds fewer than 2^32
// work-items).
__global__ __launch_bounds__(256) void probe_copy_kernel(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                         uint64_t n4) {
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride) dst[i] = src[i];
}

// The update's HBM pattern without its stencil or arithmetic: per site, the
// 10 momentum planes are read and rewritten in place and the 10 field planes
// of copy `in` are read and written to copy `out` (planes `plane` elements
// apart).  c = 1 and z = 0 leave every value unchanged.
template <typename T, bool NT>
__global__ __launch_bounds__(256) void probe_pattern_kernel(T *state, uint64_t plane, uint32_t S, int in, T c, T z) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i >= S) return;
    const T *fin = state + (size_t)in * 10 * plane;
    T *fout = state + (size_t)(1 - in) * 10 * plane;
    T *mom = state + (size_t)20 * plane;
    T m[10], f[10];
#pragma unroll
    for (int k = 0; k < 10; k++) {
        m[k] = mom[(size_t)k * plane + i];
        f[k] = fin[(size_t)k * plane + i];
    }
#pragma unroll
    for (int k = 0; k < 10; k++) {
        st_stream<NT>(&mom[(size_t)k * plane + i], m[k] * c);
        st_stream<NT>(&fout[(size_t)k * plane + i], f[k] + m[k] * z);
    }
}

}  // namespace

hipError_t launch_probe_copy(void *state, uint64_t bytes_per_copy, hipStream_t st) {
    const uint64_t n4 = bytes_per_copy / 16;
    const float4 *src = static_cast<const float4 *>(state);
    float4 *dst = reinterpret_cast<float4 *>(static_cast<char *>(state) + bytes_per_copy);
    const uint64_t nb = std::min<uint64_t>((n4 + 255) / 256, (uint64_t)1 << 23);
    probe_copy_kernel<<<(unsigned)nb, 256, 0, st>>>(src, dst, n4);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_probe_pattern(T *state, uint64_t plane, uint32_t S, int in, bool nt, hipStream_t st) {
    const unsigned nb = (S + 255) / 256;
    if (nt)
        probe_pattern_kernel<T, true><<<nb, 256, 0, st>>>(state, plane, S, in, T(1), T(0));
    else
        probe_pattern_kernel<T, false><<<nb, 256, 0, st>>>(state, plane, S, in, T(1), T(0));
    return hipGetLastError();
}

template hipError_t launch_probe_pattern<float>(float *, uint64_t, uint32_t, int, bool, hipStream_t);
template hipError_t launch_probe_pattern<double>(double *, uint64_t, uint32_t, int, bool, hipStream_t);

}  // namespace mts
