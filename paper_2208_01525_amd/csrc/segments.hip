// segments.hip -- robust-method bound-state segments on the GPU (Correia &
// Martins, arXiv:2208.01525, Sec. III.B and Sec. V.B).
//
// The fast method marks a pierced cell of one sector that has a pierced cell
// of the other sector in its (2r+1)^3 neighbourhood (either way round).  The
// robust method groups the marked cells into connected regions -- cells that
// share at least a corner, periodic -- each region being one pq segment of
// (N_cells - 1) dx, and drops regions below a minimum length.
//
// Connected components by lock-free union-find: every marked cell starts as
// its own root; each cell links to its 13 "forward" neighbours with a
// compare-and-swap that always hangs the larger root under the smaller one,
// so parent indices only decrease (no cycles, every loop is bounded) and the
// final root of a region is its smallest cell index whatever the schedule.
// Parent reads inside the union use device-coherent atomic loads.
#include "device.h"
#include "kernels.h"

namespace mts {

namespace {

constexpr uint32_t NONE = 0xFFFFFFFFu;

__device__ __forceinline__ int wrapc(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__device__ __forceinline__ uint32_t ld_parent(const uint32_t *parent, uint32_t a) {
    return __hip_atomic_load(parent + a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t root_of(const uint32_t *parent, uint32_t a) {
    for (;;) {   // parent[a] <= a, strictly decreasing until a root
        const uint32_t p = ld_parent(parent, a);
        if (p == a) return a;
        a = p;
    }
}

}  // namespace

__global__ __launch_bounds__(256) void seg_mark_kernel(Geom g, const uint8_t *cells, uint32_t plane, int radius,
                                                       uint32_t *parent) {
    const int x = blockIdx.x * 64 + threadIdx.x, y = blockIdx.y * 4 + threadIdx.y, z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const uint32_t s = x + g.nx * y + g.nxy * z;
    bool marked = false;
    for (int sec = 0; sec < 2 && !marked; sec++) {
        if (cells[(size_t)sec * plane + s] == 0) continue;
        const uint8_t *o = cells + (size_t)(1 - sec) * plane;
        for (int dz = -radius; dz <= radius && !marked; dz++)
            for (int dy = -radius; dy <= radius && !marked; dy++)
                for (int dx = -radius; dx <= radius && !marked; dx++)
                    marked = o[wrapc(x + dx, g.nx) + g.nx * wrapc(y + dy, g.ny) + g.nxy * wrapc(z + dz, g.nz)] != 0;
    }
    parent[s] = marked ? s : NONE;
}

__global__ __launch_bounds__(256) void seg_union_kernel(Geom g, uint32_t *parent) {
    const int x = blockIdx.x * 64 + threadIdx.x, y = blockIdx.y * 4 + threadIdx.y, z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const uint32_t s = x + g.nx * y + g.nxy * z;
    if (parent[s] == NONE) return;
    // the 13 neighbours that come after s in (dz, dy, dx) order
    for (int dz = 0; dz <= 1; dz++)
        for (int dy = (dz ? -1 : 0); dy <= 1; dy++)
            for (int dx = ((dz || dy) ? -1 : 1); dx <= 1; dx++) {
                const uint32_t t = wrapc(x + dx, g.nx) + g.nx * wrapc(y + dy, g.ny) + g.nxy * wrapc(z + dz, g.nz);
                if (ld_parent(parent, t) == NONE) continue;
                uint32_t a = s, b = t;
                for (;;) {   // each retry lowers a: at most S rounds
                    a = root_of(parent, a);
                    b = root_of(parent, b);
                    if (a == b) break;
                    if (a < b) {
                        const uint32_t tmp = a;
                        a = b;
                        b = tmp;
                    }
                    const uint32_t old = atomicCAS(parent + a, a, b);
                    if (old == a) break;
                    a = old;
                }
            }
}

__global__ __launch_bounds__(256) void seg_flatten_count_kernel(uint32_t S, uint32_t *parent, uint32_t *count) {
    const uint32_t s = blockIdx.x * 256 + threadIdx.x;
    if (s >= S || parent[s] == NONE) return;
    const uint32_t r = root_of(parent, s);
    atomicAdd(count + r, 1u);
}

__global__ __launch_bounds__(256) void seg_collect_kernel(uint32_t S, const uint32_t *parent, const uint32_t *count,
                                                          uint32_t *sizes, uint32_t *n_out, uint32_t cap) {
    const uint32_t s = blockIdx.x * 256 + threadIdx.x;
    if (s >= S || parent[s] != s) return;
    const uint32_t i = atomicAdd(n_out, 1u);
    if (i < cap) sizes[i] = count[s];
}

__global__ __launch_bounds__(256) void fill_u32_kernel(uint32_t *p, uint32_t n, uint32_t v) {
    const uint32_t i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_segments(const Geom &g, const uint8_t *cells, uint32_t plane, int radius, uint32_t *parent,
                           uint32_t *count, uint32_t *sizes, uint32_t *n_out, uint32_t cap, hipStream_t st) {
    const uint32_t S = g.nxy * (uint32_t)g.nz;
    const dim3 block(64, 4, 1), grid((g.nx + 63) / 64, (g.ny + 3) / 4, g.nz);
    const uint32_t nb = (S + 255) / 256;
    fill_u32_kernel<<<nb, 256, 0, st>>>(count, S, 0u);
    fill_u32_kernel<<<1, 256, 0, st>>>(n_out, 1, 0u);
    seg_mark_kernel<<<grid, block, 0, st>>>(g, cells, plane, radius, parent);
    seg_union_kernel<<<grid, block, 0, st>>>(g, parent);
    seg_flatten_count_kernel<<<nb, 256, 0, st>>>(S, parent, count);
    seg_collect_kernel<<<nb, 256, 0, st>>>(S, parent, count, sizes, n_out, cap);
    return hipGetLastError();
}

}  // namespace mts
