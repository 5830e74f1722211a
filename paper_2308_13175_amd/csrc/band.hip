// Band and index construction (once per shape).
//
// Sec. 3 of the paper: a uniform grid localises queries; pulling is done only
// in the cells within M1 of a cell that holds a point, TV only within M2; the
// vertices of those cells are the optimised parameters.  Here the band is
// built on the device with dense per-shape scratch flags (one byte per cell
// and per vertex), separable Chebyshev dilation, then compacted into 8^3
// vertex bricks addressed through a dense brick directory.  The points are
// kept sorted by band cell (the sampler's source order).
//
// The nearest-neighbour search that stands in for the paper's KD-tree runs on
// a grid of its own per shape: the same box, cells 2^k times the band's (k >=
// 0, chosen from the point density: where the points are sparse in the band's
// cells, coarser cells hold about cell_points points each), its own Morton
// ordered brick directory, a one-bit-per-cell occupancy bitmap and the points
// bucketed by its cells (a counting layout over its brick slots).
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <memory>

#include "gp_internal.h"

namespace gp {
namespace {

constexpr int kThreads = 256;

inline unsigned blocks_for(int64_t n, int threads = kThreads)
{
    int64_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > (int64_t)1 << 30) b = (int64_t)1 << 30;
    return (unsigned)b;
}

#define GRID_STRIDE(i, n) \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// bit 1 of cell flags: the cell holds a point.  Records the lowest index of a
// point outside [lo, hi].
__global__ void k_locate_points(const float* __restrict__ px, const float* __restrict__ py,
                                const float* __restrict__ pz, ShapeDesc s, uint8_t* __restrict__ cells,
                                unsigned long long* __restrict__ bad)
{
    GRID_STRIDE(j, s.point_cnt)
    {
        int64_t g = s.point_off + j;
        Loc L = locate(s, px[g], py[g], pz[g]);
        if (!L.inside) {
            atomicMin(bad, (unsigned long long)j);
            continue;
        }
        int64_t cid = ((int64_t)L.c[0] * s.R[1] + L.c[1]) * s.R[2] + L.c[2];
        cells[cid] = 1;
    }
}

// One axis of the separable Chebyshev dilation.  Source bits (src1 for the
// M1 band, src2 for the M2 band) are ORed over |d| <= m along `axis` into
// bits 2 and 4; bit 1 (point cells) is copied.
__global__ void k_dilate(const uint8_t* __restrict__ in, uint8_t* __restrict__ out, int32_t R0, int32_t R1,
                         int32_t R2, int axis, int32_t m1, int32_t m2, uint8_t src1, uint8_t src2)
{
    int64_t n = (int64_t)R0 * R1 * R2;
    GRID_STRIDE(i, n)
    {
        int32_t cz = (int32_t)(i % R2);
        int32_t cy = (int32_t)((i / R2) % R1);
        int32_t cx = (int32_t)(i / ((int64_t)R2 * R1));
        int32_t c = axis == 0 ? cx : (axis == 1 ? cy : cz);
        int32_t Ra = axis == 0 ? R0 : (axis == 1 ? R1 : R2);
        int64_t stride = axis == 0 ? (int64_t)R1 * R2 : (axis == 1 ? (int64_t)R2 : 1);
        int32_t m = m1 > m2 ? m1 : m2;
        int32_t lo = c - m < 0 ? 0 : c - m;
        int32_t hi = c + m > Ra - 1 ? Ra - 1 : c + m;
        uint8_t o = in[i] & 1;
        for (int32_t d = lo; d <= hi; ++d) {
            uint8_t v = in[i + (int64_t)(d - c) * stride];
            int32_t ad = d > c ? d - c : c - d;
            if (ad <= m1 && (v & src1)) o |= 2;
            if (ad <= m2 && (v & src2)) o |= 4;
        }
        out[i] = o;
    }
}

// Vertex flags: bit 1 = corner of an M1- or M2-band cell, bit 2 = corner of
// an M2-band cell.
__global__ void k_vertex_flags(const uint8_t* __restrict__ cells, uint8_t* __restrict__ verts, int32_t R0,
                               int32_t R1, int32_t R2)
{
    const int64_t V1 = R1 + 1, V2 = R2 + 1;
    int64_t n = (int64_t)(R0 + 1) * V1 * V2;
    GRID_STRIDE(i, n)
    {
        int32_t k = (int32_t)(i % V2);
        int32_t j = (int32_t)((i / V2) % V1);
        int32_t ii = (int32_t)(i / (V2 * V1));
        uint8_t o = 0;
        for (int a = 0; a < 2; ++a) {
            int32_t cx = ii - a;
            if (cx < 0 || cx >= R0) continue;
            for (int b = 0; b < 2; ++b) {
                int32_t cy = j - b;
                if (cy < 0 || cy >= R1) continue;
                for (int d = 0; d < 2; ++d) {
                    int32_t cz = k - d;
                    if (cz < 0 || cz >= R2) continue;
                    uint8_t f = cells[((int64_t)cx * R1 + cy) * R2 + cz];
                    if (f & 6) o |= 1;
                    if (f & 4) o |= 2;
                }
            }
        }
        verts[i] = o;
    }
}

// A brick exists iff it holds an optimised vertex.
template <int kB>
__global__ void k_brick_active(const uint8_t* __restrict__ verts, ShapeDesc s, int32_t* __restrict__ active)
{
    const int64_t nbt = (int64_t)s.nb[0] * s.nb[1] * s.nb[2];
    const int32_t V0 = s.R[0] + 1, V1 = s.R[1] + 1, V2 = s.R[2] + 1;
    GRID_STRIDE(b, nbt)
    {
        int32_t bz = (int32_t)(b % s.nb[2]);
        int32_t by = (int32_t)((b / s.nb[2]) % s.nb[1]);
        int32_t bx = (int32_t)(b / ((int64_t)s.nb[2] * s.nb[1]));
        int32_t any = 0;
        for (int32_t lx = 0; lx < kB && !any; ++lx) {
            int32_t i = bx * kB + lx;
            if (i >= V0) break;
            for (int32_t ly = 0; ly < kB && !any; ++ly) {
                int32_t j = by * kB + ly;
                if (j >= V1) break;
                const uint8_t* row = verts + ((int64_t)i * V1 + j) * V2;
                for (int32_t lz = 0; lz < kB; ++lz) {
                    int32_t k = bz * kB + lz;
                    if (k >= V2) break;
                    if (row[k] & 1) { any = 1; break; }
                }
            }
        }
        active[b] = any;
    }
}

// Bricks are numbered along a Morton curve of their coordinates, so that
// bricks with neighbouring numbers are neighbours in space.  Everything that
// runs over bricks, or over points and queries in brick order (the points are
// sorted by slot, the sampler's sources follow that order), then moves
// through the grid region by region: a block of queries drawn from
// consecutive points stays in a compact box even where its points cross from
// one brick into the next.  Key of directory entry b: the interleaved bits of
// (bx, by, bz), or all ones for a brick without an optimised vertex.
__device__ inline uint64_t spread3_64(uint32_t v)
{
    uint64_t x = v & 0x1fffffull;   // 21 bits
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__global__ void k_brick_keys(const int32_t* __restrict__ active, ShapeDesc s, uint64_t* __restrict__ keys,
                             int32_t* __restrict__ ids)
{
    const int64_t nbt = (int64_t)s.nb[0] * s.nb[1] * s.nb[2];
    GRID_STRIDE(b, nbt)
    {
        const uint32_t bz = (uint32_t)(b % s.nb[2]);
        const uint32_t by = (uint32_t)((b / s.nb[2]) % s.nb[1]);
        const uint32_t bx = (uint32_t)(b / ((int64_t)s.nb[2] * s.nb[1]));
        keys[b] = active[b] ? (spread3_64(bx) << 2) | (spread3_64(by) << 1) | spread3_64(bz) : ~0ull;
        ids[b] = (int32_t)b;
    }
}

// index[b] = the Morton rank of active directory entry b (the active entries
// sort first: their keys are below all ones).
__global__ void k_brick_rank(const int32_t* __restrict__ sorted_ids, int64_t n_active, int32_t* __restrict__ index)
{
    GRID_STRIDE(r, n_active)
    {
        index[sorted_ids[r]] = (int32_t)r;
    }
}

__global__ void k_fill_dir(const int32_t* __restrict__ active, const int32_t* __restrict__ index, ShapeDesc s,
                           int32_t shape, int64_t brick_base, int32_t* __restrict__ dir,
                           BrickInfo* __restrict__ bricks)
{
    const int64_t nbt = (int64_t)s.nb[0] * s.nb[1] * s.nb[2];
    GRID_STRIDE(b, nbt)
    {
        if (!active[b]) {
            dir[b] = -1;
            continue;
        }
        int64_t gb = brick_base + index[b];
        dir[b] = (int32_t)gb;
        BrickInfo bi;
        bi.shape = shape;
        bi.bz = (int32_t)(b % s.nb[2]);
        bi.by = (int32_t)((b / s.nb[2]) % s.nb[1]);
        bi.bx = (int32_t)(b / ((int64_t)s.nb[2] * s.nb[1]));
        bricks[index[b]] = bi;
    }
}

// Per (brick, 32-bit word): pack the vertex and cell flags of 32 slots.
template <int kB>
__global__ void k_fill_masks(const BrickInfo* __restrict__ bricks, int64_t n_bricks, ShapeDesc s,
                             const uint8_t* __restrict__ cells, const uint8_t* __restrict__ verts,
                             uint32_t* __restrict__ m_base, uint32_t* __restrict__ m_a1,
                             uint32_t* __restrict__ m_a2, uint32_t* __restrict__ m_v,
                             uint32_t* __restrict__ m_v2)
{
    const int32_t V1 = s.R[1] + 1, V2 = s.R[2] + 1;
    using G = Geo<kB>;
    GRID_STRIDE(w, n_bricks * G::W)
    {
        int64_t b = w / G::W;
        int32_t word = (int32_t)(w % G::W);
        BrickInfo bi = bricks[b];
        uint32_t fb = 0, f1 = 0, f2 = 0, fv = 0, fv2 = 0;
        for (int bit = 0; bit < 32; ++bit) {
            int32_t local = word * 32 + bit;
            int32_t i = bi.bx * kB + (local >> (2 * G::S));
            int32_t j = bi.by * kB + ((local >> G::S) & G::M);
            int32_t k = bi.bz * kB + (local & G::M);
            if (i > s.R[0] || j > s.R[1] || k > s.R[2]) continue;
            uint8_t vf = verts[((int64_t)i * V1 + j) * V2 + k];
            if (vf & 1) fv |= 1u << bit;
            if (vf & 2) fv2 |= 1u << bit;
            if (i < s.R[0] && j < s.R[1] && k < s.R[2]) {
                uint8_t cf = cells[((int64_t)i * s.R[1] + j) * s.R[2] + k];
                if (cf & 1) fb |= 1u << bit;
                if (cf & 2) f1 |= 1u << bit;
                if (cf & 4) f2 |= 1u << bit;
            }
        }
        m_base[w] = fb;
        m_a1[w] = f1;
        m_a2[w] = f2;
        m_v[w] = fv;
        m_v2[w] = fv2;
    }
}

// Count TV vertices and optimised vertices per shape.  A wave whose words
// all belong to one shape adds its sums with one atomic per counter (one
// address per shape: per-word atomics serialise there).
template <int kB>
__global__ void k_count_masks(const BrickInfo* __restrict__ bricks, int64_t n_bricks,
                              const uint32_t* __restrict__ m_v, const uint32_t* __restrict__ m_v2,
                              unsigned long long* __restrict__ n_v, unsigned long long* __restrict__ n_v2)
{
    const int64_t n = n_bricks * Geo<kB>::W;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // every lane of a wave runs the same number of rounds (the bound is rounded up to whole strides)
    for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w - (threadIdx.x & 63) < n; w += stride) {
        const bool in = w < n;
        const int32_t s = in ? bricks[w / Geo<kB>::W].shape : -1;
        unsigned long long a = in ? (unsigned long long)__popc(m_v[w]) : 0ull;
        unsigned long long b = in ? (unsigned long long)__popc(m_v2[w]) : 0ull;
        const int32_t s0 = __shfl(s, 0, 64);
        if (__all(!in || s == s0)) {
            for (int o = 32; o > 0; o >>= 1) {
                a += __shfl_down(a, o, 64);
                b += __shfl_down(b, o, 64);
            }
            if ((threadIdx.x & 63) == 0 && s0 >= 0) {
                if (a) atomicAdd(&n_v[s0], a);
                if (b) atomicAdd(&n_v2[s0], b);
            }
        } else if (in) {
            if (a) atomicAdd(&n_v[s], a);
            if (b) atomicAdd(&n_v2[s], b);
        }
    }
}

// Sort keys of the points: the slot of the point's band cell (the slot of its
// lowest corner).
template <int kB>
__global__ void k_point_keys(const float* __restrict__ px, const float* __restrict__ py,
                             const float* __restrict__ pz, Band B, int32_t shape,
                             uint32_t* __restrict__ keys, int32_t* __restrict__ vals)
{
    using G = Geo<kB>;
    const ShapeDesc& s = B.shapes[shape];
    GRID_STRIDE(j, s.point_cnt)
    {
        int64_t g = s.point_off + j;
        Loc L = locate(s, px[g], py[g], pz[g]);
        int32_t br = brick_of(B, s, L.c[0] >> G::S, L.c[1] >> G::S, L.c[2] >> G::S);
        uint32_t slot = (uint32_t)br * G::V + (uint32_t)local_index_b<kB>(L.c[0], L.c[1], L.c[2]);
        keys[s.sorted_off + j] = slot;
        vals[s.sorted_off + j] = (int32_t)g;
    }
}

template <int kB>
__global__ void k_gather_sorted(const float* __restrict__ px, const float* __restrict__ py,
                                const float* __restrict__ pz, const uint32_t* __restrict__ keys,
                                const int32_t* __restrict__ vals, Band B, int64_t n, float4* __restrict__ spts)
{
    GRID_STRIDE(i, n)
    {
        int32_t g = vals[i];
        int32_t shape = B.bricks[keys[i] / Geo<kB>::V].shape;
        spts[i] = make_float4(px[g], py[g], pz[g], __int_as_float((int32_t)(g - B.shapes[shape].point_off)));
    }
}

// Number of cells holding a point (bit 1 of the cell flags), added to *count.
__global__ void k_count_point_cells(const uint8_t* __restrict__ cells, int64_t n_cells,
                                    unsigned long long* __restrict__ count)
{
    unsigned long long c = 0;
    GRID_STRIDE(i, n_cells) c += cells[i] & 1;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_down(c, o);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(count, c);
}

// ---- search grid ------------------------------------------------------------

// Marks the search-grid bricks that hold a point of shape n (points read from
// the original-order copy at sorted_off).
__global__ void k_nn_mark(const float* __restrict__ ox, const float* __restrict__ oy, const float* __restrict__ oz,
                          ShapeDesc n, int32_t* __restrict__ active)
{
    GRID_STRIDE(j, n.point_cnt)
    {
        const int64_t g = n.sorted_off + j;
        const Loc L = locate(n, ox[g], oy[g], oz[g]);
        const int64_t b = ((int64_t)(L.c[0] >> 3) * n.nb[1] + (L.c[1] >> 3)) * n.nb[2] + (L.c[2] >> 3);
        active[b] = 1;
    }
}

__global__ void k_nn_fill_dir(const int32_t* __restrict__ active, const int32_t* __restrict__ index, int64_t nbt,
                              int64_t brick_base, int32_t* __restrict__ dir)
{
    GRID_STRIDE(b, nbt) dir[b] = active[b] ? (int32_t)(brick_base + index[b]) : -1;
}

// Bucket keys of shape `shape`'s points in its search grid (the slot of the
// point's cell), the per-slot counts and the occupancy bits.
__global__ void k_nn_point_keys(const float* __restrict__ ox, const float* __restrict__ oy,
                                const float* __restrict__ oz, Band N, int32_t shape, uint32_t* __restrict__ keys,
                                int32_t* __restrict__ vals, unsigned* __restrict__ counts, uint32_t* __restrict__ occ)
{
    const ShapeDesc& n = N.shapes[shape];
    GRID_STRIDE(j, n.point_cnt)
    {
        const int64_t g = n.sorted_off + j;
        const Loc L = locate(n, ox[g], oy[g], oz[g]);
        const int32_t br = brick_of(N, n, L.c[0] >> 3, L.c[1] >> 3, L.c[2] >> 3);
        const uint32_t slot = (uint32_t)br * kBrickVol + (uint32_t)local_index(L.c[0], L.c[1], L.c[2]);
        keys[g] = slot;
        vals[g] = (int32_t)j;
        atomicAdd(&counts[slot], 1u);
        const int64_t bit = n.occ_off * 32 + ((int64_t)L.c[0] * n.R[1] + L.c[1]) * n.R[2] + L.c[2];
        atomicOr(&occ[bit >> 5], 1u << (bit & 31));
    }
}

__global__ void k_nn_gather(const float* __restrict__ ox, const float* __restrict__ oy, const float* __restrict__ oz,
                            const int32_t* __restrict__ vals, int64_t begin, int64_t count,
                            float4* __restrict__ spts)
{
    GRID_STRIDE(i, count)
    {
        const int32_t j = vals[begin + i];
        const int64_t g = begin + j;
        spts[begin + i] = make_float4(ox[g], oy[g], oz[g], __int_as_float(j));
    }
}

struct ShapeBricks {
    DevBuf<int32_t> dir;
    DevBuf<BrickInfo> bricks;
    DevBuf<uint32_t> m_base, m_a1, m_a2, m_v, m_v2;
    int64_t n_dir = 0;
    int64_t n_bricks = 0;
};

}  // namespace
}  // namespace gp

using namespace gp;

template <int kB>
static gp_status build_band(gp_ctx ctx, const gp_shape* shapes, int32_t n_shapes, const float* px, const float* py,
                            const float* pz, int32_t m1, int32_t m2)
{
    using G = Geo<kB>;
    hipStream_t st = ctx->stream;
    ctx->built = false;
    ctx->fwd_token = 0;

    // ---- host-side descriptors ------------------------------------------
    std::vector<ShapeDesc> hs(n_shapes);
    int64_t dir_total = 0, dense_total = 0, sorted_total = 0, tiles_total = 0;
    int64_t n_points = 0, n_queries = 0;
    for (int32_t s = 0; s < n_shapes; ++s) {
        const gp_shape& in = shapes[s];
        ShapeDesc& d = hs[s];
        for (int a = 0; a < 3; ++a) {
            d.lo[a] = in.lo[a];
            d.inv_h[a] = (double)in.dims[a] / (in.hi[a] - in.lo[a]);
            d.inv_hf[a] = (float)d.inv_h[a];
            d.h[a] = (float)((in.hi[a] - in.lo[a]) / (double)in.dims[a]);
            d.hd[a] = (in.hi[a] - in.lo[a]) / (double)in.dims[a];
            d.R[a] = in.dims[a];
            d.nb[a] = (in.dims[a] + 1 + kB - 1) / kB;
        }
        d.dir_off = dir_total;
        dir_total += (int64_t)d.nb[0] * d.nb[1] * d.nb[2];
        d.dense_off = dense_total;
        dense_total += (int64_t)(d.R[0] + 1) * (d.R[1] + 1) * (d.R[2] + 1);
        d.point_off = in.point_off;
        d.point_cnt = in.point_cnt;
        d.query_off = in.query_off;
        d.query_cnt = in.query_cnt;
        d.sorted_off = sorted_total;
        sorted_total += in.point_cnt;
        d.tile_begin = tiles_total;
        tiles_total += (in.query_cnt + kQueryTile - 1) / kQueryTile;
        d.tile_end = tiles_total;
        n_points = std::max(n_points, in.point_off + in.point_cnt);
        n_queries = std::max(n_queries, in.query_off + in.query_cnt);
        d.n_tv = 0;
        d.brick_begin = d.brick_end = 0;
        d.occ_off = 0;
    }
    if (sorted_total >= ((int64_t)1 << 31) || n_points >= ((int64_t)1 << 31))
        return gp_fail(ctx, GP_ERR_CAPACITY, "more than 2^31 points");
    if (dir_total >= kMaxSlots) return gp_fail(ctx, GP_ERR_CAPACITY, "more than 2^30 brick directory entries");

    DevBuf<unsigned long long> d_bad, d_occupied;
    GP_HIP(ctx, d_bad.alloc(1));
    GP_HIP(ctx, d_occupied.alloc(n_shapes));
    GP_HIP(ctx, hipMemsetAsync(d_occupied.p, 0, sizeof(unsigned long long) * n_shapes, st));

    std::vector<std::unique_ptr<ShapeBricks>> parts;
    int64_t brick_base = 0;
    void* cub_tmp = nullptr;
    size_t cub_bytes = 0;
    DevBuf<uint8_t> cub_buf;

    for (int32_t s = 0; s < n_shapes; ++s) {
        ShapeDesc& d = hs[s];
        const int64_t nc = (int64_t)d.R[0] * d.R[1] * d.R[2];
        const int64_t nv = (int64_t)(d.R[0] + 1) * (d.R[1] + 1) * (d.R[2] + 1);
        const int64_t nbt = (int64_t)d.nb[0] * d.nb[1] * d.nb[2];
        DevBuf<uint8_t> c0, c1, vf;
        DevBuf<int32_t> active, index;
        if (c0.alloc(nc) != hipSuccess || c1.alloc(nc) != hipSuccess || vf.alloc(nv) != hipSuccess ||
            active.alloc(nbt) != hipSuccess || index.alloc(nbt) != hipSuccess)
            return gp_fail(ctx, GP_ERR_OOM, "out of device memory for the band scratch of shape " +
                                                std::to_string(s));
        GP_HIP(ctx, hipMemsetAsync(c0.p, 0, nc, st));
        unsigned long long init = ~0ull;
        GP_HIP(ctx, hipMemcpyAsync(d_bad.p, &init, sizeof(init), hipMemcpyHostToDevice, st));
        if (d.point_cnt > 0)
            k_locate_points<<<blocks_for(d.point_cnt), kThreads, 0, st>>>(px, py, pz, d, c0.p, d_bad.p);
        unsigned long long bad = 0;
        GP_HIP(ctx, hipMemcpyAsync(&bad, d_bad.p, sizeof(bad), hipMemcpyDeviceToHost, st));
        GP_HIP(ctx, hipStreamSynchronize(st));
        if (bad != ~0ull)
            return gp_fail(ctx, GP_ERR_DOMAIN, "shape " + std::to_string(s) + ": point " + std::to_string(bad) +
                                                   " lies outside the domain");
        k_count_point_cells<<<std::min(blocks_for(nc), 4096u), kThreads, 0, st>>>(c0.p, nc, d_occupied.p + s);
        // separable Chebyshev dilation x -> y -> z; a width of the largest
        // extent minus one already reaches every cell, so wider ones are cut
        // to it (same sets, bounded work)
        const int32_t rmax = std::max(d.R[0], std::max(d.R[1], d.R[2]));
        const int32_t e1 = std::min(m1, rmax - 1), e2 = std::min(m2, rmax - 1);
        k_dilate<<<blocks_for(nc), kThreads, 0, st>>>(c0.p, c1.p, d.R[0], d.R[1], d.R[2], 0, e1, e2, 1, 1);
        k_dilate<<<blocks_for(nc), kThreads, 0, st>>>(c1.p, c0.p, d.R[0], d.R[1], d.R[2], 1, e1, e2, 2, 4);
        k_dilate<<<blocks_for(nc), kThreads, 0, st>>>(c0.p, c1.p, d.R[0], d.R[1], d.R[2], 2, e1, e2, 2, 4);
        k_vertex_flags<<<blocks_for(nv), kThreads, 0, st>>>(c1.p, vf.p, d.R[0], d.R[1], d.R[2]);
        k_brick_active<kB><<<blocks_for(nbt), kThreads, 0, st>>>(vf.p, d, active.p);
        size_t need = 0;
        GP_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, need, active.p, index.p, (int)nbt, st));
        if (need > cub_bytes) {
            GP_HIP(ctx, cub_buf.alloc(need));
            cub_tmp = cub_buf.p;
            cub_bytes = need;
        }
        GP_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(cub_tmp, need, active.p, index.p, (int)nbt, st));
        int32_t last_idx = 0, last_act = 0;
        GP_HIP(ctx, hipMemcpyAsync(&last_idx, index.p + nbt - 1, 4, hipMemcpyDeviceToHost, st));
        GP_HIP(ctx, hipMemcpyAsync(&last_act, active.p + nbt - 1, 4, hipMemcpyDeviceToHost, st));
        GP_HIP(ctx, hipStreamSynchronize(st));
        const int64_t nb_s = (int64_t)last_idx + last_act;
        if ((brick_base + nb_s) * G::V >= kMaxSlots)
            return gp_fail(ctx, GP_ERR_CAPACITY, "more than 2^30 field slots");
        {
            // brick numbers along the Morton curve (index[] of the active entries)
            DevBuf<uint64_t> kin, kout;
            DevBuf<int32_t> iin, iout;
            if (kin.alloc(nbt) != hipSuccess || kout.alloc(nbt) != hipSuccess || iin.alloc(nbt) != hipSuccess ||
                iout.alloc(nbt) != hipSuccess)
                return gp_fail(ctx, GP_ERR_OOM, "out of device memory for the brick order of shape " +
                                                    std::to_string(s));
            k_brick_keys<<<blocks_for(nbt), kThreads, 0, st>>>(active.p, d, kin.p, iin.p);
            int32_t bits = 1;
            while ((int64_t(1) << bits) < std::max(d.nb[0], std::max(d.nb[1], d.nb[2]))) ++bits;
            const int end_bit = 3 * bits + 1;   // the top bit set only in the keys of inactive entries
            size_t need3 = 0;
            GP_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(nullptr, need3, kin.p, kout.p, iin.p, iout.p, (int)nbt, 0,
                                                          end_bit, st));
            if (need3 > cub_bytes) {
                GP_HIP(ctx, cub_buf.alloc(need3));
                cub_tmp = cub_buf.p;
                cub_bytes = need3;
            }
            GP_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(cub_tmp, need3, kin.p, kout.p, iin.p, iout.p, (int)nbt, 0,
                                                          end_bit, st));
            if (nb_s > 0) k_brick_rank<<<blocks_for(nb_s), kThreads, 0, st>>>(iout.p, nb_s, index.p);
            GP_HIP(ctx, hipGetLastError());
            GP_HIP(ctx, hipStreamSynchronize(st));
        }

        auto part = std::make_unique<ShapeBricks>();
        part->n_dir = nbt;
        part->n_bricks = nb_s;
        if (part->dir.alloc(nbt) != hipSuccess || part->bricks.alloc(nb_s) != hipSuccess ||
            part->m_base.alloc(nb_s * G::W) != hipSuccess || part->m_a1.alloc(nb_s * G::W) != hipSuccess ||
            part->m_a2.alloc(nb_s * G::W) != hipSuccess || part->m_v.alloc(nb_s * G::W) != hipSuccess ||
            part->m_v2.alloc(nb_s * G::W) != hipSuccess)
            return gp_fail(ctx, GP_ERR_OOM, "out of device memory for the bricks of shape " + std::to_string(s));
        k_fill_dir<<<blocks_for(nbt), kThreads, 0, st>>>(active.p, index.p, d, s, brick_base, part->dir.p,
                                                          part->bricks.p);
        if (nb_s > 0)
            k_fill_masks<kB><<<blocks_for(nb_s * G::W), kThreads, 0, st>>>(
                part->bricks.p, nb_s, d, c1.p, vf.p, part->m_base.p, part->m_a1.p, part->m_a2.p, part->m_v.p,
                part->m_v2.p);
        GP_HIP(ctx, hipGetLastError());
        d.brick_begin = brick_base;
        d.brick_end = brick_base + nb_s;
        brick_base += nb_s;
        GP_HIP(ctx, hipStreamSynchronize(st));   // scratch buffers are freed at scope end
        parts.push_back(std::move(part));
    }

    // ---- assemble the global arrays --------------------------------------
    const int64_t n_bricks = brick_base;
    const int64_t n_slots = n_bricks * G::V;
    ctx->n_shapes = n_shapes;
    ctx->n_bricks = n_bricks;
    ctx->n_slots = n_slots;
    ctx->n_dir = dir_total;
    ctx->n_points = n_points;
    ctx->n_queries = n_queries;
    ctx->n_tiles = tiles_total;
    ctx->m1 = m1;
    ctx->m2 = m2;
    if (ctx->dir.alloc(dir_total) != hipSuccess || ctx->bricks.alloc(n_bricks) != hipSuccess ||
        ctx->m_base.alloc(n_bricks * G::W) != hipSuccess ||
        ctx->m_a1.alloc(n_bricks * G::W) != hipSuccess ||
        ctx->m_a2.alloc(n_bricks * G::W) != hipSuccess ||
        ctx->m_v.alloc(n_bricks * G::W) != hipSuccess ||
        ctx->m_v2.alloc(n_bricks * G::W) != hipSuccess || ctx->shapes.alloc(n_shapes) != hipSuccess)
        return gp_fail(ctx, GP_ERR_OOM, "out of device memory for the band");
    for (int32_t s = 0; s < n_shapes; ++s) {
        ShapeBricks& p = *parts[s];
        const ShapeDesc& d = hs[s];
        GP_HIP(ctx, hipMemcpyAsync(ctx->dir.p + d.dir_off, p.dir.p, p.n_dir * 4, hipMemcpyDeviceToDevice, st));
        if (p.n_bricks == 0) continue;
        const size_t mb = (size_t)p.n_bricks * G::W * 4;
        const int64_t mo = d.brick_begin * G::W;
        GP_HIP(ctx, hipMemcpyAsync(ctx->bricks.p + d.brick_begin, p.bricks.p, p.n_bricks * sizeof(BrickInfo),
                                   hipMemcpyDeviceToDevice, st));
        GP_HIP(ctx, hipMemcpyAsync(ctx->m_base.p + mo, p.m_base.p, mb, hipMemcpyDeviceToDevice, st));
        GP_HIP(ctx, hipMemcpyAsync(ctx->m_a1.p + mo, p.m_a1.p, mb, hipMemcpyDeviceToDevice, st));
        GP_HIP(ctx, hipMemcpyAsync(ctx->m_a2.p + mo, p.m_a2.p, mb, hipMemcpyDeviceToDevice, st));
        GP_HIP(ctx, hipMemcpyAsync(ctx->m_v.p + mo, p.m_v.p, mb, hipMemcpyDeviceToDevice, st));
        GP_HIP(ctx, hipMemcpyAsync(ctx->m_v2.p + mo, p.m_v2.p, mb, hipMemcpyDeviceToDevice, st));
    }

    // per-shape vertex counts
    DevBuf<unsigned long long> cnt;
    GP_HIP(ctx, cnt.alloc(2 * (size_t)n_shapes));
    GP_HIP(ctx, hipMemsetAsync(cnt.p, 0, 2 * sizeof(unsigned long long) * n_shapes, st));
    if (n_bricks > 0)
        k_count_masks<kB><<<blocks_for(n_bricks * G::W), kThreads, 0, st>>>(ctx->bricks.p, n_bricks, ctx->m_v.p,
                                                                             ctx->m_v2.p, cnt.p, cnt.p + n_shapes);
    std::vector<unsigned long long> hcnt(2 * (size_t)n_shapes);
    GP_HIP(ctx, hipMemcpyAsync(hcnt.data(), cnt.p, hcnt.size() * 8, hipMemcpyDeviceToHost, st));
    GP_HIP(ctx, hipStreamSynchronize(st));
    int64_t n_active = 0;
    for (int32_t s = 0; s < n_shapes; ++s) {
        hs[s].n_tv = (int64_t)hcnt[n_shapes + s];
        n_active += (int64_t)hcnt[s];
    }
    ctx->n_active = n_active;
    GP_HIP(ctx, hipMemcpyAsync(ctx->shapes.p, hs.data(), n_shapes * sizeof(ShapeDesc), hipMemcpyHostToDevice, st));
    ctx->h_occupied.assign(n_shapes, 0);
    {
        std::vector<unsigned long long> ho(n_shapes);
        GP_HIP(ctx, hipMemcpyAsync(ho.data(), d_occupied.p, n_shapes * sizeof(unsigned long long),
                                   hipMemcpyDeviceToHost, st));
        GP_HIP(ctx, hipStreamSynchronize(st));
        for (int32_t s = 0; s < n_shapes; ++s) ctx->h_occupied[s] = (int64_t)ho[s];
    }

    // ---- query tiles -------------------------------------------------------
    std::vector<int64_t> ts(tiles_total > 0 ? tiles_total : 1);
    std::vector<int32_t> tsh(tiles_total > 0 ? tiles_total : 1);
    for (int32_t s = 0; s < n_shapes; ++s)
        for (int64_t t = hs[s].tile_begin; t < hs[s].tile_end; ++t) {
            ts[t] = hs[s].query_off + (t - hs[s].tile_begin) * kQueryTile;
            tsh[t] = s;
        }
    GP_HIP(ctx, ctx->tile_start.alloc(ts.size()));
    GP_HIP(ctx, ctx->tile_shape.alloc(tsh.size()));
    GP_HIP(ctx, hipMemcpyAsync(ctx->tile_start.p, ts.data(), ts.size() * 8, hipMemcpyHostToDevice, st));
    GP_HIP(ctx, hipMemcpyAsync(ctx->tile_shape.p, tsh.data(), tsh.size() * 4, hipMemcpyHostToDevice, st));

    // ---- points sorted by band cell slot ----------------------------------
    const int64_t np = sorted_total;
    {
        DevBuf<uint32_t> k_in, k_out;
        DevBuf<int32_t> v_in;
        if (k_in.alloc(np) != hipSuccess || k_out.alloc(np) != hipSuccess || v_in.alloc(np) != hipSuccess ||
            ctx->spts.alloc(np) != hipSuccess || ctx->ox.alloc(np) != hipSuccess || ctx->oy.alloc(np) != hipSuccess ||
            ctx->oz.alloc(np) != hipSuccess)
            return gp_fail(ctx, GP_ERR_OOM, "out of device memory for the sorted points");
        for (int32_t s = 0; s < n_shapes; ++s) {
            if (hs[s].point_cnt == 0) continue;
            const size_t nb = (size_t)hs[s].point_cnt * sizeof(float);
            GP_HIP(ctx, hipMemcpyAsync(ctx->ox.p + hs[s].sorted_off, px + hs[s].point_off, nb, hipMemcpyDeviceToDevice, st));
            GP_HIP(ctx, hipMemcpyAsync(ctx->oy.p + hs[s].sorted_off, py + hs[s].point_off, nb, hipMemcpyDeviceToDevice, st));
            GP_HIP(ctx, hipMemcpyAsync(ctx->oz.p + hs[s].sorted_off, pz + hs[s].point_off, nb, hipMemcpyDeviceToDevice, st));
        }
        Band B = ctx->band();
        for (int32_t s = 0; s < n_shapes; ++s)
            if (hs[s].point_cnt > 0)
                k_point_keys<kB><<<blocks_for(hs[s].point_cnt), kThreads, 0, st>>>(px, py, pz, B, s, k_in.p, v_in.p);
        GP_HIP(ctx, hipGetLastError());
        size_t need = 0;
        int end_bit = 1;
        while (((int64_t)1 << end_bit) < n_slots + 1 && end_bit < 32) ++end_bit;
        size_t need2 = 0;
        DevBuf<int32_t> v_out;
        GP_HIP(ctx, v_out.alloc(np));
        if (np > 0)
            GP_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(nullptr, need2, k_in.p, k_out.p, v_in.p, v_out.p, (int)np,
                                                          0, end_bit, st));
        need = std::max(need, need2);
        if (need > cub_bytes) {
            GP_HIP(ctx, cub_buf.alloc(need));
            cub_tmp = cub_buf.p;
            cub_bytes = need;
        }
        if (np > 0) {
            GP_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(cub_tmp, need, k_in.p, k_out.p, v_in.p, v_out.p, (int)np, 0,
                                                          end_bit, st));
            k_gather_sorted<kB><<<blocks_for(np), kThreads, 0, st>>>(px, py, pz, k_out.p, v_out.p, B, np, ctx->spts.p);
        }
        GP_HIP(ctx, hipGetLastError());
        GP_HIP(ctx, hipStreamSynchronize(st));
    }

    // ---- scratch ----------------------------------------------------------
    if (ctx->q_part.alloc((size_t)std::max<int64_t>(tiles_total, 1) * 4 * 4) != hipSuccess ||   // up to 4 parts per tile
        ctx->tv_part.alloc((size_t)std::max<int64_t>(n_bricks, 1)) != hipSuccess ||
        ctx->tau.alloc((size_t)std::max<int64_t>(n_slots, 1)) != hipSuccess ||
        ctx->inv_qv.alloc(n_shapes) != hipSuccess || ctx->flag.alloc(1) != hipSuccess ||
        ctx->fin_part.alloc((size_t)n_shapes * 32 * 5) != hipSuccess || ctx->fin_count.alloc(n_shapes) != hipSuccess ||
        ctx->iter.alloc(1) != hipSuccess || ctx->step_c.alloc(2) != hipSuccess ||
        ctx->g_raw.alloc((size_t)std::max<int64_t>(n_slots, 1)) != hipSuccess ||
        ctx->nn_pt.alloc((size_t)std::max<int64_t>(n_queries, 1)) != hipSuccess)
        return gp_fail(ctx, GP_ERR_OOM, "out of device memory for the iteration scratch");
    GP_HIP(ctx, hipMemsetAsync(ctx->flag.p, 0, 4, st));
    GP_HIP(ctx, hipMemsetAsync(ctx->fin_count.p, 0, 4 * (size_t)n_shapes, st));
    GP_HIP(ctx, hipMemsetAsync(ctx->iter.p, 0, 4, st));
    GP_HIP(ctx, hipMemsetAsync(ctx->tau.p, 0, std::max<int64_t>(n_slots, 1) * 4, st));
    GP_HIP(ctx, hipMemsetAsync(ctx->g_raw.p, 0, std::max<int64_t>(n_slots, 1) * 4, st));
    // (all bits set: index -1, which names no point, so no record is taken before a search)
    GP_HIP(ctx, hipMemsetAsync(ctx->nn_pt.p, 0xff, std::max<int64_t>(n_queries, 1) * sizeof(float4), st));

    ctx->h_shapes = hs;
    ctx->h_slot_begin.resize(n_shapes + 1);
    for (int32_t s = 0; s < n_shapes; ++s) ctx->h_slot_begin[s] = hs[s].brick_begin * G::V;
    ctx->h_slot_begin[n_shapes] = n_slots;
    GP_HIP(ctx, hipStreamSynchronize(st));
    const gp_status ns = gp_build_nn_index(ctx, ctx->nn_params.cell_points);
    if (ns != GP_OK) return ns;
    ctx->built = true;
    return GP_OK;
}

gp_status gp_build_band_impl(gp_ctx ctx, const gp_shape* shapes, int32_t n_shapes, const float* px,
                             const float* py, const float* pz, int32_t m1, int32_t m2, int32_t brick)
{
    ctx->brick = brick;
    return with_brick(brick, [&](auto tag) {
        return build_band<decltype(tag)::value>(ctx, shapes, n_shapes, px, py, pz, m1, m2);
    });
}

// Level k of a shape's search grid (cells 2^k band cells wide per axis): the
// one that brings the mean number of points per occupied cell closest to
// cell_points on a log scale.  Points on a surface fill cells in two
// dimensions, so doubling the cell edge multiplies that mean by about 4:
// k = round(log2(cell_points / mean) / 2), within [0, 3].  The grid is never
// finer than the band: queries lie about two band cells from the surface
// (the sampler's spread), and a search for a query many cells away from every
// point costs more than dense cells do.
static int32_t nn_level(int64_t points, int64_t occupied, int32_t cell_points)
{
    if (points <= 0 || occupied <= 0) return 0;
    const double mean = (double)points / (double)occupied;
    const double k = std::nearbyint(0.5 * std::log2((double)cell_points / mean));
    return (int32_t)std::min(3.0, std::max(0.0, k));
}

// Descriptor of a search grid at level k: the band's box, 2^k times its cell
// edge (exact: a power of two), enough cells to cover the box.
static ShapeDesc nn_desc(const ShapeDesc& d, int32_t k)
{
    ShapeDesc n = d;
    const double f = std::ldexp(1.0, k);
    for (int a = 0; a < 3; ++a) {
        n.R[a] = (int32_t)((d.R[a] + ((int64_t)1 << k) - 1) >> k);
        n.inv_h[a] = d.inv_h[a] / f;
        n.inv_hf[a] = (float)n.inv_h[a];
        n.h[a] = (float)(d.hd[a] * f);
        n.hd[a] = d.hd[a] * f;
        n.nb[a] = (n.R[a] + kBrick - 1) / kBrick;
    }
    return n;
}

std::vector<int32_t> gp_nn_levels(gp_ctx ctx, int32_t cell_points)
{
    std::vector<int32_t> k(ctx->n_shapes);
    for (int32_t s = 0; s < ctx->n_shapes; ++s)
        k[s] = nn_level(ctx->h_shapes[s].point_cnt, ctx->h_occupied[s], cell_points);
    return k;
}

static gp_status build_nn_index(gp_ctx ctx, int32_t cell_points)
{
    hipStream_t st = ctx->stream;
    const int32_t n_shapes = ctx->n_shapes;
    const std::vector<ShapeDesc>& hs = ctx->h_shapes;
    std::vector<ShapeDesc> ns(n_shapes);
    std::vector<DevBuf<int32_t>> dirs(n_shapes);
    std::vector<int32_t> levels(n_shapes, 0);
    int64_t dir_total = 0, occ_total = 0, brick_base = 0;
    void* cub_tmp = nullptr;
    size_t cub_bytes = 0;
    DevBuf<uint8_t> cub_buf;
    auto cub_room = [&](size_t need) -> hipError_t {
        if (need <= cub_bytes) return hipSuccess;
        hipError_t e = cub_buf.alloc(need);
        cub_tmp = cub_buf.p;
        cub_bytes = e == hipSuccess ? need : 0;
        return e;
    };
    ctx->nn_cell_points = 0;
    for (int32_t s = 0; s < n_shapes; ++s) {
        const ShapeDesc& d = hs[s];
        const int32_t k = nn_level(d.point_cnt, ctx->h_occupied[s], cell_points);
        {
            ShapeDesc n = nn_desc(d, k);
            const int64_t nbt = (int64_t)n.nb[0] * n.nb[1] * n.nb[2];
            DevBuf<int32_t> active, index;
            if (active.alloc(nbt) != hipSuccess || index.alloc(nbt) != hipSuccess)
                return gp_fail(ctx, GP_ERR_OOM, "out of device memory for the search grid of shape " + std::to_string(s));
            GP_HIP(ctx, hipMemsetAsync(active.p, 0, nbt * sizeof(int32_t), st));
            if (n.point_cnt > 0)
                k_nn_mark<<<blocks_for(n.point_cnt), kThreads, 0, st>>>(ctx->ox.p, ctx->oy.p, ctx->oz.p, n, active.p);
            GP_HIP(ctx, hipGetLastError());
            size_t need = 0;
            GP_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, need, active.p, index.p, (int)nbt, st));
            GP_HIP(ctx, cub_room(need));
            GP_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(cub_tmp, need, active.p, index.p, (int)nbt, st));
            int32_t last_idx = 0, last_act = 0;
            GP_HIP(ctx, hipMemcpyAsync(&last_idx, index.p + nbt - 1, 4, hipMemcpyDeviceToHost, st));
            GP_HIP(ctx, hipMemcpyAsync(&last_act, active.p + nbt - 1, 4, hipMemcpyDeviceToHost, st));
            GP_HIP(ctx, hipStreamSynchronize(st));
            const int64_t nb_s = (int64_t)last_idx + last_act;
            if ((brick_base + nb_s) * kBrickVol >= kMaxSlots)
                return gp_fail(ctx, GP_ERR_CAPACITY, "more than 2^30 search grid slots");
            {
                // bricks numbered along the Morton curve
                DevBuf<uint64_t> kin, kout;
                DevBuf<int32_t> iin, iout;
                if (kin.alloc(nbt) != hipSuccess || kout.alloc(nbt) != hipSuccess || iin.alloc(nbt) != hipSuccess ||
                    iout.alloc(nbt) != hipSuccess)
                    return gp_fail(ctx, GP_ERR_OOM, "out of device memory for the search grid of shape " +
                                                        std::to_string(s));
                k_brick_keys<<<blocks_for(nbt), kThreads, 0, st>>>(active.p, n, kin.p, iin.p);
                int32_t bits = 1;
                while ((int64_t(1) << bits) < std::max(n.nb[0], std::max(n.nb[1], n.nb[2]))) ++bits;
                const int end_bit = 3 * bits + 1;
                size_t need3 = 0;
                GP_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(nullptr, need3, kin.p, kout.p, iin.p, iout.p, (int)nbt,
                                                              0, end_bit, st));
                GP_HIP(ctx, cub_room(need3));
                GP_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(cub_tmp, need3, kin.p, kout.p, iin.p, iout.p, (int)nbt,
                                                              0, end_bit, st));
                if (nb_s > 0) k_brick_rank<<<blocks_for(nb_s), kThreads, 0, st>>>(iout.p, nb_s, index.p);
                if (dirs[s].alloc(nbt) != hipSuccess)
                    return gp_fail(ctx, GP_ERR_OOM, "out of device memory for the search grid of shape " +
                                                        std::to_string(s));
                k_nn_fill_dir<<<blocks_for(nbt), kThreads, 0, st>>>(active.p, index.p, nbt, brick_base, dirs[s].p);
                GP_HIP(ctx, hipGetLastError());
                GP_HIP(ctx, hipStreamSynchronize(st));   // scratch buffers are freed at scope end
            }
            n.dir_off = dir_total;
            dir_total += nbt;
            n.occ_off = occ_total;
            occ_total += ((int64_t)n.R[0] * n.R[1] * n.R[2] + 31) / 32;
            n.brick_begin = brick_base;
            n.brick_end = brick_base + nb_s;
            brick_base += nb_s;
            ns[s] = n;
            levels[s] = k;
        }
    }
    if (dir_total >= kMaxSlots) return gp_fail(ctx, GP_ERR_CAPACITY, "more than 2^30 search grid directory entries");

    const int64_t n_slots = brick_base * kBrickVol;
    const int64_t np = n_shapes > 0 ? hs[n_shapes - 1].sorted_off + hs[n_shapes - 1].point_cnt : 0;
    if (ctx->nn_shapes.alloc(n_shapes) != hipSuccess || ctx->nn_dir.alloc(dir_total) != hipSuccess ||
        ctx->occ.alloc((size_t)std::max<int64_t>(occ_total, 1)) != hipSuccess ||
        ctx->cell_start.alloc(n_slots + 1) != hipSuccess || ctx->nn_spts.alloc(np) != hipSuccess)
        return gp_fail(ctx, GP_ERR_OOM, "out of device memory for the search grids");
    GP_HIP(ctx, hipMemcpyAsync(ctx->nn_shapes.p, ns.data(), n_shapes * sizeof(ShapeDesc), hipMemcpyHostToDevice, st));
    for (int32_t s = 0; s < n_shapes; ++s) {
        const int64_t nbt = (int64_t)ns[s].nb[0] * ns[s].nb[1] * ns[s].nb[2];
        GP_HIP(ctx, hipMemcpyAsync(ctx->nn_dir.p + ns[s].dir_off, dirs[s].p, nbt * sizeof(int32_t),
                                   hipMemcpyDeviceToDevice, st));
    }
    GP_HIP(ctx, hipMemsetAsync(ctx->occ.p, 0, std::max<int64_t>(occ_total, 1) * sizeof(uint32_t), st));
    {
        DevBuf<uint32_t> k_in, k_out;
        DevBuf<int32_t> v_in, v_out;
        DevBuf<unsigned> counts;
        if (k_in.alloc(np) != hipSuccess || k_out.alloc(np) != hipSuccess || v_in.alloc(np) != hipSuccess ||
            v_out.alloc(np) != hipSuccess || counts.alloc(n_slots + 1) != hipSuccess)
            return gp_fail(ctx, GP_ERR_OOM, "out of device memory for the search grids");
        GP_HIP(ctx, hipMemsetAsync(counts.p, 0, (n_slots + 1) * sizeof(unsigned), st));
        Band N = ctx->nn_band();
        for (int32_t s = 0; s < n_shapes; ++s)
            if (ns[s].point_cnt > 0)
                k_nn_point_keys<<<blocks_for(ns[s].point_cnt), kThreads, 0, st>>>(
                    ctx->ox.p, ctx->oy.p, ctx->oz.p, N, s, k_in.p, v_in.p, counts.p, ctx->occ.p);
        GP_HIP(ctx, hipGetLastError());
        // cell_start = exclusive prefix sum of the per-slot counts
        size_t need = 0, need2 = 0;
        GP_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, need, counts.p, (unsigned*)ctx->cell_start.p,
                                                     (int)(n_slots + 1), st));
        int end_bit = 1;
        while (((int64_t)1 << end_bit) < n_slots + 1 && end_bit < 32) ++end_bit;
        if (np > 0)
            GP_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(nullptr, need2, k_in.p, k_out.p, v_in.p, v_out.p, (int)np,
                                                          0, end_bit, st));
        GP_HIP(ctx, cub_room(std::max(need, need2)));
        need = cub_bytes;
        GP_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(cub_tmp, need, counts.p, (unsigned*)ctx->cell_start.p,
                                                     (int)(n_slots + 1), st));
        if (np > 0) {
            // a stable sort: within a cell the points keep their original order
            GP_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(cub_tmp, need, k_in.p, k_out.p, v_in.p, v_out.p, (int)np, 0,
                                                          end_bit, st));
            for (int32_t s = 0; s < n_shapes; ++s)
                if (ns[s].point_cnt > 0)
                    k_nn_gather<<<blocks_for(ns[s].point_cnt), kThreads, 0, st>>>(
                        ctx->ox.p, ctx->oy.p, ctx->oz.p, v_out.p, ns[s].sorted_off, ns[s].point_cnt, ctx->nn_spts.p);
        }
        GP_HIP(ctx, hipGetLastError());
        GP_HIP(ctx, hipStreamSynchronize(st));
    }
    ctx->h_nn_shapes = ns;
    ctx->h_nn_levels = levels;
    ctx->nn_slots = n_slots;
    ctx->nn_cell_points = cell_points;
    return GP_OK;
}

// A failed rebuild leaves the search grids half replaced: the context is
// then unusable until the next gp_build_band.
gp_status gp_build_nn_index(gp_ctx ctx, int32_t cell_points)
{
    const gp_status st = build_nn_index(ctx, cell_points);
    if (st != GP_OK) ctx->built = false;
    return st;
}
