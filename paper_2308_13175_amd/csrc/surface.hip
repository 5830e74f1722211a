// The mesh of the field's zero level set over the optimised cells: the step
// the paper runs once the optimisation ends (Sec. 3, last paragraph: cells
// that were not optimised are skipped; Sec. 4 "Details": marching cubes).
//
// Marching cubes (method 0).  A cell whose eight corners are optimised
// vertices is classified by which corners are inside (f < 0).  The triangles
// of each of the 256 classes are generated at compile time from one rule
// (no printed case table): each face is walked counter-clockwise as seen
// from outside the cube; every maximal run of inside corners gets a segment
// from the crossed edge where the walk leaves it to the one where it
// entered (so a face with two diagonal inside corners cuts them off
// separately, decided by the face alone, the same from both of its cells:
// no cracks); the segments close into loops, taken from the lowest crossed
// edge; each loop is fanned from its first edge.  Corners: (a, b, c) at
// 4a + 2b + c.  Edges along axis d: 4d + 2 u + v, with (u, v) the other two
// coordinates of its corners in axis order.
//
// Marching tetrahedra (method 1).  Each optimised cell is cut into six
// tetrahedra along its main diagonal, (0, A, B, 7) for the paths
// 0 -> A -> B -> 7 through the corners; neighbouring cells cut a shared face
// along the same diagonal.  A tetrahedron with one corner on one side gives
// one triangle, two and two give two.
//
// Either way a triangle corner is the zero of the linear interpolant on an
// edge, taken from the edge's inside end p towards its outside end q:
// p + f_p / (f_p - f_q) (q - p), in double with no fused multiply-add, so a
// grid edge gives the same point in every cell that has it.
//
// One thread per (brick, cell whose lowest corner is in the brick): a count
// pass, a scan, an emit pass, then a sort by key (cell id x-major times 16,
// plus the triangle's number in the cell: for tetrahedra, tet * 2 +
// triangle), so the output order does not depend on the brick layout.
#include <hipcub/hipcub.hpp>

#include "gp_internal.h"

namespace gp {
namespace {

constexpr int kThreads = 256;

inline unsigned blocks_for(int64_t n)
{
    int64_t b = (n + kThreads - 1) / kThreads;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, (int64_t)1 << 30));
}

__constant__ int kTet[6][4] = {{0, 4, 6, 7}, {0, 4, 5, 7}, {0, 2, 6, 7}, {0, 2, 3, 7}, {0, 1, 5, 7}, {0, 1, 3, 7}};

// ---- marching cubes triangles per corner class, built at compile time -----
constexpr int kMcMaxTri = 5;

struct McTable {
    int8_t n[256];                   // triangles of the class
    int8_t e[256][kMcMaxTri][3];     // their corners, as edges
};

constexpr int corner_at(const int x[3]) { return 4 * x[0] + 2 * x[1] + x[2]; }

// Edge between corners p and q (neighbours on the cube).
constexpr int edge_between(int p, int q)
{
    const int d = (p ^ q) == 4 ? 0 : ((p ^ q) == 2 ? 1 : 2);
    const int m = p & q;   // the shared coordinates (the other axis is 0 here)
    const int x[3] = {(m >> 2) & 1, (m >> 1) & 1, m & 1};
    const int u = d == 0 ? x[1] : x[0], v = d == 2 ? x[1] : x[2];
    return 4 * d + 2 * u + v;
}

constexpr McTable build_mc_table()
{
    McTable T{};
    for (int cls = 0; cls < 256; ++cls) {
        int next[12] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
        for (int axis = 0; axis < 3; ++axis)
            for (int side = 0; side < 2; ++side) {
                // (u, v, axis) right-handed: on the +axis face the ring
                // (0,0) (1,0) (1,1) (0,1) in (u, v) runs counter-clockwise
                // seen from outside, on the -axis face the reverse
                const int u = (axis + 1) % 3, v = (axis + 2) % 3;
                const int ru[4] = {0, 1, 1, 0}, rv[4] = {0, 0, 1, 1};
                int ring[4] = {0, 0, 0, 0};
                for (int k = 0; k < 4; ++k) {
                    const int kk = side ? k : (4 - k) % 4;
                    int x[3] = {0, 0, 0};
                    x[axis] = side;
                    x[u] = ru[kk];
                    x[v] = rv[kk];
                    ring[k] = corner_at(x);
                }
                for (int k = 0; k < 4; ++k) {
                    const bool here = (cls >> ring[k]) & 1, after = (cls >> ring[(k + 1) % 4]) & 1;
                    if (!here || after) continue;        // only where the walk leaves an inside run
                    int b = k;
                    while ((cls >> ring[b]) & 1) b = (b + 3) % 4;
                    next[edge_between(ring[k], ring[(k + 1) % 4])] = edge_between(ring[b], ring[(b + 1) % 4]);
                }
            }
        bool seen[12] = {};
        int nt = 0;
        for (int start = 0; start < 12; ++start) {
            if (next[start] < 0 || seen[start]) continue;
            int loop[12] = {}, m = 0;
            for (int e = start; m == 0 || e != start; e = next[e]) {
                seen[e] = true;
                loop[m++] = e;
            }
            for (int i = 1; i + 1 < m; ++i) {
                T.e[cls][nt][0] = (int8_t)loop[0];
                T.e[cls][nt][1] = (int8_t)loop[i];
                T.e[cls][nt][2] = (int8_t)loop[i + 1];
                ++nt;
            }
        }
        T.n[cls] = (int8_t)nt;
    }
    return T;
}

constexpr McTable kMcHost = build_mc_table();

constexpr bool mc_table_fits()
{
    for (int c = 0; c < 256; ++c)
        if (kMcHost.n[c] < 0 || kMcHost.n[c] > kMcMaxTri) return false;
    return kMcHost.n[0] == 0 && kMcHost.n[255] == 0;
}
static_assert(mc_table_fits(), "marching cubes classes give 0 to 5 triangles");

__constant__ McTable kMc = kMcHost;

// Corners at the ends of edge e (the lower first).
__device__ inline void edge_corners(int e, int& p, int& q)
{
    const int d = e >> 2, u = (e >> 1) & 1, v = e & 1;
    int x[3] = {0, 0, 0};
    x[d == 0 ? 1 : 0] = u;
    x[d == 2 ? 1 : 2] = v;
    p = corner_at(x);
    q = p | (4 >> d);
}

// Corners of the cell with lowest corner at local cell l of brick `brick`:
// global cell c, and whether all eight corners are optimised (then slot[] and
// the values f[] are filled).
template <int kB>
__device__ inline bool optimised_cell(const Band& B, const ShapeDesc& s, int32_t brick, int32_t l, int32_t c[3],
                                      const float* __restrict__ field, float f[8])
{
    using G = Geo<kB>;
    const BrickInfo bi = B.bricks[brick];
    c[0] = bi.bx * kB + (l >> (2 * G::S));
    c[1] = bi.by * kB + ((l >> G::S) & G::M);
    c[2] = bi.bz * kB + (l & G::M);
    if (c[0] >= s.R[0] || c[1] >= s.R[1] || c[2] >= s.R[2]) return false;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                const int32_t i = c[0] + a, j = c[1] + b, k = c[2] + d;
                const int32_t br = brick_of(B, s, i >> G::S, j >> G::S, k >> G::S);
                if (br < 0) return false;
                const int32_t loc = local_index_b<kB>(i, j, k);
                if (!mask_bit_b<kB>(B.m_v, br, loc)) return false;
                f[4 * a + 2 * b + d] = field[(int64_t)br * G::V + loc];
            }
    return true;
}

__device__ inline int tet_count(const float f[8], int t)
{
    int ni = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) ni += f[kTet[t][i]] < 0.f;
    return ni == 0 || ni == 4 ? 0 : (ni == 2 ? 2 : 1);
}

__device__ inline int32_t corner_class(const float f[8])
{
    int32_t cls = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) cls |= (f[i] < 0.f ? 1 : 0) << i;
    return cls;
}

template <int kB>
__global__ void k_surf_count(Band B, int32_t shape, const float* __restrict__ field, int32_t method,
                             int32_t* __restrict__ count)
{
    const ShapeDesc& s = B.shapes[shape];
    const int64_t n = (s.brick_end - s.brick_begin) * Geo<kB>::V;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
        int32_t c[3];
        float f[8];
        int32_t m = 0;
        if (optimised_cell<kB>(B, s, (int32_t)(s.brick_begin + g / Geo<kB>::V), (int32_t)(g % Geo<kB>::V), c, field,
                               f)) {
            if (method == 0) m = kMc.n[corner_class(f)];
            else
                for (int t = 0; t < 6; ++t) m += tet_count(f, t);
        }
        count[g] = m;
    }
}

__device__ inline void edge_point(const double P[8][3], const double fd[8], int a, int b, float* out)
{
#pragma clang fp contract(off)
    const double t = fd[a] / (fd[a] - fd[b]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double d = P[b][k] - P[a][k];
        const double v = P[a][k] + t * d;
        out[k] = (float)v;
    }
}

template <int kB>
__global__ void k_surf_emit(Band B, int32_t shape, const float* __restrict__ field, int32_t method,
                            const int32_t* __restrict__ offset, float* __restrict__ xyz, int64_t* __restrict__ key,
                            int32_t* __restrict__ idx)
{
#pragma clang fp contract(off)
    const ShapeDesc& s = B.shapes[shape];
    const int64_t n = (s.brick_end - s.brick_begin) * Geo<kB>::V;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n; g += (int64_t)gridDim.x * blockDim.x) {
        if (offset[g + 1] == offset[g]) continue;
        int32_t c[3];
        float f[8];
        if (!optimised_cell<kB>(B, s, (int32_t)(s.brick_begin + g / Geo<kB>::V), (int32_t)(g % Geo<kB>::V), c, field,
                                f))
            continue;
        double P[8][3], fd[8];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int d = 0; d < 2; ++d) {
                    const int i = 4 * a + 2 * b + d;
                    P[i][0] = s.lo[0] + (double)(c[0] + a) * s.hd[0];
                    P[i][1] = s.lo[1] + (double)(c[1] + b) * s.hd[1];
                    P[i][2] = s.lo[2] + (double)(c[2] + d) * s.hd[2];
                    fd[i] = (double)f[i];
                }
        const int64_t cid = ((int64_t)c[0] * s.R[1] + c[1]) * s.R[2] + c[2];
        int32_t o = offset[g];
        if (method == 0) {
            const int32_t cls = corner_class(f);
            for (int t = 0; t < kMc.n[cls]; ++t) {
                float* tri = xyz + (int64_t)o * 9;
                for (int v = 0; v < 3; ++v) {
                    int p, q;
                    edge_corners(kMc.e[cls][t][v], p, q);
                    if (!(f[p] < 0.f)) {   // from the inside end
                        const int x = p;
                        p = q;
                        q = x;
                    }
                    edge_point(P, fd, p, q, tri + 3 * v);
                }
                key[o] = cid * 16 + t;
                idx[o] = o;
                ++o;
            }
            continue;
        }
        for (int t = 0; t < 6; ++t) {
            int in[4], out[4], ni = 0, no = 0;
            for (int i = 0; i < 4; ++i) {
                const int v = kTet[t][i];
                if (f[v] < 0.f) in[ni++] = v;
                else out[no++] = v;
            }
            if (ni == 0 || no == 0) continue;
            float* tri = xyz + (int64_t)o * 9;
            if (ni == 1 || no == 1) {
                for (int k = 0; k < 3; ++k) {
                    if (ni == 1) edge_point(P, fd, in[0], out[k], tri + 3 * k);
                    else edge_point(P, fd, in[k], out[0], tri + 3 * k);
                }
                key[o] = cid * 16 + t * 2;
                idx[o] = o;
                ++o;
            } else {
                float ac[3], ad[3], bd[3], bc[3];
                edge_point(P, fd, in[0], out[0], ac);
                edge_point(P, fd, in[0], out[1], ad);
                edge_point(P, fd, in[1], out[1], bd);
                edge_point(P, fd, in[1], out[0], bc);
                for (int k = 0; k < 3; ++k) {
                    tri[k] = ac[k];
                    tri[3 + k] = ad[k];
                    tri[6 + k] = bd[k];
                    tri[9 + k] = ac[k];
                    tri[12 + k] = bd[k];
                    tri[15 + k] = bc[k];
                }
                key[o] = cid * 16 + t * 2;
                key[o + 1] = cid * 16 + t * 2 + 1;
                idx[o] = o;
                idx[o + 1] = o + 1;
                o += 2;
            }
        }
    }
}

__global__ void k_surf_gather(const float* __restrict__ xyz, const int32_t* __restrict__ order, int64_t n,
                              float* __restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n * 9; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = xyz[(int64_t)order[i / 9] * 9 + i % 9];
}

}  // namespace
}  // namespace gp

using namespace gp;

gp_status gp_extract_surface_impl(gp_ctx ctx, int32_t shape, const float* field, float* tri_xyz, int64_t* tri_key,
                                  int64_t capacity, int64_t* n_out, int32_t method)
{
    *n_out = 0;
    const ShapeDesc& d = ctx->h_shapes[shape];
    const int64_t n = (d.brick_end - d.brick_begin) * ((int64_t)ctx->brick * ctx->brick * ctx->brick);
    if (n == 0) return GP_OK;
    if (n >= ((int64_t)1 << 31)) return gp_fail(ctx, GP_ERR_CAPACITY, "too many cells for the surface pass");
    hipStream_t st = ctx->stream;
    const Band B = ctx->band();
    DevBuf<int32_t> count, offset;
    if (count.alloc(n + 1) != hipSuccess || offset.alloc(n + 1) != hipSuccess)
        return gp_fail(ctx, GP_ERR_OOM, "out of device memory for the surface pass");
    GP_HIP(ctx, hipMemsetAsync(count.p + n, 0, sizeof(int32_t), st));
    with_brick(ctx->brick, [&](auto tag) {
        k_surf_count<decltype(tag)::value><<<blocks_for(n), kThreads, 0, st>>>(B, shape, field, method, count.p);
    });
    GP_HIP(ctx, hipGetLastError());
    size_t need = 0;
    GP_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(nullptr, need, count.p, offset.p, (int)(n + 1), st));
    DevBuf<uint8_t> tmp;
    if (tmp.alloc(std::max<size_t>(need, 1)) != hipSuccess)
        return gp_fail(ctx, GP_ERR_OOM, "out of device memory for the surface pass");
    GP_HIP(ctx, hipcub::DeviceScan::ExclusiveSum(tmp.p, need, count.p, offset.p, (int)(n + 1), st));
    int32_t total = 0;
    GP_HIP(ctx, hipMemcpyAsync(&total, offset.p + n, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GP_HIP(ctx, hipStreamSynchronize(st));
    *n_out = total;
    if (total > capacity)
        return gp_fail(ctx, GP_ERR_CAPACITY, "the outputs hold " + std::to_string(capacity) + " triangles, " +
                                                 std::to_string(total) + " needed");
    if (total == 0) return GP_OK;
    DevBuf<float> xyz;
    DevBuf<int64_t> key;
    DevBuf<int32_t> idx, order;
    if (xyz.alloc((size_t)total * 9) != hipSuccess || key.alloc(total) != hipSuccess ||
        idx.alloc(total) != hipSuccess || order.alloc(total) != hipSuccess)
        return gp_fail(ctx, GP_ERR_OOM, "out of device memory for the surface pass");
    with_brick(ctx->brick, [&](auto tag) {
        k_surf_emit<decltype(tag)::value><<<blocks_for(n), kThreads, 0, st>>>(B, shape, field, method, offset.p, xyz.p,
                                                                            key.p, idx.p);
    });
    GP_HIP(ctx, hipGetLastError());
    size_t need2 = 0;
    GP_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(nullptr, need2, key.p, tri_key, idx.p, order.p, total, 0, 64, st));
    DevBuf<uint8_t> tmp2;
    if (tmp2.alloc(std::max<size_t>(need2, 1)) != hipSuccess)
        return gp_fail(ctx, GP_ERR_OOM, "out of device memory for the surface pass");
    GP_HIP(ctx, hipcub::DeviceRadixSort::SortPairs(tmp2.p, need2, key.p, tri_key, idx.p, order.p, total, 0, 64, st));
    k_surf_gather<<<blocks_for((int64_t)total * 9), kThreads, 0, st>>>(xyz.p, order.p, total, tri_xyz);
    GP_HIP(ctx, hipGetLastError());
    GP_HIP(ctx, hipStreamSynchronize(st));
    return GP_OK;
}
