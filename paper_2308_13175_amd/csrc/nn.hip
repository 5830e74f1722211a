// Nearest surface point NN(q) of every query (Eq. 4).
//
// The paper organises the points in a KD-tree.  On the GPU the points are
// instead bucketed by grid cell (sorted by the slot of their cell, built once
// in band.hip), and each query searches cells ring by ring around its own
// cell.  A cell is opened only if its box can hold a point at least as close
// as the best so far, and the search stops once every unopened cell is
// provably farther.  Distances are compared exactly in double without fused
// multiply-add, ties going to the lowest point index, so the result equals a
// brute-force search bit for bit.
//
// A block handles a tile of 1024 queries that the sampler drew from
// neighbouring points.  Before searching, the block stages the bounding box
// of its queries' cells (grown by one cell) in LDS: a per-cell offset table
// and the points of those cells, copied cooperatively.  Ring searches then read
// cells inside the box from LDS and only cells outside it from global memory,
// so the result does not depend on the staging.
#include "gp_internal.h"

namespace gp {
namespace {

constexpr int kNnExpand = 1;           // cells added on every side of the tile's query box
constexpr int kNnMaxCells = 4096;      // staged cells
constexpr int kNnMaxPoints = 4096;     // staged points

struct Best {
    double d2;
    int32_t id;
};

__device__ inline double exact_d2(float qx, float qy, float qz, float sx, float sy, float sz)
{
#pragma clang fp contract(off)
    double dx = (double)qx - (double)sx;
    double dy = (double)qy - (double)sy;
    double dz = (double)qz - (double)sz;
    double xx = dx * dx;
    double yy = dy * dy;
    double zz = dz * dz;
    double s = xx + yy;
    return s + zz;
}

__device__ inline void consider(double d2, int32_t id, Best& best)
{
    if (d2 < best.d2 || (d2 == best.d2 && id < best.id)) {
        best.d2 = d2;
        best.id = id;
    }
}

// Gap in cells between the query's local coordinate du (relative to its own
// cell) and the cell at integer offset d on one axis, shrunk by a margin that
// covers float rounding, never negative.
__device__ inline float cell_gap(float du, int32_t d, float margin)
{
    float g = fmaxf((float)d - du, du - (float)(d + 1));
    return fmaxf(g - margin, 0.f);
}

struct Global {
    const int32_t* cell_start;
    const float* spx;
    const float* spy;
    const float* spz;
    const int32_t* sid;
};

struct Staged {
    int32_t lo[3], dim[3];
    bool ok;
    const uint16_t* off;   // [ncell + 1] first staged point of each cell
    const float4* pts;     // x, y, z, id (bit pattern)
};

// Global range of the points of cell (x, y, z): false if the cell holds none.
__device__ inline bool cell_range(const Band& B, const ShapeDesc& s, const Global& G, int32_t x, int32_t y, int32_t z,
                                  int32_t& b, int32_t& e)
{
    const int32_t br = brick_of(B, s, x >> 3, y >> 3, z >> 3);
    if (br < 0) return false;
    const int32_t local = local_index(x, y, z);
    if (!mask_bit(B.m_base, br, local)) return false;
    const int32_t slot = br * kBrickVol + local;
    b = G.cell_start[slot];
    e = G.cell_start[slot + 1];
    return e > b;
}

__device__ inline void visit_cell(const Band& B, const ShapeDesc& s, const Global& G, const Staged& S, int32_t x,
                                  int32_t y, int32_t z, float qx, float qy, float qz, Best& best)
{
    if (S.ok) {
        const int32_t lx = x - S.lo[0], ly = y - S.lo[1], lz = z - S.lo[2];
        if ((uint32_t)lx < (uint32_t)S.dim[0] && (uint32_t)ly < (uint32_t)S.dim[1] &&
            (uint32_t)lz < (uint32_t)S.dim[2]) {
            const int32_t li = (lx * S.dim[1] + ly) * S.dim[2] + lz;
            const int32_t b = S.off[li], e = S.off[li + 1];
            for (int32_t i = b; i < e; ++i) {
                const float4 p = S.pts[i];
                consider(exact_d2(qx, qy, qz, p.x, p.y, p.z), __float_as_int(p.w), best);
            }
            return;
        }
    }
    int32_t b, e;
    if (!cell_range(B, s, G, x, y, z, b, e)) return;
    for (int32_t i = b; i < e; ++i) consider(exact_d2(qx, qy, qz, G.spx[i], G.spy[i], G.spz[i]), G.sid[i], best);
}

// Query's clamped cell and its local coordinate within that cell.
__device__ inline void query_cell(const ShapeDesc& s, float x, float y, float z, int32_t c0[3], float du[3])
{
    const float p[3] = {x, y, z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double u = ((double)p[a] - s.lo[a]) * s.inv_h[a];
        double fl = fmin(fmax(floor(u), 0.0), (double)(s.R[a] - 1));
        c0[a] = (int32_t)fl;
        du[a] = (float)(u - fl);
    }
}

__device__ inline int32_t search(const Band& B, const ShapeDesc& s, const Global& G, const Staged& S, float x,
                                 float y, float z)
{
    if (s.point_cnt <= 0) return -1;
    int32_t c0[3];
    float du[3], margin[3];
    query_cell(s, x, y, z, c0, du);
#pragma unroll
    for (int a = 0; a < 3; ++a) margin[a] = 1e-4f * (1.f + fabsf(du[a]));
    const float h2[3] = {s.h[0] * s.h[0], s.h[1] * s.h[1], s.h[2] * s.h[2]};
    Best best{__builtin_inf(), 0x7fffffff};
    for (int32_t r = 0;; ++r) {
        const int32_t xl = max(c0[0] - r, 0), xh = min(c0[0] + r, s.R[0] - 1);
        const int32_t yl = max(c0[1] - r, 0), yh = min(c0[1] + r, s.R[1] - 1);
        const int32_t zl = max(c0[2] - r, 0), zh = min(c0[2] + r, s.R[2] - 1);
        for (int32_t cx = xl; cx <= xh; ++cx) {
            const int32_t dx = cx - c0[0];
            const float gx = cell_gap(du[0], dx, margin[0]);
            const float lbx = gx * gx * h2[0];
            if ((double)lbx > best.d2) continue;
            const bool on_x = (dx == -r || dx == r);
            for (int32_t cy = yl; cy <= yh; ++cy) {
                const int32_t dy = cy - c0[1];
                const float gy = cell_gap(du[1], dy, margin[1]);
                const float lbxy = fmaf(gy * gy, h2[1], lbx);
                if ((double)lbxy > best.d2) continue;
                const bool on_xy = on_x || dy == -r || dy == r;
                // on the ring's x/y faces every z is on the ring; inside, only z = +-r
                const int32_t z_first = on_xy ? zl : c0[2] - r;
                const int32_t z_step = on_xy ? 1 : (r > 0 ? 2 * r : 1);
                const int32_t z_last = on_xy ? zh : c0[2] + r;
                for (int32_t cz = z_first; cz <= z_last; cz += z_step) {
                    if (cz < 0 || cz >= s.R[2]) continue;
                    const float gz = cell_gap(du[2], cz - c0[2], margin[2]);
                    const float lb = fmaf(gz * gz, h2[2], lbxy) * (1.f - 1e-6f);
                    if ((double)lb > best.d2) continue;
                    visit_cell(B, s, G, S, cx, cy, cz, x, y, z, best);
                }
            }
        }
        // every cell with Chebyshev offset <= r is done; bound the rest
        float bound = __builtin_inff();
        bool more = false;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (c0[a] - r - 1 >= 0) {
                more = true;
                float g = fmaxf(du[a] + (float)r - margin[a], 0.f);
                bound = fminf(bound, g * g * h2[a]);
            }
            if (c0[a] + r + 1 <= s.R[a] - 1) {
                more = true;
                float g = fmaxf((float)(r + 1) - du[a] - margin[a], 0.f);
                bound = fminf(bound, g * g * h2[a]);
            }
        }
        if (!more) break;
        if (best.d2 < (double)(bound * (1.f - 1e-6f))) break;
    }
    return best.id;
}

// Exclusive prefix sum of one int per thread over the block (blockDim = 256).
__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t* scratch /* [4] */, int32_t& total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        int32_t w = __shfl_up(incl, o, 64);
        if (lane >= o) incl += w;
    }
    if (lane == 63) scratch[wave] = incl;
    __syncthreads();
    int32_t base = 0;
    total = 0;
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) {
        if (w < wave) base += scratch[w];
        total += scratch[w];
    }
    __syncthreads();
    return base + incl - v;
}

__global__ __launch_bounds__(kQueryBlock) void k_nn(Band B, Global G, const float* __restrict__ qx,
                                                    const float* __restrict__ qy, const float* __restrict__ qz,
                                                    int32_t* __restrict__ nn)
{
    __shared__ uint16_t s_off[kNnMaxCells + 1];
    __shared__ float4 s_pts[kNnMaxPoints];
    __shared__ int32_t s_red[4 * 6];
    __shared__ int32_t s_flag;

    const int64_t tile = blockIdx.x;
    const int32_t shape = B.tile_shape[tile];
    const ShapeDesc& s = B.shapes[shape];
    const int64_t q0 = B.tile_start[tile];
    const int64_t qe = min(q0 + (int64_t)kQueryTile, s.query_off + s.query_cnt);

    // ---- bounding box of the tile's query cells ---------------------------
    int32_t box[6] = {0x7fffffff, 0x7fffffff, 0x7fffffff, -1, -1, -1};
    for (int64_t k = q0 + threadIdx.x; k < qe; k += blockDim.x) {
        int32_t c0[3];
        float du[3];
        query_cell(s, qx[k], qy[k], qz[k], c0, du);
        for (int a = 0; a < 3; ++a) {
            box[a] = min(box[a], c0[a]);
            box[3 + a] = max(box[3 + a], c0[a]);
        }
    }
    block_minmax6(box, s_red);
    Staged S;
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
        S.lo[a] = max(box[a] - kNnExpand, 0);
        S.dim[a] = min(box[3 + a] + kNnExpand, s.R[a] - 1) - S.lo[a] + 1;
        ncell *= S.dim[a];
    }
    S.off = s_off;
    S.pts = s_pts;
    S.ok = s.point_cnt > 0 && ncell <= kNnMaxCells;

    // ---- stage the box: counts, prefix sum, copy ---------------------------
    if (S.ok) {
        const int32_t nc = (int32_t)ncell;
        const int32_t chunk = (nc + blockDim.x - 1) / blockDim.x;
        const int32_t c_begin = min((int32_t)threadIdx.x * chunk, nc), c_end = min(c_begin + chunk, nc);
        if (threadIdx.x == 0) s_flag = 0;
        __syncthreads();
        int32_t mine = 0;
        for (int32_t i = c_begin; i < c_end; ++i) {
            const int32_t lz = i % S.dim[2], ly = (i / S.dim[2]) % S.dim[1], lx = i / (S.dim[2] * S.dim[1]);
            int32_t b = 0, e = 0;
            cell_range(B, s, G, S.lo[0] + lx, S.lo[1] + ly, S.lo[2] + lz, b, e);
            const int32_t c = e - b;
            if (c > kNnMaxPoints) s_flag = 1;
            s_off[i] = (uint16_t)min(c, kNnMaxPoints);
            mine += c;
        }
        int32_t total = 0;
        int32_t base = block_exclusive_scan(mine, s_red, total);
        if (total > kNnMaxPoints) s_flag = 1;
        for (int32_t i = c_begin; i < c_end; ++i) {
            const int32_t c = s_off[i];
            s_off[i] = (uint16_t)min(base, kNnMaxPoints);
            base += c;
        }
        if (threadIdx.x == blockDim.x - 1) s_off[nc] = (uint16_t)min(total, kNnMaxPoints);
        __syncthreads();
        S.ok = s_flag == 0;
        if (S.ok) {
            for (int32_t i = threadIdx.x; i < nc; i += blockDim.x) {
                const int32_t lz = i % S.dim[2], ly = (i / S.dim[2]) % S.dim[1], lx = i / (S.dim[2] * S.dim[1]);
                int32_t b = 0, e = 0;
                if (!cell_range(B, s, G, S.lo[0] + lx, S.lo[1] + ly, S.lo[2] + lz, b, e)) continue;
                int32_t d = s_off[i];
                for (int32_t j = b; j < e; ++j, ++d)
                    s_pts[d] = make_float4(G.spx[j], G.spy[j], G.spz[j], __int_as_float(G.sid[j]));
            }
        }
        __syncthreads();
    }

    // ---- exact ring search per query -----------------------------------------
    for (int64_t k = q0 + threadIdx.x; k < qe; k += blockDim.x) nn[k] = search(B, s, G, S, qx[k], qy[k], qz[k]);
}

}  // namespace
}  // namespace gp

using namespace gp;

gp_status gp_nn_impl(gp_ctx ctx, const float* qx, const float* qy, const float* qz, int32_t* nn)
{
    if (ctx->n_tiles == 0) return GP_OK;
    Global G{ctx->cell_start.p, ctx->spx.p, ctx->spy.p, ctx->spz.p, ctx->sid.p};
    GP_TIMED(ctx, "k_nn");
    k_nn<<<(unsigned)ctx->n_tiles, kQueryBlock, 0, ctx->stream>>>(ctx->band(), G, qx, qy, qz, nn);
    GP_HIP(ctx, hipGetLastError());
    return GP_OK;
}
