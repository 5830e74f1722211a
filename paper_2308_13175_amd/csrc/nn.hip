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
#include "gp_internal.h"

namespace gp {
namespace {

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

// Gap in cells between the query's local coordinate du (relative to its own
// cell) and the cell at integer offset d on one axis, shrunk by a margin that
// covers float rounding, never negative.
__device__ inline float cell_gap(float du, int32_t d, float margin)
{
    float g = fmaxf((float)d - du, du - (float)(d + 1));
    return fmaxf(g - margin, 0.f);
}

__device__ inline void visit_cell(const Band& B, const ShapeDesc& s, const int32_t* __restrict__ cell_start,
                                  const float* __restrict__ spx, const float* __restrict__ spy,
                                  const float* __restrict__ spz, const int32_t* __restrict__ sid, int32_t x,
                                  int32_t y, int32_t z, float qx, float qy, float qz, Best& best)
{
    int32_t br = brick_of(B, s, x >> 3, y >> 3, z >> 3);
    if (br < 0) return;
    int32_t slot = br * kBrickVol + local_index(x, y, z);
    int32_t b = cell_start[slot], e = cell_start[slot + 1];
    for (int32_t i = b; i < e; ++i) {
        double d2 = exact_d2(qx, qy, qz, spx[i], spy[i], spz[i]);
        int32_t id = sid[i];
        if (d2 < best.d2 || (d2 == best.d2 && id < best.id)) {
            best.d2 = d2;
            best.id = id;
        }
    }
}

__global__ __launch_bounds__(kQueryBlock) void k_nn(Band B, const int32_t* __restrict__ cell_start,
                                                    const float* __restrict__ spx, const float* __restrict__ spy,
                                                    const float* __restrict__ spz, const int32_t* __restrict__ sid,
                                                    const float* __restrict__ qx, const float* __restrict__ qy,
                                                    const float* __restrict__ qz, int32_t* __restrict__ nn)
{
    const int64_t tile = blockIdx.x;
    const int32_t shape = B.tile_shape[tile];
    const ShapeDesc& s = B.shapes[shape];
    const int64_t q0 = B.tile_start[tile];
    const int64_t qe = min(q0 + (int64_t)kQueryTile, s.query_off + s.query_cnt);
    const float h2[3] = {s.h[0] * s.h[0], s.h[1] * s.h[1], s.h[2] * s.h[2]};

    for (int64_t k = q0 + threadIdx.x; k < qe; k += blockDim.x) {
        const float x = qx[k], y = qy[k], z = qz[k];
        int32_t c0[3];
        float du[3], margin[3];
        const float p[3] = {x, y, z};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            double u = ((double)p[a] - s.lo[a]) * s.inv_h[a];
            double fl = fmin(fmax(floor(u), 0.0), (double)(s.R[a] - 1));
            c0[a] = (int32_t)fl;
            du[a] = (float)(u - fl);
            margin[a] = 1e-4f * (1.f + fabsf(du[a]));
        }
        Best best{__builtin_inf(), 0x7fffffff};
        if (s.point_cnt > 0) {
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
                            visit_cell(B, s, cell_start, spx, spy, spz, sid, cx, cy, cz, x, y, z, best);
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
        }
        nn[k] = s.point_cnt > 0 ? best.id : -1;
    }
}

}  // namespace
}  // namespace gp

using namespace gp;

gp_status gp_nn_impl(gp_ctx ctx, const float* qx, const float* qy, const float* qz, int32_t* nn)
{
    if (ctx->n_tiles == 0) return GP_OK;
    GP_TIMED(ctx, "k_nn");
    k_nn<<<(unsigned)ctx->n_tiles, kQueryBlock, 0, ctx->stream>>>(ctx->band(), ctx->cell_start.p, ctx->spx.p,
                                                                  ctx->spy.p, ctx->spz.p, ctx->sid.p, qx, qy, qz, nn);
    GP_HIP(ctx, hipGetLastError());
    return GP_OK;
}
