// Query sampling (Sec. 3: queries drawn from a Gaussian around randomly chosen
// surface points, resampled every iteration).
//
// Sources are stratified over the points in their cell-sorted order, so a
// block of consecutive queries stays inside a small region of the grid (good
// locality for every later kernel) while each point is used floor(Q/J) or
// ceil(Q/J) times per iteration; a random rotation per iteration changes which
// points are used when Q < J.  Offsets come from the counter-based
// Philox4x32-10 generator (Salmon et al., SC'11) and the Box-Muller transform,
// so query k of iteration t is reproducible from (seed, t, shape, k) alone.
#include "gp_internal.h"

namespace gp {
namespace {

struct U4 {
    uint32_t x[4];
};

__device__ inline U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1)
{
    U4 c{{c0, c1, c2, c3}};
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c.x[0];
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c.x[2];
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.x[2]);
        U4 n{{hi1 ^ c.x[1] ^ k0, lo1, hi0 ^ c.x[3] ^ k1, lo0}};
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ inline float unit_open(uint32_t x)
{
    // ((x >> 8) + 1/2) * 2^-24: exact in float, strictly inside (0, 1)
    return ((float)(x >> 8) + 0.5f) * 5.9604644775390625e-8f;
}

__global__ __launch_bounds__(kQueryBlock) void k_sample(Band B, const float4* __restrict__ spts,
                                                        const float* __restrict__ sigma, float sigma_const,
                                                        uint32_t key0, uint32_t key1, int32_t iteration_arg,
                                                        const int32_t* __restrict__ iter_counter,
                                                        float* __restrict__ qx, float* __restrict__ qy,
                                                        float* __restrict__ qz, int32_t* __restrict__ src)
{
    const int64_t tile = blockIdx.x;
    const int32_t shape = B.tile_shape[tile];
    const ShapeDesc& s = B.shapes[shape];
    const int64_t q0 = B.tile_start[tile];
    const int64_t qe = min(q0 + (int64_t)kQueryTile, s.query_off + s.query_cnt);
    const int64_t J = s.point_cnt, Q = s.query_cnt;
    const uint32_t iteration = (uint32_t)(iteration_arg >= 0 ? iteration_arg : *iter_counter + 1);
    if (J <= 0) {
        for (int64_t k = q0 + threadIdx.x; k < qe; k += blockDim.x) {
            qx[k] = qy[k] = qz[k] = __builtin_nanf("");
            if (src) src[k] = -1;
        }
        return;
    }
    // per-iteration rotation of the source order
    const U4 ro = philox4x32_10(0xFFFFFFFFu, 0xFFFFFFFFu, iteration, (uint32_t)shape, key0, key1);
    const int64_t rot = (int64_t)(ro.x[0] % (uint32_t)J);
    for (int64_t k = q0 + threadIdx.x; k < qe; k += blockDim.x) {
        const int64_t kk = k - s.query_off;
        int64_t j = (kk * J) / Q + rot;
        if (j >= J) j -= J;
        const int64_t p = s.sorted_off + j;
        const float4 sp = spts[p];
        const int32_t orig = __float_as_int(sp.w);
        const float sg = sigma ? sigma[s.point_off + orig] : sigma_const;
        const U4 r = philox4x32_10((uint32_t)kk, (uint32_t)((uint64_t)kk >> 32), iteration, (uint32_t)shape, key0, key1);
        const float u0 = unit_open(r.x[0]), u1 = unit_open(r.x[1]);
        const float u2 = unit_open(r.x[2]), u3 = unit_open(r.x[3]);
        const float r0 = sqrtf(-2.f * logf(u0));
        const float r1 = sqrtf(-2.f * logf(u2));
        float s1, c1, s3, c3;
        sincospif(2.f * u1, &s1, &c1);
        sincospif(2.f * u3, &s3, &c3);
        qx[k] = fmaf(sg, r0 * c1, sp.x);
        qy[k] = fmaf(sg, r0 * s1, sp.y);
        qz[k] = fmaf(sg, r1 * c3, sp.z);
        if (src) src[k] = orig;
    }
}

}  // namespace
}  // namespace gp

using namespace gp;

gp_status gp_sample_impl(gp_ctx ctx, uint64_t seed, int32_t iteration, const float* sigma, float sigma_const,
                         float* qx, float* qy, float* qz, int32_t* src)
{
    if (ctx->n_tiles == 0) return GP_OK;
    GP_TIMED(ctx, "k_sample");
    k_sample<<<(unsigned)ctx->n_tiles, kQueryBlock, 0, ctx->stream>>>(
        ctx->band(), ctx->spts.p, sigma, sigma_const, (uint32_t)seed,
        (uint32_t)(seed >> 32), iteration, ctx->iter.p, qx, qy, qz, src);
    GP_HIP(ctx, hipGetLastError());
    return GP_OK;
}
