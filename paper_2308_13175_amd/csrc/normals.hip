// Normal supervision (Sec. 4, normals paragraph): when ground-truth normals
// of the points are known, the field's gradient at the surface points is
// supervised by them.  Reading: the same cosine form as the gradient-
// consistency term, with the point's normal in place of the query's gradient,
//   L_N = (1/Q_v) sum over valid queries of (1 - gh_s . n_s),
// s = NN(q), gh_s = grad f(s) / |grad f(s)| (below the norm threshold the term
// is 1 with zero gradient), valid queries as for the pull loss (in the grid,
// in an M1-band cell).  Its gradient with respect to grad f(s) is
// -(n_s - (gh_s . n_s) gh_s) / |grad f(s)|, scattered into the 8 corners of
// s's cell through the derivatives of the trilinear weights.
//
// Three launches: per-block partial sums (term, count), a per-shape mean
// (and the gradient scale weight * dloss / Q_v), and the scatter (float
// atomics on the gradient: an optional term, kept out of the fused pass).
#include "gp_internal.h"

namespace gp {
namespace {

constexpr int kNrmBlock = 256;

struct SurfEval {
    int32_t slot[8];
    float t[3];
    double gh[3];
    double n;
    bool ok;
    int64_t point;   // global index of s in the caller's point and normal arrays
};

// Validity of query (x, y, z) and the field at its nearest point; false for
// an invalid query or an index outside the shape's points.
template <int kB>
__device__ inline bool eval_nearest(const Band& B, const ShapeDesc& s, const float* __restrict__ D, float x, float y,
                                    float z, int64_t k, int32_t nn, const PointView& P, SurfEval& e)
{
    const Loc L = locate(s, x, y, z);
    if (!L.inside) return false;
    using G = Geo<kB>;
    const int32_t br = brick_of(B, s, L.c[0] >> G::S, L.c[1] >> G::S, L.c[2] >> G::S);
    if (br < 0 || !mask_bit_b<kB>(B.m_a1, br, local_index_b<kB>(L.c[0], L.c[1], L.c[2]))) return false;
    if (nn < 0 || nn >= s.point_cnt) return false;
    float sx, sy, sz;
    nearest_point(s, P, k, nn, sx, sy, sz);
    const Loc Ls = locate(s, sx, sy, sz);
    corner_slots<kB>(B, s, Ls.c, e.slot);
    float v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = D[e.slot[i]];
    const Interp it = trilinear(v, Ls.t, s.inv_h);
    e.n = sqrt(fma(it.g[0], it.g[0], fma(it.g[1], it.g[1], it.g[2] * it.g[2])));
    e.ok = e.n >= kEpsNorm;
    const double inv = e.ok ? 1.0 / e.n : 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        e.gh[a] = it.g[a] * inv;
        e.t[a] = (float)Ls.t[a];
    }
    e.point = s.point_off + nn;
    return true;
}

__device__ inline double block_sum256(double v, double* lds)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    const double r = (lds[0] + lds[1]) + (lds[2] + lds[3]);
    __syncthreads();
    return r;
}

template <int kB>
__global__ __launch_bounds__(kNrmBlock) void k_normal_terms(Band B, const float* __restrict__ qx,
                                                            const float* __restrict__ qy,
                                                            const float* __restrict__ qz,
                                                            const int32_t* __restrict__ nn,
                                                            PointView P, const float* __restrict__ D,
                                                            const float* __restrict__ nx,
                                                            const float* __restrict__ ny,
                                                            const float* __restrict__ nz, double* __restrict__ part)
{
    static_assert(kNrmBlock == 256, "four waves");
    __shared__ double lds[4];
    const int64_t tile = blockIdx.x / 4;
    const int32_t shape = B.tile_shape[tile];
    const ShapeDesc& s = B.shapes[shape];
    const int64_t k = B.tile_start[tile] + (int64_t)(blockIdx.x % 4) * kNrmBlock + threadIdx.x;
    const int64_t qe = min(B.tile_start[tile] + (int64_t)kQueryTile, s.query_off + s.query_cnt);
    double term = 0.0, cnt = 0.0;
    SurfEval e;
    if (k < qe && eval_nearest<kB>(B, s, D, qx[k], qy[k], qz[k], k, nn[k], P, e)) {
        const double n[3] = {(double)nx[e.point], (double)ny[e.point], (double)nz[e.point]};
        term = e.ok ? 1.0 - fma(e.gh[0], n[0], fma(e.gh[1], n[1], e.gh[2] * n[2])) : 1.0;
        cnt = 1.0;
    }
    term = block_sum256(term, lds);
    cnt = block_sum256(cnt, lds);
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = term;
        part[2 * blockIdx.x + 1] = cnt;
    }
}

// One thread per shape: the mean and the gradient scale.
__global__ void k_normal_mean(Band B, int32_t n_shapes, const double* __restrict__ part, float weight,
                              const double* __restrict__ dloss, double* __restrict__ term_out,
                              float* __restrict__ scale)
{
    const int32_t shape = blockIdx.x * blockDim.x + threadIdx.x;
    if (shape >= n_shapes) return;
    const ShapeDesc& s = B.shapes[shape];
    double t = 0.0, c = 0.0;
    for (int64_t b = s.tile_begin * 4; b < s.tile_end * 4; ++b) {
        t += part[2 * b];
        c += part[2 * b + 1];
    }
    term_out[shape] = c > 0.0 ? t / c : 0.0;
    scale[shape] = c > 0.0 ? (float)((double)weight * (dloss ? dloss[shape] : 1.0) / c) : 0.f;
}

template <int kB>
__global__ __launch_bounds__(kNrmBlock) void k_normal_scatter(Band B, const float* __restrict__ qx,
                                                              const float* __restrict__ qy,
                                                              const float* __restrict__ qz,
                                                              const int32_t* __restrict__ nn,
                                                              PointView P,
                                                              const float* __restrict__ D,
                                                              const float* __restrict__ nx,
                                                              const float* __restrict__ ny,
                                                              const float* __restrict__ nz,
                                                              const float* __restrict__ scale, float* __restrict__ G)
{
    const int64_t tile = blockIdx.x / 4;
    const int32_t shape = B.tile_shape[tile];
    const ShapeDesc& s = B.shapes[shape];
    const int64_t k = B.tile_start[tile] + (int64_t)(blockIdx.x % 4) * kNrmBlock + threadIdx.x;
    const int64_t qe = min(B.tile_start[tile] + (int64_t)kQueryTile, s.query_off + s.query_cnt);
    SurfEval e;
    if (k >= qe || !eval_nearest<kB>(B, s, D, qx[k], qy[k], qz[k], k, nn[k], P, e) || !e.ok) return;
    const double n[3] = {(double)nx[e.point], (double)ny[e.point], (double)nz[e.point]};
    const double c = fma(e.gh[0], n[0], fma(e.gh[1], n[1], e.gh[2] * n[2]));
    float dg[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) dg[a] = (float)(-(n[a] - c * e.gh[a]) / e.n);
    float out[8];
    trilinear_adjoint(e.t, s.inv_hf, 0.f, dg, out);
    const float sc = scale[shape];
#pragma unroll
    for (int i = 0; i < 8; ++i) atomicAdd(&G[e.slot[i]], sc * out[i]);
}

}  // namespace
}  // namespace gp

using namespace gp;

gp_status gp_normals_impl(gp_ctx ctx, const float* qx, const float* qy, const float* qz, const int32_t* nn,
                          const float* field, const float* nx, const float* ny, const float* nz, float weight,
                          const double* dloss, double* term_out, float* grad)
{
    hipStream_t st = ctx->stream;
    const Band B = ctx->band();
    const int64_t blocks = ctx->n_tiles * 4;
    if ((int64_t)ctx->nrm_part.n < std::max<int64_t>(2 * blocks, 1)) GP_HIP(ctx, ctx->nrm_part.alloc(std::max<int64_t>(2 * blocks, 1)));
    if ((int64_t)ctx->nrm_scale.n < ctx->n_shapes) GP_HIP(ctx, ctx->nrm_scale.alloc(ctx->n_shapes));
    if (blocks > 0) {
        GP_TIMED(ctx, "k_normal_terms");
        with_brick(ctx->brick, [&](auto tag) {
            k_normal_terms<decltype(tag)::value><<<(unsigned)blocks, kNrmBlock, 0, st>>>(
                B, qx, qy, qz, nn, ctx->points(), field, nx, ny, nz, ctx->nrm_part.p);
        });
    }
    k_normal_mean<<<(unsigned)((ctx->n_shapes + 63) / 64), 64, 0, st>>>(B, ctx->n_shapes, ctx->nrm_part.p, weight,
                                                                        dloss, term_out, ctx->nrm_scale.p);
    if (grad && blocks > 0) {
        GP_TIMED(ctx, "k_normal_scatter");
        with_brick(ctx->brick, [&](auto tag) {
            k_normal_scatter<decltype(tag)::value><<<(unsigned)blocks, kNrmBlock, 0, st>>>(
                B, qx, qy, qz, nn, ctx->points(), field, nx, ny, nz, ctx->nrm_scale.p, grad);
        });
    }
    GP_HIP(ctx, hipGetLastError());
    return GP_OK;
}
