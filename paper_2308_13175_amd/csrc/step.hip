// Adam step over the field slots (Sec. 4 "Details": Adam with a stepwise
// decayed learning rate; only band variables are optimised, Sec. 3) and the
// layout helpers that convert between the brick slots and dense vertex ids.
#include <hipcub/hipcub.hpp>

#include "gp_internal.h"

namespace gp {
namespace {

constexpr int kThreads = 256;

inline unsigned blocks_for(int64_t n)
{
    int64_t b = (n + kThreads - 1) / kThreads;
    if (b < 1) b = 1;
    if (b > (int64_t)1 << 30) b = (int64_t)1 << 30;
    return (unsigned)b;
}

#define GRID_STRIDE(i, n) \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (int64_t)gridDim.x * blockDim.x)

// Step constants on the device, so that a captured graph of a whole
// iteration advances the schedule on every replay.  t_arg >= 1 sets the
// iteration; t_arg == 0 advances the stored counter by one.
__global__ void k_step_consts(int32_t* __restrict__ iter, float* __restrict__ c, int32_t t_arg, float lr0,
                              float decay, int32_t decay_every, float beta1, float beta2)
{
    const int32_t t = t_arg > 0 ? t_arg : *iter + 1;
    *iter = t;
    const double lr = (double)lr0 * pow((double)decay, (double)((t - 1) / decay_every));
    const double bc1 = 1.0 - pow((double)beta1, (double)t);
    const double bc2 = 1.0 - pow((double)beta2, (double)t);
    c[0] = (float)(lr / bc1);
    c[1] = (float)(1.0 / sqrt(bc2));
}

// One thread per slot; c[0] = lr_t / (1 - beta1^t), c[1] = 1 / sqrt(1 - beta2^t).
__global__ void k_adam(const uint32_t* __restrict__ m_v, int64_t n_slots, float* __restrict__ D,
                       float* __restrict__ G, float* __restrict__ M, float* __restrict__ V,
                       const float* __restrict__ c, float beta1, float beta2, float eps)
{
    const float lr_over_bc1 = c[0], inv_sqrt_bc2 = c[1];
    GRID_STRIDE(i, n_slots)
    {
        const uint32_t word = m_v[i >> 5];
        const float g = G[i];
        if ((word >> (i & 31)) & 1u) {
            const float m = fmaf(beta1, M[i], (1.f - beta1) * g);
            const float v = fmaf(beta2, V[i], (1.f - beta2) * g * g);
            M[i] = m;
            V[i] = v;
            D[i] -= lr_over_bc1 * m / fmaf(sqrtf(v), inv_sqrt_bc2, eps);
        }
        G[i] = 0.f;
    }
}

template <int kB>
__device__ inline int64_t slot_vertex(const Band& B, int64_t slot, int32_t& shape, int32_t ijk[3])
{
    using G = Geo<kB>;
    const BrickInfo bi = B.bricks[slot / G::V];
    const int32_t local = (int32_t)(slot % G::V);
    const ShapeDesc& s = B.shapes[bi.shape];
    shape = bi.shape;
    ijk[0] = bi.bx * kB + (local >> (2 * G::S));
    ijk[1] = bi.by * kB + ((local >> G::S) & G::M);
    ijk[2] = bi.bz * kB + (local & G::M);
    if (ijk[0] > s.R[0] || ijk[1] > s.R[1] || ijk[2] > s.R[2]) return -1;
    return ((int64_t)ijk[0] * (s.R[1] + 1) + ijk[1]) * (s.R[2] + 1) + ijk[2];
}

template <int kB>
__global__ void k_layout(Band B, const uint32_t* __restrict__ m_base, const uint32_t* __restrict__ m_a2,
                         int64_t n_slots, int64_t* __restrict__ vid, uint8_t* __restrict__ flags)
{
    GRID_STRIDE(i, n_slots)
    {
        int32_t shape, ijk[3];
        const int64_t v = slot_vertex<kB>(B, i, shape, ijk);
        if (vid) vid[i] = v;
        if (flags) {
            const int64_t w = i >> 5;
            const uint32_t bit = 1u << (i & 31);
            uint8_t f = 0;
            if (B.m_v[w] & bit) f |= 1;
            if (B.m_v2[w] & bit) f |= 2;
            if (B.m_a1[w] & bit) f |= 4;
            if (m_a2[w] & bit) f |= 8;
            if (m_base[w] & bit) f |= 16;
            flags[i] = f;
        }
    }
}

// Linear id of the M1-band cell whose lowest corner is each slot of one
// shape's slot range, or -1.
template <int kB>
__global__ void k_active_cells(Band B, int64_t slot0, int64_t n, int64_t* __restrict__ ids)
{
    GRID_STRIDE(i, n)
    {
        const int64_t slot = slot0 + i;
        int32_t shape, ijk[3];
        int64_t id = -1;
        if ((B.m_a1[slot >> 5] >> (slot & 31)) & 1u) {
            slot_vertex<kB>(B, slot, shape, ijk);
            const ShapeDesc& s = B.shapes[shape];
            id = ((int64_t)ijk[0] * s.R[1] + ijk[1]) * s.R[2] + ijk[2];
        }
        ids[i] = id;
    }
}

struct NonNegative {
    __device__ bool operator()(const int64_t& v) const { return v >= 0; }
};

template <int kB>
__global__ void k_gather(Band B, int64_t n_slots, const float* __restrict__ dense, float* __restrict__ field,
                         int to_field)
{
    GRID_STRIDE(i, n_slots)
    {
        int32_t shape, ijk[3];
        const int64_t v = slot_vertex<kB>(B, i, shape, ijk);
        const int64_t off = B.shapes[shape].dense_off;
        if (to_field) {
            field[i] = v >= 0 ? dense[off + v] : 0.f;
        } else if (v >= 0 && ((B.m_v[i >> 5] >> (i & 31)) & 1u)) {
            const_cast<float*>(dense)[off + v] = field[i];
        }
    }
}

template <int kB>
__global__ void k_init_sphere(Band B, int64_t n_slots, const double* __restrict__ centre,
                              const double* __restrict__ radius, float* __restrict__ field)
{
    GRID_STRIDE(i, n_slots)
    {
        int32_t shape, ijk[3];
        const int64_t v = slot_vertex<kB>(B, i, shape, ijk);
        if (v < 0) {
            field[i] = 0.f;
            continue;
        }
        const ShapeDesc& s = B.shapes[shape];
        double r2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double x = s.lo[a] + (double)ijk[a] / s.inv_h[a] - centre[3 * shape + a];
            r2 += x * x;
        }
        field[i] = (float)(sqrt(r2) - radius[shape]);
    }
}

}  // namespace
}  // namespace gp

using namespace gp;

gp_status gp_step_consts_impl(gp_ctx ctx, int32_t t, float lr0, float decay, int32_t decay_every, float beta1,
                              float beta2)
{
    GP_TIMED(ctx, "k_step_consts");
    k_step_consts<<<1, 1, 0, ctx->stream>>>(ctx->iter.p, ctx->step_c.p, t, lr0, decay, decay_every, beta1, beta2);
    GP_HIP(ctx, hipGetLastError());
    return GP_OK;
}

gp_status gp_step_impl(gp_ctx ctx, float* field, float* grad, float* m, float* v, float beta1, float beta2, float eps)
{
    if (ctx->n_slots == 0) return GP_OK;
    GP_TIMED(ctx, "k_adam");
    k_adam<<<blocks_for(ctx->n_slots), kThreads, 0, ctx->stream>>>(ctx->m_v.p, ctx->n_slots, field, grad, m, v,
                                                                   ctx->step_c.p, beta1, beta2, eps);
    GP_HIP(ctx, hipGetLastError());
    return GP_OK;
}

gp_status gp_layout_impl(gp_ctx ctx, int64_t* vid, uint8_t* flags)
{
    if (ctx->n_slots == 0) return GP_OK;
    with_brick(ctx->brick, [&](auto tag) {
        k_layout<decltype(tag)::value><<<blocks_for(ctx->n_slots), kThreads, 0, ctx->stream>>>(
            ctx->band(), ctx->m_base.p, ctx->m_a2.p, ctx->n_slots, vid, flags);
    });
    GP_HIP(ctx, hipGetLastError());
    return GP_OK;
}

gp_status gp_gather_impl(gp_ctx ctx, const float* dense, float* field, bool to_field)
{
    if (ctx->n_slots == 0) return GP_OK;
    with_brick(ctx->brick, [&](auto tag) {
        k_gather<decltype(tag)::value><<<blocks_for(ctx->n_slots), kThreads, 0, ctx->stream>>>(
            ctx->band(), ctx->n_slots, dense, field, to_field ? 1 : 0);
    });
    GP_HIP(ctx, hipGetLastError());
    return GP_OK;
}

gp_status gp_init_sphere_impl(gp_ctx ctx, const double* centre, const double* radius, float* field)
{
    if (ctx->n_slots == 0) return GP_OK;
    const int32_t n = ctx->n_shapes;
    DevBuf<double> d;
    GP_HIP(ctx, d.alloc(4 * (size_t)n));
    GP_HIP(ctx, hipMemcpyAsync(d.p, centre, 3 * sizeof(double) * n, hipMemcpyHostToDevice, ctx->stream));
    GP_HIP(ctx, hipMemcpyAsync(d.p + 3 * n, radius, sizeof(double) * n, hipMemcpyHostToDevice, ctx->stream));
    with_brick(ctx->brick, [&](auto tag) {
        k_init_sphere<decltype(tag)::value><<<blocks_for(ctx->n_slots), kThreads, 0, ctx->stream>>>(
            ctx->band(), ctx->n_slots, d.p, d.p + 3 * n, field);
    });
    GP_HIP(ctx, hipGetLastError());
    GP_HIP(ctx, hipStreamSynchronize(ctx->stream));   // the scratch is freed on return
    return GP_OK;
}

gp_status gp_active_cells_impl(gp_ctx ctx, int32_t shape, int64_t* cell_ids, int64_t capacity, int64_t* n_out)
{
    const int64_t b = ctx->h_slot_begin[shape], e = ctx->h_slot_begin[shape + 1], n = e - b;
    *n_out = 0;
    if (n == 0) return GP_OK;
    hipStream_t st = ctx->stream;
    DevBuf<int64_t> ids, sel;
    DevBuf<int64_t> cnt;
    if (ids.alloc(n) != hipSuccess || sel.alloc(n) != hipSuccess || cnt.alloc(1) != hipSuccess)
        return gp_fail(ctx, GP_ERR_OOM, "out of device memory for the cell export");
    with_brick(ctx->brick, [&](auto tag) {
        k_active_cells<decltype(tag)::value><<<blocks_for(n), kThreads, 0, st>>>(ctx->band(), b, n, ids.p);
    });
    GP_HIP(ctx, hipGetLastError());
    size_t need = 0;
    GP_HIP(ctx, hipcub::DeviceSelect::If(nullptr, need, ids.p, sel.p, cnt.p, (int)n, NonNegative(), st));
    DevBuf<uint8_t> tmp;
    if (tmp.alloc(need) != hipSuccess) return gp_fail(ctx, GP_ERR_OOM, "out of device memory for the cell export");
    GP_HIP(ctx, hipcub::DeviceSelect::If(tmp.p, need, ids.p, sel.p, cnt.p, (int)n, NonNegative(), st));
    int64_t m = 0;
    GP_HIP(ctx, hipMemcpyAsync(&m, cnt.p, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    GP_HIP(ctx, hipStreamSynchronize(st));
    *n_out = m;
    if (m > capacity)
        return gp_fail(ctx, GP_ERR_CAPACITY, "cell_ids holds " + std::to_string(capacity) + " ids, " +
                                                 std::to_string(m) + " needed");
    if (m == 0) return GP_OK;
    // slot order is brick-major: sort the ids
    size_t need2 = 0;
    GP_HIP(ctx, hipcub::DeviceRadixSort::SortKeys(nullptr, need2, sel.p, cell_ids, (int)m, 0, 64, st));
    DevBuf<uint8_t> tmp2;
    if (tmp2.alloc(need2) != hipSuccess) return gp_fail(ctx, GP_ERR_OOM, "out of device memory for the cell export");
    GP_HIP(ctx, hipcub::DeviceRadixSort::SortKeys(tmp2.p, need2, sel.p, cell_ids, (int)m, 0, 64, st));
    GP_HIP(ctx, hipStreamSynchronize(st));
    return GP_OK;
}
