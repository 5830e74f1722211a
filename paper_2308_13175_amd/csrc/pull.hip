// Forward and backward of the GridPull loss (Eq. 4-8).
//
// Query side, one thread per query of a 1024-query tile:
//   locate q (double), check the M1 band, gather the 8 corners of its cell,
//   f(q) and grad f(q) by trilinear interpolation (Eq. 1 / Eq. 3), the pull
//   p = q - f grad f / |grad f|, the residual p - s to the query's nearest
//   point s = NN(q) (Eq. 4), and at s: f(s) (Eq. 6) and grad f(s) for the
//   cosine term (Eq. 7).  The forward writes per-tile sums (double); the
//   backward (fused with the forward in k_query_grad) takes the adjoint of
//   the same quantities and adds it to the 8 corners at q and the 8 corners
//   at s: summed per block in LDS (fixed point, in rows of the 64-byte
//   gradient lines the block touches), then one float atomic per non-zero
//   entry (or straight to the gradient when the block's box would take too
//   many slabs).
// Vertex side, per brick (a block, or a wave): tau_i over the six axis
//   neighbours that are TV vertices (Eq. 5) in the forward; in the backward
//   the gradient is gathered per vertex (each vertex writes only its own
//   slot).
#include <algorithm>
#include <mutex>

#include "gp_internal.h"

namespace gp {
namespace {

// One side (the query q or its surface point s): the cell, the slots of its
// corners and the field there.  Value, gradient and normalised gradient are
// kept in double: the pull residual and the adjoint below subtract nearly
// equal quantities both far from the surface (|f| >> |q - s|) and near
// convergence (p close to s).
struct Side {
    int32_t c[3];      // cell
    int32_t slot[8];
    float t[3];        // local coordinate (for the adjoint weights)
    double f;          // f
    double g[3];       // grad f
    double n;          // |grad f|
    double gh[3];      // grad f / |grad f| (0 if |grad f| < eps)
    double inv_n;      // 1 / |grad f| (0 if |grad f| < eps)
    bool ok;           // |grad f| >= eps
};

template <int kB>
__device__ inline void eval_side(const Band& B, const ShapeDesc& s, const float* __restrict__ D, const Loc& L,
                                 Side& out)
{
    out.c[0] = L.c[0];
    out.c[1] = L.c[1];
    out.c[2] = L.c[2];
    corner_slots<kB>(B, s, L.c, out.slot);
    float v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = *at32(D, (uint32_t)out.slot[i]);
    out.t[0] = (float)L.t[0];
    out.t[1] = (float)L.t[1];
    out.t[2] = (float)L.t[2];
    const Interp it = trilinear(v, L.t, s.inv_h);
    out.f = it.f;
    out.g[0] = it.g[0];
    out.g[1] = it.g[1];
    out.g[2] = it.g[2];
    out.n = sqrt(fma(it.g[0], it.g[0], fma(it.g[1], it.g[1], it.g[2] * it.g[2])));
    out.ok = out.n >= kEpsNorm;
    const double inv = out.ok ? 1.0 / out.n : 0.0;
    out.inv_n = inv;
    out.gh[0] = it.g[0] * inv;
    out.gh[1] = it.g[1] * inv;
    out.gh[2] = it.g[2] * inv;
}

// Everything one valid query contributes.  Returns false for an invalid query.
struct QueryState {
    Side q, s;
    double d[3];     // q - s (exact)
    double r[3];     // residual p - s = (q - s) - f gh
    double lp;       // |p - s|
};

template <int kB>
__device__ inline bool eval_query(const Band& B, const ShapeDesc& s, const float* __restrict__ D, float x, float y,
                                  float z, int64_t k, int32_t nn, const PointView& P, int32_t* bad_nn, QueryState& st)
{
    // the loads of both sides are issued before any of them is tested
    const Loc L = locate(s, x, y, z);
    const bool nn_ok = nn >= 0 && nn < s.point_cnt;
    float sx = 0.f, sy = 0.f, sz = 0.f;
    if (s.point_cnt > 0) nearest_point(s, P, k, nn_ok ? nn : 0, sx, sy, sz);
    using G = Geo<kB>;
    const int32_t br = L.inside ? brick_of(B, s, L.c[0] >> G::S, L.c[1] >> G::S, L.c[2] >> G::S) : -1;
    if (br < 0 || !mask_bit_b<kB>(B.m_a1, br, local_index_b<kB>(L.c[0], L.c[1], L.c[2]))) return false;
    if (!nn_ok) {
        atomicOr(bad_nn, 2);   // reported as an argument error by the next gp_sync
        return false;
    }
    const Loc Ls = locate(s, sx, sy, sz);
    eval_side<kB>(B, s, D, L, st.q);
    eval_side<kB>(B, s, D, Ls, st.s);
    st.d[0] = (double)x - (double)sx;
    st.d[1] = (double)y - (double)sy;
    st.d[2] = (double)z - (double)sz;
    const double f = st.q.f;
#pragma unroll
    for (int a = 0; a < 3; ++a) st.r[a] = fma(-f, st.q.gh[a], st.d[a]);
    st.lp = sqrt(fma(st.r[0], st.r[0], fma(st.r[1], st.r[1], st.r[2] * st.r[2])));
    return true;
}

template <int N>
__device__ inline void block_sum(double (&v)[N], double* lds /* [4 waves][N] */)
{
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = wave_sum_f64(v[i]);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
        for (int i = 0; i < N; ++i) lds[wave * N + i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = blockDim.x >> 6;
        for (int i = 0; i < N; ++i) {
            double a = 0.0;
            for (int w = 0; w < nw; ++w) a += lds[w * N + i];
            v[i] = a;
        }
    }
}

template <int kB>
__global__ __launch_bounds__(kQueryBlock) void k_forward_query(Band B, const float* __restrict__ qx,
                                                               const float* __restrict__ qy,
                                                               const float* __restrict__ qz,
                                                               const int32_t* __restrict__ nn, PointView P,
                                                               const float* __restrict__ D,
                                                               double* __restrict__ q_part, int32_t* flag)
{
    __shared__ double lds[4 * 4];
    const int64_t tile = xcd_work_item(blockIdx.x, gridDim.x);
    const int32_t shape = B.tile_shape[tile];
    const ShapeDesc& s = B.shapes[shape];
    const int64_t q0 = B.tile_start[tile];
    const int64_t qe = min(q0 + (int64_t)kQueryTile, s.query_off + s.query_cnt);
    double sp = 0.0, ss = 0.0, sg = 0.0;
    int cnt = 0;
    for (int64_t k = q0 + threadIdx.x; k < qe; k += blockDim.x) {
        QueryState st;
        if (!eval_query<kB>(B, s, D, qx[k], qy[k], qz[k], k, nn[k], P, flag, st)) continue;
        const double lg = (st.q.ok && st.s.ok)
                              ? 1.0 - fma(st.q.gh[0], st.s.gh[0], fma(st.q.gh[1], st.s.gh[1], st.q.gh[2] * st.s.gh[2]))
                              : 1.0;
        sp += st.lp;
        ss += fabs(st.s.f);
        sg += lg;
        ++cnt;
    }
    double v[4] = {sp, ss, sg, (double)cnt};
    block_sum<4>(v, lds);
    if (threadIdx.x == 0)
        for (int i = 0; i < 4; ++i) q_part[tile * 4 + i] = v[i];
}

constexpr int kGradParts = 4;                          // blocks per query tile in the gradient pass
constexpr int kGradBlock = kQueryTile / kGradParts;    // one query per thread

// Adjoint of one valid query (Eq. 4, 6, 7 differentiated): the contributions
// to the 8 corners of q's cell and the 8 corners of s's cell.
__device__ inline void query_adjoint(const ShapeDesc& s, const QueryState& st, gp_weights w, float cq[8], float cs[8])
{
    // pull term, d l / d f = -gh.e with e = r/|r|; d l / d grad f is the
    // projection of -f e orthogonal to gh over |grad f|, which equals
    // -f/(|grad f| |r|) (I - gh gh^T)(q - s) because r = (q - s) - f gh
    const double inv_lp = st.lp > 0.0 ? 1.0 / st.lp : 0.0;
    const double* gh = st.q.gh;
    const double* ghs = st.s.gh;
    const double df = -(gh[0] * st.r[0] + gh[1] * st.r[1] + gh[2] * st.r[2]) * inv_lp;
    double dg[3] = {0.0, 0.0, 0.0}, dgs[3] = {0.0, 0.0, 0.0};
    if (st.q.ok) {
        const double k = -st.q.f * inv_lp * st.q.inv_n;
        const double dd = gh[0] * st.d[0] + gh[1] * st.d[1] + gh[2] * st.d[2];
#pragma unroll
        for (int a = 0; a < 3; ++a) dg[a] = k * fma(-dd, gh[a], st.d[a]);
    }
    // gradient-consistency term through both normalised gradients
    if (st.q.ok && st.s.ok) {
        const double c = gh[0] * ghs[0] + gh[1] * ghs[1] + gh[2] * ghs[2];
        const double kq = (double)w.gamma * st.q.inv_n, ks = (double)w.gamma * st.s.inv_n;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            dg[a] -= kq * fma(-c, gh[a], ghs[a]);
            dgs[a] = -ks * fma(-c, ghs[a], gh[a]);
        }
    }
    const double fs = st.s.f;
    const float dfs = w.beta * (fs > 0.0 ? 1.f : (fs < 0.0 ? -1.f : 0.f));
    const float dgf[3] = {(float)dg[0], (float)dg[1], (float)dg[2]};
    const float dgsf[3] = {(float)dgs[0], (float)dgs[1], (float)dgs[2]};
    trilinear_adjoint(st.q.t, s.inv_hf, (float)df, dgf, cq);
    trilinear_adjoint(st.s.t, s.inv_hf, dfs, dgsf, cs);
}

// Accumulation of the contributions of a block.  Its queries come from
// neighbouring points (bricks are numbered along a Morton curve, so
// neighbouring points stay neighbours across brick faces), so their 16 corner
// contributions fall in a small box of the grid, the box of the block's query
// and nearest-point cells, but fill only about a quarter of its vertices: the
// queries lie in a shell around the surface.  The block therefore sums them
// in LDS rows of 16 consecutive slots (one 64-byte line of the gradient: in a
// brick of edge kB, 16 / kB neighbouring y columns of kB vertices each) for
// the lines it touches only:
// - a line map, one 16-bit entry per line of the box (ordered by x, then
//   z-brick, then y line), is marked at every touched line;
// - each wave numbers the marked entries of its share of the map in map order
//   (one LDS counter per block, one atomic per wave and step), so the touched
//   lines get rows 0, 1, ..., lines next to each other in memory mostly on
//   consecutive rows;
// - each contribution is added to its entry (slot mod 16) of its line's row,
//   and the row records its line (slot / 16);
// - the flush walks the rows in order, 16 lanes per row, so that a wave adds
//   whole lines, mostly contiguous runs of them, to the gradient (one float
//   atomic per non-zero entry) and clears what it reads.
// A block touching more lines than there are rows takes the rows in turns
// (each turn adds the contributions of its rows and flushes them).  A box with
// more lines than the map takes slabs of whole x layers, each marked,
// numbered and flushed on its own; a box that would take more than the
// context's maximum number of slabs sends its contributions straight to the
// gradient (global float atomics).  The rows' size (LDS allocated at launch)
// and that maximum are settings of the context (gp_set_grad_params).
// The entries hold fixed point with 32 fraction bits in 64-bit integers:
// integer LDS atomics run at full rate where float ones do not (measured:
// float accumulators made the pass several times slower), and the sums inside
// a block are exact and independent of the order of the adds.  A
// contribution of 2^19 or more in magnitude bypasses the rows, so no sum
// leaves the range of the fixed point (a vertex receives at most 2
// contributions from each of the 256 queries).  The conversion adds
// 1.5 * 2^52 to the scaled value in double: for |v| < 2^51 the sum lies in
// [2^52, 2^53), where the double's ulp is 1, so the addition rounds v to the
// nearest integer (ties to even, as a rounding conversion would) and the
// sum's bits minus those of 1.5 * 2^52 are that integer in two's complement.
constexpr int32_t kRowSlots = 16;   // slots per row (one 64-byte line of the gradient)
constexpr int32_t kLineMap = 2048;  // line-map entries (16 bits each)

// LDS of a query block: the rows (cap 64-bit entries), each row's line, then the line map.
__host__ __device__ constexpr int32_t win_lds_bytes(int32_t cap)
{
    return cap * 8 + (cap / kRowSlots) * 4 + kLineMap * 2;
}
static_assert(win_lds_bytes(4096) + 512 <= 160 * 1024 / 4, "default rows: four blocks per CU");
static_assert(win_lds_bytes(kWinCapMax) <= 64 * 1024 - 512, "rows within one workgroup's 64 KB");
constexpr double kFixScale = 4294967296.0;   // 2^32
constexpr float kFixLimit = 524288.f;        // 2^19
constexpr double kFixMagic = 6755399441055744.0;   // 1.5 * 2^52

// Lines of a brick of edge kB: 16 / kB = 2^L neighbouring y columns each.
template <int kB>
struct LineGeo {
    static constexpr int32_t L = 4 - Geo<kB>::S;
};

// The box of a block in lines: x vertices lo .. lo + nx - 1, z-bricks
// zb0 .. zb0 + nzb - 1, y lines yl0 .. yl0 + nyl - 1; the x layers per slab
// and the number of slabs (0: no rows, the contributions go straight to the
// gradient).
struct LineBox {
    int32_t lo;
    int32_t nx;
    int32_t zb0, nzb;
    int32_t yl0, nyl;
    int32_t layers;
    int32_t slabs;
};

template <int kB>
__device__ inline LineBox choose_linebox(const int32_t box[6], int32_t max_slabs)
{
    constexpr int32_t S = Geo<kB>::S, L = LineGeo<kB>::L;
    LineBox C;
    C.slabs = 0;
    C.layers = 0;
    C.lo = box[0];
    C.nx = box[3] - box[0] + 2;
    C.zb0 = box[2] >> S;
    C.nzb = ((box[5] + 1) >> S) - C.zb0 + 1;
    C.yl0 = box[1] >> L;
    C.nyl = ((box[4] + 1) >> L) - C.yl0 + 1;
    if (box[3] < 0) return C;   // no valid query
    const int64_t cross = (int64_t)C.nzb * C.nyl;
    if (cross > kLineMap) return C;
    C.layers = (int32_t)min((int64_t)C.nx, kLineMap / cross);
    const int32_t slabs = (C.nx + C.layers - 1) / C.layers;
    if (slabs <= max_slabs) C.slabs = slabs;
    return C;
}

// Line-map index (in the slab of x layers [a0, a1)) of every corner of cell
// c, or -1 outside the slab.
template <int kB>
__device__ inline void line_corners(const LineBox& C, int32_t a0, int32_t a1, const int32_t c[3], int32_t idx[8])
{
    constexpr int32_t S = Geo<kB>::S, L = LineGeo<kB>::L;
    const int32_t rx = c[0] - C.lo - a0, na = a1 - a0;
    const int32_t z0 = (c[2] >> S) - C.zb0, y0 = (c[1] >> L) - C.yl0;
    // corner (a, b, d) = base + a * sx + b * dy + d * dz
    const int32_t base = (rx * C.nzb + z0) * C.nyl + y0, sx = C.nzb * C.nyl;
    const int32_t dz = (((c[2] + 1) >> S) - (c[2] >> S)) * C.nyl, dy = ((c[1] + 1) >> L) - (c[1] >> L);
    const bool in0 = (uint32_t)rx < (uint32_t)na, in1 = (uint32_t)(rx + 1) < (uint32_t)na;   // y, z inside the box
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int32_t off = ((i >> 2) ? sx : 0) + (((i >> 1) & 1) ? dy : 0) + ((i & 1) ? dz : 0);
        idx[i] = ((i >> 2) ? in1 : in0) ? base + off : -1;
    }
}

// Mark the lines of the corners of cell c that lie in the slab.
template <int kB>
__device__ inline void line_mark(const LineBox& C, int32_t a0, int32_t a1, const int32_t c[3], uint16_t* map)
{
    int32_t idx[8];
    line_corners<kB>(C, a0, a1, c, idx);
#pragma unroll
    for (int i = 0; i < 8; ++i)
        if (idx[i] >= 0 && ((i & 1) == 0 || idx[i] != idx[i - 1])) map[idx[i]] = 1;
}

// Number the marked entries of the map (first n entries): each becomes its
// row + 1; *cnt ends as the number of rows.  Every thread of the block calls
// it (a wave's lanes take the same steps).
__device__ inline void line_number(uint16_t* map, int32_t n, int32_t* cnt)
{
    const uint32_t lane = threadIdx.x & 63;
    for (int32_t i0 = 0; i0 < n; i0 += blockDim.x) {
        const int32_t i = i0 + (int32_t)threadIdx.x;
        const bool m = i < n && map[i] != 0;
        const uint64_t mask = __ballot(m);
        if (mask == 0) continue;
        int32_t base = 0;
        if (lane == 0) base = atomicAdd(cnt, (int32_t)__popcll(mask));
        base = __builtin_amdgcn_readfirstlane(base);
        const int32_t below = (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        if (m) map[i] = (uint16_t)(base + below + 1);
    }
}

// The contributions of one cell whose lines have rows [row0, row0 + nrows)
// (and lie in the slab): into entry (slot mod 16) of the row, which records
// its line; contributions too large for the fixed point go straight to the
// gradient in the block's first turn (bypass).
template <int kB>
__device__ inline void line_add(const LineBox& C, int32_t a0, int32_t a1, const int32_t c[3], const int32_t slot[8],
                                const float v[8], int32_t row0, int32_t nrows, bool first, const uint16_t* map,
                                unsigned long long* acc, int32_t* rowkey, float* __restrict__ G, float scale)
{
    int32_t idx[8];
    line_corners<kB>(C, a0, a1, c, idx);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        // (converted here, in its turn: kept opaque so that the conversions
        // are not hoisted out of the loop and held as 16 64-bit values)
        float x = v[i];
        asm volatile("" : "+v"(x));
        const bool big = !(fabsf(x) < kFixLimit);
        if (idx[i] >= 0 && !big) {
            const int32_t row = (int32_t)map[idx[i]] - 1 - row0;
            if ((uint32_t)row < (uint32_t)nrows) {
                atomicAdd(&acc[row * kRowSlots + (slot[i] & (kRowSlots - 1))],
                          (unsigned long long)(__double_as_longlong(fma((double)x, kFixScale, kFixMagic)) -
                                               __double_as_longlong(kFixMagic)));
                rowkey[row] = slot[i] >> 4;   // (every add names its row's line: a corner of the same
                                              // line may have bypassed the rows)
            }
        } else if (first && big) {
            atomicAdd(at32(G, (uint32_t)slot[i]), scale * x);
        }
    }
}

// Add every non-zero entry of the first nrows rows to the gradient, in row
// order (16 consecutive slots per row), and clear it.  kf = scale / 2^32.
__device__ inline void line_flush(int32_t nrows, unsigned long long* acc, const int32_t* rowkey,
                                  float* __restrict__ G, double kf)
{
    const int32_t n = nrows * kRowSlots;
    for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const long long v = (long long)acc[i];
        if (v == 0) continue;
        acc[i] = 0ull;
        atomicAdd(at32(G, (uint32_t)(rowkey[i >> 4] * kRowSlots + (i & (kRowSlots - 1)))), (float)((double)v * kf));
    }
}

// Every contribution of one cell straight to the gradient (no rows).
__device__ inline void direct_add(const int32_t slot[8], const float v[8], float* __restrict__ G, float scale)
{
#pragma unroll
    for (int i = 0; i < 8; ++i) atomicAdd(at32(G, (uint32_t)slot[i]), scale * v[i]);
}

// One thread per query of a quarter tile: evaluate, take the adjoint, add
// the 16 corner contributions to the block's rows (or straight to the
// gradient), then flush the rows.  kLoss: also the tile's loss partials, and
// the contributions go out unscaled (the per-shape scale 1/valid count is
// applied when they are folded into the gradient); otherwise they are scaled
// by dloss / valid count.
template <bool kLoss, int kB>
__global__ __launch_bounds__(kGradBlock, 4) void k_query_grad(Band B, const float* __restrict__ qx,
                                                           const float* __restrict__ qy,
                                                           const float* __restrict__ qz,
                                                           const int32_t* __restrict__ nn, PointView P,
                                                           const float* __restrict__ D, gp_weights w,
                                                           const double* __restrict__ dloss,
                                                           const double* __restrict__ inv_qv,
                                                           float* __restrict__ G, double* __restrict__ q_part,
                                                           int32_t* flag, int32_t cap, int32_t max_slabs)
{
    extern __shared__ __align__(16) unsigned long long s_acc[];   // [cap] rows, then row lines, then the map
    __shared__ double s_red[kGradBlock / 64 * 4];
    __shared__ int32_t s_box[kGradBlock / 64 * 6];
    __shared__ int32_t s_cnt;
    const int32_t nrows_cap = cap / kRowSlots;
    int32_t* const s_rowkey = reinterpret_cast<int32_t*>(s_acc + cap);
    uint16_t* const s_map = reinterpret_cast<uint16_t*>(s_rowkey + nrows_cap);
    const int64_t item = xcd_work_item(blockIdx.x, gridDim.x);
    const int64_t tile = item / kGradParts;
    const int32_t quarter = (int32_t)(item % kGradParts);
    const int32_t shape = B.tile_shape[tile];
    const ShapeDesc& s = B.shapes[shape];
    const int64_t q0 = B.tile_start[tile] + (int64_t)quarter * kGradBlock;
    const int64_t qe = min(B.tile_start[tile] + (int64_t)kQueryTile, s.query_off + s.query_cnt);
    const float scale = kLoss ? 1.f : (float)(dloss[shape] * inv_qv[shape]);

    for (int32_t i = threadIdx.x; i < cap / 2; i += blockDim.x)
        reinterpret_cast<ulonglong2*>(s_acc)[i] = make_ulonglong2(0ull, 0ull);

    const int64_t k = q0 + threadIdx.x;
    float cq[8], cs[8];
    int32_t sq[8], ss[8], ccq[3] = {0, 0, 0}, ccs[3] = {0, 0, 0};
    bool valid = false;
    double part[4] = {0.0, 0.0, 0.0, 0.0};
    if (k < qe) {
        QueryState st;
        valid = eval_query<kB>(B, s, D, qx[k], qy[k], qz[k], k, nn[k], P, flag, st);
        if (valid) {
            if (kLoss) {
                part[0] = st.lp;
                part[1] = fabs(st.s.f);
                part[2] = (st.q.ok && st.s.ok) ? 1.0 - fma(st.q.gh[0], st.s.gh[0],
                                                           fma(st.q.gh[1], st.s.gh[1], st.q.gh[2] * st.s.gh[2]))
                                               : 1.0;
            }
            query_adjoint(s, st, w, cq, cs);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                sq[i] = st.q.slot[i];
                ss[i] = st.s.slot[i];
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                ccq[a] = st.q.c[a];
                ccs[a] = st.s.c[a];
            }
        }
    }
    if (kLoss) {
        // tile partials in a fixed order: lanes, then waves (the count exactly, from the valid lanes)
#pragma unroll
        for (int i = 0; i < 3; ++i) part[i] = wave_sum_f64(part[i]);
        part[3] = (double)__popcll(__ballot(valid));
        const int wave = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0)
            for (int i = 0; i < 4; ++i) s_red[wave * 4 + i] = part[i];
        __syncthreads();
        if (threadIdx.x < 4) {
            double a = 0.0;
            for (int wv = 0; wv < kGradBlock / 64; ++wv) a += s_red[wv * 4 + threadIdx.x];
            q_part[item * 4 + threadIdx.x] = a;
        }
    }

    // the box of the block's query and nearest-point cells
    int32_t box[6];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        box[a] = valid ? min(ccq[a], ccs[a]) : 0x7fffffff;
        box[3 + a] = valid ? max(ccq[a], ccs[a]) : -1;
    }
    block_minmax6(box, s_box);   // (its barriers also order the row clear)
#pragma unroll
    for (int a = 0; a < 6; ++a) box[a] = __builtin_amdgcn_readfirstlane(box[a]);
    const LineBox C = choose_linebox<kB>(box, max_slabs);
    if (C.slabs == 0) {
        if (valid) {
            direct_add(sq, cq, G, scale);
            direct_add(ss, cs, G, scale);
        }
    } else {
        const double kf = (double)scale * (1.0 / kFixScale);
        const int32_t cross = C.nzb * C.nyl;
        for (int32_t p = 0; p < C.slabs; ++p) {
            const int32_t a0 = p * C.layers, a1 = min(a0 + C.layers, C.nx);
            const int32_t nmap = (a1 - a0) * cross;
            for (int32_t i = threadIdx.x; i < (nmap + 1) / 2; i += blockDim.x)
                reinterpret_cast<uint32_t*>(s_map)[i] = 0u;
            if (threadIdx.x == 0) s_cnt = 0;
            __syncthreads();
            if (valid) {
                line_mark<kB>(C, a0, a1, ccq, s_map);
                line_mark<kB>(C, a0, a1, ccs, s_map);
            }
            __syncthreads();
            line_number(s_map, nmap, &s_cnt);
            __syncthreads();
            const int32_t n_rows = __builtin_amdgcn_readfirstlane(s_cnt);
            // (at least one turn, so that the bypass of the first slab runs)
            for (int32_t r0 = 0; r0 == 0 || r0 < n_rows; r0 += nrows_cap) {
                const int32_t nrows = min(nrows_cap, n_rows - r0);
                if (valid) {
                    line_add<kB>(C, a0, a1, ccq, sq, cq, r0, nrows, p == 0 && r0 == 0, s_map, s_acc, s_rowkey, G,
                                 scale);
                    line_add<kB>(C, a0, a1, ccs, ss, cs, r0, nrows, p == 0 && r0 == 0, s_map, s_acc, s_rowkey, G,
                                 scale);
                }
                __syncthreads();
                line_flush(max(nrows, 0), s_acc, s_rowkey, G, kf);
                __syncthreads();
            }
        }
    }
}

// ---- TV (Eq. 5).  A vertex takes part only if it is a TV vertex (V2 mask),
// and so does each of its six axis neighbours; a missing brick or a vertex
// outside the grid is not a TV vertex.  The forward stores 1/tau (0 where
// tau = 0) for the backward, which then divides nothing (unless it is given
// no array for it: the loss alone).  Two layouts of the
// same arithmetic:
// - one block per brick, one thread per vertex, the brick and a one-vertex
//   halo staged in LDS: many waves for a band of few bricks;
// - one wave per brick, lane (i, j) owning the column of vertices
//   (i, j, 0..7), which are contiguous slots: the z neighbours are in its own
//   column, the x and y neighbours in the columns of lanes i +- 1, j +- 1
//   (shuffles), and what lies across a brick face is loaded from the
//   neighbouring brick by the lanes on that face.  Five times as many bricks
//   are in flight per CU, which large bands need.

constexpr int kTvWaves = 4;                              // bricks per block in the wave layout

// Block-per-brick layout for bricks of edge kB: up to 512 threads, each
// taking V / threads of the brick's vertices; the brick and a one-vertex halo
// staged in LDS.
template <int kB>
struct TvBrick {
    static constexpr int H = kB + 2;                                  // staged vertices per axis
    static constexpr int HV = H * H * H;
    static constexpr int T = Geo<kB>::V < 512 ? Geo<kB>::V : 512;     // threads per block
};

template <int kB>
__device__ inline int32_t halo_index(int32_t i, int32_t j, int32_t k)   // brick-local, -1..kB
{
    constexpr int H = kB + 2;
    return ((i + 1) * H + (j + 1)) * H + (k + 1);
}

// Stage values of one or two slot arrays (b may be null) and the TV flags.
template <int kB>
__device__ inline void stage_brick(const Band& B, const ShapeDesc& s, int32_t brick, const BrickInfo& bi,
                                   const float* __restrict__ a, const float* __restrict__ b, float* sa, float* sb,
                                   uint8_t* tv)
{
    using G = Geo<kB>;
    for (int t = threadIdx.x; t < G::V; t += blockDim.x) {   // the brick's own vertex t
        const int32_t li = t >> (2 * G::S), lj = (t >> G::S) & G::M, lk = t & G::M;
        const int32_t h = halo_index<kB>(li, lj, lk);
        const int32_t slot = brick * G::V + t;
        sa[h] = a[slot];
        if (b) sb[h] = b[slot];
        tv[h] = (uint8_t)mask_bit_b<kB>(B.m_v2, brick, t);
    }
    for (int t = threadIdx.x; t < 6 * kB * kB; t += blockDim.x) {
        // face f: axis f / 2, side -1 (even f) or +1 (odd f); kB^2 vertices each
        const int f = t >> (2 * G::S), w = t & (kB * kB - 1), axis = f >> 1, side = (f & 1) ? 1 : -1;
        int32_t l[3];
        l[axis] = side > 0 ? kB : -1;
        l[(axis + 1) % 3] = w >> G::S;
        l[(axis + 2) % 3] = w & G::M;
        const int32_t gi = bi.bx * kB + l[0], gj = bi.by * kB + l[1], gk = bi.bz * kB + l[2];
        const int32_t h = halo_index<kB>(l[0], l[1], l[2]);
        float va = 0.f, vb = 0.f;
        uint8_t flag = 0;
        if (gi >= 0 && gj >= 0 && gk >= 0 && gi <= s.R[0] && gj <= s.R[1] && gk <= s.R[2]) {
            const int32_t nb = brick_of(B, s, gi >> G::S, gj >> G::S, gk >> G::S);
            if (nb >= 0) {
                const int32_t loc = local_index_b<kB>(gi, gj, gk);
                const int32_t slot = nb * G::V + loc;
                va = a[slot];
                if (b) vb = b[slot];
                flag = (uint8_t)mask_bit_b<kB>(B.m_v2, nb, loc);
            }
        }
        sa[h] = va;
        if (b) sb[h] = vb;
        tv[h] = flag;
    }
}

template <int kB>
__global__ __launch_bounds__(TvBrick<kB>::T) void k_tv_forward_brick(Band B, const float* __restrict__ D,
                                                                   float* __restrict__ itau,
                                                                   double* __restrict__ tv_part)
{
    using G = Geo<kB>;
    constexpr int H = TvBrick<kB>::H;
    __shared__ float s_d[TvBrick<kB>::HV];
    __shared__ uint8_t s_tv[TvBrick<kB>::HV];
    __shared__ double lds[TvBrick<kB>::T / 64 + 1];
    const int32_t brick = blockIdx.x;
    const BrickInfo bi = B.bricks[brick];
    const ShapeDesc& s = B.shapes[bi.shape];
    stage_brick<kB>(B, s, brick, bi, D, nullptr, s_d, nullptr, s_tv);
    __syncthreads();
    double v = 0.0;
    for (int t = threadIdx.x; t < G::V; t += blockDim.x) {
        const int32_t li = t >> (2 * G::S), lj = (t >> G::S) & G::M, lk = t & G::M;
        const int32_t h = halo_index<kB>(li, lj, lk);
        if (!s_tv[h]) continue;
        const float dv = s_d[h];
        const int32_t nbh[6] = {h + H * H, h - H * H, h + H, h - H, h + 1, h - 1};
        float s2 = 0.f;
#pragma unroll
        for (int o = 0; o < 6; ++o) {
            if (!s_tv[nbh[o]]) continue;
            const float d = dv - s_d[nbh[o]];
            s2 = fmaf(d, d, s2);
        }
        const float tau_v = sqrtf(s2);
        if (itau) itau[brick * G::V + t] = tau_v > 0.f ? 1.f / tau_v : 0.f;
        v += (double)tau_v;
    }
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int t = threadIdx.x;
    if ((t & 63) == 0) lds[t >> 6] = v;
    __syncthreads();
    if (t == 0) {
        double a = 0.0;
        for (int wv = 0; wv < (int)(blockDim.x >> 6); ++wv) a += lds[wv];
        tv_part[brick] = a;
    }
}

// Gradient of alpha * L_TV in gather form (every vertex sums over its own
// neighbours and writes only its own slot), scaled by dloss.  With raw, also
// adds dloss / valid count times the unscaled query contributions of the
// fused pass and clears them.
template <int kB>
__global__ __launch_bounds__(TvBrick<kB>::T) void k_tv_backward_brick(Band B, const float* __restrict__ D,
                                                                    const float* __restrict__ itau, gp_weights w,
                                                                    const double* __restrict__ dloss,
                                                                    const double* __restrict__ inv_qv,
                                                                    float* __restrict__ raw, float* __restrict__ G)
{
    using Gm = Geo<kB>;
    constexpr int H = TvBrick<kB>::H;
    __shared__ float s_d[TvBrick<kB>::HV], s_t[TvBrick<kB>::HV];
    __shared__ uint8_t s_tv[TvBrick<kB>::HV];
    const int32_t brick = blockIdx.x;
    const BrickInfo bi = B.bricks[brick];
    const ShapeDesc& s = B.shapes[bi.shape];
    const bool tv_on = s.n_tv > 0;
    if (tv_on) stage_brick<kB>(B, s, brick, bi, D, itau, s_d, s_t, s_tv);
    __syncthreads();
    const float scale = tv_on ? (float)((double)w.alpha * dloss[bi.shape] / (double)s.n_tv) : 0.f;
    const float rscale = raw ? (float)(dloss[bi.shape] * inv_qv[bi.shape]) : 0.f;
    for (int t = threadIdx.x; t < Gm::V; t += blockDim.x) {
        const int32_t slot = brick * Gm::V + t;
        float add = 0.f;
        bool touch = false;
        if (raw) {
            const float r = raw[slot];
            if (r != 0.f) {
                add = rscale * r;
                raw[slot] = 0.f;
                touch = true;
            }
        }
        const int32_t li = t >> (2 * Gm::S), lj = (t >> Gm::S) & Gm::M, lk = t & Gm::M;
        const int32_t h = halo_index<kB>(li, lj, lk);
        if (tv_on && s_tv[h]) {
            const float dv = s_d[h];
            const float inv_tv = s_t[h];
            const int32_t nbh[6] = {h + H * H, h - H * H, h + H, h - H, h + 1, h - 1};
            float acc = 0.f;
#pragma unroll
            for (int o = 0; o < 6; ++o) {
                if (!s_tv[nbh[o]]) continue;
                acc = fmaf(dv - s_d[nbh[o]], inv_tv + s_t[nbh[o]], acc);
            }
            add = fmaf(scale, acc, add);
            touch = true;
        }
        if (touch) G[slot] += add;
    }
}

// The 8 mask bits of column col (0..63) of a brick: vertices col * 8 + k.
__device__ inline uint32_t col_mask(const uint32_t* m, int32_t brick, int32_t col)
{
    const uint32_t w = m[(int64_t)brick * kMaskWords + (col >> 2)];
    return (w >> ((col & 3) * 8)) & 0xffu;
}

__device__ inline void load_col(const float* __restrict__ a, int32_t slot0, float v[8])
{
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = *at32(a, (uint32_t)(slot0 + k));
}

// Directory entry of the brick at offset (dx, dy, dz) from bi, or -1.
__device__ inline int32_t nbr_brick(const Band& B, const ShapeDesc& s, const BrickInfo& bi, int dx, int dy, int dz)
{
    const int32_t x = bi.bx + dx, y = bi.by + dy, z = bi.bz + dz;
    if (x < 0 || y < 0 || z < 0 || x >= s.nb[0] || y >= s.nb[1] || z >= s.nb[2]) return -1;
    return brick_of(B, s, x, y, z);
}

// The directory entries of the six face neighbours of a brick, in the order
// x+1, x-1, y+1, y-1, z-1, z+1 (-1: none); the same for every lane of the
// wave, so they are looked up once, all together, before any is needed.
__device__ inline void face_nbrs(const Band& B, const ShapeDesc& s, const BrickInfo& bi, int32_t nbr[6])
{
    nbr[0] = nbr_brick(B, s, bi, 1, 0, 0);
    nbr[1] = nbr_brick(B, s, bi, -1, 0, 0);
    nbr[2] = nbr_brick(B, s, bi, 0, 1, 0);
    nbr[3] = nbr_brick(B, s, bi, 0, -1, 0);
    nbr[4] = nbr_brick(B, s, bi, 0, 0, -1);
    nbr[5] = nbr_brick(B, s, bi, 0, 0, 1);
}

// The neighbour column of this lane's column in direction (di, dj) of the
// i-j plane: from lane (i + di, j + dj), or across the brick face into brick
// br (the face neighbour in that direction).  Values of up to two arrays (b
// may be null) and the neighbours' V2 bits.
__device__ inline uint32_t side_col(const Band& B, int32_t br, int lane, int di, int dj, const float va[8],
                                    const float vb[8], uint32_t m, const float* __restrict__ a,
                                    const float* __restrict__ b, float na[8], float nb[8])
{
    const int32_t i = lane >> 3, j = lane & 7, ii = i + di, jj = j + dj;
    const int src = (lane + di * 8 + dj) & 63;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        na[k] = __shfl(va[k], src, 64);
        if (b) nb[k] = __shfl(vb[k], src, 64);
    }
    uint32_t nm = (uint32_t)__shfl((int)m, src, 64);
    if (ii < 0 || ii > 7 || jj < 0 || jj > 7) {
        const int32_t ncol = ((ii & 7) << 3) | (jj & 7);
        nm = 0u;
        if (br >= 0) {
            load_col(a, br * kBrickVol + ncol * 8, na);
            if (b) load_col(b, br * kBrickVol + ncol * 8, nb);
            nm = col_mask(B.m_v2, br, ncol);
        }
    }
    return nm;
}

__global__ __launch_bounds__(kTvWaves * 64) void k_tv_forward_wave(Band B, const float* __restrict__ D,
                                                                   float* __restrict__ itau,
                                                                   double* __restrict__ tv_part, int32_t n_bricks)
{
    const int lane = threadIdx.x & 63;
    const int32_t brick = (int32_t)blockIdx.x * kTvWaves + (int32_t)(threadIdx.x >> 6);
    if (brick >= n_bricks) return;
    const BrickInfo bi = B.bricks[brick];
    const ShapeDesc& s = B.shapes[bi.shape];
    const int32_t slot0 = brick * kBrickVol + lane * 8;
    int32_t nbr[6];
    face_nbrs(B, s, bi, nbr);
    float v[8], s2[8];
    load_col(D, slot0, v);
    const uint32_t m = col_mask(B.m_v2, brick, lane);
#pragma unroll
    for (int k = 0; k < 8; ++k) s2[k] = 0.f;
    // z neighbours: inside the column, then across the two z faces
#pragma unroll
    for (int k = 0; k < 7; ++k)
        if ((m >> k) & (m >> (k + 1)) & 1u) {
            const float d = v[k] - v[k + 1];
            s2[k] = fmaf(d, d, s2[k]);
            s2[k + 1] = fmaf(d, d, s2[k + 1]);
        }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int32_t br = nbr[4 + e];
        const int k = e ? 7 : 0, kn = e ? 0 : 7;
        if (br >= 0 && ((m >> k) & 1u) && ((col_mask(B.m_v2, br, lane) >> kn) & 1u)) {
            const float d = v[k] - *at32(D, (uint32_t)(br * kBrickVol + lane * 8 + kn));
            s2[k] = fmaf(d, d, s2[k]);
        }
    }
    // x and y neighbours
#pragma unroll 1
    for (int dir = 0; dir < 4; ++dir) {
        const int di = dir == 0 ? 1 : (dir == 1 ? -1 : 0), dj = dir == 2 ? 1 : (dir == 3 ? -1 : 0);
        float n[8];
        const uint32_t nm = side_col(B, nbr[dir], lane, di, dj, v, nullptr, m, D, nullptr, n, nullptr);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if ((m & nm) >> k & 1u) {
                const float d = v[k] - n[k];
                s2[k] = fmaf(d, d, s2[k]);
            }
    }
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if ((m >> k) & 1u) {
            const float t = sqrtf(s2[k]);
            if (itau) *at32(itau, (uint32_t)(slot0 + k)) = t > 0.f ? 1.f / t : 0.f;
            sum += (double)t;
        }
    for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
    if (lane == 0) tv_part[brick] = sum;
}

__global__ __launch_bounds__(kTvWaves * 64, 5) void k_tv_backward_wave(Band B, const float* __restrict__ D,
                                                                    const float* __restrict__ itau, gp_weights w,
                                                                    const double* __restrict__ dloss,
                                                                    const double* __restrict__ inv_qv,
                                                                    float* __restrict__ raw, float* __restrict__ G,
                                                                    int32_t n_bricks)
{
    const int lane = threadIdx.x & 63;
    const int32_t brick = (int32_t)blockIdx.x * kTvWaves + (int32_t)(threadIdx.x >> 6);
    if (brick >= n_bricks) return;
    const BrickInfo bi = B.bricks[brick];
    const ShapeDesc& s = B.shapes[bi.shape];
    const bool tv_on = s.n_tv > 0;
    const float scale = tv_on ? (float)((double)w.alpha * dloss[bi.shape] / (double)s.n_tv) : 0.f;
    const float rscale = raw ? (float)(dloss[bi.shape] * inv_qv[bi.shape]) : 0.f;
    const int32_t slot0 = brick * kBrickVol + lane * 8;
    float add[8];
    uint32_t touched = 0u;
#pragma unroll
    for (int k = 0; k < 8; ++k) add[k] = 0.f;
    if (raw) {
        float r[8];
        load_col(raw, slot0, r);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (r[k] != 0.f) {
                add[k] = rscale * r[k];
                touched |= 1u << k;
            }
        if (touched)
#pragma unroll
            for (int k = 0; k < 8; ++k) *at32(raw, (uint32_t)(slot0 + k)) = 0.f;
    }
    const uint32_t m = tv_on ? col_mask(B.m_v2, brick, lane) : 0u;
    if (__ballot(m != 0u)) {
        int32_t nbr[6];
        face_nbrs(B, s, bi, nbr);
        float v[8], it[8], acc[8];
        load_col(D, slot0, v);
        load_col(itau, slot0, it);
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[k] = 0.f;
#pragma unroll
        for (int k = 0; k < 7; ++k)
            if ((m >> k) & (m >> (k + 1)) & 1u) {
                const float d = v[k] - v[k + 1], c = it[k] + it[k + 1];
                acc[k] = fmaf(d, c, acc[k]);
                acc[k + 1] = fmaf(-d, c, acc[k + 1]);
            }
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int32_t br = nbr[4 + e];
            const int k = e ? 7 : 0, kn = e ? 0 : 7;
            if (br >= 0 && ((m >> k) & 1u) && ((col_mask(B.m_v2, br, lane) >> kn) & 1u)) {
                const uint32_t ns = (uint32_t)(br * kBrickVol + lane * 8 + kn);
                acc[k] = fmaf(v[k] - *at32(D, ns), it[k] + *at32(itau, ns), acc[k]);
            }
        }
#pragma unroll 1
        for (int dir = 0; dir < 4; ++dir) {
            const int di = dir == 0 ? 1 : (dir == 1 ? -1 : 0), dj = dir == 2 ? 1 : (dir == 3 ? -1 : 0);
            float n[8], nt[8];
            const uint32_t nm = side_col(B, nbr[dir], lane, di, dj, v, it, m, D, itau, n, nt);
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if ((m & nm) >> k & 1u) acc[k] = fmaf(v[k] - n[k], it[k] + nt[k], acc[k]);
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if ((m >> k) & 1u) add[k] = fmaf(scale, acc[k], add[k]);
        touched |= m;
    }
    if (touched)
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if ((touched >> k) & 1u) *at32(G, (uint32_t)(slot0 + k)) += add[k];
}

// Per-shape loss from the tile and brick partials, deterministically:
// kFinChunks blocks per shape (fewer were measured slower, even for small
// shapes) each sum a fixed contiguous chunk of them and write their five sums
// to fin_part; the last block of the shape to finish (a per-shape counter,
// reset by that block for the next call) adds the chunks in order.  The tile
// partials are pairs of doubles, (pull, surface) then (gradient term, count);
// a chunk starts on an even pair and the block stride is even, so a thread
// always adds to the same two of the four sums.
constexpr int kFinalizeBlock = 256;
constexpr int kFinChunks = 32;

__global__ __launch_bounds__(kFinalizeBlock) void k_finalize(Band B, const double* __restrict__ q_part,
                                                             const double* __restrict__ tv_part, gp_weights w,
                                                             double* __restrict__ loss_out,
                                                             int64_t* __restrict__ n_valid_out,
                                                             double* __restrict__ inv_qv, int32_t* __restrict__ flag,
                                                             int32_t parts, double* __restrict__ fin_part,
                                                             int32_t* __restrict__ fin_count)
{
    __shared__ double lds[kFinalizeBlock / 64 * 5];
    __shared__ int32_t s_last;
    const int32_t chunk = blockIdx.x, nch = gridDim.x, shape = blockIdx.y;
    const ShapeDesc& s = B.shapes[shape];
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    // q_part holds `parts` partial sums per tile, 4 doubles each
    const double2* qp = reinterpret_cast<const double2*>(q_part);
    const int64_t np = (s.tile_end - s.tile_begin) * parts;            // pairs of pairs
    const int64_t pb = s.tile_begin * parts * 2 + 2 * (np * chunk / nch);
    const int64_t pe = s.tile_begin * parts * 2 + 2 * (np * (chunk + 1) / nch);
    const int hi = threadIdx.x & 1;
    // four independent accumulators so that four loads are in flight per thread
    double a0[4] = {0.0, 0.0, 0.0, 0.0}, a1[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t m = pb + threadIdx.x;
    for (; m + 3 * (int64_t)blockDim.x < pe; m += 4 * (int64_t)blockDim.x) {
        double2 d[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) d[u] = qp[m + u * (int64_t)blockDim.x];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a0[u] += d[u].x;
            a1[u] += d[u].y;
        }
    }
#pragma unroll
    for (int u = 0; u < 3; ++u) {   // at most three left
        if (m < pe) {
            const double2 d = qp[m];
            a0[u] += d.x;
            a1[u] += d.y;
        }
        m += blockDim.x;
    }
    const double s0 = (a0[0] + a0[1]) + (a0[2] + a0[3]), s1 = (a1[0] + a1[1]) + (a1[2] + a1[3]);
    v[0] = hi ? 0.0 : s0;
    v[1] = hi ? 0.0 : s1;
    v[2] = hi ? s0 : 0.0;
    v[3] = hi ? s1 : 0.0;
    const int64_t nbk = s.brick_end - s.brick_begin;
    const int64_t bb = s.brick_begin + nbk * chunk / nch, be = s.brick_begin + nbk * (chunk + 1) / nch;
    for (int64_t b = bb + threadIdx.x; b < be; b += blockDim.x) v[4] += tv_part[b];
#pragma unroll
    for (int i = 0; i < 5; ++i)
        for (int o = 32; o > 0; o >>= 1) v[i] += __shfl_xor(v[i], o, 64);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
        for (int i = 0; i < 5; ++i) lds[wave * 5 + i] = v[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        double* out = fin_part + ((int64_t)shape * kFinChunks + chunk) * 5;
        for (int i = 0; i < 5; ++i) {
            double a = 0.0;
            for (int wv = 0; wv < kFinalizeBlock / 64; ++wv) a += lds[wv * 5 + i];
            out[i] = a;
        }
        __threadfence();
        s_last = atomicAdd(&fin_count[shape], 1) == nch - 1;
    }
    __syncthreads();
    if (!s_last) return;
    // the shape's last block: every chunk's sums are visible after the fence;
    // one load per thread, then the chunks are added in order
static_assert(kFinChunks * 5 <= kFinalizeBlock, "one chunk sum per thread");
    __shared__ double s_chunk[kFinChunks * 5];
    __threadfence();
    if (threadIdx.x < nch * 5)
        s_chunk[threadIdx.x] = __hip_atomic_load(fin_part + (int64_t)shape * kFinChunks * 5 + threadIdx.x,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (threadIdx.x != 0) return;
    double t[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
    for (int c = 0; c < nch; ++c)
#pragma unroll
        for (int i = 0; i < 5; ++i) t[i] += s_chunk[c * 5 + i];
    atomicExch(&fin_count[shape], 0);
    const double nq = t[3];
    const double iq = nq > 0.0 ? 1.0 / nq : 0.0;
    const double pull = t[0] * iq, surf = t[1] * iq, grad = t[2] * iq;
    const double tv = s.n_tv > 0 ? t[4] / (double)s.n_tv : 0.0;
    const double total = pull + (double)w.alpha * tv + (double)w.beta * surf + (double)w.gamma * grad;
    loss_out[shape * 5 + 0] = total;
    loss_out[shape * 5 + 1] = pull;
    loss_out[shape * 5 + 2] = tv;
    loss_out[shape * 5 + 3] = surf;
    loss_out[shape * 5 + 4] = grad;
    n_valid_out[shape] = (int64_t)nq;
    inv_qv[shape] = iq;
    if (!isfinite(total)) atomicOr(flag, 1);
}

}  // namespace
}  // namespace gp

using namespace gp;

// TV layout: block per brick for a small band (more waves), wave per brick
// for a large one (more bricks in flight), from the context's thresholds
// (defaults from measured crossovers: the forward gains from about 2000
// bricks, 0.44 -> 0.26 ms at 137k bricks and 24 -> 19 us at 6k; the
// backward, which moves two arrays and keeps more registers, only far above
// 6k bricks, 0.71 -> 0.54 ms at 137k and 32 -> 34 us at 6k).
static bool tv_wave_layout(gp_ctx ctx, int64_t wave_from)
{
    return ctx->brick == kBrick && ctx->n_bricks >= wave_from;   // the wave layout is written for 8^3 bricks
}

// itau may be null (the loss alone); tv_part receives the per-brick sums.
static void launch_tv_forward(gp_ctx ctx, const Band& B, const float* field, float* itau, double* tv_part,
                              hipStream_t st)
{
    if (tv_wave_layout(ctx, ctx->grad_params.tv_fwd_wave_from))
        k_tv_forward_wave<<<(unsigned)((ctx->n_bricks + kTvWaves - 1) / kTvWaves), kTvWaves * 64, 0, st>>>(
            B, field, itau, tv_part, (int32_t)ctx->n_bricks);
    else
        with_brick(ctx->brick, [&](auto tag) {
            constexpr int kB = decltype(tag)::value;
            k_tv_forward_brick<kB><<<(unsigned)ctx->n_bricks, TvBrick<kB>::T, 0, st>>>(B, field, itau, tv_part);
        });
}

static void launch_tv_backward(gp_ctx ctx, const Band& B, const float* field, gp_weights w, const double* dloss,
                               float* raw, float* grad, hipStream_t st)
{
    if (tv_wave_layout(ctx, ctx->grad_params.tv_bwd_wave_from))
        k_tv_backward_wave<<<(unsigned)((ctx->n_bricks + kTvWaves - 1) / kTvWaves), kTvWaves * 64, 0, st>>>(
            B, field, ctx->tau.p, w, dloss, ctx->inv_qv.p, raw, grad, (int32_t)ctx->n_bricks);
    else
        with_brick(ctx->brick, [&](auto tag) {
            constexpr int kB = decltype(tag)::value;
            k_tv_backward_brick<kB><<<(unsigned)ctx->n_bricks, TvBrick<kB>::T, 0, st>>>(B, field, ctx->tau.p, w, dloss,
                                                                                      ctx->inv_qv.p, raw, grad);
        });
}

gp_status gp_forward_impl(gp_ctx ctx, const float* qx, const float* qy, const float* qz, const int32_t* nn,
                          const float* field, gp_weights w, double* loss_out, int64_t* n_valid_out)
{
    hipStream_t st = ctx->stream;
    Band B = ctx->band();
    if (ctx->n_tiles > 0) {
        GP_TIMED(ctx, "k_forward_query");
        with_brick(ctx->brick, [&](auto tag) {
            k_forward_query<decltype(tag)::value><<<(unsigned)ctx->n_tiles, kQueryBlock, 0, st>>>(
                B, qx, qy, qz, nn, ctx->points(), field, ctx->q_part.p, ctx->flag.p);
        });
    }
    if (ctx->n_bricks > 0) {
        GP_TIMED(ctx, "k_tv_forward");
        launch_tv_forward(ctx, B, field, ctx->tau.p, ctx->tv_part.p, st);
    }
    GP_TIMED(ctx, "k_finalize");
    k_finalize<<<dim3(kFinChunks, (unsigned)ctx->n_shapes), kFinalizeBlock, 0, st>>>(
        B, ctx->q_part.p, ctx->tv_part.p, w, loss_out, n_valid_out, ctx->inv_qv.p, ctx->flag.p, 1, ctx->fin_part.p,
        ctx->fin_count.p);
    GP_HIP(ctx, hipGetLastError());
    return GP_OK;
}

gp_status gp_backward_impl(gp_ctx ctx, const float* qx, const float* qy, const float* qz, const int32_t* nn,
                           const float* field, gp_weights w, const double* dloss, float* grad)
{
    hipStream_t st = ctx->stream;
    Band B = ctx->band();
    if (ctx->n_tiles > 0) {
        GP_TIMED(ctx, "k_backward_query");
        const GradParams& gpar = ctx->grad_params;
        with_brick(ctx->brick, [&](auto tag) {
            constexpr int kB = decltype(tag)::value;
            k_query_grad<false, kB><<<(unsigned)(ctx->n_tiles * kGradParts), kGradBlock, win_lds_bytes(gpar.win_cap),
                                      st>>>(B, qx, qy, qz, nn, ctx->points(), field, w, dloss, ctx->inv_qv.p, grad,
                                            nullptr, ctx->flag.p, gpar.win_cap, gpar.win_max_passes);
        });
    }
    if (ctx->n_bricks > 0) {
        GP_TIMED(ctx, "k_tv_backward");
        launch_tv_backward(ctx, B, field, w, dloss, nullptr, grad, st);
    }
    GP_HIP(ctx, hipGetLastError());
    return GP_OK;
}

gp_status gp_forward_backward_impl(gp_ctx ctx, const float* qx, const float* qy, const float* qz,
                                   const int32_t* nn, const float* field, gp_weights w, const double* dloss,
                                   double* loss_out, int64_t* n_valid_out, float* grad)
{
    hipStream_t st = ctx->stream;
    Band B = ctx->band();
    if (ctx->n_tiles > 0) {
        GP_TIMED(ctx, "k_query_grad");
        const GradParams& gpar = ctx->grad_params;
        with_brick(ctx->brick, [&](auto tag) {
            constexpr int kB = decltype(tag)::value;
            k_query_grad<true, kB><<<(unsigned)(ctx->n_tiles * kGradParts), kGradBlock, win_lds_bytes(gpar.win_cap),
                                     st>>>(B, qx, qy, qz, nn, ctx->points(), field, w, dloss, ctx->inv_qv.p,
                                           ctx->g_raw.p, ctx->q_part.p, ctx->flag.p, gpar.win_cap,
                                           gpar.win_max_passes);
        });
    }
    if (ctx->n_bricks > 0) {
        GP_TIMED(ctx, "k_tv_forward");
        launch_tv_forward(ctx, B, field, ctx->tau.p, ctx->tv_part.p, st);
    }
    {
        GP_TIMED(ctx, "k_finalize");
        k_finalize<<<dim3(kFinChunks, (unsigned)ctx->n_shapes), kFinalizeBlock, 0, st>>>(
            B, ctx->q_part.p, ctx->tv_part.p, w, loss_out, n_valid_out, ctx->inv_qv.p, ctx->flag.p, kGradParts,
            ctx->fin_part.p, ctx->fin_count.p);
    }
    if (ctx->n_bricks > 0) {
        GP_TIMED(ctx, "k_tv_backward");
        launch_tv_backward(ctx, B, field, w, dloss, ctx->g_raw.p, grad, st);
    }
    GP_HIP(ctx, hipGetLastError());
    return GP_OK;
}

// ---------------------------------------------------------------------------
// gp_pull_forward_static: the loss of gp_pull_forward with no allocation and
// no context scratch.  Its scratch (the per-tile and per-brick partial sums,
// the chunk sums and counter of the reduction, the reciprocal valid counts)
// lives in the file-scope device array `scratch`; every GPU holds its own copy
// until the process ends, and host code reaches it only through the address
// hipGetSymbolAddress gives for that device (the array's name is no device
// address on the host).  The copy keeps the last call's contents, so the
// reduction counter is cleared (by a small kernel, never a memset node) at
// the start of every call; calls that overlap on one GPU share the array and
// race.
constexpr size_t kStaticScratchBytes = (size_t)8 << 20;
constexpr int kStaticMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

static std::mutex g_scratch_mutex;
static void* g_scratch_ptr[kStaticMaxDevices] = {};

// The device address of `scratch` on the context's device (current), found
// once per device.
static gp_status static_scratch(gp_ctx ctx, unsigned char** out)
{
    if (ctx->device < 0 || ctx->device >= kStaticMaxDevices)
        return gp_fail(ctx, GP_ERR_DEVICE, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[ctx->device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) return gp_hip_fail(ctx, e == hipSuccess ? hipErrorInvalidSymbol : e,
                                                      "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[ctx->device] = p;
    }
    *out = static_cast<unsigned char*>(g_scratch_ptr[ctx->device]);
    return GP_OK;
}

namespace gp {
namespace {

__global__ void k_zero_i32(int32_t* __restrict__ p, int32_t n)
{
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n) p[i] = 0;
}

}  // namespace
}  // namespace gp

gp_status gp_forward_static_impl(gp_ctx ctx, const float* qx, const float* qy, const float* qz, const int32_t* nn,
                                 const float* field, gp_weights w, double* loss_out, int64_t* n_valid_out)
{
    // layout (in doubles): tile partials [n_tiles * 4], brick partials
    // [n_bricks], chunk sums [n_shapes * kFinChunks * 5], reciprocal valid
    // counts [n_shapes], then the chunk counters [n_shapes] (int32)
    const int64_t n_q = std::max<int64_t>(ctx->n_tiles, 1) * 4, n_t = std::max<int64_t>(ctx->n_bricks, 1);
    const int64_t n_f = (int64_t)ctx->n_shapes * kFinChunks * 5, n_i = ctx->n_shapes;
    const int64_t need = (n_q + n_t + n_f + n_i) * 8 + (int64_t)ctx->n_shapes * 4;
    if (need > (int64_t)kStaticScratchBytes)
        return gp_fail(ctx, GP_ERR_CAPACITY, "gp_pull_forward_static needs " + std::to_string(need) +
                                                 " bytes of scratch for this band, beyond its " +
                                                 std::to_string(kStaticScratchBytes));
    unsigned char* base = nullptr;
    gp_status stt = static_scratch(ctx, &base);
    if (stt != GP_OK) return stt;
    double* q_part = reinterpret_cast<double*>(base);
    double* tv_part = q_part + n_q;
    double* fin_part = tv_part + n_t;
    double* inv_qv = fin_part + n_f;
    int32_t* fin_count = reinterpret_cast<int32_t*>(inv_qv + n_i);
    hipStream_t st = ctx->stream;
    Band B = ctx->band();
    k_zero_i32<<<(unsigned)((ctx->n_shapes + 255) / 256), 256, 0, st>>>(fin_count, ctx->n_shapes);
    if (ctx->n_tiles > 0)
        with_brick(ctx->brick, [&](auto tag) {
            k_forward_query<decltype(tag)::value><<<(unsigned)ctx->n_tiles, kQueryBlock, 0, st>>>(
                B, qx, qy, qz, nn, ctx->points(), field, q_part, ctx->flag.p);
        });
    if (ctx->n_bricks > 0) launch_tv_forward(ctx, B, field, nullptr, tv_part, st);
    k_finalize<<<dim3(kFinChunks, (unsigned)ctx->n_shapes), kFinalizeBlock, 0, st>>>(
        B, q_part, tv_part, w, loss_out, n_valid_out, inv_qv, ctx->flag.p, 1, fin_part, fin_count);
    GP_HIP(ctx, hipGetLastError());
    return GP_OK;
}

// ---------------------------------------------------------------------------
// gp_autotune_grad: the row and slab settings of the fused query pass, then the TV
// layouts at this band's size, each timed between events on the context's
// stream (one untimed run, then the smallest of reps runs).  The query pass
// accumulates into the context's own accumulator, cleared afterwards; the TV
// backward writes a scratch gradient.
template <int kB>
static gp_status autotune_grad(gp_ctx ctx, const float* qx, const float* qy, const float* qz, const int32_t* nn,
                               const float* field, gp_weights w, int32_t reps, GradParams* best_out,
                               float* best_ms_out)
{
    static const int32_t kPasses[] = {4, 16, 64};
    hipStream_t st = ctx->stream;
    const Band B = ctx->band();
    const GradParams current = ctx->grad_params;
    GradParams best = current;
    float ms[3] = {-1.f, -1.f, -1.f};
    hipEvent_t ev[2];
    GP_HIP(ctx, hipEventCreate(&ev[0]));
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        return gp_fail(ctx, GP_ERR_DEVICE, "hipEventCreate failed");
    }
    hipError_t e = hipSuccess;
    auto time_it = [&](auto&& launch) -> float {
        float t_min = -1.f;
        for (int32_t r = 0; r <= reps && e == hipSuccess; ++r) {
            if (r > 0) e = hipEventRecord(ev[0], st);
            if (e == hipSuccess) launch();
            if (e == hipSuccess) e = hipGetLastError();
            if (r > 0 && e == hipSuccess) e = hipEventRecord(ev[1], st);
            if (r > 0 && e == hipSuccess) e = hipEventSynchronize(ev[1]);
            float t = 0.f;
            if (r > 0 && e == hipSuccess) e = hipEventElapsedTime(&t, ev[0], ev[1]);
            if (r > 0 && e == hipSuccess && (t_min < 0.f || t < t_min)) t_min = t;
        }
        return t_min;
    };
    DevBuf<float> grad;
    DevBuf<double> dloss;
    if (ctx->n_tiles > 0) {
        auto query_pass = [&](int32_t cap, int32_t passes) {
            return time_it([&] {
                k_query_grad<true, kB><<<(unsigned)(ctx->n_tiles * kGradParts), kGradBlock, win_lds_bytes(cap), st>>>(
                    B, qx, qy, qz, nn, ctx->points(), field, w, nullptr, nullptr, ctx->g_raw.p, ctx->q_part.p,
                    ctx->flag.p, cap, passes);
            });
        };
        float best_t = query_pass(current.win_cap, current.win_max_passes);
        for (int32_t cap : kWinCaps)
            for (int32_t passes : kPasses) {
                if (cap == current.win_cap && passes == current.win_max_passes) continue;
                const float t = query_pass(cap, passes);
                if (e != hipSuccess || t < 0.f) continue;
                const bool holding = best.win_cap == current.win_cap && best.win_max_passes == current.win_max_passes;
                if (t < best_t * (holding ? 0.98f : 1.f)) {
                    best_t = t;
                    best.win_cap = cap;
                    best.win_max_passes = passes;
                }
            }
        ms[0] = best_t;
        if (e == hipSuccess) e = hipMemsetAsync(ctx->g_raw.p, 0, (size_t)std::max<int64_t>(ctx->n_slots, 1) * 4, st);
    }
    if (kB == kBrick && ctx->n_bricks > 0 && e == hipSuccess) {   // (other bricks have the block layout only)
        const int64_t nb = ctx->n_bricks;
        const unsigned waves_grid = (unsigned)((nb + kTvWaves - 1) / kTvWaves);
        // forward: writes the context's 1/tau and per-brick partials (scratch until the next forward)
        const float t_wave = time_it([&] {
            k_tv_forward_wave<<<waves_grid, kTvWaves * 64, 0, st>>>(B, field, ctx->tau.p, ctx->tv_part.p, (int32_t)nb);
        });
        const float t_brick = time_it([&] {
            k_tv_forward_brick<kB><<<(unsigned)nb, TvBrick<kB>::T, 0, st>>>(B, field, ctx->tau.p, ctx->tv_part.p);
        });
        const bool wave_now = nb >= current.tv_fwd_wave_from;
        const float t_now = wave_now ? t_wave : t_brick, t_other = wave_now ? t_brick : t_wave;
        if (e == hipSuccess && t_other >= 0.f && t_other < 0.98f * t_now)
            best.tv_fwd_wave_from = wave_now ? nb + 1 : std::min(current.tv_fwd_wave_from, nb);
        ms[1] = (t_other >= 0.f && t_other < 0.98f * t_now) ? t_other : t_now;
        // backward (the TV gradient alone, into a scratch gradient)
        if (e == hipSuccess) e = grad.alloc((size_t)std::max<int64_t>(ctx->n_slots, 1));
        if (e == hipSuccess) e = dloss.alloc((size_t)ctx->n_shapes);
        if (e == hipSuccess) {
            std::vector<double> ones((size_t)ctx->n_shapes, 1.0);
            e = hipMemcpyAsync(dloss.p, ones.data(), ones.size() * sizeof(double), hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
        }
        const float b_wave = time_it([&] {
            k_tv_backward_wave<<<waves_grid, kTvWaves * 64, 0, st>>>(B, field, ctx->tau.p, w, dloss.p, ctx->inv_qv.p,
                                                                    nullptr, grad.p, (int32_t)nb);
        });
        const float b_brick = time_it([&] {
            k_tv_backward_brick<kB><<<(unsigned)nb, TvBrick<kB>::T, 0, st>>>(B, field, ctx->tau.p, w, dloss.p, ctx->inv_qv.p,
                                                                 nullptr, grad.p);
        });
        const bool bwave_now = nb >= current.tv_bwd_wave_from;
        const float b_now = bwave_now ? b_wave : b_brick, b_other = bwave_now ? b_brick : b_wave;
        if (e == hipSuccess && b_other >= 0.f && b_other < 0.98f * b_now)
            best.tv_bwd_wave_from = bwave_now ? nb + 1 : std::min(current.tv_bwd_wave_from, nb);
        ms[2] = (b_other >= 0.f && b_other < 0.98f * b_now) ? b_other : b_now;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    GP_HIP(ctx, e);
    ctx->grad_params = best;
    if (best_out) *best_out = best;
    if (best_ms_out)
        for (int i = 0; i < 3; ++i) best_ms_out[i] = ms[i];
    return GP_OK;
}

gp_status gp_autotune_grad_impl(gp_ctx ctx, const float* qx, const float* qy, const float* qz, const int32_t* nn,
                                const float* field, gp_weights w, int32_t reps, GradParams* best_out,
                                float* best_ms_out)
{
    return with_brick(ctx->brick, [&](auto tag) {
        return autotune_grad<decltype(tag)::value>(ctx, qx, qy, qz, nn, field, w, reps, best_out, best_ms_out);
    });
}
