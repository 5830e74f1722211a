// Internal definitions of the gfx950 GridPull library: device-side shape
// descriptors, the brick-sparse field layout and the helpers every kernel
// shares (cell location, brick lookup, trilinear value and gradient).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <type_traits>
#include <vector>

#include "gridpull.h"

namespace gp {

// Bricks of the band: kB^3 vertices, kB in {4, 8, 16} (gp_build_band's
// brick argument); every kernel that walks the band is instantiated per size.
// The search grid of the nearest-neighbour search always uses 8^3 bricks
// (kBrick, kBrickVol and the untemplated helpers below).
template <int kB>
struct Geo {
    static_assert(kB == 4 || kB == 8 || kB == 16, "brick edge 4, 8 or 16");
    static constexpr int32_t B = kB;                           // vertices per edge
    static constexpr int32_t S = kB == 4 ? 2 : (kB == 8 ? 3 : 4);   // log2 B
    static constexpr int32_t M = kB - 1;
    static constexpr int32_t V = kB * kB * kB;                 // vertices per brick
    static constexpr int32_t W = V / 32;                       // 32-bit mask words per brick
};
template <int kB>
struct BrickTag {
    static constexpr int value = kB;
};

constexpr int kBrick = 8;                 // the search grid's brick edge (and the default band brick)
constexpr int kBrickVol = 512;
constexpr int kMaskWords = kBrickVol / 32;
constexpr int kQueryBlock = 256;          // threads per block of the query kernels
constexpr int kQueriesPerThread = 4;
constexpr int kQueryTile = kQueryBlock * kQueriesPerThread;
// Field slots and brick directory entries stay below 2^30, so that 4-byte
// elements are addressed with 32-bit byte offsets (see at32).
constexpr int64_t kMaxSlots = (int64_t)1 << 30;
constexpr double kEpsNorm = 1e-12;        // |grad f| below this: no normalised gradient

// Per-shape constants as the kernels see them.
struct ShapeDesc {
    double lo[3];
    double inv_h[3];       // R_a / (hi_a - lo_a)
    float inv_hf[3];       // the same in float (gradient factors)
    float h[3];
    double hd[3];          // (hi_a - lo_a) / R_a in double (vertex positions)
    int32_t R[3];          // cells per axis
    int32_t nb[3];         // bricks per axis = ceil((R+1)/8)
    int64_t dir_off;       // first directory entry of this shape
    int64_t brick_begin;   // global brick range [brick_begin, brick_end)
    int64_t brick_end;
    int64_t point_off;
    int64_t point_cnt;
    int64_t query_off;
    int64_t query_cnt;
    int64_t tile_begin;    // query tiles [tile_begin, tile_end)
    int64_t tile_end;
    int64_t dense_off;     // offset of the shape's (R+1)^3 dense vertex array
    int64_t sorted_off;    // first entry of the shape's points in the sorted copy
    int64_t n_tv;          // number of TV vertices
    int64_t occ_off;       // search grids only: first word of the shape's cell occupancy bitmap
};

// Brick metadata: owning shape and brick coordinates.
struct BrickInfo {
    int32_t shape;
    int32_t bx, by, bz;
};

// Read-only view of the band structures.
struct Band {
    const ShapeDesc* shapes;
    const int32_t* dir;          // brick directory, -1 = no brick
    const BrickInfo* bricks;
    const uint32_t* m_base;      // [n_bricks][16] cell (lowest corner) holds a point
    const uint32_t* m_a1;        // [n_bricks][16] cell (lowest corner) in the M1 band
    const uint32_t* m_v;         // [n_bricks][16] optimised vertex
    const uint32_t* m_v2;        // [n_bricks][16] TV vertex
    const int64_t* tile_start;   // [n_tiles] first query of each tile
    const int32_t* tile_shape;   // [n_tiles]
    const uint32_t* occ;         // search grids only: per shape, 1 bit per cell (x-major id), set if the cell holds a point
};

// Nearest-neighbour search shape: a group of queries is cut where its cells
// would span `span` or more cells on an axis, its lockstep box is the group's
// cell box grown by `shell` cells, `parts` blocks (1, 2 or 4) share each
// query tile, with skip_empty every column of cells is first trimmed to its
// first and last occupied cell (occupancy bitmap), and without sort the
// groups are cut along the input order.  Any values give the
// same exact result; they only move work between the lockstep and per-query
// passes, between blocks, and between loads of bitmap words and of ranges.
struct NnParams {
    int32_t span = 8;
    int32_t shell = 1;
    int32_t parts = 1;
    int32_t skip_empty = 0;   // trim each scanned column to its occupied cells first
    int32_t sort = 1;         // Morton-sort each tile before grouping (else the input order)
    int32_t cell_points = 8;  // target points per occupied cell of the search grid (host side only)
};
constexpr int32_t kNnSpanMax = 64;
constexpr int32_t kNnShellMax = 4;
constexpr int32_t kNnCellPointsMax = 65536;

// Settings of the gradient pass and the TV kernels (any values give the same
// arithmetic; only the speed changes): the LDS rows of the query pass in
// vertices (kWinCaps; 8 bytes each, in rows of 16 consecutive slots,
// allocated at launch), the most slabs a block takes before its contributions
// go straight to the gradient, and the band sizes (bricks) from which the TV
// forward and backward take one wave per brick instead of one block.
constexpr int32_t kWinCaps[3] = {2048, 4096, 6144};
constexpr int32_t kWinCapMax = 6144;
constexpr int32_t kWinPassesMax = 64;
struct GradParams {
    int32_t win_cap = 4096;
    int32_t win_max_passes = 16;
    int64_t tv_fwd_wave_from = 2048;
    int64_t tv_bwd_wave_from = 16384;
};

struct Loc {
    int32_t c[3];
    double t[3];     // exact local coordinate in [0, 1]
    bool inside;
};

// Cell location in double, shared by every kernel: u = (x - lo) * inv_h,
// c = floor(u) clamped to R-1; inside iff 0 <= u <= R.
__device__ inline Loc locate(const ShapeDesc& s, float x, float y, float z)
{
#pragma clang fp contract(off)
    Loc L;
    const float p[3] = {x, y, z};
    bool in = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double u = ((double)p[a] - s.lo[a]) * s.inv_h[a];
        in = in && (u >= 0.0) && (u <= (double)s.R[a]);
        double fl = floor(u);
        // clamp also for positions outside (their result is not used for values)
        fl = fmin(fmax(fl, 0.0), (double)(s.R[a] - 1));
        int32_t ci = (int32_t)fl;
        L.c[a] = ci;
        L.t[a] = u - (double)ci;
    }
    L.inside = in;
    return L;
}

// Element i (< 2^30) of a 4-byte array through a 32-bit byte offset: with a
// uniform base the load takes the scalar-base plus vector-offset form, with
// no 64-bit address arithmetic per lane.
template <class T>
__device__ inline T* at32(T* base, uint32_t i)
{
    static_assert(sizeof(T) == 4, "4-byte elements");
    using Byte = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return reinterpret_cast<T*>(reinterpret_cast<Byte*>(base) + i * 4u);
}

__device__ inline int32_t brick_of(const Band& B, const ShapeDesc& s, int32_t bx, int32_t by, int32_t bz)
{
    return B.dir[s.dir_off + ((int64_t)bx * s.nb[1] + by) * s.nb[2] + bz];
}

// Index of vertex (i, j, k) inside its brick: x-major over the brick's edge.
template <int kB>
__device__ inline int32_t local_index_b(int32_t i, int32_t j, int32_t k)
{
    using G = Geo<kB>;
    return (((i & G::M) << G::S | (j & G::M)) << G::S) | (k & G::M);
}

__device__ inline int32_t local_index(int32_t i, int32_t j, int32_t k)
{
    return local_index_b<kBrick>(i, j, k);
}

template <int kB>
__device__ inline bool mask_bit_b(const uint32_t* m, int32_t brick, int32_t local)
{
    return (m[(int64_t)brick * Geo<kB>::W + (local >> 5)] >> (local & 31)) & 1u;
}

__device__ inline bool mask_bit(const uint32_t* m, int32_t brick, int32_t local)
{
    return mask_bit_b<kBrick>(m, brick, local);
}

// Slots of the eight corners of cell c, corner (a,b,c) at index 4a+2b+c.
// Every corner of an M1-band cell exists, so no -1 is returned for them.
// The corner one step up an axis lies in the next brick only when the cell
// sits on the brick's last layer of that axis, so the eight directory
// entries are one base entry plus fixed strides.
template <int kB>
__device__ inline void corner_slots(const Band& B, const ShapeDesc& s, const int32_t c[3], int32_t slot[8])
{
    using G = Geo<kB>;
    const uint32_t e0 =
        (uint32_t)s.dir_off + ((uint32_t)(c[0] >> G::S) * s.nb[1] + (c[1] >> G::S)) * s.nb[2] + (c[2] >> G::S);
    const uint32_t st[3] = {(c[0] & G::M) == G::M ? (uint32_t)(s.nb[1] * s.nb[2]) : 0u,
                            (c[1] & G::M) == G::M ? (uint32_t)s.nb[2] : 0u, (c[2] & G::M) == G::M ? 1u : 0u};
    const int32_t lx[2] = {(c[0] & G::M) << (2 * G::S), ((c[0] + 1) & G::M) << (2 * G::S)};
    const int32_t ly[2] = {(c[1] & G::M) << G::S, ((c[1] + 1) & G::M) << G::S};
    const int32_t lz[2] = {c[2] & G::M, (c[2] + 1) & G::M};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                const int32_t br = *at32(B.dir, e0 + a * st[0] + b * st[1] + d * st[2]);
                slot[4 * a + 2 * b + d] = br * G::V + lx[a] + ly[b] + lz[d];
            }
}

// Work item of block b among n: the chip dispatches consecutive blocks to
// its eight XCDs in turn, and each XCD has its own L2, so neighbouring work
// items (which read the same points and field values) would land in
// different L2s.  Renumbered, each run of 8 * kXcdChunk blocks gives every
// XCD kXcdChunk consecutive items (neighbours share its L2), while the runs
// still spread every region of the work over all eight XCDs (balance); the
// last n mod (8 * kXcdChunk) blocks keep their numbers.  A bijection of
// [0, n), so every item is done once whatever the mapping of blocks to XCDs
// really is.
constexpr int64_t kXcdChunk = 16;

__device__ inline int64_t xcd_work_item(int64_t b, int64_t n)
{
    constexpr int64_t run = 8 * kXcdChunk;
    if (b >= n / run * run) return b;
    const int64_t r = b % run;
    return b - r + (r & 7) * kXcdChunk + (r >> 3);
}

// Coordinates of a query's nearest point nn (an index among its shape's
// points, valid: 0 <= nn < point_cnt).  The NN search records, per query,
// the coordinates of its result together with the result's index; when that
// index is nn, the point is read there, 16 contiguous bytes of the query's
// own record (no dependent load).  Otherwise (nearest points that did not
// come from the search, or a record of an earlier search) it is read from
// the original order.  Either way the same coordinates.
struct PointView {
    const float4* pt;       // [n_queries] last NN result per query: x, y, z, its index within the shape (bits)
    const float* ox;        // original order, at sorted_off + index
    const float* oy;
    const float* oz;
};

__device__ inline void nearest_point(const ShapeDesc& s, const PointView& P, int64_t k, int32_t nn, float& sx,
                                     float& sy, float& sz)
{
    const float4 v = P.pt[k];
    if (__float_as_int(v.w) == nn) {
        sx = v.x;
        sy = v.y;
        sz = v.z;
    } else {
        const int64_t g = s.sorted_off + nn;
        sx = P.ox[g];
        sy = P.oy[g];
        sz = P.oz[g];
    }
}

// Wave-wide reductions: DPP steps inside each row of 16 lanes (pairs, quads,
// half rows, rows), then the four row results read from lanes 0, 16, 32 and
// 48.  Every lane of the wave must be active; the result is wave-uniform.
// The sums are taken in that fixed order (each step adds two partial sums,
// the same in both lanes), so they do not depend on timing.
template <int Ctrl>
__device__ inline int32_t dpp_i32(int32_t v)
{
    return __builtin_amdgcn_update_dpp(v, v, Ctrl, 0xf, 0xf, false);
}

template <int Ctrl>
__device__ inline double dpp_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int32_t lo = dpp_i32<Ctrl>((int32_t)b), hi = dpp_i32<Ctrl>((int32_t)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)(uint32_t)hi << 32) | (uint32_t)lo));
}

__device__ inline double readlane_f64(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(b >> 32), lane);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ inline int32_t wave_min_i32(int32_t v)
{
    v = min(v, dpp_i32<0xB1>(v));    // quad_perm [1, 0, 3, 2]
    v = min(v, dpp_i32<0x4E>(v));    // quad_perm [2, 3, 0, 1]
    v = min(v, dpp_i32<0x141>(v));   // row_half_mirror
    v = min(v, dpp_i32<0x140>(v));   // row_mirror
    return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

__device__ inline int32_t wave_max_i32(int32_t v)
{
    v = max(v, dpp_i32<0xB1>(v));
    v = max(v, dpp_i32<0x4E>(v));
    v = max(v, dpp_i32<0x141>(v));
    v = max(v, dpp_i32<0x140>(v));
    return max(max(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               max(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
}

__device__ inline double wave_sum_f64(double v)
{
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    v += dpp_f64<0x141>(v);
    v += dpp_f64<0x140>(v);
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// Block-wide minimum of v[0..2] and maximum of v[3..5] (blockDim = 256).
// Every thread receives the result.  scratch: shared int [4 * 6].
__device__ inline void block_minmax6(int32_t v[6], int32_t* scratch)
{
#pragma unroll
    for (int i = 0; i < 6; ++i) v[i] = i < 3 ? wave_min_i32(v[i]) : wave_max_i32(v[i]);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
        for (int i = 0; i < 6; ++i) scratch[wave * 6 + i] = v[i];
    __syncthreads();
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < 6; ++i) {
        int32_t r = scratch[i];
        for (int w = 1; w < nw; ++w) r = i < 3 ? min(r, scratch[w * 6 + i]) : max(r, scratch[w * 6 + i]);
        v[i] = r;
    }
    __syncthreads();
}

// Trilinear value and gradient from the eight corner values (Eq. 1 / Eq. 3),
// in double from the float corner values and the exact double local
// coordinate: the gradient is a sum of corner differences that can cancel,
// and its error would be amplified by the normalisation 1/|grad f|.
struct Interp {
    double f;
    double g[3];
};

__device__ inline Interp trilinear(const float D[8], const double t[3], const double inv_h[3])
{
    // interpolate along z, then y, then x; keep the partial differences
    double e[4], dz[4];
#pragma unroll
    for (int ab = 0; ab < 4; ++ab) {
        dz[ab] = (double)D[2 * ab + 1] - (double)D[2 * ab];
        e[ab] = fma(t[2], dz[ab], (double)D[2 * ab]);
    }
    double fa[2], fya[2], fza[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        fya[a] = e[2 * a + 1] - e[2 * a];
        fa[a] = fma(t[1], fya[a], e[2 * a]);
        fza[a] = fma(t[1], dz[2 * a + 1] - dz[2 * a], dz[2 * a]);
    }
    Interp r;
    const double fx = fa[1] - fa[0];
    r.f = fma(t[0], fx, fa[0]);
    r.g[0] = fx * inv_h[0];
    r.g[1] = fma(t[0], fya[1] - fya[0], fya[0]) * inv_h[1];
    r.g[2] = fma(t[0], fza[1] - fza[0], fza[0]) * inv_h[2];
    return r;
}

// Adjoint of trilinear(): contribution to each corner value given
// dl/df and dl/dgrad f.
__device__ inline void trilinear_adjoint(const float t[3], const float inv_h[3], float df,
                                         const float dg[3], float out[8])
{
    const float gx = dg[0] * inv_h[0], gy = dg[1] * inv_h[1], gz = dg[2] * inv_h[2];
    const float wx[2] = {1.f - t[0], t[0]}, wy[2] = {1.f - t[1], t[1]}, wz[2] = {1.f - t[2], t[2]};
    const float sg[2] = {-1.f, 1.f};
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int d = 0; d < 2; ++d) {
                float wyz = wy[b] * wz[d];
                float v = wyz * fmaf(wx[a], df, sg[a] * gx);
                v = fmaf(wx[a] * wz[d] * sg[b], gy, v);
                v = fmaf(wx[a] * wy[b] * sg[d], gz, v);
                out[4 * a + 2 * b + d] = v;
            }
}

}  // namespace gp

// ---------------------------------------------------------------------------
// Host-side context
// ---------------------------------------------------------------------------

template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    hipError_t alloc(size_t count)
    {
        release();
        if (count == 0) count = 1;
        hipError_t e = hipMalloc(&p, count * sizeof(T));
        if (e == hipSuccess) n = count;
        else p = nullptr;
        return e;
    }
};

struct gp_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;

    // band state
    bool built = false;
    int32_t brick = 8;          // band brick edge (4, 8 or 16)
    int32_t n_shapes = 0;
    int32_t m1 = 0, m2 = 0;
    int64_t n_bricks = 0;
    int64_t n_slots = 0;
    int64_t n_active = 0;
    int64_t n_points = 0;       // end of the last point slice
    int64_t n_queries = 0;      // end of the last query slice
    int64_t n_tiles = 0;
    int64_t n_dir = 0;
    std::vector<gp::ShapeDesc> h_shapes;
    std::vector<int64_t> h_slot_begin;

    DevBuf<gp::ShapeDesc> shapes;
    DevBuf<int32_t> dir;
    DevBuf<gp::BrickInfo> bricks;
    DevBuf<uint32_t> m_a1, m_a2, m_base, m_v, m_v2;
    DevBuf<int64_t> tile_start;
    DevBuf<int32_t> tile_shape;
    std::vector<int64_t> h_occupied;   // [n_shapes] band cells holding a point

    DevBuf<float4> spts;          // points sorted by band cell slot (the sampler's source order): x, y, z,
                                  // original index within the shape (bits)
    DevBuf<float> ox, oy, oz;     // points in their original order, at sorted_off + index

    // nearest-neighbour search grid: per shape a grid over the same box with
    // cells 2^k times the band's, its own brick directory, occupancy bitmap
    // and points bucketed by its cells
    std::vector<gp::ShapeDesc> h_nn_shapes;
    std::vector<int32_t> h_nn_levels;   // [n_shapes] k: search cells are 2^k band cells wide
    int32_t nn_cell_points = 0;   // the target the current search grids were built for (0: none)
    int64_t nn_slots = 0;
    DevBuf<gp::ShapeDesc> nn_shapes;
    DevBuf<int32_t> nn_dir;
    DevBuf<uint32_t> occ;         // occupancy bitmaps of all search grids
    DevBuf<int32_t> cell_start;   // [nn_slots + 1]
    DevBuf<float4> nn_spts;       // points sorted by search-grid slot: x, y, z, original index (bits)
    DevBuf<float4> nn_pt;         // [n_queries] the last NN result per query: coordinates and index (bits)

    // per-iteration scratch
    DevBuf<double> q_part;        // [n_tiles][4] sum pull, surf, grad, count
    DevBuf<double> tv_part;       // [n_bricks] sum tau
    DevBuf<float> tau;            // [n_slots] 1 / tau of the last forward (0 where tau = 0)
    DevBuf<double> inv_qv;        // [n_shapes] 1 / valid count (0 if none)
    DevBuf<double> fin_part;      // [n_shapes][32][5] chunk sums of the loss reduction
    DevBuf<int32_t> fin_count;    // [n_shapes] chunks finished (back to 0 after each reduction)
    DevBuf<double> nrm_part;      // normal supervision: per-block (term, count), allocated on first use
    DevBuf<float> nrm_scale;      // normal supervision: per-shape gradient scale
    DevBuf<int32_t> flag;         // device error flag
    DevBuf<int32_t> iter;         // device-resident iteration counter (last Adam t)
    DevBuf<float> step_c;         // [2] lr_t / (1 - beta1^t), 1 / sqrt(1 - beta2^t)
    DevBuf<float> g_raw;          // [n_slots] unscaled query contributions of a fused pass (kept zero between passes)
    // The last forward (gp_pull_forward or gp_pull_forward_backward): its
    // token (0 = none, or invalidated) and the arrays it read.  A backward
    // must name that token and the same arrays; a later call of the library
    // that writes one of those arrays, or rebuilds the band, invalidates it.
    uint64_t token_counter = 0;
    uint64_t fwd_token = 0;
    const void* fwd_arrays[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // qx, qy, qz, nn, field

    gp::NnParams nn_params;       // set by gp_set_nn_params or gp_autotune_nn
    gp::GradParams grad_params;   // set by gp_set_grad_params, gp_set_tv_layout or gp_autotune_grad

    // optional per-kernel timing with events on the context's stream
    struct TimedLaunch {
        const char* name;
        hipEvent_t a, b;
    };
    bool timing = false;
    std::vector<TimedLaunch> timed;
    std::vector<hipEvent_t> event_pool;

    gp::PointView points() const
    {
        return gp::PointView{nn_pt.p, ox.p, oy.p, oz.p};
    }

    // The band view with the search grids' descriptors, directory and
    // occupancy in place of the band's (for the nearest-neighbour search).
    gp::Band nn_band() const
    {
        gp::Band b = band();
        b.shapes = nn_shapes.p;
        b.dir = nn_dir.p;
        b.bricks = nullptr;
        b.occ = occ.p;
        return b;
    }

    gp::Band band() const
    {
        gp::Band b;
        b.shapes = shapes.p;
        b.dir = dir.p;
        b.bricks = bricks.p;
        b.m_base = m_base.p;
        b.m_a1 = m_a1.p;
        b.m_v = m_v.p;
        b.m_v2 = m_v2.p;
        b.tile_start = tile_start.p;
        b.tile_shape = tile_shape.p;
        b.occ = nullptr;
        return b;
    }
};

// Calls f(BrickTag<kB>{}) for the band's brick edge kB (4, 8 or 16), so that
// a launch site picks the kernel instance of the context's bricks.
template <class F>
inline auto with_brick(int32_t brick, F&& f) -> decltype(f(gp::BrickTag<8>{}))
{
    switch (brick) {
    case 4: return f(gp::BrickTag<4>{});
    case 16: return f(gp::BrickTag<16>{});
    default: return f(gp::BrickTag<8>{});
    }
}

// Brackets one kernel launch with events when timing is enabled.
hipEvent_t gp_timer_begin(gp_ctx ctx);
void gp_timer_end(gp_ctx ctx, const char* name, hipEvent_t begin);

struct GpTimed {
    gp_ctx c;
    const char* name;
    hipEvent_t a;
    GpTimed(gp_ctx c_, const char* n) : c(c_), name(n), a(gp_timer_begin(c_)) {}
    ~GpTimed() { gp_timer_end(c, name, a); }
};
#define GP_TIMED(ctx, name) GpTimed gp_timed_scope_(ctx, name)

// status helpers (defined in gp_api.hip)
gp_status gp_fail(gp_ctx ctx, gp_status st, const std::string& msg);
gp_status gp_hip_fail(gp_ctx ctx, hipError_t e, const char* what);

#define GP_HIP(ctx, call)                                              \
    do {                                                               \
        hipError_t e_ = (call);                                        \
        if (e_ != hipSuccess) return gp_hip_fail((ctx), e_, #call);    \
    } while (0)

// kernel launch wrappers implemented in the other translation units
gp_status gp_build_band_impl(gp_ctx ctx, const gp_shape* shapes, int32_t n_shapes,
                             const float* px, const float* py, const float* pz,
                             int32_t m1, int32_t m2, int32_t brick);
gp_status gp_build_nn_index(gp_ctx ctx, int32_t cell_points);
std::vector<int32_t> gp_nn_levels(gp_ctx ctx, int32_t cell_points);   // per shape, before the size limits
gp_status gp_nn_impl(gp_ctx ctx, const float* qx, const float* qy, const float* qz, int32_t* nn);
gp_status gp_autotune_nn_impl(gp_ctx ctx, const float* qx, const float* qy, const float* qz, int32_t* nn,
                              int32_t reps, gp::NnParams* best_out, float* best_ms_out);
gp_status gp_sample_impl(gp_ctx ctx, uint64_t seed, int32_t iteration, const float* sigma,
                         float sigma_const, float* qx, float* qy, float* qz, int32_t* src);
gp_status gp_step_consts_impl(gp_ctx ctx, int32_t t, float lr0, float decay, int32_t decay_every, float beta1,
                              float beta2);
gp_status gp_autotune_grad_impl(gp_ctx ctx, const float* qx, const float* qy, const float* qz, const int32_t* nn,
                                const float* field, gp_weights w, int32_t reps, gp::GradParams* best_out,
                                float* best_ms_out);
gp_status gp_forward_impl(gp_ctx ctx, const float* qx, const float* qy, const float* qz,
                          const int32_t* nn, const float* field, gp_weights w,
                          double* loss_out, int64_t* n_valid_out);
gp_status gp_forward_static_impl(gp_ctx ctx, const float* qx, const float* qy, const float* qz, const int32_t* nn,
                                 const float* field, gp_weights w, double* loss_out, int64_t* n_valid_out);
gp_status gp_backward_impl(gp_ctx ctx, const float* qx, const float* qy, const float* qz,
                           const int32_t* nn, const float* field, gp_weights w,
                           const double* dloss, float* grad);
gp_status gp_forward_backward_impl(gp_ctx ctx, const float* qx, const float* qy, const float* qz,
                                   const int32_t* nn, const float* field, gp_weights w, const double* dloss,
                                   double* loss_out, int64_t* n_valid_out, float* grad);
gp_status gp_step_impl(gp_ctx ctx, float* field, float* grad, float* m, float* v, float beta1, float beta2,
                       float eps);
gp_status gp_layout_impl(gp_ctx ctx, int64_t* vid, uint8_t* flags);
gp_status gp_active_cells_impl(gp_ctx ctx, int32_t shape, int64_t* cell_ids, int64_t capacity, int64_t* n_out);
gp_status gp_normals_impl(gp_ctx ctx, const float* qx, const float* qy, const float* qz, const int32_t* nn,
                          const float* field, const float* nx, const float* ny, const float* nz, float weight,
                          const double* dloss, double* term_out, float* grad);
gp_status gp_extract_surface_impl(gp_ctx ctx, int32_t shape, const float* field, float* tri_xyz, int64_t* tri_key,
                                  int64_t capacity, int64_t* n_out, int32_t method);
gp_status gp_gather_impl(gp_ctx ctx, const float* dense, float* field, bool to_field);
gp_status gp_init_sphere_impl(gp_ctx ctx, const double* centre, const double* radius, float* field);
