// Nearest surface point NN(q) of every query (Eq. 4).
//
// The paper organises the points in a KD-tree.  Here the points are bucketed
// by the cells of a search grid per shape (built in band.hip: the shape's box
// in cells 2^k times the band's, k chosen from the point density so that an
// occupied cell holds a few points whatever the band resolution), sorted by
// the slot of their cell; a cell's points are contiguous, and so are the
// points of a run of cells along z inside one brick.  Every "cell" below is a
// search-grid cell.
//
// A block takes a tile of 1024 queries and sorts them by the Morton code of
// their cell; each wave cuts its quarter of the sorted list into groups of at
// most 64 queries whose cells span fewer than group_span cells per axis
// (default 8) and serves the groups one at a time in two passes.  Blocks take
// their tiles in an XCD-aware order (xcd_work_item).
//
// Lockstep pass (lane = query): the box of the group's cells grown by one
// cell.  Its rows (x, y) are laid out one per lane and cut into z-runs inside
// one brick (each run's points are contiguous), staged in LDS 64 at a time;
// their point ranges are fetched in one round trip and the concatenated
// points streamed in chunks of 64 through LDS, each point broadcast to every
// lane.  Each lane keeps its smallest and second-smallest float distance: when
// the second exceeds the first by more than the float error bound, the float
// argmin is the exact argmin; when in addition the best distance is below the
// query's gap to the box, no other point can be as close and the query is
// resolved.
//
// Point-parallel pass (lane = point) for the few queries left open: up to 6
// at a time, the cells meeting the bounding box of the ball of each one's
// candidate distance, outside the box already scanned, are streamed once;
// every lane tests its point against each of the queries, and the per-lane
// minima are reduced over the wave.  Afterwards no unseen point can beat the
// candidate, so a unique float minimum is the answer.
//
// Near ties (and queries with no candidate, or a very large ball) run an
// exact ring search: distances in double without fused multiply-add, ties to
// the lowest point index, so every result equals a brute-force search bit
// for bit.
#include <hipcub/hipcub.hpp>

#include <algorithm>

#include "gp_internal.h"

namespace gp {
namespace {

constexpr int kNnMaxGrow = 8;     // growth beyond which a group with no point in its box goes to the ring search

struct Best {
    double d2;
    int32_t id;     // original index within the shape (the tie rule)
    int32_t pos;    // global position in the search grid's sorted copy
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

__device__ inline void consider(double d2, int32_t id, int32_t pos, Best& best)
{
    if (d2 < best.d2 || (d2 == best.d2 && id < best.id)) {
        best.d2 = d2;
        best.id = id;
        best.pos = pos;
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
    const float4* pts;    // x, y, z, original index (bits)
};

// The search passes carry, in .w of each staged point, its position in the
// search grid's sorted copy instead of its original index (float pass ties are not
// decided there: they go to the exact search, which uses the original index).

// Global range of the points of cells (x, y, za..zb) (one brick): empty if none.
__device__ inline void run_range(const Band& B, const ShapeDesc& s, const Global& G, int32_t x, int32_t y,
                                 int32_t za, int32_t zb, int32_t& b, int32_t& e)
{
    b = e = 0;
    const int32_t br = brick_of(B, s, x >> 3, y >> 3, za >> 3);
    if (br < 0) return;
    b = G.cell_start[br * kBrickVol + local_index(x, y, za)];
    e = G.cell_start[br * kBrickVol + local_index(x, y, zb) + 1];
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

// Exact ring search: cells in rings of growing Chebyshev radius around the
// query's cell, each opened only if its box can hold a point at least as close
// as the best so far; stops once every unopened cell is provably farther.
// Returns the winner's position in the sorted copy (-1 for a shape without points).
__device__ inline int32_t search(const Band& B, const ShapeDesc& s, const Global& G, float x, float y, float z)
{
    if (s.point_cnt <= 0) return -1;
    int32_t c0[3];
    float du[3], margin[3];
    query_cell(s, x, y, z, c0, du);
#pragma unroll
    for (int a = 0; a < 3; ++a) margin[a] = 1e-4f * (1.f + fabsf(du[a]));
    const float h2[3] = {s.h[0] * s.h[0], s.h[1] * s.h[1], s.h[2] * s.h[2]};
    Best best{__builtin_inf(), 0x7fffffff, -1};
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
                    int32_t b, e;
                    run_range(B, s, G, cx, cy, cz, cz, b, e);
                    for (int32_t i = b; i < e; ++i) {
                        const float4 p = G.pts[i];
                        consider(exact_d2(x, y, z, p.x, p.y, p.z), __float_as_int(p.w), i, best);
                    }
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
    return best.pos;
}

// Wave-wide minimum of v[0..2] and maximum of v[3..5] (the same in every
// lane afterwards, so kept in scalar registers).
__device__ inline void wave_minmax6(int32_t v[6])
{
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        for (int o = 32; o > 0; o >>= 1) {
            int32_t w = __shfl_xor(v[i], o, 64);
            v[i] = i < 3 ? min(v[i], w) : max(v[i], w);
        }
        v[i] = __builtin_amdgcn_readfirstlane(v[i]);
    }
}

__device__ inline uint32_t spread3(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// Per-lane scan state.
struct Scan {
    float x, y, z;
    int32_t c0[3];
    float du[3];
    float best1, best2;
    int32_t id1;
    bool open;   // live and not yet resolved
};

// Orders the LDS accesses of the lanes of one wave.
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int32_t wave_exclusive_sum(int32_t v, int32_t& total)
{
    const int lane = threadIdx.x & 63;
    int32_t incl = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int32_t w = __shfl_up(incl, o, 64);
        if (lane >= o) incl += w;
    }
    total = __shfl(incl, 63, 64);
    return incl - v;
}

// Rank of this lane among the lanes set in m.
__device__ inline int32_t lane_rank(uint64_t m)
{
    return (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Evaluate the staged chunk buf[0..cnt) (an LDS broadcast per point) for every lane.
__device__ inline void eval_chunk(const float4* __restrict__ buf, int32_t cnt, Scan& q)
{
    float b1 = q.best1, b2 = q.best2;
    int32_t id = q.id1;
#pragma unroll 8
    for (int32_t t = 0; t < cnt; ++t) {
        const float4 p = buf[t];
        const float dx = q.x - p.x, dy = q.y - p.y, dz = q.z - p.z;
        const float d2f = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
        // (b1 <= b2: the second smallest of b1, b2, d2f is their median)
        const bool lt = d2f < b1;
        b2 = __builtin_amdgcn_fmed3f(b1, b2, d2f);
        id = lt ? __float_as_int(p.w) : id;
        b1 = lt ? d2f : b1;   // a select on the same compare (no NaN canonicalisation of a min)
    }
    q.best1 = b1;
    q.best2 = b2;
    q.id1 = id;
}

template <int Ctrl>
__device__ inline uint32_t dpp_u(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int32_t)v, (int32_t)v, Ctrl, 0xf, 0xf, false);
}

// Wave-wide minimum of non-negative floats (their bits order as integers).
__device__ inline float wave_min_pos(float v)
{
    uint32_t u = __float_as_uint(v);
    u = min(u, dpp_u<0xB1>(u));    // quad_perm [1, 0, 3, 2]
    u = min(u, dpp_u<0x4E>(u));    // quad_perm [2, 3, 0, 1]
    u = min(u, dpp_u<0x141>(u));   // row_half_mirror
    u = min(u, dpp_u<0x140>(u));   // row_mirror
    u = min(min((uint32_t)__builtin_amdgcn_readlane((int32_t)u, 0), (uint32_t)__builtin_amdgcn_readlane((int32_t)u, 16)),
            min((uint32_t)__builtin_amdgcn_readlane((int32_t)u, 32), (uint32_t)__builtin_amdgcn_readlane((int32_t)u, 48)));
    return __uint_as_float(u);
}

// Smallest and second-smallest distance over the wave and an argmin: the
// smallest of the lanes' b1; its lane; then the second smallest is the
// smaller of that lane's b2 and every other lane's b1 (two lanes tying on
// the smallest give b2 == b1, which never counts as unique).
__device__ inline void wave_best2(float& b1, float& b2, int32_t& id)
{
    const float m = wave_min_pos(b1);
    const uint64_t at = __ballot(b1 == m);
    const int32_t lead = (int32_t)__builtin_ctzll(at);
    const int lane = threadIdx.x & 63;
    const float second = wave_min_pos(lane == lead ? b2 : b1);
    id = __builtin_amdgcn_readlane(id, lead);
    b1 = m;
    b2 = second;
}

// Inclusive prefix maximum over the lanes of non-negative values: within
// rows of 16 by DPP row shifts, then across rows from the rows' last lanes.
__device__ inline int32_t wave_prefix_max(int32_t v)
{
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false));   // row_shr:1
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false));   // row_shr:2
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false));   // row_shr:4
    v = max(v, __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false));   // row_shr:8
    const int32_t r0 = __builtin_amdgcn_readlane(v, 15);
    const int32_t r1 = max(r0, __builtin_amdgcn_readlane(v, 31));
    const int32_t r2 = max(r1, __builtin_amdgcn_readlane(v, 47));
    const int row = (threadIdx.x & 63) >> 4;
    return max(v, row == 0 ? 0 : (row == 1 ? r0 : (row == 2 ? r1 : r2)));
}

constexpr int kRunCap = 128;   // runs staged per wave (a batch of 64 plus one append round)
constexpr int kRunArea = kRunCap + 16;   // per wave: the runs, then 64 ints marking run starts in a chunk
constexpr int kTail = 6;       // open queries served together by the point-parallel pass
constexpr int kTailSpan = 24;  // larger balls (cells per axis) go to the ring search

// Lockstep evaluation: lane = query, each staged point broadcast from LDS.
struct Lockstep {
    Scan* q;
    float4* buf;   // this wave's 64-point staging area
    __device__ void stage(const float4& p) const
    {
        buf[threadIdx.x & 63] = p;
        wave_sync();
    }
    __device__ void eval(const float4&, int32_t cnt) const
    {
        eval_chunk(buf, cnt, *q);
        wave_sync();
    }
};

// Point-parallel evaluation: lane = point, each of up to kTail queries (slot
// k at tq[k]) keeps per-lane smallest / second-smallest distance and argmin,
// reduced over the wave afterwards.
struct Tail {
    const float4* tq;
    int32_t ns;
    float b1[kTail], b2[kTail];
    int32_t id[kTail];
    __device__ void stage(const float4&) const {}
    __device__ void eval(const float4& p, int32_t cnt)
    {
        const bool ok = (int32_t)(threadIdx.x & 63) < cnt;
#pragma unroll
        for (int k = 0; k < kTail; ++k) {
            if (k < ns) {
                const float4 t = tq[k];
                const float dx = t.x - p.x, dy = t.y - p.y, dz = t.z - p.z;
                float d = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
                d = ok ? d : __builtin_inff();
                const bool lt = d < b1[k];
                b2[k] = __builtin_amdgcn_fmed3f(b1[k], b2[k], d);
                id[k] = lt ? __float_as_int(p.w) : id[k];
                b1[k] = lt ? d : b1[k];
            }
        }
    }
};

// Scan the points of the first min(n, 64) staged runs (x, y, z0, z1) with
// the evaluator, drop those runs from the stage and return how many are left.
template <class Ev>
__device__ inline int32_t flush_runs(const Band& B, const ShapeDesc& s, const Global& G, int4* __restrict__ runs,
                                     int32_t n, Ev& ev)
{
    const int lane = threadIdx.x & 63;
    const int32_t cnt = min(n, 64);
    int32_t pb = 0, pe = 0;
    if (lane < cnt) {
        const int4 r = runs[lane];
        run_range(B, s, G, r.x, r.y, r.z, r.w, pb, pe);
    }
    int32_t total;
    const int32_t off = wave_exclusive_sum(pe - pb, total);
    total = __builtin_amdgcn_readfirstlane(total);
    // Stream position c + lane -> the last non-empty run starting at or before
    // it: every non-empty run starting inside the chunk marks its start (no
    // two share one), a prefix maximum spreads the marks over the lanes, and
    // the run covering the chunk's first position comes from the previous
    // chunk's last lane.  Chunks are taken in order.
    int32_t* starts = reinterpret_cast<int32_t*>(runs + kRunCap);
    int32_t carry = 0;   // 1 + run covering the next chunk's first position
    auto chunk_at = [&](int32_t c) -> float4 {
        starts[lane] = 0;
        wave_sync();
        const int32_t h = off - c;
        if (lane < cnt && pe > pb && h >= 0 && h < 64) starts[h] = lane + 1;
        wave_sync();
        const int32_t v = wave_prefix_max(max(starts[lane], carry));
        carry = __builtin_amdgcn_readlane(v, 63);
        const int32_t j = max(v - 1, 0);
        const int32_t p = c + lane;
        const int32_t idx = __shfl(pb, j, 64) + (p - __shfl(off, j, 64));
        const float4 x = G.pts[p < total ? idx : 0];   // a scan only happens for a shape with points
        return p < total ? make_float4(x.x, x.y, x.z, __int_as_float(idx)) : make_float4(0.f, 0.f, 0.f, 0.f);
    };
    float4 nxt = total > 0 ? chunk_at(0) : make_float4(0.f, 0.f, 0.f, 0.f);
    for (int32_t c = 0; c < total; c += 64) {
        const float4 cur = nxt;
        ev.stage(cur);
        nxt = chunk_at(c + 64);    // the next chunk's loads fly during the evaluation
        ev.eval(cur, min(64, total - c));
    }
    const int32_t rest = n - cnt;
    int4 keep = make_int4(0, 0, 0, 0);
    if (lane < rest) keep = runs[64 + lane];
    wave_sync();
    if (lane < rest) runs[lane] = keep;
    wave_sync();
    return rest;
}

// The first and last cell of column (x, y) in [za, zb] that hold a point,
// from the occupancy bitmap (za > zb afterwards: none).
__device__ inline void trim_column(const Band& B, const ShapeDesc& s, int32_t x, int32_t y, int32_t& za, int32_t& zb)
{
    if (za > zb) return;
    const int64_t base = s.occ_off * 32 + ((int64_t)x * s.R[1] + y) * s.R[2];   // bit of cell (x, y, 0)
    const int64_t i0 = base + za, i1 = base + zb;
    const int64_t w0 = i0 >> 5, w1 = i1 >> 5;
    const uint32_t m0 = ~0u << (i0 & 31), m1 = ~0u >> (31 - (i1 & 31));
    int64_t first = -1, last = -1;
#pragma unroll 1
    for (int64_t w = w0; w <= w1; ++w) {
        uint32_t v = B.occ[w] & (w == w0 ? m0 : ~0u) & (w == w1 ? m1 : ~0u);
        if (v) {
            first = w * 32 + __builtin_ctz(v);
            break;
        }
    }
    if (first < 0) {
        za = 1;
        zb = 0;
        return;
    }
#pragma unroll 1
    for (int64_t w = w1; w >= (first >> 5); --w) {
        uint32_t v = B.occ[w] & (w == w0 ? m0 : ~0u) & (w == w1 ? m1 : ~0u);
        if (v) {
            last = w * 32 + 31 - __builtin_clz(v);
            break;
        }
    }
    za = (int32_t)(first - base);
    zb = (int32_t)(last - base);
}

// Stage the brick-aligned pieces of this lane's z range [za, zb] on row
// (x, y) (an empty range adds nothing), flushing whenever 64 are staged.
// With trim, the range is first cut to its occupied cells.
template <class Ev>
__device__ inline void stage_range(const Band& B, const ShapeDesc& s, const Global& G, int4* __restrict__ runs,
                                   int32_t& n, Ev& ev, int32_t x, int32_t y, int32_t za, int32_t zb, bool trim)
{
    if (trim) trim_column(B, s, x, y, za, zb);
    int32_t z0 = za;
    for (;;) {
        const bool has = z0 <= zb;
        const uint64_t m = __ballot(has);
        if (m == 0) break;
        const int32_t z1 = min(zb, z0 | 7);
        if (has) runs[n + lane_rank(m)] = make_int4(x, y, z0, z1);
        n += __popcll(m);
        z0 = has ? z1 + 1 : z0;
        if (n >= 64) {
            wave_sync();
            n = flush_runs(B, s, G, runs, n, ev);
        }
    }
}

// Stage every cell of box [lo, hi] outside box [olo, ohi] (which may be
// empty), rows (x, y) one per lane, and scan them all.  With balls (x, y, z,
// r^2; a negative r^2 is an unused place), a column is taken only where it
// comes within r of one of the nb ball centres, and only the cells meeting
// the union of those chords.
template <class Ev>
__device__ inline void scan_box(const Band& B, const ShapeDesc& s, const Global& G, int4* __restrict__ runs, Ev& ev,
                                const int32_t lo[3], const int32_t hi[3], const int32_t olo[3], const int32_t ohi[3],
                                bool trim, const float4* balls = nullptr, int32_t nb = 0)
{
    const int lane = threadIdx.x & 63;
    if (lo[0] > hi[0] || lo[1] > hi[1] || lo[2] > hi[2]) return;
    int32_t n = 0;
    const int32_t ny = hi[1] - lo[1] + 1;
    const int32_t nrows = (hi[0] - lo[0] + 1) * ny;
    const float lo0 = (float)s.lo[0], lo1 = (float)s.lo[1], lo2 = (float)s.lo[2];
    const float ih2 = (float)s.inv_h[2];
    for (int32_t base = 0; base < nrows; base += 64) {
        const int32_t r = base + lane;
        bool row = r < nrows;
        const int32_t x = lo[0] + (row ? r / ny : 0);
        const int32_t y = lo[1] + (row ? r % ny : 0);
        int32_t za = lo[2], zb = hi[2];
        if (balls) {
            const float xl = fmaf((float)x, s.h[0], lo0), yl = fmaf((float)y, s.h[1], lo1);
            const float mx = 1e-3f * s.h[0], my = 1e-3f * s.h[1];
            int32_t zlo = 0x7fffffff, zhi = -1;
            for (int k = 0; k < nb; ++k) {
                const float4 t = balls[k];
                const float gx = fmaxf(fmaxf(xl - t.x, t.x - (xl + s.h[0])) - mx, 0.f);
                const float gy = fmaxf(fmaxf(yl - t.y, t.y - (yl + s.h[1])) - my, 0.f);
                const float lxy = fmaf(gx, gx, gy * gy);
                if (lxy <= t.w) {
                    const float rz = sqrtf(t.w - lxy) + 1e-3f * s.h[2];
                    const float ua = fminf(fmaxf((t.z - rz - lo2) * ih2, -1.f), 1e8f);
                    const float ub = fminf(fmaxf((t.z + rz - lo2) * ih2, -1.f), 1e8f);
                    zlo = min(zlo, (int32_t)floorf(ua));
                    zhi = max(zhi, (int32_t)floorf(ub));
                }
            }
            za = max(za, zlo);
            zb = min(zb, zhi);
        }
        if (!row) zb = -1;
        const bool inner = x >= olo[0] && x <= ohi[0] && y >= olo[1] && y <= ohi[1];
        int32_t zc = 0, zd = -1;
        if (row && inner) {
            zc = max(za, ohi[2] + 1);
            zd = zb;
            zb = min(zb, olo[2] - 1);
        }
        stage_range(B, s, G, runs, n, ev, x, y, za, zb, trim);
        stage_range(B, s, G, runs, n, ev, x, y, zc, zd, trim);
    }
    if (n > 0) {
        wave_sync();
        flush_runs(B, s, G, runs, n, ev);
    }
}

using BlockSort = hipcub::BlockRadixSort<uint32_t, kQueryBlock, kQueriesPerThread, int32_t>;

__device__ inline uint32_t compact3(uint32_t v)
{
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030c30c3u;
    v = (v | (v >> 4)) & 0x0300f00fu;
    v = (v | (v >> 8)) & 0x030000ffu;
    v = (v | (v >> 16)) & 0x000003ffu;
    return v;
}

constexpr int kWaves = kQueryBlock / 64;
constexpr int kWaveSpan = kQueryTile / kWaves;   // sorted positions grouped and scanned by one wave

// kTuning only names the instance: the autotuner launches k_nn<true>, so
// kernel traces keep its trial launches apart from the search itself.
template <bool kTuning>
__global__ __launch_bounds__(kQueryBlock, 4) void k_nn(Band B, Global G, NnParams P, const float* __restrict__ qx,
                                                    const float* __restrict__ qy, const float* __restrict__ qz,
                                                    int32_t* __restrict__ nn, float4* __restrict__ nn_pt)
{
    __shared__ typename BlockSort::TempStorage sort_tmp;
    __shared__ int16_t s_order[kQueryTile];
    __shared__ uint32_t s_cell[kQueryTile];          // sorted position -> packed cell (10 bits per axis)
    __shared__ int32_t s_red[kWaves * 6];
    __shared__ float4 s_buf[kQueryBlock];
    __shared__ int4 s_runs[kWaves][kRunArea];
    __shared__ int16_t s_group[kWaves][kWaveSpan + 1];
    __shared__ int32_t s_ngroups[kWaves];
    __shared__ float4 s_tq[kWaves][kTail];

    // P.parts blocks share a tile: each sorts all of it and scans its own
    // contiguous share of the sorted positions (more blocks for small batches)
    const int64_t item = xcd_work_item(blockIdx.x, gridDim.x);
    const int64_t tile = item / P.parts;
    const int32_t part = (int32_t)(item % P.parts);
    const int32_t shape = B.tile_shape[tile];
    const ShapeDesc& s = B.shapes[shape];
    const int64_t q0 = B.tile_start[tile];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    float4* wbuf = s_buf + wave * 64;
    int4* runs = s_runs[wave];
    const int32_t nq = (int32_t)min((int64_t)kQueryTile, s.query_off + s.query_cnt - q0);

    // ---- sort the tile's queries by the Morton code of their cell ----------
    uint32_t key[kQueriesPerThread];
    int32_t val[kQueriesPerThread];
    int32_t cells[kQueriesPerThread][3];
    int32_t box[6] = {0x7fffffff, 0x7fffffff, 0x7fffffff, -1, -1, -1};
#pragma unroll
    for (int j = 0; j < kQueriesPerThread; ++j) {
        const int32_t li = threadIdx.x * kQueriesPerThread + j;
        val[j] = li;
        float du[3];
        cells[j][0] = cells[j][1] = cells[j][2] = 0;
        if (li < nq) {
            query_cell(s, qx[q0 + li], qy[q0 + li], qz[q0 + li], cells[j], du);
            for (int a = 0; a < 3; ++a) {
                box[a] = min(box[a], cells[j][a]);
                box[3 + a] = max(box[3 + a], cells[j][a]);
            }
        }
    }
    block_minmax6(box, s_red);
#pragma unroll
    for (int j = 0; j < kQueriesPerThread; ++j) {
        const int32_t li = threadIdx.x * kQueriesPerThread + j;
        key[j] = 0xffffffffu;
        if (li < nq)
            key[j] = spread3((uint32_t)min(cells[j][0] - box[0], 1023)) |
                     (spread3((uint32_t)min(cells[j][1] - box[1], 1023)) << 1) |
                     (spread3((uint32_t)min(cells[j][2] - box[2], 1023)) << 2);
    }
    // only the bits the tile's cell box needs (3 per axis per doubling of its span)
    int32_t span = 1;
    for (int a = 0; a < 3; ++a) span = max(span, box[3 + a] - box[a] + 1);
    const int32_t bits = min(3 * (32 - __builtin_clz((uint32_t)span - 1u | 1u)), 30);
    if (P.sort) BlockSort(sort_tmp).Sort(key, val, 0, bits);   // (uniform: every thread or none)
#pragma unroll
    for (int j = 0; j < kQueriesPerThread; ++j) {
        const int32_t pos = threadIdx.x * kQueriesPerThread + j;
        s_order[pos] = (int16_t)val[j];
        s_cell[pos] = compact3(key[j]) | (compact3(key[j] >> 1) << 10) | (compact3(key[j] >> 2) << 20);
    }
    __syncthreads();

    // ---- greedy groups along this wave's part of the sorted order: at most
    // 64 queries whose cells span fewer than P.span cells per axis.  From
    // each group's first position the next 64 cells are loaded one per lane;
    // prefix minima and maxima over the lanes give the span of every prefix,
    // and the group ends before the first lane whose prefix does not fit.
    const int32_t wspan = kWaveSpan / P.parts;
    const int32_t wb0 = __builtin_amdgcn_readfirstlane(min((part * kWaves + wave) * wspan, nq));
    const int32_t we0 = __builtin_amdgcn_readfirstlane(min(wb0 + wspan, nq));
    {
        int32_t ng = 0;
        for (int32_t g = wb0; g < we0; ++ng) {
            const int32_t pos = g + lane;
            const bool in = pos < we0;
            const uint32_t pc = in ? s_cell[pos] : 0u;
            int32_t lo[3] = {(int32_t)(pc & 1023u), (int32_t)((pc >> 10) & 1023u), (int32_t)(pc >> 20)};
            int32_t hi[3] = {lo[0], lo[1], lo[2]};
            for (int o = 1; o < 64; o <<= 1) {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int32_t l = __shfl_up(lo[a], o, 64), h = __shfl_up(hi[a], o, 64);
                    if (lane >= o) {
                        lo[a] = min(lo[a], l);
                        hi[a] = max(hi[a], h);
                    }
                }
            }
            const bool fits = in && hi[0] - lo[0] < P.span && hi[1] - lo[1] < P.span && hi[2] - lo[2] < P.span;
            const uint64_t bad = __ballot(!fits);
            const int32_t len = bad ? max((int32_t)__builtin_ctzll(bad), 1) : 64;
            if (lane == 0) s_group[wave][ng] = (int16_t)g;
            g += len;
        }
        if (lane == 0) {
            s_group[wave][ng] = (int16_t)we0;
            s_ngroups[wave] = ng;
        }
    }
    wave_sync();
    const int32_t ngroups = s_ngroups[wave];

    const float inv_h[3] = {1.f / s.h[0], 1.f / s.h[1], 1.f / s.h[2]};
    float4* tq = s_tq[wave];
    for (int32_t gi = 0; gi < ngroups; ++gi) {
        const int32_t pos = s_group[wave][gi] + lane;
        const bool live = pos < s_group[wave][gi + 1];
        const int32_t li = live ? s_order[pos] : 0;
        const int64_t k = q0 + li;
        Scan q;
        q.x = live ? qx[k] : 0.f;
        q.y = live ? qy[k] : 0.f;
        q.z = live ? qz[k] : 0.f;
        query_cell(s, q.x, q.y, q.z, q.c0, q.du);
        q.best1 = q.best2 = __builtin_inff();
        q.id1 = -1;
        q.open = live && s.point_cnt > 0;
        int32_t wb[6] = {0x7fffffff, 0x7fffffff, 0x7fffffff, -1, -1, -1};
        if (live)
            for (int a = 0; a < 3; ++a) {
                wb[a] = q.c0[a];
                wb[3 + a] = q.c0[a];
            }
        wave_minmax6(wb);
        if (__any(q.open)) {
            // ---- lockstep pass over the group's box grown by P.shell cells,
            // grown further one cell at a time while it holds no point
            int32_t lo[3], hi[3];
            {
                int32_t olo[3] = {0, 0, 0}, ohi[3] = {-1, -1, -1};
                for (int e = P.shell;; ++e) {
                    for (int a = 0; a < 3; ++a) {
                        lo[a] = max(wb[a] - e, 0);
                        hi[a] = min(wb[3 + a] + e, s.R[a] - 1);
                    }
                    Lockstep ev{&q, wbuf};
                    scan_box(B, s, G, runs, ev, lo, hi, olo, ohi, P.skip_empty != 0);
                    if (__any(q.id1 >= 0) || e >= kNnMaxGrow) break;
                    for (int a = 0; a < 3; ++a) {
                        olo[a] = lo[a];
                        ohi[a] = hi[a];
                    }
                }
            }
            // resolved: a unique float minimum that no point outside the box can match
            if (q.open && q.id1 >= 0 && q.best2 > q.best1 * (1.f + 1e-6f)) {
                float gap = __builtin_inff();
                for (int a = 0; a < 3; ++a) {
                    if (lo[a] > 0) gap = fminf(gap, fmaxf((float)(q.c0[a] - lo[a]) + q.du[a] - 1e-3f, 0.f) * s.h[a]);
                    if (hi[a] < s.R[a] - 1)
                        gap = fminf(gap, fmaxf((float)(hi[a] + 1 - q.c0[a]) - q.du[a] - 1e-3f, 0.f) * s.h[a]);
                }
                if (q.best1 * (1.f + 1e-6f) < gap * gap * (1.f - 1e-5f)) q.open = false;
            }

            // ---- point-parallel pass for the open lanes that have a candidate:
            // the cells meeting the bounding box of the ball of the candidate
            // distance, outside the box already scanned, kTail lanes at a time.
            // Afterwards every point that can beat the candidate has been seen.
            int32_t ball[6] = {0x7fffffff, 0x7fffffff, 0x7fffffff, -1, -1, -1};
            bool tail = q.open && q.id1 >= 0;
            if (tail) {
                const float r = sqrtf(q.best1);
    #pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const float ra = r * inv_h[a] * (1.f + 1e-5f) + 1e-3f;
                    ball[a] = max(q.c0[a] + (int32_t)floorf(q.du[a] - ra), 0);
                    ball[3 + a] = min(q.c0[a] + (int32_t)floorf(q.du[a] + ra), s.R[a] - 1);
                    tail = tail && ball[3 + a] - ball[a] < kTailSpan;
                }
            }
            uint64_t pend = __ballot(tail);
            while (pend != 0) {
                uint64_t batch = 0;
                for (int t = 0; t < kTail && pend != 0; ++t) {
                    batch |= pend & (~pend + 1);
                    pend &= pend - 1;
                }
                const bool inb = (batch >> lane) & 1;
                if (inb) tq[lane_rank(batch)] = make_float4(q.x, q.y, q.z, q.best1 * (1.f + 4e-5f) + 1e-30f);
                int32_t reg[6];
                for (int a = 0; a < 6; ++a) reg[a] = inb ? ball[a] : (a < 3 ? 0x7fffffff : -1);
                wave_minmax6(reg);
                wave_sync();
                Tail ev;
                ev.tq = tq;
                ev.ns = __popcll(batch);
    #pragma unroll
                for (int t = 0; t < kTail; ++t) {
                    ev.b1[t] = ev.b2[t] = __builtin_inff();
                    ev.id[t] = -1;
                }
                scan_box(B, s, G, runs, ev, reg, reg + 3, lo, hi, P.skip_empty != 0, tq, ev.ns);
                // reduce every slot over the wave and merge it into its lane
                uint64_t own = batch;
#pragma unroll
                for (int t = 0; t < kTail; ++t) {
                    if (t < ev.ns) {
                        float b1 = ev.b1[t], b2 = ev.b2[t];
                        int32_t id = ev.id[t];
                        wave_best2(b1, b2, id);
                        const int32_t owner = __builtin_ctzll(own);
                        own &= own - 1;
                        if (lane == owner) {
                            q.best2 = fminf(fminf(q.best2, b2), fmaxf(q.best1, b1));
                            q.id1 = b1 < q.best1 ? id : q.id1;
                            q.best1 = fminf(q.best1, b1);
                        }
                    }
                }
                wave_sync();
            }
            if (tail && q.best2 > q.best1 * (1.f + 1e-6f)) q.open = false;
        }
        if (!live) continue;
        // the winner's position in the sorted copy; its original index is
        // stored there too (a load from the same small region as the scan)
        const int32_t at = (s.point_cnt > 0 && !q.open) ? q.id1 : search(B, s, G, q.x, q.y, q.z);
        const float4 w = at >= 0 ? G.pts[at] : make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
        nn[k] = __float_as_int(w.w);
        nn_pt[k] = w;
    }
}

}  // namespace
}  // namespace gp

using namespace gp;

gp_status gp_nn_impl(gp_ctx ctx, const float* qx, const float* qy, const float* qz, int32_t* nn)
{
    if (ctx->n_tiles == 0) return GP_OK;
    Global G{ctx->cell_start.p, ctx->nn_spts.p};
    GP_TIMED(ctx, "k_nn");
    k_nn<false><<<(unsigned)(ctx->n_tiles * ctx->nn_params.parts), kQueryBlock, 0, ctx->stream>>>(
        ctx->nn_band(), G, ctx->nn_params, qx, qy, qz, nn, ctx->nn_pt.p);
    GP_HIP(ctx, hipGetLastError());
    return GP_OK;
}

// Times k_nn on the caller's queries (the results are the same for every
// setting): first on the search grids of 4, 16, ... times the current target
// density while each is faster than the last (a factor of 4 moves each
// shape's grid by one level), else of 1/4, 1/16, ... of it; then, on the
// fastest grid, every (span, shell) pair of a small grid, then the number of
// blocks per tile for the best pair (and, if that changed, every pair again
// at the new number), then the other skip_empty setting, then the other sort
// setting, and keeps the fastest in the context.
// Each candidate runs once, then `reps` times, between events; its time is
// the smallest of the repeats (a candidate whose first run takes 4 times the
// best time so far is not repeated).  The context's current setting is timed
// first and is only replaced by one at least 2% faster, so timing noise does
// not move a setting that is already as good.
gp_status gp_autotune_nn_impl(gp_ctx ctx, const float* qx, const float* qy, const float* qz, int32_t* nn,
                              int32_t reps, NnParams* best_out, float* best_ms_out)
{
    static const int32_t spans[] = {4, 6, 8, 12, 16, 24, 32};
    static const int32_t shells[] = {0, 1, 2};
    static const int32_t parts[] = {1, 2, 4};
    const NnParams current = ctx->nn_params;
    NnParams best = current;
    float best_ms = -1.f;
    if (ctx->n_tiles > 0) {
        if (ctx->nn_cell_points != current.cell_points) {
            const gp_status rs = gp_build_nn_index(ctx, current.cell_points);
            if (rs != GP_OK) return rs;
        }
        hipEvent_t ev[2];
        GP_HIP(ctx, hipEventCreate(&ev[0]));
        if (hipEventCreate(&ev[1]) != hipSuccess) {
            (void)hipEventDestroy(ev[0]);
            ctx->err = "hipEventCreate failed";
            return GP_ERR_DEVICE;
        }
        hipError_t e = hipSuccess;
        gp_status rebuilt = GP_OK;
        auto time_one = [&](const NnParams& P) -> float {
            const Global G{ctx->cell_start.p, ctx->nn_spts.p};
            float t_min = -1.f;
            for (int32_t r = 0; r <= reps && e == hipSuccess; ++r) {
                e = hipEventRecord(ev[0], ctx->stream);
                k_nn<true><<<(unsigned)(ctx->n_tiles * P.parts), kQueryBlock, 0, ctx->stream>>>(ctx->nn_band(), G, P,
                                                                                            qx, qy, qz, nn, ctx->nn_pt.p);
                if (e == hipSuccess) e = hipGetLastError();
                if (e == hipSuccess) e = hipEventRecord(ev[1], ctx->stream);
                if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
                if (e != hipSuccess) break;
                if (r == 0) {
                    if (best_ms > 0.f && ms > 4.f * best_ms) return ms;   // far off: not worth the repeats
                    continue;
                }
                if (t_min < 0.f || ms < t_min) t_min = ms;
            }
            return t_min;
        };
        auto same = [](const NnParams& a, const NnParams& b) {
            return a.span == b.span && a.shell == b.shell && a.parts == b.parts && a.skip_empty == b.skip_empty &&
                   a.sort == b.sort && a.cell_points == b.cell_points;
        };
        // a challenger must beat the current setting by 2%, anything else plainly
        auto offer = [&](const NnParams& P) {
            const float t = time_one(P);
            if (e != hipSuccess || t < 0.f) return;
            if (best_ms < 0.f || t < best_ms * (same(best, current) ? 0.98f : 1.f)) {
                best_ms = t;
                best = P;
            }
        };
        offer(current);
        // the search grids of other targets, one level at a time; a target
        // that gives grids already timed ends its direction (all levels at
        // their limit)
        std::vector<std::vector<int32_t>> tried{gp_nn_levels(ctx, current.cell_points)};
        auto try_grid = [&](int32_t cp) -> bool {   // true if it is the fastest so far
            if (e != hipSuccess || rebuilt != GP_OK) return false;
            const std::vector<int32_t> lv = gp_nn_levels(ctx, cp);
            if (std::find(tried.begin(), tried.end(), lv) != tried.end()) return false;
            tried.push_back(lv);
            rebuilt = gp_build_nn_index(ctx, cp);
            if (rebuilt != GP_OK) return false;
            NnParams P = current;
            P.cell_points = cp;
            offer(P);
            return same(best, P);
        };
        for (int64_t cp = (int64_t)current.cell_points * 4; cp <= kNnCellPointsMax && try_grid((int32_t)cp); cp *= 4) {
        }
        if (best.cell_points == current.cell_points)
            for (int32_t cp = current.cell_points / 4; cp >= 1 && try_grid(cp); cp /= 4) {
            }
        if (rebuilt == GP_OK && e == hipSuccess && ctx->nn_cell_points != best.cell_points)
            rebuilt = gp_build_nn_index(ctx, best.cell_points);
        if (rebuilt != GP_OK) {
            (void)hipEventDestroy(ev[0]);
            (void)hipEventDestroy(ev[1]);
            return rebuilt;
        }
        const NnParams gridded = best;
        for (int32_t sp : spans)
            for (int32_t sh : shells) {
                NnParams P = gridded;
                P.span = sp;
                P.shell = sh;
                if (sp != gridded.span || sh != gridded.shell) offer(P);
            }
        const NnParams shaped = best;
        for (int32_t pa : parts) {
            NnParams P = shaped;
            P.parts = pa;
            if (pa != shaped.parts) offer(P);
        }
        if (best.parts != shaped.parts) {   // the pairs again, at the new number of blocks per tile
            const NnParams parted = best;
            for (int32_t sp : spans)
                for (int32_t sh : shells) {
                    NnParams P = parted;
                    P.span = sp;
                    P.shell = sh;
                    if (sp != parted.span || sh != parted.shell) offer(P);
                }
        }
        {
            NnParams P = best;
            P.skip_empty = !best.skip_empty;
            offer(P);
        }
        {
            NnParams P = best;
            P.sort = !best.sort;
            offer(P);
        }
        (void)hipEventDestroy(ev[0]);
        (void)hipEventDestroy(ev[1]);
        GP_HIP(ctx, e);
        // leave nn holding the chosen configuration's (identical) result
        const Global G{ctx->cell_start.p, ctx->nn_spts.p};
        k_nn<true><<<(unsigned)(ctx->n_tiles * best.parts), kQueryBlock, 0, ctx->stream>>>(ctx->nn_band(), G, best, qx,
                                                                                       qy, qz, nn, ctx->nn_pt.p);
        GP_HIP(ctx, hipGetLastError());
    }
    ctx->nn_params = best;
    if (best_out) *best_out = best;
    if (best_ms_out) *best_ms_out = best_ms;
    return GP_OK;
}
