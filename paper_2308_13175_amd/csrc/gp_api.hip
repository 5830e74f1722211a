// The C ABI: argument validation, status codes, stream handling.  The
// numerical work lives in band.hip, nn.hip, sample.hip, pull.hip, step.hip,
// normals.hip and surface.hip.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include "gp_internal.h"

hipEvent_t gp_timer_begin(gp_ctx ctx)
{
    if (!ctx || !ctx->timing) return nullptr;
    hipEvent_t e = nullptr;
    if (!ctx->event_pool.empty()) {
        e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        return nullptr;
    }
    if (hipEventRecord(e, ctx->stream) != hipSuccess) {
        ctx->event_pool.push_back(e);
        return nullptr;
    }
    return e;
}

void gp_timer_end(gp_ctx ctx, const char* name, hipEvent_t begin)
{
    if (!ctx || !begin) return;
    hipEvent_t e = nullptr;
    if (!ctx->event_pool.empty()) {
        e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
    } else if (hipEventCreate(&e) != hipSuccess) {
        ctx->event_pool.push_back(begin);
        return;
    }
    (void)hipEventRecord(e, ctx->stream);
    ctx->timed.push_back({name, begin, e});
}

gp_status gp_fail(gp_ctx ctx, gp_status st, const std::string& msg)
{
    if (ctx) ctx->err = msg;
    return st;
}

gp_status gp_hip_fail(gp_ctx ctx, hipError_t e, const char* what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    if (e == hipErrorOutOfMemory) return gp_fail(ctx, GP_ERR_OOM, m);
    return gp_fail(ctx, GP_ERR_DEVICE, m);
}

namespace {

gp_status ready(gp_ctx ctx)
{
    if (!ctx) return GP_ERR_ARG;
    ctx->err.clear();
    if (!ctx->built) return gp_fail(ctx, GP_ERR_STATE, "gp_build_band has not completed on this context");
    if (hipSetDevice(ctx->device) != hipSuccess) return gp_fail(ctx, GP_ERR_DEVICE, "hipSetDevice failed");
    return GP_OK;
}

gp_status check_queries(gp_ctx ctx, const void* a, const void* b, const void* c, int64_t n)
{
    if (n != ctx->n_queries)
        return gp_fail(ctx, GP_ERR_ARG, "n_queries (" + std::to_string(n) + ") must equal the end of the last query "
                                        "slice (" + std::to_string(ctx->n_queries) + ")");
    if (n > 0 && (!a || !b || !c)) return gp_fail(ctx, GP_ERR_ARG, "null query array");
    return GP_OK;
}

// The forward that just ran on these arrays becomes the one a backward may follow.
void record_forward(gp_ctx ctx, const void* qx, const void* qy, const void* qz, const void* nn, const void* field)
{
    ctx->fwd_token = ++ctx->token_counter;
    const void* a[5] = {qx, qy, qz, nn, field};
    for (int i = 0; i < 5; ++i) ctx->fwd_arrays[i] = a[i];
}

// A call of the library is about to write array p: a forward that read it is
// no longer the state a backward may use.
void invalidate_forward(gp_ctx ctx, const void* p)
{
    if (!p) return;
    for (int i = 0; i < 5; ++i)
        if (ctx->fwd_arrays[i] == p) ctx->fwd_token = 0;
}

}  // namespace

extern "C" {

gp_status gp_create(gp_ctx* out, int device, void* hip_stream)
{
    if (!out) return GP_ERR_ARG;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return GP_ERR_ARG;
    if (hipSetDevice(device) != hipSuccess) return GP_ERR_DEVICE;
    gp_ctx c = new (std::nothrow) gp_ctx_s();
    if (!c) return GP_ERR_OOM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    *out = c;
    return GP_OK;
}

void gp_destroy(gp_ctx ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (auto& r : ctx->timed) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
    delete ctx;
}

const char* gp_last_error(gp_ctx ctx)
{
    return ctx ? ctx->err.c_str() : "null context";
}

gp_status gp_set_stream(gp_ctx ctx, void* hip_stream)
{
    if (!ctx) return GP_ERR_ARG;
    ctx->stream = (hipStream_t)hip_stream;
    return GP_OK;
}

gp_status gp_sync(gp_ctx ctx)
{
    if (!ctx) return GP_ERR_ARG;
    ctx->err.clear();
    (void)hipSetDevice(ctx->device);
    GP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (!ctx->built) return GP_OK;
    int32_t f = 0;
    GP_HIP(ctx, hipMemcpy(&f, ctx->flag.p, 4, hipMemcpyDeviceToHost));
    if (f) {
        int32_t z = 0;
        GP_HIP(ctx, hipMemcpy(ctx->flag.p, &z, 4, hipMemcpyHostToDevice));
        if (f & 2) return gp_fail(ctx, GP_ERR_ARG, "a nearest-point index was outside its shape's points");
        return gp_fail(ctx, GP_ERR_NUMERIC, "a loss was not finite");
    }
    return GP_OK;
}

gp_status gp_build_band(gp_ctx ctx, const gp_shape* shapes, int32_t n_shapes, const float* px, const float* py,
                        const float* pz, int32_t m1, int32_t m2, int32_t brick, int64_t* n_slots_out,
                        int64_t* n_active_vertices_out)
{
    if (!ctx) return GP_ERR_ARG;
    ctx->err.clear();
    if (!shapes || n_shapes < 1) return gp_fail(ctx, GP_ERR_ARG, "need at least one shape");
    if (m1 < 0 || m2 < 0 || m1 > 1024 || m2 > 1024)
        return gp_fail(ctx, GP_ERR_ARG, "m1 and m2 must lie in [0, 1024]");
    if (brick != 4 && brick != 8 && brick != 16) return gp_fail(ctx, GP_ERR_ARG, "brick must be 4, 8 or 16");
    bool any_points = false;
    for (int32_t s = 0; s < n_shapes; ++s) {
        const gp_shape& d = shapes[s];
        for (int a = 0; a < 3; ++a) {
            if (d.dims[a] < 1 || d.dims[a] > (1 << 20))
                return gp_fail(ctx, GP_ERR_ARG, "shape " + std::to_string(s) + ": dims must lie in [1, 2^20]");
            if (!(d.hi[a] > d.lo[a]) || !std::isfinite(d.lo[a]) || !std::isfinite(d.hi[a]))
                return gp_fail(ctx, GP_ERR_ARG, "shape " + std::to_string(s) + ": need finite lo < hi");
        }
        if (d.point_off < 0 || d.point_cnt < 0 || d.query_off < 0 || d.query_cnt < 0)
            return gp_fail(ctx, GP_ERR_ARG, "shape " + std::to_string(s) + ": negative slice");
        any_points = any_points || d.point_cnt > 0;
        // slices of different shapes must not overlap
        for (int32_t t = 0; t < s; ++t) {
            const gp_shape& e = shapes[t];
            if (d.point_cnt > 0 && e.point_cnt > 0 && d.point_off < e.point_off + e.point_cnt &&
                e.point_off < d.point_off + d.point_cnt)
                return gp_fail(ctx, GP_ERR_ARG, "point slices of shapes overlap");
            if (d.query_cnt > 0 && e.query_cnt > 0 && d.query_off < e.query_off + e.query_cnt &&
                e.query_off < d.query_off + d.query_cnt)
                return gp_fail(ctx, GP_ERR_ARG, "query slices of shapes overlap");
        }
    }
    if (any_points && (!px || !py || !pz)) return gp_fail(ctx, GP_ERR_ARG, "null point array");
    if (hipSetDevice(ctx->device) != hipSuccess) return gp_fail(ctx, GP_ERR_DEVICE, "hipSetDevice failed");
    ctx->fwd_token = 0;
    gp_status st = gp_build_band_impl(ctx, shapes, n_shapes, px, py, pz, m1, m2, brick);
    if (st != GP_OK) {
        (void)hipStreamSynchronize(ctx->stream);
        return st;
    }
    if (n_slots_out) *n_slots_out = ctx->n_slots;
    if (n_active_vertices_out) *n_active_vertices_out = ctx->n_active;
    return GP_OK;
}

gp_status gp_nn_query(gp_ctx ctx, const float* qx, const float* qy, const float* qz, int64_t n_queries,
                      int32_t* nn_out)
{
    gp_status st = ready(ctx);
    if (st != GP_OK) return st;
    if ((st = check_queries(ctx, qx, qy, qz, n_queries)) != GP_OK) return st;
    if (n_queries > 0 && !nn_out) return gp_fail(ctx, GP_ERR_ARG, "null nn_out");
    invalidate_forward(ctx, nn_out);
    return gp_nn_impl(ctx, qx, qy, qz, nn_out);
}

gp_status gp_set_nn_params(gp_ctx ctx, const gp_nn_params* params)
{
    if (!ctx) return GP_ERR_ARG;
    if (!params) return gp_fail(ctx, GP_ERR_ARG, "null params");
    if (params->group_span < 1 || params->group_span > gp::kNnSpanMax)
        return gp_fail(ctx, GP_ERR_ARG, "group_span must be in [1, 64]");
    if (params->first_shell < 0 || params->first_shell > gp::kNnShellMax)
        return gp_fail(ctx, GP_ERR_ARG, "first_shell must be in [0, 4]");
    if (params->tile_parts != 1 && params->tile_parts != 2 && params->tile_parts != 4)
        return gp_fail(ctx, GP_ERR_ARG, "tile_parts must be 1, 2 or 4");
    if (params->skip_empty != 0 && params->skip_empty != 1) return gp_fail(ctx, GP_ERR_ARG, "skip_empty must be 0 or 1");
    if (params->morton_sort != 0 && params->morton_sort != 1)
        return gp_fail(ctx, GP_ERR_ARG, "morton_sort must be 0 or 1");
    if (params->cell_points < 1 || params->cell_points > gp::kNnCellPointsMax)
        return gp_fail(ctx, GP_ERR_ARG, "cell_points must be in [1, 65536]");
    if (ctx->built && params->cell_points != ctx->nn_cell_points) {
        if (hipSetDevice(ctx->device) != hipSuccess) return gp_fail(ctx, GP_ERR_DEVICE, "hipSetDevice failed");
        const gp_status st = gp_build_nn_index(ctx, params->cell_points);
        if (st != GP_OK) return st;
    }
    ctx->nn_params.cell_points = params->cell_points;
    ctx->nn_params.span = params->group_span;
    ctx->nn_params.shell = params->first_shell;
    ctx->nn_params.parts = params->tile_parts;
    ctx->nn_params.skip_empty = params->skip_empty;
    ctx->nn_params.sort = params->morton_sort;
    return GP_OK;
}

static void nn_params_out(const gp::NnParams& p, gp_nn_params* out)
{
    out->group_span = p.span;
    out->first_shell = p.shell;
    out->tile_parts = p.parts;
    out->skip_empty = p.skip_empty;
    out->morton_sort = p.sort;
    out->cell_points = p.cell_points;
}

gp_status gp_get_nn_params(gp_ctx ctx, gp_nn_params* params)
{
    if (!ctx) return GP_ERR_ARG;
    if (!params) return gp_fail(ctx, GP_ERR_ARG, "null output");
    nn_params_out(ctx->nn_params, params);
    return GP_OK;
}

gp_status gp_get_nn_grid(gp_ctx ctx, int32_t shape, int32_t* dims_out, int32_t* level_out)
{
    gp_status st = ready(ctx);
    if (st != GP_OK) return st;
    if (shape < 0 || shape >= ctx->n_shapes) return gp_fail(ctx, GP_ERR_ARG, "shape out of range");
    if (!dims_out) return gp_fail(ctx, GP_ERR_ARG, "null dims_out");
    for (int a = 0; a < 3; ++a) dims_out[a] = ctx->h_nn_shapes[shape].R[a];
    if (level_out) *level_out = ctx->h_nn_levels[shape];
    return GP_OK;
}

gp_status gp_set_tv_layout(gp_ctx ctx, int32_t layout)
{
    if (!ctx) return GP_ERR_ARG;
    if (layout < 0 || layout > 2) return gp_fail(ctx, GP_ERR_ARG, "layout must be 0, 1 or 2");
    const gp::GradParams d;
    gp::GradParams& g = ctx->grad_params;
    g.tv_fwd_wave_from = layout == 0 ? d.tv_fwd_wave_from : (layout == 1 ? INT64_MAX : 0);
    g.tv_bwd_wave_from = layout == 0 ? d.tv_bwd_wave_from : (layout == 1 ? INT64_MAX : 0);
    return GP_OK;
}

gp_status gp_set_grad_params(gp_ctx ctx, const gp_grad_params* params)
{
    if (!ctx) return GP_ERR_ARG;
    if (!params) return gp_fail(ctx, GP_ERR_ARG, "null params");
    bool cap_ok = false;
    for (int32_t c : gp::kWinCaps) cap_ok = cap_ok || params->window_cap == c;
    if (!cap_ok) return gp_fail(ctx, GP_ERR_ARG, "window_cap must be 2048, 4096 or 6144");
    if (params->window_max_passes < 1 || params->window_max_passes > gp::kWinPassesMax)
        return gp_fail(ctx, GP_ERR_ARG, "window_max_passes must be in [1, 64]");
    if (params->tv_forward_wave_from < 0 || params->tv_backward_wave_from < 0)
        return gp_fail(ctx, GP_ERR_ARG, "the TV thresholds must be >= 0");
    gp::GradParams& g = ctx->grad_params;
    g.win_cap = params->window_cap;
    g.win_max_passes = params->window_max_passes;
    g.tv_fwd_wave_from = params->tv_forward_wave_from;
    g.tv_bwd_wave_from = params->tv_backward_wave_from;
    return GP_OK;
}

static void grad_params_out(const gp::GradParams& g, gp_grad_params* out)
{
    out->window_cap = g.win_cap;
    out->window_max_passes = g.win_max_passes;
    out->tv_forward_wave_from = g.tv_fwd_wave_from;
    out->tv_backward_wave_from = g.tv_bwd_wave_from;
}

gp_status gp_get_grad_params(gp_ctx ctx, gp_grad_params* params)
{
    if (!ctx) return GP_ERR_ARG;
    if (!params) return gp_fail(ctx, GP_ERR_ARG, "null output");
    grad_params_out(ctx->grad_params, params);
    return GP_OK;
}

gp_status gp_autotune_grad(gp_ctx ctx, const float* qx, const float* qy, const float* qz, const int32_t* nn,
                           int64_t n_queries, const float* field, gp_weights w, int32_t reps,
                           gp_grad_params* chosen_out, float* best_ms_out)
{
    gp_status st = ready(ctx);
    if (st != GP_OK) return st;
    if ((st = check_queries(ctx, qx, qy, qz, n_queries)) != GP_OK) return st;
    if ((n_queries > 0 && !nn) || !field) return gp_fail(ctx, GP_ERR_ARG, "null nn or field");
    if (reps < 1 || reps > 100) return gp_fail(ctx, GP_ERR_ARG, "reps must be in [1, 100]");
    ctx->fwd_token = 0;
    gp::GradParams best;
    st = gp_autotune_grad_impl(ctx, qx, qy, qz, nn, field, w, reps, &best, best_ms_out);
    if (st != GP_OK) return st;
    if (chosen_out) grad_params_out(best, chosen_out);
    return GP_OK;
}

gp_status gp_autotune_nn(gp_ctx ctx, const float* qx, const float* qy, const float* qz, int64_t n_queries,
                         int32_t* nn_out, int32_t reps, gp_nn_params* chosen_out, float* best_ms_out)
{
    gp_status st = ready(ctx);
    if (st != GP_OK) return st;
    if ((st = check_queries(ctx, qx, qy, qz, n_queries)) != GP_OK) return st;
    if (n_queries > 0 && !nn_out) return gp_fail(ctx, GP_ERR_ARG, "null nn_out");
    if (reps < 1 || reps > 100) return gp_fail(ctx, GP_ERR_ARG, "reps must be in [1, 100]");
    invalidate_forward(ctx, nn_out);
    gp::NnParams best;
    float ms = -1.f;
    if ((st = gp_autotune_nn_impl(ctx, qx, qy, qz, nn_out, reps, &best, &ms)) != GP_OK) return st;
    if (chosen_out) nn_params_out(best, chosen_out);
    if (best_ms_out) *best_ms_out = ms;
    return GP_OK;
}

gp_status gp_sample_queries(gp_ctx ctx, uint64_t seed, int32_t iteration, const float* sigma, float sigma_const,
                            float* qx, float* qy, float* qz, int32_t* src_out)
{
    gp_status st = ready(ctx);
    if (st != GP_OK) return st;
    if (ctx->n_queries > 0 && (!qx || !qy || !qz)) return gp_fail(ctx, GP_ERR_ARG, "null query array");
    if (!sigma && !(sigma_const >= 0.f)) return gp_fail(ctx, GP_ERR_ARG, "sigma_const must be >= 0");
    invalidate_forward(ctx, qx);
    invalidate_forward(ctx, qy);
    invalidate_forward(ctx, qz);
    return gp_sample_impl(ctx, seed, iteration, sigma, sigma_const, qx, qy, qz, src_out);
}

gp_status gp_pull_forward(gp_ctx ctx, const float* qx, const float* qy, const float* qz, const int32_t* nn,
                          int64_t n_queries, const float* field, gp_weights w, double* loss_out,
                          int64_t* n_valid_out)
{
    gp_status st = ready(ctx);
    if (st != GP_OK) return st;
    if ((st = check_queries(ctx, qx, qy, qz, n_queries)) != GP_OK) return st;
    if ((n_queries > 0 && !nn) || !field || !loss_out || !n_valid_out)
        return gp_fail(ctx, GP_ERR_ARG, "null argument");
    if ((st = gp_forward_impl(ctx, qx, qy, qz, nn, field, w, loss_out, n_valid_out)) != GP_OK) return st;
    record_forward(ctx, qx, qy, qz, nn, field);
    return GP_OK;
}

gp_status gp_pull_forward_static(gp_ctx ctx, const float* qx, const float* qy, const float* qz, const int32_t* nn,
                                 int64_t n_queries, const float* field, gp_weights w, double* loss_out,
                                 int64_t* n_valid_out)
{
    gp_status st = ready(ctx);
    if (st != GP_OK) return st;
    if ((st = check_queries(ctx, qx, qy, qz, n_queries)) != GP_OK) return st;
    if ((n_queries > 0 && !nn) || !field || !loss_out || !n_valid_out)
        return gp_fail(ctx, GP_ERR_ARG, "null argument");
    return gp_forward_static_impl(ctx, qx, qy, qz, nn, field, w, loss_out, n_valid_out);
}

uint64_t gp_forward_token(gp_ctx ctx)
{
    return ctx ? ctx->fwd_token : 0;
}

gp_status gp_pull_backward(gp_ctx ctx, const float* qx, const float* qy, const float* qz, const int32_t* nn,
                           int64_t n_queries, const float* field, gp_weights w, const double* dloss, float* grad,
                           uint64_t forward_token)
{
    gp_status st = ready(ctx);
    if (st != GP_OK) return st;
    if (ctx->fwd_token == 0)
        return gp_fail(ctx, GP_ERR_STATE, "gp_pull_backward needs a preceding gp_pull_forward whose queries, "
                                          "nearest points and field have not been written since");
    if (forward_token != ctx->fwd_token)
        return gp_fail(ctx, GP_ERR_STATE, "forward_token names another forward than the last one");
    {
        const void* a[5] = {qx, qy, qz, nn, field};
        for (int i = 0; i < 5; ++i)
            if (a[i] != ctx->fwd_arrays[i])
                return gp_fail(ctx, GP_ERR_STATE, "gp_pull_backward must see the arrays of its forward");
    }
    if ((st = check_queries(ctx, qx, qy, qz, n_queries)) != GP_OK) return st;
    if ((n_queries > 0 && !nn) || !field || !dloss || !grad) return gp_fail(ctx, GP_ERR_ARG, "null argument");
    return gp_backward_impl(ctx, qx, qy, qz, nn, field, w, dloss, grad);
}

gp_status gp_pull_forward_backward(gp_ctx ctx, const float* qx, const float* qy, const float* qz,
                                   const int32_t* nn, int64_t n_queries, const float* field, gp_weights w,
                                   const double* dloss, double* loss_out, int64_t* n_valid_out, float* grad)
{
    gp_status st = ready(ctx);
    if (st != GP_OK) return st;
    if ((st = check_queries(ctx, qx, qy, qz, n_queries)) != GP_OK) return st;
    if ((n_queries > 0 && !nn) || !field || !dloss || !loss_out || !n_valid_out || !grad)
        return gp_fail(ctx, GP_ERR_ARG, "null argument");
    if ((st = gp_forward_backward_impl(ctx, qx, qy, qz, nn, field, w, dloss, loss_out, n_valid_out, grad)) != GP_OK)
        return st;
    record_forward(ctx, qx, qy, qz, nn, field);
    return GP_OK;
}

gp_status gp_pull_normals(gp_ctx ctx, const float* qx, const float* qy, const float* qz, const int32_t* nn,
                          int64_t n_queries, const float* field, const float* nx, const float* ny, const float* nz,
                          float weight, const double* dloss, double* term_out, float* grad)
{
    gp_status st = ready(ctx);
    if (st != GP_OK) return st;
    if ((st = check_queries(ctx, qx, qy, qz, n_queries)) != GP_OK) return st;
    if ((n_queries > 0 && !nn) || !field || !term_out) return gp_fail(ctx, GP_ERR_ARG, "null argument");
    if (ctx->n_points > 0 && (!nx || !ny || !nz)) return gp_fail(ctx, GP_ERR_ARG, "null normal array");
    if (!std::isfinite(weight)) return gp_fail(ctx, GP_ERR_ARG, "weight must be finite");
    return gp_normals_impl(ctx, qx, qy, qz, nn, field, nx, ny, nz, weight, dloss, term_out, grad);
}

gp_status gp_step(gp_ctx ctx, float* field, float* grad, float* m, float* v, int32_t t, float lr0, float decay,
                  int32_t decay_every, float beta1, float beta2, float eps)
{
    gp_status st = ready(ctx);
    if (st != GP_OK) return st;
    if (!field || !grad || !m || !v) return gp_fail(ctx, GP_ERR_ARG, "null argument");
    if (t < 0 || decay_every < 1) return gp_fail(ctx, GP_ERR_ARG, "need t >= 0 and decay_every >= 1");
    if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps >= 0.f))
        return gp_fail(ctx, GP_ERR_ARG, "need 0 <= beta < 1 and eps >= 0");
    invalidate_forward(ctx, field);
    if ((st = gp_step_consts_impl(ctx, t, lr0, decay, decay_every, beta1, beta2)) != GP_OK) return st;
    return gp_step_impl(ctx, field, grad, m, v, beta1, beta2, eps);
}

gp_status gp_timing_enable(gp_ctx ctx, int enable)
{
    if (!ctx) return GP_ERR_ARG;
    ctx->timing = enable != 0;
    return GP_OK;
}

gp_status gp_timing_report(gp_ctx ctx, char* buf, int64_t buf_size)
{
    if (!ctx || !buf || buf_size < 1) return GP_ERR_ARG;
    ctx->err.clear();
    (void)hipSetDevice(ctx->device);
    GP_HIP(ctx, hipStreamSynchronize(ctx->stream));
    std::vector<std::pair<std::string, std::pair<int64_t, double>>> agg;
    for (auto& r : ctx->timed) {
        float ms = 0.f;
        GP_HIP(ctx, hipEventElapsedTime(&ms, r.a, r.b));
        size_t i = 0;
        while (i < agg.size() && agg[i].first != r.name) ++i;
        if (i == agg.size()) agg.push_back({r.name, {0, 0.0}});
        agg[i].second.first += 1;
        agg[i].second.second += ms;
        ctx->event_pool.push_back(r.a);
        ctx->event_pool.push_back(r.b);
    }
    ctx->timed.clear();
    std::string out;
    for (auto& a : agg) {
        char line[256];
        snprintf(line, sizeof(line), "%s %lld %.6f\n", a.first.c_str(), (long long)a.second.first, a.second.second);
        out += line;
    }
    if ((int64_t)out.size() + 1 > buf_size) {
        buf[0] = 0;
        return gp_fail(ctx, GP_ERR_CAPACITY, "timing report does not fit the buffer");
    }
    memcpy(buf, out.c_str(), out.size() + 1);
    return GP_OK;
}

gp_status gp_shape_slots(gp_ctx ctx, int64_t* slot_begin)
{
    gp_status st = ready(ctx);
    if (st != GP_OK) return st;
    if (!slot_begin) return gp_fail(ctx, GP_ERR_ARG, "null slot_begin");
    for (size_t i = 0; i < ctx->h_slot_begin.size(); ++i) slot_begin[i] = ctx->h_slot_begin[i];
    return GP_OK;
}

gp_status gp_export_layout(gp_ctx ctx, int64_t* vertex_id_of_slot, uint8_t* slot_flags)
{
    gp_status st = ready(ctx);
    if (st != GP_OK) return st;
    if (!vertex_id_of_slot && !slot_flags) return gp_fail(ctx, GP_ERR_ARG, "nothing to export");
    return gp_layout_impl(ctx, vertex_id_of_slot, slot_flags);
}

gp_status gp_export_active_cells(gp_ctx ctx, int32_t shape, int64_t* cell_ids, int64_t capacity, int64_t* n_out)
{
    gp_status st = ready(ctx);
    if (st != GP_OK) return st;
    if (!n_out || shape < 0 || shape >= ctx->n_shapes || capacity < 0 || (capacity > 0 && !cell_ids))
        return gp_fail(ctx, GP_ERR_ARG, "need a shape index in range, n_out, and cell_ids when capacity > 0");
    return gp_active_cells_impl(ctx, shape, cell_ids, capacity, n_out);
}

gp_status gp_extract_surface(gp_ctx ctx, int32_t shape, const float* field, float* tri_xyz, int64_t* tri_key,
                             int64_t capacity, int64_t* n_out, int32_t method)
{
    gp_status st = ready(ctx);
    if (st != GP_OK) return st;
    if (!n_out || !field || shape < 0 || shape >= ctx->n_shapes || capacity < 0 ||
        (capacity > 0 && (!tri_xyz || !tri_key)))
        return gp_fail(ctx, GP_ERR_ARG, "need a shape index in range, field, n_out, and outputs when capacity > 0");
    if (method != 0 && method != 1) return gp_fail(ctx, GP_ERR_ARG, "method must be 0 (marching cubes) or 1 (tetrahedra)");
    return gp_extract_surface_impl(ctx, shape, field, tri_xyz, tri_key, capacity, n_out, method);
}

gp_status gp_gather_vertices(gp_ctx ctx, const float* dense, float* field)
{
    gp_status st = ready(ctx);
    if (st != GP_OK) return st;
    if (!dense || !field) return gp_fail(ctx, GP_ERR_ARG, "null argument");
    invalidate_forward(ctx, field);
    return gp_gather_impl(ctx, dense, field, true);
}

gp_status gp_scatter_vertices(gp_ctx ctx, const float* field, float* dense)
{
    gp_status st = ready(ctx);
    if (st != GP_OK) return st;
    if (!dense || !field) return gp_fail(ctx, GP_ERR_ARG, "null argument");
    return gp_gather_impl(ctx, dense, const_cast<float*>(field), false);
}

gp_status gp_init_sphere(gp_ctx ctx, const double* centre, const double* radius, float* field)
{
    gp_status st = ready(ctx);
    if (st != GP_OK) return st;
    if (!centre || !radius || !field) return gp_fail(ctx, GP_ERR_ARG, "null argument");
    invalidate_forward(ctx, field);
    return gp_init_sphere_impl(ctx, centre, radius, field);
}

}  // extern "C"
