/*
 * gridpull_oracle.c -- plain, slow FP64 reference of the GridPull pull step.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker for the HIP library:
 * only the tests, the smoke check and the benchmark's CPU-baseline leg load
 * it.  It shares no code, header, table or helper with the HIP path.
 *
 * Everything is double precision, single threaded, in the order the paper
 * states the method (Chen, Liu, Han: "GridPull: Towards Scalability in
 * Learning Implicit Representations from 3D Point Clouds", ICCV 2023):
 *
 *   Sec. 3 "Overview" / Eq. 1       field D on the (R+1)^3 grid vertices,
 *                                   f(q) = trilinear interpolation of D
 *   Sec. 3 "Signed Distance Inference", Eq. 3
 *                                   interpolation as the 8-term polynomial
 *                                   a0 + a1 x + ... + a7 xyz through the
 *                                   8 cell corners (same function as Eq. 1)
 *   same paragraph                  pull p = q - f(q) grad f / |grad f|
 *   Eq. 4                           L_Pull = |p - NN(q)|
 *   same section, band paragraph    pulling only in cells within M1 of the
 *                                   cells holding points
 *   Eq. 5 and the M2 paragraph      TV term per vertex, six axis neighbours,
 *                                   on the M2 band
 *   Eq. 6                           L_Surface = |f(s)|
 *   Eq. 7                           L_grad = 1 - cos(grad f(q), grad f(NN(q)))
 *   Eq. 8 (second "objective")      L = L_Pull + a L_TV + b L_Surface + c L_grad
 *   Sec. 4 "Details"                Adam, lr decay x0.3 every 400 iterations
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - cells/vertices: R counts cells, vertices are R+1 per axis;
 *   - cell location: u = (q - lo) * inv_h in double, c = floor(u) clamped to
 *     R-1, valid iff 0 <= u <= R on every axis (a point on hi lands in the last
 *     cell with t = 1);
 *   - band: Chebyshev dilation of the point cells by M, clipped to the grid;
 *   - L_Surface uses s = NN(q) per query; every query-side term is a mean
 *     over the valid queries (cell inside the M1 band);
 *   - TV: tau_i = sqrt(sum over the six neighbours j that are also M2-band
 *     vertices of (D_i - D_j)^2); L_TV = mean of tau over the M2-band vertices;
 *   - |grad f| < eps_n: the normalised gradient is 0 (no derivative) and the
 *     gradient-consistency term is 1 (no derivative); e = r/|r| is 0 at r = 0;
 *     the derivative of |f_s| is sign(f_s), 0 at 0;
 *   - nearest neighbour: smallest d2 = ((dx*dx + dy*dy) + dz*dz) with
 *     dx = (double)q_x - (double)s_x, no fused multiply-add, ties to the
 *     lowest point index.
 *
 * Parity unpinned: nothing in the paper fixes whether these readings, the
 * sampler, the marching cubes face rule or the normal term are what the
 * authors ran, nor the reconstruction quality of its tables (no datasets or
 * trained fields here).  Each function is pinned against closed forms,
 * invariants and brute force instead; the tests name the pins.
 *
 * Linear ids are x-major: cell (cx*Ry + cy)*Rz + cz, vertex
 * (i*(Ry+1) + j)*(Rz+1) + k.
 *
 * Flags: cell_flags bit 1 = contains a point, bit 2 = M1 band, bit 4 = M2 band;
 *        vert_flags bit 1 = corner of an M1- or M2-band cell (optimised),
 *        bit 2 = corner of an M2-band cell (TV set).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Grid geometry (Sec. 3, "Discrete Grids")                                   */
/* ------------------------------------------------------------------------- */

typedef struct {
    int64_t R[3];      /* cells per axis */
    int64_t V[3];      /* vertices per axis = R + 1 */
    double lo[3];
    double h[3];       /* cell size (hi - lo) / R */
    double inv_h[3];   /* R / (hi - lo) */
} grid_t;

static void grid_init(grid_t* g, const int32_t* R, const double* lo, const double* hi)
{
    for (int a = 0; a < 3; ++a) {
        g->R[a] = R[a];
        g->V[a] = (int64_t)R[a] + 1;
        g->lo[a] = lo[a];
        g->h[a] = (hi[a] - lo[a]) / (double)R[a];
        g->inv_h[a] = (double)R[a] / (hi[a] - lo[a]);
    }
}

static int64_t cell_id(const grid_t* g, const int64_t c[3])
{
    return (c[0] * g->R[1] + c[1]) * g->R[2] + c[2];
}

static int64_t vertex_id(const grid_t* g, int64_t i, int64_t j, int64_t k)
{
    return (i * g->V[1] + j) * g->V[2] + k;
}

/* Locate a position in the grid: cell c and local coordinate t in [0,1].
 * Returns 1 if 0 <= u_a <= R_a on every axis, else 0 (c, t then undefined). */
static int locate(const grid_t* g, const double x[3], int64_t c[3], double t[3])
{
    for (int a = 0; a < 3; ++a) {
        double u = (x[a] - g->lo[a]) * g->inv_h[a];
        if (!(u >= 0.0) || !(u <= (double)g->R[a])) return 0;
        double fl = floor(u);
        int64_t ci = (int64_t)fl;
        if (ci > g->R[a] - 1) ci = g->R[a] - 1;
        c[a] = ci;
        t[a] = u - (double)ci;
    }
    return 1;
}

/* ------------------------------------------------------------------------- */
/* Bands (Sec. 3: M1 band for pulling, M2 band for TV)                        */
/* ------------------------------------------------------------------------- */

static void dilate(const grid_t* g, const uint8_t* cell_flags_in, uint8_t bit_in,
                   uint8_t* cell_flags, uint8_t bit_out, int64_t M)
{
    for (int64_t cx = 0; cx < g->R[0]; ++cx)
    for (int64_t cy = 0; cy < g->R[1]; ++cy)
    for (int64_t cz = 0; cz < g->R[2]; ++cz) {
        int64_t b[3] = {cx, cy, cz};
        if (!(cell_flags_in[cell_id(g, b)] & bit_in)) continue;
        for (int64_t x = cx - M; x <= cx + M; ++x) {
            if (x < 0 || x >= g->R[0]) continue;
            for (int64_t y = cy - M; y <= cy + M; ++y) {
                if (y < 0 || y >= g->R[1]) continue;
                for (int64_t z = cz - M; z <= cz + M; ++z) {
                    if (z < 0 || z >= g->R[2]) continue;
                    int64_t c[3] = {x, y, z};
                    cell_flags[cell_id(g, c)] |= bit_out;
                }
            }
        }
    }
}

static void mark_corners(const grid_t* g, const uint8_t* cell_flags, uint8_t cell_bits,
                         uint8_t* vert_flags, uint8_t vbit)
{
    for (int64_t cx = 0; cx < g->R[0]; ++cx)
    for (int64_t cy = 0; cy < g->R[1]; ++cy)
    for (int64_t cz = 0; cz < g->R[2]; ++cz) {
        int64_t c[3] = {cx, cy, cz};
        if (!(cell_flags[cell_id(g, c)] & cell_bits)) continue;
        for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
        for (int d = 0; d < 2; ++d)
            vert_flags[vertex_id(g, cx + a, cy + b, cz + d)] |= vbit;
    }
}

/* Base cells, M1/M2 bands and the optimised / TV vertex sets.
 * cell_flags [R_x R_y R_z] and vert_flags [(R+1)^3] are written in full.
 * Returns -1 on success, else the index of the first point outside [lo, hi]. */
int64_t og_build_band(const int32_t* R, const double* lo, const double* hi,
                      const float* px, const float* py, const float* pz, int64_t n_points,
                      int32_t m1, int32_t m2, uint8_t* cell_flags, uint8_t* vert_flags)
{
    grid_t g;
    grid_init(&g, R, lo, hi);
    int64_t nc = g.R[0] * g.R[1] * g.R[2];
    int64_t nv = g.V[0] * g.V[1] * g.V[2];
    memset(cell_flags, 0, (size_t)nc);
    memset(vert_flags, 0, (size_t)nv);
    for (int64_t j = 0; j < n_points; ++j) {
        double x[3] = {px[j], py[j], pz[j]};
        int64_t c[3];
        double t[3];
        if (!locate(&g, x, c, t)) return j;
        cell_flags[cell_id(&g, c)] |= 1;
    }
    dilate(&g, cell_flags, 1, cell_flags, 2, m1);
    dilate(&g, cell_flags, 1, cell_flags, 4, m2);
    mark_corners(&g, cell_flags, 2 | 4, vert_flags, 1);
    mark_corners(&g, cell_flags, 4, vert_flags, 2);
    return -1;
}

/* ------------------------------------------------------------------------- */
/* Nearest surface point NN(q) (Eq. 4), brute force over all points          */
/* ------------------------------------------------------------------------- */

static double dist2(const float* q, float sx, float sy, float sz)
{
    double dx = (double)q[0] - (double)sx;
    double dy = (double)q[1] - (double)sy;
    double dz = (double)q[2] - (double)sz;
    double xx = dx * dx;
    double yy = dy * dy;
    double zz = dz * dz;
    double s = xx + yy;
    return s + zz;
}

void og_nn_bruteforce(const float* qx, const float* qy, const float* qz, int64_t n_queries,
                      const float* px, const float* py, const float* pz, int64_t n_points,
                      int32_t* nn)
{
    for (int64_t k = 0; k < n_queries; ++k) {
        float q[3] = {qx[k], qy[k], qz[k]};
        double best = INFINITY;
        int64_t arg = -1;
        for (int64_t j = 0; j < n_points; ++j) {
            double d = dist2(q, px[j], py[j], pz[j]);
            if (d < best) { best = d; arg = j; }   /* strict: ties keep the lowest j */
        }
        nn[k] = (int32_t)arg;
    }
}

/* ------------------------------------------------------------------------- */
/* Trilinear interpolation and its gradient (Eq. 1 / Eq. 3)                   */
/* ------------------------------------------------------------------------- */

typedef struct {
    int64_t vid[8];     /* corner (a,b,c) at index 4a + 2b + c */
    double w[8];        /* W_a(t_x) W_b(t_y) W_c(t_z), W_0 = 1 - t, W_1 = t */
    double dw[8][3];    /* derivative of w with respect to q_x, q_y, q_z */
    double f;           /* f(q) */
    double g[3];        /* grad f(q) */
    double n;           /* |grad f(q)| */
} interp_t;

static void interpolate(const grid_t* g, const double* D, const int64_t c[3], const double t[3],
                        interp_t* it)
{
    double W[3][2] = {{1.0 - t[0], t[0]}, {1.0 - t[1], t[1]}, {1.0 - t[2], t[2]}};
    double dW[2] = {-1.0, 1.0};
    it->f = 0.0;
    it->g[0] = it->g[1] = it->g[2] = 0.0;
    for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
    for (int d = 0; d < 2; ++d) {
        int k = 4 * a + 2 * b + d;
        it->vid[k] = vertex_id(g, c[0] + a, c[1] + b, c[2] + d);
        it->w[k] = W[0][a] * W[1][b] * W[2][d];
        it->dw[k][0] = dW[a] * g->inv_h[0] * W[1][b] * W[2][d];
        it->dw[k][1] = W[0][a] * dW[b] * g->inv_h[1] * W[2][d];
        it->dw[k][2] = W[0][a] * W[1][b] * dW[d] * g->inv_h[2];
        double Dv = D[it->vid[k]];
        it->f += it->w[k] * Dv;
        for (int e = 0; e < 3; ++e) it->g[e] += it->dw[k][e] * Dv;
    }
    it->n = sqrt(it->g[0] * it->g[0] + it->g[1] * it->g[1] + it->g[2] * it->g[2]);
}

/* Field value and gradient at an arbitrary position (for the closed-form
 * checks).  Returns 0 if the position is outside the grid. */
int og_eval(const int32_t* R, const double* lo, const double* hi, const double* D,
            double x, double y, double z, double* f_out, double* g_out)
{
    grid_t g;
    grid_init(&g, R, lo, hi);
    double p[3] = {x, y, z};
    int64_t c[3];
    double t[3];
    if (!locate(&g, p, c, t)) return 0;
    interp_t it;
    interpolate(&g, D, c, t, &it);
    *f_out = it.f;
    for (int a = 0; a < 3; ++a) g_out[a] = it.g[a];
    return 1;
}

/* ------------------------------------------------------------------------- */
/* Loss (Eq. 4-8) and its exact gradient with respect to D                    */
/* ------------------------------------------------------------------------- */

static void scatter(double* G, const interp_t* it, double scale, double dl_df, const double dl_dg[3])
{
    for (int k = 0; k < 8; ++k) {
        double v = it->w[k] * dl_df;
        for (int a = 0; a < 3; ++a) v += it->dw[k][a] * dl_dg[a];
        G[it->vid[k]] += scale * v;
    }
}

/*
 * terms_out[5] = { total, L_Pull, L_TV, L_Surface, L_grad }:
 *   L_Pull, L_Surface, L_grad are means over the valid queries (a query is
 *   valid when it lies in the grid and its cell is in the M1 band), L_TV is the
 *   mean of tau over the M2-band vertices, total = L_Pull + alpha L_TV +
 *   beta L_Surface + gamma L_grad.
 * grad_out (nullable, [(R+1)^3]) receives d total / d D (zeroed first).
 * per_query (nullable, [n_queries][4]) receives l_pull, l_surf, l_grad and a
 *   validity flag per query.
 * tau_out (nullable, [(R+1)^3]) receives tau at the M2-band vertices.
 * Returns the number of valid queries, or -1 if a nearest point lies outside
 * the grid.
 */
int64_t og_loss_grad(const int32_t* R, const double* lo, const double* hi,
                     const uint8_t* cell_flags, const uint8_t* vert_flags, const double* D,
                     const float* qx, const float* qy, const float* qz, const int32_t* nn,
                     int64_t n_queries,
                     const float* px, const float* py, const float* pz,
                     double alpha, double beta, double gamma, double eps_n,
                     double* terms_out, double* grad_out, double* per_query, double* tau_out)
{
    grid_t g;
    grid_init(&g, R, lo, hi);
    int64_t nv = g.V[0] * g.V[1] * g.V[2];
    if (grad_out) memset(grad_out, 0, (size_t)nv * sizeof(double));

    /* Pass 1: count the valid queries, so that the gradient of each mean can
     * be scattered directly. */
    int64_t n_valid = 0;
    for (int64_t k = 0; k < n_queries; ++k) {
        double q[3] = {qx[k], qy[k], qz[k]};
        int64_t c[3];
        double t[3];
        if (locate(&g, q, c, t) && (cell_flags[cell_id(&g, c)] & 2)) ++n_valid;
    }
    double inv_q = n_valid > 0 ? 1.0 / (double)n_valid : 0.0;

    double sum_pull = 0.0, sum_surf = 0.0, sum_grad = 0.0;
    for (int64_t k = 0; k < n_queries; ++k) {
        double q[3] = {qx[k], qy[k], qz[k]};
        int64_t c[3];
        double t[3];
        if (per_query) { per_query[4 * k] = per_query[4 * k + 1] = per_query[4 * k + 2] = 0.0;
                         per_query[4 * k + 3] = 0.0; }
        if (!locate(&g, q, c, t) || !(cell_flags[cell_id(&g, c)] & 2)) continue;

        /* f and grad f at the query (Eq. 1, Eq. 3). */
        interp_t iq;
        interpolate(&g, D, c, t, &iq);
        double gh[3] = {0.0, 0.0, 0.0};
        int q_ok = iq.n >= eps_n;
        if (q_ok) for (int a = 0; a < 3; ++a) gh[a] = iq.g[a] / iq.n;

        /* The nearest surface point s = NN(q) and f, grad f there. */
        int64_t j = nn[k];
        double s[3] = {px[j], py[j], pz[j]};
        int64_t cs[3];
        double ts[3];
        if (!locate(&g, s, cs, ts)) return -1;
        interp_t is;
        interpolate(&g, D, cs, ts, &is);
        double ghs[3] = {0.0, 0.0, 0.0};
        int s_ok = is.n >= eps_n;
        if (s_ok) for (int a = 0; a < 3; ++a) ghs[a] = is.g[a] / is.n;

        /* Pull (Sec. 3): p = q - f(q) * grad f / |grad f|; residual p - s (Eq. 4). */
        double r[3];
        for (int a = 0; a < 3; ++a) {
            double p = q[a] - iq.f * gh[a];
            r[a] = p - s[a];
        }
        double l_pull = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        double e[3] = {0.0, 0.0, 0.0};
        if (l_pull > 0.0) for (int a = 0; a < 3; ++a) e[a] = r[a] / l_pull;

        /* Surface term (Eq. 6). */
        double l_surf = fabs(is.f);
        double sgn = is.f > 0.0 ? 1.0 : (is.f < 0.0 ? -1.0 : 0.0);

        /* Gradient consistency (Eq. 7). */
        double cosv = 0.0, l_grad = 1.0;
        int grad_ok = q_ok && s_ok;
        if (grad_ok) {
            cosv = gh[0] * ghs[0] + gh[1] * ghs[1] + gh[2] * ghs[2];
            l_grad = 1.0 - cosv;
        }

        sum_pull += l_pull;
        sum_surf += l_surf;
        sum_grad += l_grad;
        if (per_query) { per_query[4 * k] = l_pull; per_query[4 * k + 1] = l_surf;
                         per_query[4 * k + 2] = l_grad; per_query[4 * k + 3] = 1.0; }

        if (!grad_out) continue;

        /* Adjoint at the query: l = l_pull + gamma l_grad as a function of f, grad f. */
        double dl_df = -(gh[0] * e[0] + gh[1] * e[1] + gh[2] * e[2]);
        double dl_dg[3] = {0.0, 0.0, 0.0};
        if (q_ok) {
            /* d l_pull / d gh = -f e; through gh = g / |g|: (I - gh gh^T) / |g| */
            double u[3] = {-iq.f * e[0], -iq.f * e[1], -iq.f * e[2]};
            double ug = u[0] * gh[0] + u[1] * gh[1] + u[2] * gh[2];
            for (int a = 0; a < 3; ++a) dl_dg[a] = (u[a] - ug * gh[a]) / iq.n;
        }
        double dls_dg[3] = {0.0, 0.0, 0.0};
        if (grad_ok) {
            for (int a = 0; a < 3; ++a) {
                dl_dg[a] += gamma * (-(ghs[a] - cosv * gh[a]) / iq.n);
                dls_dg[a] = gamma * (-(gh[a] - cosv * ghs[a]) / is.n);
            }
        }
        scatter(grad_out, &iq, inv_q, dl_df, dl_dg);
        /* Adjoint at the surface point: beta |f_s| + gamma l_grad. */
        scatter(grad_out, &is, inv_q, beta * sgn, dls_dg);
    }

    /* TV term (Eq. 5) over the M2-band vertices. */
    int64_t n_tv = 0;
    for (int64_t v = 0; v < nv; ++v) if (vert_flags[v] & 2) ++n_tv;
    double* tau = (double*)calloc((size_t)nv, sizeof(double));
    double sum_tv = 0.0;
    const int off[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    for (int64_t i = 0; i < g.V[0]; ++i)
    for (int64_t jj = 0; jj < g.V[1]; ++jj)
    for (int64_t kk = 0; kk < g.V[2]; ++kk) {
        int64_t v = vertex_id(&g, i, jj, kk);
        if (!(vert_flags[v] & 2)) continue;
        double s2 = 0.0;
        for (int o = 0; o < 6; ++o) {
            int64_t a = i + off[o][0], b = jj + off[o][1], cc = kk + off[o][2];
            if (a < 0 || b < 0 || cc < 0 || a >= g.V[0] || b >= g.V[1] || cc >= g.V[2]) continue;
            int64_t u = vertex_id(&g, a, b, cc);
            if (!(vert_flags[u] & 2)) continue;
            double d = D[v] - D[u];
            s2 += d * d;
        }
        tau[v] = sqrt(s2);
        sum_tv += tau[v];
    }
    double l_tv = n_tv > 0 ? sum_tv / (double)n_tv : 0.0;
    if (grad_out && n_tv > 0) {
        double sc = alpha / (double)n_tv;
        for (int64_t i = 0; i < g.V[0]; ++i)
        for (int64_t jj = 0; jj < g.V[1]; ++jj)
        for (int64_t kk = 0; kk < g.V[2]; ++kk) {
            int64_t v = vertex_id(&g, i, jj, kk);
            if (!(vert_flags[v] & 2)) continue;
            double acc = 0.0;
            for (int o = 0; o < 6; ++o) {
                int64_t a = i + off[o][0], b = jj + off[o][1], cc = kk + off[o][2];
                if (a < 0 || b < 0 || cc < 0 || a >= g.V[0] || b >= g.V[1] || cc >= g.V[2]) continue;
                int64_t u = vertex_id(&g, a, b, cc);
                if (!(vert_flags[u] & 2)) continue;
                double d = D[v] - D[u];
                /* d tau_v / d D_v and d tau_u / d D_v; a zero tau has d = 0 here. */
                if (tau[v] > 0.0) acc += d / tau[v];
                if (tau[u] > 0.0) acc += d / tau[u];
            }
            grad_out[v] += sc * acc;
        }
    }
    if (tau_out) memcpy(tau_out, tau, (size_t)nv * sizeof(double));
    free(tau);

    double l_pull = sum_pull * inv_q, l_surf = sum_surf * inv_q, l_grad = sum_grad * inv_q;
    terms_out[1] = l_pull;
    terms_out[2] = l_tv;
    terms_out[3] = l_surf;
    terms_out[4] = l_grad;
    terms_out[0] = l_pull + alpha * l_tv + beta * l_surf + gamma * l_grad;
    return n_valid;
}

/* ------------------------------------------------------------------------- */
/* Adam (Sec. 4 "Details": Adam, lr0, x decay every decay_every iterations;   */
/* Kingma and Ba, ICLR 2015)                                                  */
/* ------------------------------------------------------------------------- */

void og_adam(int64_t n, double* D, const double* G, double* m, double* v, const uint8_t* vert_flags,
             int32_t t, double lr0, double decay, int32_t decay_every,
             double beta1, double beta2, double eps)
{
    double lr = lr0 * pow(decay, (double)((t - 1) / decay_every));
    double bc1 = 1.0 - pow(beta1, (double)t);
    double bc2 = 1.0 - pow(beta2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        if (!(vert_flags[i] & 1)) continue;
        m[i] = beta1 * m[i] + (1.0 - beta1) * G[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * G[i] * G[i];
        double mh = m[i] / bc1;
        double vh = v[i] / bc2;
        D[i] = D[i] - lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------------------------- */
/* Query offsets: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the   */
/* Box-Muller transform.  Query k of a batch draws one Philox block with      */
/* counter (k mod 2^32, k >> 32, iteration, stream) and key (seed mod 2^32,    */
/* seed >> 32); the four words become uniforms U = ((x >> 8) + 1/2) 2^-24 and   */
/* the offsets are z0, z1 = sqrt(-2 ln U0) (cos, sin)(2 pi U1) and             */
/* z2 = sqrt(-2 ln U2) cos(2 pi U3).                                           */
/* ------------------------------------------------------------------------- */

void og_philox4x32_10(const uint32_t* ctr_in, const uint32_t* key_in, uint32_t* out)
{
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k[2] = {key_in[0], key_in[1]};
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k[0];
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c[3] ^ k[1];
        uint32_t n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
        k[0] += 0x9E3779B9u;
        k[1] += 0xBB67AE85u;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

void og_query_offsets(uint64_t seed, uint32_t iteration, uint32_t stream, int64_t k0, int64_t n,
                      double* z_out /* [n][3] */)
{
    const double two_pi = 6.283185307179586476925286766559;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t i = 0; i < n; ++i) {
        uint64_t k = (uint64_t)(k0 + i);
        uint32_t ctr[4] = {(uint32_t)k, (uint32_t)(k >> 32), iteration, stream};
        uint32_t x[4];
        og_philox4x32_10(ctr, key, x);
        double U[4];
        for (int a = 0; a < 4; ++a) U[a] = ((double)(x[a] >> 8) + 0.5) * (1.0 / 16777216.0);
        double r0 = sqrt(-2.0 * log(U[0]));
        double r1 = sqrt(-2.0 * log(U[2]));
        z_out[3 * i + 0] = r0 * cos(two_pi * U[1]);
        z_out[3 * i + 1] = r0 * sin(two_pi * U[1]);
        z_out[3 * i + 2] = r1 * cos(two_pi * U[3]);
    }
}

/* ------------------------------------------------------------------------ */
/* Surface extraction (the mesh step after the optimisation, Sec. 3/4: the    */
/* zero level set of the field over the cells that were optimised).          */
/* Reading taken here: marching tetrahedra instead of the marching-cubes      */
/* case table.  Every cell whose eight corners are optimised vertices is cut  */
/* into six tetrahedra along its main diagonal (corner (0,0,0) to (1,1,1),   */
/* corner (a,b,c) at index 4a + 2b + c); the cut is the same on both sides of */
/* every face, so the mesh has no cracks.  A vertex is inside where f < 0.   */
/* A tetrahedron with one vertex on one side and three on the other gives    */
/* one triangle, two and two give two; each triangle vertex sits on an edge  */
/* (p, q), p inside, where the linear interpolant vanishes:                 */
/* p + f_p / (f_p - f_q) (q - p).                                           */
/* Triangles are listed by cell id, then tetrahedron, then triangle; the     */
/* key of a triangle is cell_id * 16 + tet * 2 + triangle.                   */
/* ------------------------------------------------------------------------ */

/* the six tetrahedra: (0, A, B, 7) along the paths 0 -> A -> B -> 7 */
static const int kTets[6][4] = {{0, 4, 6, 7}, {0, 4, 5, 7}, {0, 2, 6, 7},
                                {0, 2, 3, 7}, {0, 1, 5, 7}, {0, 1, 3, 7}};

static void edge_point(const double P[8][3], const double f[8], int a, int b, double out[3])
{
    double t = f[a] / (f[a] - f[b]);
    for (int k = 0; k < 3; ++k) out[k] = P[a][k] + t * (P[b][k] - P[a][k]);
}

/* Triangles of one tetrahedron (corner indices v[4] into P, f): returns how
 * many (0, 1 or 2) and writes their vertices to tri[2][3][3]. */
static int tet_triangles(const double P[8][3], const double f[8], const int v[4], double tri[2][3][3])
{
    int in[4], out[4], ni = 0, no = 0;
    for (int i = 0; i < 4; ++i) {
        if (f[v[i]] < 0.0) in[ni++] = v[i];
        else out[no++] = v[i];
    }
    if (ni == 0 || no == 0) return 0;
    if (ni == 1 || no == 1) {
        /* the lone vertex and the three edges leaving it; every edge point is
         * taken from its inside end, so that a grid edge gives the same point
         * in every tetrahedron that has it */
        for (int k = 0; k < 3; ++k) {
            if (ni == 1) edge_point(P, f, in[0], out[k], tri[0][k]);
            else edge_point(P, f, in[k], out[0], tri[0][k]);
        }
        return 1;
    }
    /* two in (a, b), two out (c, d): the quad ac, ad, bd, bc as two triangles */
    double ac[3], ad[3], bd[3], bc[3];
    edge_point(P, f, in[0], out[0], ac);
    edge_point(P, f, in[0], out[1], ad);
    edge_point(P, f, in[1], out[1], bd);
    edge_point(P, f, in[1], out[0], bc);
    for (int k = 0; k < 3; ++k) {
        tri[0][0][k] = ac[k]; tri[0][1][k] = ad[k]; tri[0][2][k] = bd[k];
        tri[1][0][k] = ac[k]; tri[1][1][k] = bd[k]; tri[1][2][k] = bc[k];
    }
    return 2;
}

/* D: dense vertex values; vert_flags bit 1: optimised vertex.  Writes at most
 * capacity triangles (keys and 9 coordinates each) and returns how many the
 * field has in total. */
int64_t og_extract_surface(const int32_t* R_in, const double* lo, const double* hi, const double* D,
                           const uint8_t* vert_flags, int64_t capacity, int64_t* keys, double* xyz)
{
    grid_t g;
    grid_init(&g, R_in, lo, hi);
    int64_t n = 0;
    for (int64_t cx = 0; cx < g.R[0]; ++cx)
    for (int64_t cy = 0; cy < g.R[1]; ++cy)
    for (int64_t cz = 0; cz < g.R[2]; ++cz) {
        double P[8][3], f[8];
        int all = 1;
        for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
        for (int c = 0; c < 2; ++c) {
            int64_t vid = vertex_id(&g, cx + a, cy + b, cz + c);
            int i = 4 * a + 2 * b + c;
            if (!(vert_flags[vid] & 1)) all = 0;
            f[i] = D[vid];
            P[i][0] = g.lo[0] + (double)(cx + a) * g.h[0];
            P[i][1] = g.lo[1] + (double)(cy + b) * g.h[1];
            P[i][2] = g.lo[2] + (double)(cz + c) * g.h[2];
        }
        if (!all) continue;
        int64_t c3[3] = {cx, cy, cz};
        int64_t cid = cell_id(&g, c3);
        for (int t = 0; t < 6; ++t) {
            double tri[2][3][3];
            int m = tet_triangles(P, f, kTets[t], tri);
            for (int r = 0; r < m; ++r) {
                if (n < capacity) {
                    keys[n] = cid * 16 + t * 2 + r;
                    for (int v = 0; v < 3; ++v)
                        for (int k = 0; k < 3; ++k) xyz[9 * n + 3 * v + k] = tri[r][v][k];
                }
                ++n;
            }
        }
    }
    return n;
}

/* ------------------------------------------------------------------------ */
/* Marching cubes (Lorensen and Cline, SIGGRAPH 1987): the mesh the paper     */
/* extracts over the optimised cells (Sec. 3, last paragraph; Sec. 4        */
/* "Details").  The triangles of a cell depend only on which of its eight     */
/* corners are inside (f < 0), one of 256 configurations.  They are derived  */
/* here from one rule rather than taken from a printed case table:          */
/*  - each face is walked through its corners counter-clockwise as seen from */
/*    outside the cube; an edge whose ends differ is crossed;                */
/*  - on each face, every maximal run of inside corners along the walk gets  */
/*    a segment from the crossed edge where the walk leaves it to the one    */
/*    where it entered (on a face with two diagonal inside corners the two    */
/*    are cut off separately: the ambiguity is resolved by the face alone,  */
/*    the same way in both cells that share it, so the mesh has no cracks);   */
/*  - a crossed edge ends a segment on one of its faces and starts one on the */
/*    other, so the segments close into loops; loops are taken from the      */
/*    smallest unused crossed edge (edge numbers below), and each loop        */
/*    v0, v1, ..., v_k-1 becomes the fan (v0, v_i, v_i+1), i = 1 .. k-2.     */
/* Corner (a,b,c) has index 4a + 2b + c.  Edges: along x, 2b + c; along y,   */
/* 4 + 2a + c; along z, 8 + 2a + b.  A triangle vertex is the zero of the    */
/* linear interpolant on its edge, from the inside end p: as edge_point.     */
/* Keys: cell_id * 16 + the triangle's number in its cell.                    */
/* ------------------------------------------------------------------------ */

/* the faces, counter-clockwise from outside: x = 0, x = 1, y = 0, y = 1, z = 0, z = 1 */
static const int mc_faces[6][4] = {{0, 1, 3, 2}, {4, 6, 7, 5}, {0, 4, 5, 1},
                                   {2, 3, 7, 6}, {0, 2, 6, 4}, {1, 5, 7, 3}};

static int mc_edge(int p, int q)
{
    int lo = p < q ? p : q, a = (lo >> 2) & 1, b = (lo >> 1) & 1, c = lo & 1;
    switch (p ^ q) {
    case 4: return 2 * b + c;          /* along x */
    case 2: return 4 + 2 * a + c;      /* along y */
    default: return 8 + 2 * a + b;     /* along z */
    }
}

static void mc_edge_ends(int e, int* p, int* q)
{
    if (e < 4) { *p = e; *q = 4 + e; }                                      /* (0,b,c)-(1,b,c) */
    else if (e < 8) { int a = (e - 4) >> 1, c = (e - 4) & 1; *p = 4 * a + c; *q = 4 * a + 2 + c; }
    else { int a = (e - 8) >> 1, b = (e - 8) & 1; *p = 4 * a + 2 * b; *q = *p + 1; }
}

/* Triangles (as edge triples) of configuration cfg (bit i: corner i inside);
 * returns how many, or -1 if the segments do not close into loops. */
static int mc_triangles(int cfg, int tri[16][3])
{
    int next[12], used[12], n = 0;
    for (int e = 0; e < 12; ++e) { next[e] = -1; used[e] = 0; }
    for (int F = 0; F < 6; ++F) {
        const int* c = mc_faces[F];
        for (int j = 0; j < 4; ++j) {
            int in_j = (cfg >> c[j]) & 1, in_n = (cfg >> c[(j + 1) % 4]) & 1;
            if (!(in_j && !in_n)) continue;          /* not where the walk leaves a run */
            int k = j;
            while ((cfg >> c[k]) & 1) k = (k + 3) % 4; /* back to the corner before the run */
            next[mc_edge(c[j], c[(j + 1) % 4])] = mc_edge(c[k], c[(k + 1) % 4]);
        }
    }
    for (int e = 0; e < 12; ++e) {
        if (next[e] < 0 || used[e]) continue;
        int loop[12], m = 0, v = e;
        do {
            if (v < 0 || m == 12) return -1;         /* segments that do not close: no valid rule */
            loop[m++] = v;
            used[v] = 1;
            v = next[v];
        } while (v != e);
        for (int i = 1; i + 1 < m; ++i) {
            tri[n][0] = loop[0]; tri[n][1] = loop[i]; tri[n][2] = loop[i + 1];
            ++n;
        }
    }
    return n;
}

/* The same inputs and outputs as og_extract_surface, by marching cubes
 * (-1 if the rule fails to close a configuration's segments). */
int64_t og_marching_cubes(const int32_t* R_in, const double* lo, const double* hi, const double* D,
                          const uint8_t* vert_flags, int64_t capacity, int64_t* keys, double* xyz)
{
    grid_t g;
    grid_init(&g, R_in, lo, hi);
    int64_t n = 0;
    for (int64_t cx = 0; cx < g.R[0]; ++cx)
    for (int64_t cy = 0; cy < g.R[1]; ++cy)
    for (int64_t cz = 0; cz < g.R[2]; ++cz) {
        double P[8][3], f[8];
        int all = 1, cfg = 0;
        for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
        for (int c = 0; c < 2; ++c) {
            int64_t vid = vertex_id(&g, cx + a, cy + b, cz + c);
            int i = 4 * a + 2 * b + c;
            if (!(vert_flags[vid] & 1)) all = 0;
            f[i] = D[vid];
            if (f[i] < 0.0) cfg |= 1 << i;
            P[i][0] = g.lo[0] + (double)(cx + a) * g.h[0];
            P[i][1] = g.lo[1] + (double)(cy + b) * g.h[1];
            P[i][2] = g.lo[2] + (double)(cz + c) * g.h[2];
        }
        if (!all || cfg == 0 || cfg == 255) continue;
        int64_t c3[3] = {cx, cy, cz};
        int64_t cid = cell_id(&g, c3);
        int tri[16][3];
        int m = mc_triangles(cfg, tri);
        if (m < 0) return -1;
        for (int r = 0; r < m; ++r) {
            if (n < capacity) {
                keys[n] = cid * 16 + r;
                for (int v = 0; v < 3; ++v) {
                    int p, q;
                    mc_edge_ends(tri[r][v], &p, &q);
                    if (!(f[p] < 0.0)) { int t = p; p = q; q = t; }   /* p: the inside end */
                    edge_point(P, f, p, q, xyz + 9 * n + 3 * v);
                }
            }
            ++n;
        }
    }
    return n;
}

/* The triangle count of every configuration (for the pins). */
void og_mc_counts(int32_t* out)
{
    int tri[16][3];
    for (int cfg = 0; cfg < 256; ++cfg) out[cfg] = mc_triangles(cfg, tri);
}

/* ------------------------------------------------------------------------ */
/* Normal supervision (Sec. 4, normals paragraph: with ground-truth normals, */
/* the gradient of the field at the surface points is supervised by them).  */
/* Reading taken here: the same cosine form as the gradient-consistency term */
/* with the given normal in place of the query's gradient,                  */
/*   L_N = (1/Q_v) sum over valid queries of (1 - gh_s . n_s),               */
/* s = NN(q), gh_s = grad f(s) / |grad f(s)| (below eps_n the term is 1 with */
/* zero gradient), Q_v and validity as in og_loss_grad.  Writes L_N to       */
/* term_out and adds weight * d L_N / d D to grad_out (nullable; not zeroed).*/
/* Returns Q_v, or -1 if a nearest point lies outside the grid.              */
/* ------------------------------------------------------------------------ */
int64_t og_normal_term(const int32_t* R, const double* lo, const double* hi, const uint8_t* cell_flags,
                       const double* D, const float* qx, const float* qy, const float* qz, const int32_t* nn,
                       int64_t n_queries, const float* px, const float* py, const float* pz,
                       const float* nx, const float* ny, const float* nz, double weight, double eps_n,
                       double* term_out, double* grad_out)
{
    grid_t g;
    grid_init(&g, R, lo, hi);
    int64_t n_valid = 0;
    for (int64_t k = 0; k < n_queries; ++k) {
        double q[3] = {qx[k], qy[k], qz[k]};
        int64_t c[3];
        double t[3];
        if (locate(&g, q, c, t) && (cell_flags[cell_id(&g, c)] & 2)) ++n_valid;
    }
    double inv_q = n_valid > 0 ? 1.0 / (double)n_valid : 0.0;
    double sum = 0.0;
    for (int64_t k = 0; k < n_queries; ++k) {
        double q[3] = {qx[k], qy[k], qz[k]};
        int64_t c[3];
        double t[3];
        if (!locate(&g, q, c, t) || !(cell_flags[cell_id(&g, c)] & 2)) continue;
        int64_t j = nn[k];
        double s[3] = {px[j], py[j], pz[j]};
        int64_t cs[3];
        double ts[3];
        if (!locate(&g, s, cs, ts)) return -1;
        interp_t is;
        interpolate(&g, D, cs, ts, &is);
        double nj[3] = {nx[j], ny[j], nz[j]};
        if (is.n < eps_n) {
            sum += 1.0;
            continue;
        }
        double ghs[3], cosv = 0.0;
        for (int a = 0; a < 3; ++a) {
            ghs[a] = is.g[a] / is.n;
            cosv += ghs[a] * nj[a];
        }
        sum += 1.0 - cosv;
        if (!grad_out) continue;
        /* d (1 - gh . n) / d grad f = -(n - (gh . n) gh) / |grad f| */
        double dl_dg[3];
        for (int a = 0; a < 3; ++a) dl_dg[a] = -(nj[a] - cosv * ghs[a]) / is.n;
        scatter(grad_out, &is, weight * inv_q, 0.0, dl_dg);
    }
    *term_out = sum * inv_q;
    return n_valid;
}
