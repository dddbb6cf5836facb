/*
 * gsc_oracle.c -- plain, slow FP64 CPU oracle for the per-frame hot path of a
 * cache-centric structured-3DGS stereo renderer (GS-Cache, arXiv 2502.14938).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker that the GPU library is
 * compared against; the GPU library never links, calls or includes it, and it
 * shares no code with the GPU library.  Only the tests, the smoke check and
 * the benchmark's CPU-baseline leg use it.
 *
 * Every routine works in double precision on float32 scene data and follows
 * one step of the method in the paper's order:
 *   - unified camera of a stereo pair          Section 4, eqs. 5-6
 *   - anchor selection (LOD + frustum)          Section 3.1 (Octree-GS LOD),
 *                                               Section 3.2 (anchor filtering)
 *   - neural-Gaussian derivation                Section 3.1 eq. 3, eq. 2
 *   - EWA projection to 2D                      Section 3.1 (splatting)
 *   - opacity-aware exact tile lists            Section 6 (RasterizeGaussians)
 *   - stable (tile, depth) ordering             Section 6 (key-value pairs)
 *   - front-to-back alpha compositing           Section 3.1 (rasterization)
 * Where the paper is silent the documented readings are used (pinhole camera
 * with rows right/down/forward, 0.3 px^2 dilation, alpha clamp 0.99, skip
 * below 1/255, stop when T(1-alpha) < 1e-4, 16x16 tiles).
 *
 * "Band" outputs flag decisions whose FP64 margin is so small that an FP32
 * implementation may legitimately take the other side.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_TILE 16

typedef struct {
    double R[9];      /* world -> camera, rows: right, down, forward */
    double pos[3];    /* camera centre, world */
    double fovx, fovy;
    int32_t width, height;
    double znear;
} orc_camera;

/* ---------------------------------------------------------------- helpers */

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static double norm3(const double* a) { return sqrt(dot3(a, a)); }
static void cross3(const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
/* camera coordinates of a world point: t = R (x - p) */
static void to_camera(const orc_camera* c, const double* x, double* t) {
    double v[3] = {x[0] - c->pos[0], x[1] - c->pos[1], x[2] - c->pos[2]};
    for (int i = 0; i < 3; ++i) t[i] = c->R[3 * i] * v[0] + c->R[3 * i + 1] * v[1] + c->R[3 * i + 2] * v[2];
}
static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* ------------------------------------------------- precision emulation */

/* Round to nearest, ties to even, keeping `bits` significant bits. */
static double round_sig(double x, int bits) {
    if (x == 0.0 || !isfinite(x)) return x;
    int e;
    frexp(x, &e);                         /* x = m 2^e, 0.5 <= |m| < 1 */
    double q = ldexp(1.0, e - bits);      /* spacing of `bits`-bit significands */
    return nearbyint(x / q) * q;          /* default rounding mode: ties to even */
}
/* bfloat16: 8 significant bits, float32 exponent range. */
double orc_round_bf16(double x) { return round_sig(x, 8); }
/* OCP float8 e4m3fn: 4 significant bits, normal range [2^-6, 448],
 * subnormal spacing 2^-9, no infinities; saturate at +-448. */
double orc_round_e4m3(double x) {
    if (x == 0.0 || !isfinite(x)) return x;
    double a = fabs(x), r;
    if (a < ldexp(1.0, -6)) r = nearbyint(a / ldexp(1.0, -9)) * ldexp(1.0, -9);
    else r = round_sig(a, 4);
    if (r > 448.0) r = 448.0;
    return x < 0 ? -r : r;
}

/* ---------------------------------------------------- unified camera */
/* Section 4, eqs. 5-6: the unified camera looks along the normalised mean of
 * the eyes' forward axes and sits behind the eyes' midpoint by
 * |p1 - p2| / (2 tan(fovx / 2)), so that its horizontal field of view covers
 * both eyes'.  Reading for roll: right axis = mean of the eyes' right axes,
 * made orthogonal to the forward axis; down = forward x right.  Intrinsics
 * are those of the (identical) eyes. */
void orc_unified_camera(const orc_camera* l, const orc_camera* r, orc_camera* u) {
    double d[3], p[3], rt[3], dn[3];
    for (int i = 0; i < 3; ++i) d[i] = 0.5 * (l->R[6 + i] + r->R[6 + i]);
    double nd = norm3(d);
    for (int i = 0; i < 3; ++i) d[i] /= nd;
    double base[3] = {l->pos[0] - r->pos[0], l->pos[1] - r->pos[1], l->pos[2] - r->pos[2]};
    double setback = norm3(base) / (2.0 * tan(0.5 * l->fovx));
    for (int i = 0; i < 3; ++i) p[i] = 0.5 * (l->pos[i] + r->pos[i]) - d[i] * setback;
    for (int i = 0; i < 3; ++i) rt[i] = 0.5 * (l->R[i] + r->R[i]);
    double proj = dot3(rt, d);
    for (int i = 0; i < 3; ++i) rt[i] -= proj * d[i];
    double nr = norm3(rt);
    for (int i = 0; i < 3; ++i) rt[i] /= nr;
    cross3(d, rt, dn);
    *u = *l;
    for (int i = 0; i < 3; ++i) {
        u->R[i] = rt[i];
        u->R[3 + i] = dn[i];
        u->R[6 + i] = d[i];
        u->pos[i] = p[i];
    }
}

/* ---------------------------------------------------- anchor selection */
/* Keep anchor a iff
 *   (LOD)     level_a == 0  or  |x_a - p_u| <= d_l = d_ref * 2^-level_a, and
 *   (frustum) its bounding sphere (x_a, rho_a) is not wholly outside any of
 *             the unified camera's four side planes or its near plane.
 * With fade (the fractional level transition, a reading of the cited
 * Octree-GS distance-driven LOD): a level-l anchor (l > 0) is kept iff
 * |x_a - p_u| < 2 d_l, with the weight w_a = clamp(2 - |x_a - p_u| / d_l,
 * 0, 1) on the opacities of its Gaussians: 1 up to d_l, falling linearly to
 * 0 at 2 d_l, so a level comes in over the octave of distance before it is
 * fully present instead of appearing at once.  Level 0: w = 1.  w_out (may
 * be NULL) receives w for every anchor (1 without fade).
 * Output: the kept ids in ascending order; band[a] = 1 when either test's
 * margin is below 1e-6 relative. Returns the count. */
int64_t orc_select(int64_t n, const float* pos, const uint8_t* level, const float* radius,
                   const orc_camera* u, double d_ref, int fade, int32_t* out_ids, uint8_t* band, double* w_out) {
    double tx = tan(0.5 * u->fovx), ty = tan(0.5 * u->fovy);
    double nx = sqrt(1.0 + tx * tx), ny = sqrt(1.0 + ty * ty);
    uint8_t* keep = (uint8_t*)malloc(n > 0 ? (size_t)n : 1);
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < n; ++a) {
        double x[3] = {pos[3 * a], pos[3 * a + 1], pos[3 * a + 2]};
        double v[3] = {x[0] - u->pos[0], x[1] - u->pos[1], x[2] - u->pos[2]};
        double dist = norm3(v);
        double rho = radius[a];
        int lod_ok = 1, b = 0;
        double w = 1.0;
        if (level[a] != 0) {
            double dl = d_ref * ldexp(1.0, -(int)level[a]);
            double lim = fade ? 2.0 * dl : dl;
            lod_ok = fade ? dist < lim : dist <= lim;
            if (fabs(dist - lim) < 1e-6 * (lim + dist)) b = 1;
            if (fade) w = fmin(fmax(2.0 - dist / dl, 0.0), 1.0);
        }
        if (w_out) w_out[a] = w;
        double t[3];
        to_camera(u, x, t);
        double s[5];
        s[0] = t[2] - u->znear;
        s[1] = (t[0] + tx * t[2]) / nx;
        s[2] = (-t[0] + tx * t[2]) / nx;
        s[3] = (t[1] + ty * t[2]) / ny;
        s[4] = (-t[1] + ty * t[2]) / ny;
        double mag = fabs(t[0]) + fabs(t[1]) + fabs(t[2]) + rho + u->znear + 1.0;
        int fr_ok = 1;
        for (int i = 0; i < 5; ++i) {
            if (s[i] < -rho) fr_ok = 0;
            if (fabs(s[i] + rho) < 1e-6 * mag) b = 1;
        }
        keep[a] = (uint8_t)(lod_ok && fr_ok);
        if (band) band[a] = (uint8_t)b;
    }
    int64_t m = 0;
    for (int64_t a = 0; a < n; ++a)
        if (keep[a]) out_ids[m++] = (int32_t)a;
    free(keep);
    return m;
}

/* ---------------------------------------------------------- derivation */
/* Section 3.1, eq. 3 with the documented readings: for anchor a seen from the
 * unified camera centre p_u,
 *   d = (x_a - p_u) / |x_a - p_u|,  z = [f_a ; d]                 (F + 3)
 *   or, with a distance input (dist_unit > 0, the cited methods' optional
 *   camera-distance feature), z = [f_a ; d ; |x_a - p_u| / dist_unit] (F + 4)
 *   per head (alpha c=1, color c=3, cov c=7):
 *       h = ReLU(W1 z + b1) (H),   o = W2 h + b2 (c k), output index j*c + ch
 *   alpha_j = tanh(o_alpha[j])
 *   rgb_j   = sigmoid(o_color[3j .. 3j+2])
 *   scale_j = s_a[3:6] * sigmoid(o_cov[7j .. 7j+2])
 *   q_j     = o_cov[7j+3 .. 7j+6] / |.|  (w, x, y, z); zero -> (1, 0, 0, 0)
 *   Sigma_j = R(q_j) diag(scale_j)^2 R(q_j)^T                      (eq. 2)
 *   mu_j    = x_a + s_a[0:3] * O_aj
 * prec: 0 = exact FP64; 1 = bfloat16 weights and activations (z and h rounded
 * to bf16, biases and accumulation exact); 2 = as 1 but W1/W2 rounded to
 * e4m3fn with a per-output-row scale absmax/448.
 * Outputs (m*k rows): mu[3], cov[6] (xx xy xz yy yz zz), rgb[3], alpha[1],
 * alpha_pre[1] (the tanh argument, for band checks). */
static void quantise_weights(const float* W, int rows, int cols, int prec, double* out) {
    for (int r = 0; r < rows; ++r) {
        double amax = 0.0, s = 1.0;
        if (prec == 2) {
            for (int c = 0; c < cols; ++c) amax = fmax(amax, fabs((double)W[r * cols + c]));
            s = amax > 0.0 ? amax / 448.0 : 1.0;
        }
        for (int c = 0; c < cols; ++c) {
            double w = W[r * cols + c];
            if (prec == 1) w = orc_round_bf16(w);
            else if (prec == 2) w = orc_round_e4m3(w / s) * s;
            out[r * cols + c] = w;
        }
    }
}

void orc_derive(int64_t m, const int32_t* ids, const float* pos, const float* feat, const float* scale,
                const float* offsets, int F, int H, int k, const float* const* mlp, const double* pu,
                int prec, double dist_unit, double* mu, double* cov, double* rgb, double* alpha,
                double* alpha_pre) {
    const int C[3] = {1, 3, 7};
    const int NI = dist_unit > 0.0 ? F + 4 : F + 3;  /* inputs per anchor */
    double* W1[3];
    double* W2[3];
    for (int h = 0; h < 3; ++h) {
        W1[h] = (double*)malloc(sizeof(double) * H * NI);
        W2[h] = (double*)malloc(sizeof(double) * C[h] * k * H);
        quantise_weights(mlp[4 * h + 0], H, NI, prec, W1[h]);
        quantise_weights(mlp[4 * h + 2], C[h] * k, H, prec, W2[h]);
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < m; ++i) {
        int64_t a = ids[i];
        double x[3] = {pos[3 * a], pos[3 * a + 1], pos[3 * a + 2]};
        double v[3] = {x[0] - pu[0], x[1] - pu[1], x[2] - pu[2]};
        double nv = norm3(v);
        double* z = (double*)malloc(sizeof(double) * NI);
        double* hid = (double*)malloc(sizeof(double) * H);
        double* o[3];
        for (int f = 0; f < F; ++f) z[f] = feat[a * F + f];
        for (int c = 0; c < 3; ++c) z[F + c] = v[c] / nv;
        if (NI == F + 4) z[F + 3] = nv / dist_unit;
        if (prec) for (int f = 0; f < NI; ++f) z[f] = orc_round_bf16(z[f]);
        for (int h = 0; h < 3; ++h) {
            const float* b1 = mlp[4 * h + 1];
            const float* b2 = mlp[4 * h + 3];
            o[h] = (double*)malloc(sizeof(double) * C[h] * k);
            for (int r = 0; r < H; ++r) {
                double acc = 0.0;
                for (int c = 0; c < NI; ++c) acc += W1[h][r * NI + c] * z[c];
                acc += b1[r];
                hid[r] = acc > 0.0 ? acc : 0.0;
                if (prec) hid[r] = orc_round_bf16(hid[r]);
            }
            for (int r = 0; r < C[h] * k; ++r) {
                double acc = 0.0;
                for (int c = 0; c < H; ++c) acc += W2[h][r * H + c] * hid[c];
                o[h][r] = acc + b2[r];
            }
        }
        const float* s = scale + 6 * a;
        for (int j = 0; j < k; ++j) {
            int64_t g = i * k + j;
            const float* O = offsets + (a * k + j) * 3;
            for (int c = 0; c < 3; ++c) mu[3 * g + c] = x[c] + (double)s[c] * (double)O[c];
            alpha_pre[g] = o[0][j];
            alpha[g] = tanh(o[0][j]);
            for (int c = 0; c < 3; ++c) rgb[3 * g + c] = sigmoid(o[1][3 * j + c]);
            double sc[3];
            for (int c = 0; c < 3; ++c) sc[c] = (double)s[3 + c] * sigmoid(o[2][7 * j + c]);
            double qw = o[2][7 * j + 3], qx = o[2][7 * j + 4], qy = o[2][7 * j + 5], qz = o[2][7 * j + 6];
            double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
            if (qn > 0.0) { qw /= qn; qx /= qn; qy /= qn; qz /= qn; }
            else { qw = 1.0; qx = qy = qz = 0.0; }
            double R[3][3] = {
                {1.0 - 2.0 * (qy * qy + qz * qz), 2.0 * (qx * qy - qw * qz), 2.0 * (qx * qz + qw * qy)},
                {2.0 * (qx * qy + qw * qz), 1.0 - 2.0 * (qx * qx + qz * qz), 2.0 * (qy * qz - qw * qx)},
                {2.0 * (qx * qz - qw * qy), 2.0 * (qy * qz + qw * qx), 1.0 - 2.0 * (qx * qx + qy * qy)}};
            double S[3][3];
            for (int r = 0; r < 3; ++r)
                for (int c = 0; c < 3; ++c) {
                    double acc = 0.0;
                    for (int l = 0; l < 3; ++l) acc += R[r][l] * sc[l] * sc[l] * R[c][l];
                    S[r][c] = acc;
                }
            double* cv = cov + 6 * g;
            cv[0] = S[0][0]; cv[1] = S[0][1]; cv[2] = S[0][2];
            cv[3] = S[1][1]; cv[4] = S[1][2]; cv[5] = S[2][2];
        }
        for (int h = 0; h < 3; ++h) free(o[h]);
        free(z);
        free(hid);
    }
    for (int h = 0; h < 3; ++h) { free(W1[h]); free(W2[h]); }
}

/* ---------------------------------------------------------- projection */
/* EWA splatting (Section 3.1) with the documented constants.  Per Gaussian:
 *   t = R_e (mu - p_e); cull if t_z <= znear
 *   J = [[fx/tz, 0, -fx tx'/tz^2], [0, fy/tz, -fy ty'/tz^2]], with tx'/tz and
 *       ty'/tz clamped to +-1.3 tan(fov/2)
 *   Sigma2D = J R_e Sigma R_e^T J^T + 0.3 I; cull if det <= 0
 *   conic = Sigma2D^-1; mean2D = (fx tx/tz + W/2, fy ty/tz + H/2)
 *   cull if alpha < 1/255; depth = t_z
 * Outputs per Gaussian: mean2d[2], conic[3] (a b c of [[a b][b c]]),
 * sigma2d[3], depth, keep; band = 1 if the alpha or near test is marginal. */
void orc_preprocess(int64_t n, const double* mu, const double* cov, const double* alpha,
                    const orc_camera* e, double* mean2d, double* conic, double* sigma2d,
                    double* depth, uint8_t* keep, uint8_t* band) {
    double fx = e->width / (2.0 * tan(0.5 * e->fovx));
    double fy = e->height / (2.0 * tan(0.5 * e->fovy));
    double limx = 1.3 * tan(0.5 * e->fovx), limy = 1.3 * tan(0.5 * e->fovy);
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < n; ++g) {
        double t[3];
        to_camera(e, mu + 3 * g, t);
        keep[g] = 0;
        band[g] = 0;
        depth[g] = t[2];
        if (fabs(t[2] - e->znear) < 1e-6 * (fabs(t[2]) + 1.0)) band[g] = 1;
        if (fabs(alpha[g] - 1.0 / 255.0) < 1e-6) band[g] = 1;
        if (!(t[2] > e->znear)) continue;
        double rx = t[0] / t[2], ry = t[1] / t[2];
        rx = rx < -limx ? -limx : (rx > limx ? limx : rx);
        ry = ry < -limy ? -limy : (ry > limy ? limy : ry);
        double J[2][3] = {{fx / t[2], 0.0, -fx * rx / t[2]}, {0.0, fy / t[2], -fy * ry / t[2]}};
        const double* c = cov + 6 * g;
        double S[3][3] = {{c[0], c[1], c[2]}, {c[1], c[3], c[4]}, {c[2], c[4], c[5]}};
        double T[2][3];
        for (int r = 0; r < 2; ++r)
            for (int k = 0; k < 3; ++k) {
                double acc = 0.0;
                for (int l = 0; l < 3; ++l) acc += J[r][l] * e->R[3 * l + k];
                T[r][k] = acc;
            }
        double M[2][2];
        for (int r = 0; r < 2; ++r)
            for (int s = 0; s < 2; ++s) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) acc += T[r][k] * S[k][l] * T[s][l];
                M[r][s] = acc;
            }
        double a = M[0][0] + 0.3, b = M[0][1], cc = M[1][1] + 0.3;
        double det = a * cc - b * b;
        if (!(det > 0.0)) continue;
        if (!(alpha[g] >= 1.0 / 255.0)) continue;
        conic[3 * g] = cc / det;
        conic[3 * g + 1] = -b / det;
        conic[3 * g + 2] = a / det;
        sigma2d[3 * g] = a;
        sigma2d[3 * g + 1] = b;
        sigma2d[3 * g + 2] = cc;
        mean2d[2 * g] = fx * t[0] / t[2] + 0.5 * e->width;
        mean2d[2 * g + 1] = fy * t[1] / t[2] + 0.5 * e->height;
        keep[g] = 1;
    }
}

/* --------------------------------------------------------- tile lists */
/* Opacity-aware exact tile coverage (Section 6).  The Gaussian's footprint is
 * the set where alpha * exp(-q/2) >= 1/255, i.e. q <= 2 ln(255 alpha), with
 * q(p) = (p - m)^T conic (p - m).  A 16x16 tile is listed iff the minimum of q
 * over the rectangle spanned by its pixel centres is within that bound.
 * Because q is convex, the minimum is 0 when m lies in the rectangle and
 * otherwise lies on one of the four edges (a 1-D quadratic, clamped). */
static double edge_min(double a, double b, double c, double fixed_d, double lo, double hi, int fixed_is_x) {
    /* minimise q over a segment where one coordinate offset is fixed */
    double best;
    if (fixed_is_x) {       /* dx fixed, free dy in [lo, hi]: q = a dx^2 + 2 b dx dy + c dy^2 */
        double dy = -b * fixed_d / c;
        dy = dy < lo ? lo : (dy > hi ? hi : dy);
        best = a * fixed_d * fixed_d + 2.0 * b * fixed_d * dy + c * dy * dy;
    } else {                /* dy fixed, free dx */
        double dx = -b * fixed_d / a;
        dx = dx < lo ? lo : (dx > hi ? hi : dx);
        best = a * dx * dx + 2.0 * b * dx * fixed_d + c * fixed_d * fixed_d;
    }
    return best;
}

double orc_rect_min_q(double mx, double my, double a, double b, double c, double x0, double x1, double y0,
                      double y1) {
    if (mx >= x0 && mx <= x1 && my >= y0 && my <= y1) return 0.0;
    double q = edge_min(a, b, c, x0 - mx, y0 - my, y1 - my, 1);
    double q2 = edge_min(a, b, c, x1 - mx, y0 - my, y1 - my, 1);
    if (q2 < q) q = q2;
    q2 = edge_min(a, b, c, y0 - my, x0 - mx, x1 - mx, 0);
    if (q2 < q) q = q2;
    q2 = edge_min(a, b, c, y1 - my, x0 - mx, x1 - mx, 0);
    if (q2 < q) q = q2;
    return q;
}

/* Screen-position resolution of a float32 implementation at (mx, my) in a
 * W x H image: two float32 ulps of the coordinate scale |mx| + |my| + W + H.
 * A float32 pixel coordinate is rounded once itself, and the camera
 * transform, the division by depth and the focal scaling before it round
 * at scales no larger than that (far Gaussians near x = 2000 px resolve only
 * ~1e-4 px).  A decision whose margin in q is below |grad q| * delta (at
 * most 2 sqrt(q (a + c)) * delta, a + c bounding the conic's largest
 * eigenvalue) can go either way in float32 and is marginal. */
static double pos_delta(double mx, double my, int W, int H) {
    return ldexp(fabs(mx) + fabs(my) + (double)W + (double)H, -23);
}

/* Candidate tiles come from the ellipse's bounding box (half extents
 * sqrt(tau * Sigma2D_xx), sqrt(tau * Sigma2D_yy)) padded by one pixel, so the
 * exact test alone decides.  Emission order: g ascending, tiles row-major.
 * flags: bit0 = listed, bit1 = |min q - tau| within 1e-5 relative plus the
 * change the float32 screen position allows (pos_delta) (band).
 * Pairs are written when listed or in band.  Returns the number written, or
 * the negative of the number needed when cap is too small. */
static int64_t tiles_of(double mx, double my, const double* cn, const double* sg, double al, int W, int H,
                        int32_t* tile, uint8_t* flags, int64_t cap) {
    int ntx = (W + ORC_TILE - 1) / ORC_TILE, nty = (H + ORC_TILE - 1) / ORC_TILE;
    double tau = 2.0 * log(255.0 * al);
    if (tau < 0.0) tau = 0.0;
    double ex = sqrt(tau * sg[0]) + 1.0, ey = sqrt(tau * sg[2]) + 1.0;
    int tx0 = (int)floor((mx - ex - 0.5) / ORC_TILE), tx1 = (int)floor((mx + ex - 0.5) / ORC_TILE);
    int ty0 = (int)floor((my - ey - 0.5) / ORC_TILE), ty1 = (int)floor((my + ey - 0.5) / ORC_TILE);
    if (tx0 < 0) tx0 = 0;
    if (ty0 < 0) ty0 = 0;
    if (tx1 > ntx - 1) tx1 = ntx - 1;
    if (ty1 > nty - 1) ty1 = nty - 1;
    int64_t cnt = 0;
    const double qband = 1e-5 * (tau + 1.0) + 2.0 * sqrt(tau * (cn[0] + cn[2])) * pos_delta(mx, my, W, H);
    for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx) {
            double x0 = ORC_TILE * tx + 0.5, y0 = ORC_TILE * ty + 0.5;
            double x1 = (ORC_TILE * tx + ORC_TILE - 1 < W - 1 ? ORC_TILE * tx + ORC_TILE - 1 : W - 1) + 0.5;
            double y1 = (ORC_TILE * ty + ORC_TILE - 1 < H - 1 ? ORC_TILE * ty + ORC_TILE - 1 : H - 1) + 0.5;
            double q = orc_rect_min_q(mx, my, cn[0], cn[1], cn[2], x0, x1, y0, y1);
            int listed = q <= tau;
            int bnd = fabs(q - tau) <= qband;
            if (listed || bnd) {
                if (tile && cnt < cap) {
                    tile[cnt] = ty * ntx + tx;
                    flags[cnt] = (uint8_t)(listed | (bnd << 1));
                }
                ++cnt;
            }
        }
    return cnt;
}

int64_t orc_tile_pairs(int64_t n, const double* mean2d, const double* conic, const double* sigma2d,
                       const double* alpha, const uint8_t* keep, int W, int H, int64_t cap,
                       int32_t* out_tile, int32_t* out_g, uint8_t* out_flags) {
    int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t g = 0; g < n; ++g)
        cnt[g] = keep[g] ? tiles_of(mean2d[2 * g], mean2d[2 * g + 1], conic + 3 * g, sigma2d + 3 * g,
                                    alpha[g], W, H, NULL, NULL, 0)
                         : 0;
    int64_t total = 0;
    for (int64_t g = 0; g < n; ++g) {
        int64_t c = cnt[g];
        cnt[g] = total;
        total += c;
    }
    if (total > cap) {
        free(cnt);
        return -total;
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t g = 0; g < n; ++g) {
        if (!keep[g]) continue;
        int64_t off = cnt[g];
        int64_t c = tiles_of(mean2d[2 * g], mean2d[2 * g + 1], conic + 3 * g, sigma2d + 3 * g, alpha[g], W, H,
                             out_tile + off, out_flags + off, total - off);
        for (int64_t i = 0; i < c; ++i) out_g[off + i] = (int32_t)g;
    }
    free(cnt);
    return total;
}

/* --------------------------------------------------------------- sort */
/* Order pairs by (tile, float32(depth)) with ties kept in emission order.
 * The FP64 depth is rounded to float32 (nearest, ties to even) as the key. */
typedef struct {
    int32_t tile;
    float depth;
    int64_t idx;
} orc_key;

static int cmp_key(const void* pa, const void* pb) {
    const orc_key* a = (const orc_key*)pa;
    const orc_key* b = (const orc_key*)pb;
    if (a->tile != b->tile) return a->tile < b->tile ? -1 : 1;
    if (a->depth != b->depth) return a->depth < b->depth ? -1 : 1;
    return a->idx < b->idx ? -1 : (a->idx > b->idx ? 1 : 0);
}

void orc_sort_pairs(int64_t n, const int32_t* tile, const int32_t* g, const double* depth, int64_t* order) {
    orc_key* k = (orc_key*)malloc(sizeof(orc_key) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        k[i].tile = tile[i];
        k[i].depth = (float)depth[g[i]];
        k[i].idx = i;
    }
    qsort(k, (size_t)n, sizeof(orc_key), cmp_key);
    for (int64_t i = 0; i < n; ++i) order[i] = k[i].idx;
    free(k);
}

/* ------------------------------------------------------------- blend */
/* Front-to-back compositing per pixel centre p = (u + 0.5, v + 0.5) over its
 * tile's sorted list:
 *   T = 1, C = 0; for each g: q = d^T conic d (d = p - mean2D);
 *   alpha = min(0.99, alpha_g exp(-q/2)); skip if alpha < 1/255;
 *   stop (without adding g) if T (1 - alpha) < 1e-4;
 *   C += rgb_g alpha T;  T *= 1 - alpha.
 * Outputs planar RGB [3,H,W] (background 0), final T [H,W], and the number
 * of Gaussians added per pixel.  pix_band[p] = 1 when any decision at that
 * pixel is marginal: alpha vs 1/255 within alpha_band (1e-7; wider where the
 * opacities carry a weight computed in float32 on the other side) plus
 * alpha's change under the float32 screen-position resolution (pos_delta),
 * or q vs 2 ln(255 alpha_g) within the tile test's band; the stop test within
 * 1e-9 plus T times that change; two consecutive added Gaussians whose
 * depths are within 4 float32 ulps so their order is not fixed by float32
 * keys; or a marginal pair the tile test left out (ghost_*: per-tile ranges
 * into ghost_g, may be NULL) reaching the threshold at the pixel. */
/* Is the alpha threshold of Gaussian g at a pixel with quadratic form q
 * marginal?  In q: alpha_g exp(-q/2) >= 1/255 <=> q <= tau = 2 ln(255
 * alpha_g), the tile test's inequality at the pixel, with the tile test's
 * band (1e-5 relative plus the float32 screen-position term). */
static int alpha_q_marginal(double q, double al, const double* cn, double mx, double my, int W, int H) {
    if (!(al > 0.0)) return 0;
    double tau = 2.0 * log(255.0 * al);
    double qband = 1e-5 * (fabs(tau) + 1.0) + 2.0 * sqrt(q * (cn[0] + cn[2])) * pos_delta(mx, my, W, H);
    return fabs(q - tau) <= qband;
}

void orc_blend(int W, int H, const int64_t* tile_start, const int64_t* tile_end, const int32_t* sorted_g,
               const double* mean2d, const double* conic, const double* alpha, const double* rgb,
               const double* depth, double* out_rgb, double* out_T, int32_t* n_contrib, uint8_t* pix_band,
               int32_t* n_eval, double alpha_band, const int64_t* ghost_start, const int64_t* ghost_end,
               const int32_t* ghost_g) {
    int ntx = (W + ORC_TILE - 1) / ORC_TILE;
    int64_t npx = (int64_t)W * H;
#pragma omp parallel for schedule(dynamic, 4)
    for (int v = 0; v < H; ++v)
        for (int u = 0; u < W; ++u) {
            int tile = (v / ORC_TILE) * ntx + (u / ORC_TILE);
            double px = u + 0.5, py = v + 0.5;
            double T = 1.0, C[3] = {0.0, 0.0, 0.0};
            int32_t nc = 0, ne = 0;
            uint8_t bnd = 0;
            double prev_depth = -1.0;
            for (int64_t i = tile_start[tile]; i < tile_end[tile]; ++i) {
                int32_t g = sorted_g[i];
                ++ne; /* visited, whether it contributes, is skipped or ends the pixel */
                double dx = px - mean2d[2 * g], dy = py - mean2d[2 * g + 1];
                const double* cn = conic + 3 * g;
                double q = cn[0] * dx * dx + 2.0 * cn[1] * dx * dy + cn[2] * dy * dy;
                double a = alpha[g] * exp(-0.5 * q);
                if (a > 0.99) a = 0.99;
                /* alpha's uncertainty from the float32 screen position */
                double da = a * sqrt(q * (cn[0] + cn[2])) * pos_delta(mean2d[2 * g], mean2d[2 * g + 1], W, H);
                if (fabs(a - 1.0 / 255.0) < alpha_band + da ||
                    alpha_q_marginal(q, alpha[g], cn, mean2d[2 * g], mean2d[2 * g + 1], W, H))
                    bnd = 1;
                if (a < 1.0 / 255.0) continue;
                double tn = T * (1.0 - a);
                if (fabs(tn - 1e-4) < 1e-9 + T * da) bnd = 1;
                if (tn < 1e-4) break;
                float fd = (float)depth[g];
                if (prev_depth >= 0.0 && fabs(depth[g] - prev_depth) <= 4.0 * (nextafterf(fd, INFINITY) - fd))
                    bnd = 1;
                prev_depth = depth[g];
                for (int c = 0; c < 3; ++c) C[c] += rgb[3 * g + c] * a * T;
                T = tn;
                ++nc;
            }
            /* marginal pairs the tile test left out: the other side may list
             * them, and then composites them wherever alpha reaches 1/255 */
            if (ghost_start)
                for (int64_t i = ghost_start[tile]; i < ghost_end[tile] && !bnd; ++i) {
                    int32_t g = ghost_g[i];
                    double dx = px - mean2d[2 * g], dy = py - mean2d[2 * g + 1];
                    const double* cn = conic + 3 * g;
                    double q = cn[0] * dx * dx + 2.0 * cn[1] * dx * dy + cn[2] * dy * dy;
                    double a = alpha[g] * exp(-0.5 * q);
                    if (a >= 1.0 / 255.0 - alpha_band ||
                        alpha_q_marginal(q, alpha[g], cn, mean2d[2 * g], mean2d[2 * g + 1], W, H))
                        bnd = 1;
                }
            int64_t p = (int64_t)v * W + u;
            for (int c = 0; c < 3; ++c) out_rgb[c * npx + p] = C[c];
            out_T[p] = T;
            n_contrib[p] = nc;
            pix_band[p] = bnd;
            n_eval[p] = ne;
        }
}

/* Threads the parallel loops above run on (1 without OpenMP). */
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Sets the thread count of the parallel loops above (for timing the oracle
   on a given number of host cores); n <= 0 leaves it unchanged. */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
