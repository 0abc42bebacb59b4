/*
 * ivrgs_oracle.c -- CPU reference of the editable-Gaussian rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously-correct
 * definition that the HIP path is checked against.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark load it.  It shares no
 * code with the HIP library.
 *
 * Arithmetic is FP64, except the depth sort key, which both sides round to
 * FP32 step by step (no fused multiply-add) so that the front-to-back order is
 * bit-identical.  Build with -ffp-contract=off.
 *
 * What is computed (paper sections/equations):
 *   - 3D Gaussian, covariance from rotation and scale (Sec. 3, Eq. 1):
 *       Sigma = R(q) diag(s)^2 R(q)^T.
 *   - EWA projection (Sec. 3): Sigma' = J W Sigma W^T J^T, with J the Jacobian
 *     of the perspective map at the camera-space mean, plus a screen-space
 *     low-pass eps*I (a reading; the paper only says "approximated as").
 *   - Blinn-Phong colour per Gaussian (Sec. 3, Eq. 3; Sec. 4.3):
 *       c' = k_a c_v + k_d c_v |n.l| + k_s |n.h|^beta [|n.l| > 0] (1,1,1),
 *     with I_a = I_d = c_v, I_s = white, h = (v+l)/|v+l|, v the unit direction
 *     from the Gaussian to the camera, l = v for the headlight or the model's
 *     orbital light direction (Sec. 3, the two light kinds).
 *   - Front-to-back compositing sorted by depth (Sec. 3, Eq. 2):
 *       C = sum_i T_i alpha_i c_i,  T_i = prod_{j<i} (1 - alpha_j),
 *       alpha = o * G (the 2D Gaussian at the pixel).
 *     Readings (the paper is silent): alpha is capped at alpha_max, skipped
 *     below alpha_min, and the pass stops before a Gaussian that would drop the
 *     transmittance below T_min.  The image is RGB = C + T_final * bg and the
 *     alpha channel A = sum_i T_i alpha_i (the alpha channel is supervised in
 *     Sec. 4.2).
 *   - Backward: the exact gradient of a linear functional of RGBA, analytic
 *     for the compositing (back-to-front suffix sums) and, per Gaussian, the
 *     Jacobian of the projection computed by complex-step differentiation of
 *     the same complex-valued projection code (no hand-derived chain rule).
 *
 * A per-Gaussian pixel box prunes the per-pixel loop.  It is conservative
 * (every pixel with alpha >= alpha_min lies inside it, plus a 2 px margin);
 * the test-suite proves pruning changes nothing against a brute-force
 * evaluation of every Gaussian at every pixel.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* ---------------------------------------------------------------- inputs */
typedef struct {
    int64_t n;
    const float *mean;      /* [3][n] */
    const float *log_scale; /* [3][n] */
    const float *quat;      /* [4][n]  (w, x, y, z), not necessarily unit */
    const float *opacity;   /* [1][n]  used as given */
    const float *normal;    /* [3][n]  not necessarily unit */
    const float *color;     /* [3][n]  render-ready voxel colour c_v */
    const float *shade;     /* [4][n]  k_a, k_d, k_s, beta */
    const int32_t *model_id;/* [n] or NULL (all model 0) */
} og_gauss;

typedef struct { float R[9], t[3], fx, fy, cx, cy; } og_camera;

typedef struct {
    double alpha_min, alpha_max, T_min, lowpass, z_near;
    double bg[3];
    int32_t width, height;
} og_params;

/* Per-Gaussian projection record (real parts). */
enum {
    P_VALID = 0, P_Z32, P_MX, P_MY, P_COV00, P_COV01, P_COV11,
    P_Q00, P_Q01, P_Q11, P_O, P_R, P_G, P_B, P_EXTX, P_EXTY,
    P_TX, P_TY, P_TZ, P_NL, P_NH, P_DM, P_KAPPA, P_ERGB, P_WIDTH
};
/* The nine differentiable record values, in this order. */
enum { R_MX = 0, R_MY, R_Q00, R_Q01, R_Q11, R_O, R_CR, R_CG, R_CB, R_N };
#define N_PARAM 21

/* Gaussian parameters as one vector of 21: mean 3, log_scale 3, quat 4,
 * opacity 1, normal 3, color 3, shade 4 (the order of the planes). */
static void gather_params(const og_gauss *g, int64_t i, double p[N_PARAM])
{
    int64_t n = g->n;
    int k = 0;
    for (int c = 0; c < 3; ++c) p[k++] = g->mean[c * n + i];
    for (int c = 0; c < 3; ++c) p[k++] = g->log_scale[c * n + i];
    for (int c = 0; c < 4; ++c) p[k++] = g->quat[c * n + i];
    p[k++] = g->opacity[i];
    for (int c = 0; c < 3; ++c) p[k++] = g->normal[c * n + i];
    for (int c = 0; c < 3; ++c) p[k++] = g->color[c * n + i];
    for (int c = 0; c < 4; ++c) p[k++] = g->shade[c * n + i];
}

/* Depth sort key: camera-space z of the mean, each product and sum rounded
 * to FP32 in this order: ((R20*x + R21*y) + R22*z) + t2. */
static float depth_key(const og_camera *cam, float x, float y, float z)
{
    float a = cam->R[6] * x;
    float b = cam->R[7] * y;
    float c = cam->R[8] * z;
    float s = a + b;
    s = s + c;
    s = s + cam->t[2];
    return s;
}

/* |x| continued analytically for the complex step: sign taken from Re x. */
static cplx cabs_cs(cplx x) { return creal(x) < 0.0 ? -x : x; }

static cplx csqrt_pos(cplx x) { return csqrt(x); }

/* Unit quaternion (w, x, y, z) -> rotation matrix (row-major), the textbook
 * formula for R(q) v = q v q^*. */
static void quat_rot(const cplx q[4], cplx R[9])
{
    cplx w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

/*
 * Project one Gaussian.  p: 21 parameters (complex for the complex step).
 * light: row of the model edit table (dir at [12..14], headlight flag bits
 * at [15]); ldir, when not NULL, replaces the row's (unnormalised) orbital
 * light direction, so that the complex step can differentiate with respect
 * to it.  Writes the nine record values to rec and, when aux != NULL, the
 * real-valued diagnostics (P_* layout).  Returns 1 if the Gaussian is kept.
 */
static int project_one(const cplx p[N_PARAM], float z32, const og_camera *cam,
                       const float *light, const cplx *ldir, const og_params *prm, cplx rec[R_N],
                       double *aux)
{
    const cplx *mu = p + 0, *ls = p + 3, *q = p + 6, *op = p + 10;
    const cplx *nrm = p + 11, *col = p + 14, *shd = p + 17;
    int valid = 1;

    /* covariance Sigma = R diag(s^2) R^T (Sec. 3) */
    cplx s[3];
    for (int k = 0; k < 3; ++k) s[k] = cexp(ls[k]);
    cplx qn = csqrt_pos(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    cplx qu[4];
    for (int k = 0; k < 4; ++k) qu[k] = q[k] / qn;
    cplx Rq[9];
    quat_rot(qu, Rq);
    cplx Sig[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += Rq[i * 3 + k] * s[k] * s[k] * Rq[j * 3 + k];
            Sig[i * 3 + j] = acc;
        }

    /* camera-space mean t = W mu + t_wc */
    double W[9];
    for (int k = 0; k < 9; ++k) W[k] = cam->R[k];
    cplx t[3];
    for (int i = 0; i < 3; ++i)
        t[i] = W[i * 3 + 0] * mu[0] + W[i * 3 + 1] * mu[1] + W[i * 3 + 2] * mu[2] + (double)cam->t[i];
    if (!((double)z32 > prm->z_near)) valid = 0;

    /* EWA: J at the mean, Sigma' = (J W) Sigma (J W)^T + eps I */
    double fx = cam->fx, fy = cam->fy;
    cplx J[6];
    J[0] = fx / t[2]; J[1] = 0.0; J[2] = -fx * t[0] / (t[2] * t[2]);
    J[3] = 0.0; J[4] = fy / t[2]; J[5] = -fy * t[1] / (t[2] * t[2]);
    cplx T[6];
    for (int a = 0; a < 2; ++a)
        for (int j = 0; j < 3; ++j) {
            cplx acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += J[a * 3 + k] * W[k * 3 + j];
            T[a * 3 + j] = acc;
        }
    cplx S2[4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            cplx acc = 0.0;
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) acc += T[a * 3 + i] * Sig[i * 3 + j] * T[b * 3 + j];
            S2[a * 2 + b] = acc + (a == b ? prm->lowpass : 0.0);
        }
    cplx det = S2[0] * S2[3] - S2[1] * S2[2];
    if (!(creal(det) > 0.0)) valid = 0;
    cplx Q00 = S2[3] / det, Q01 = -S2[1] / det, Q11 = S2[0] / det;
    cplx mx = fx * t[0] / t[2] + (double)cam->cx;
    cplx my = fy * t[1] / t[2] + (double)cam->cy;

    /* Blinn-Phong colour (Eq. 3), I_a = I_d = c_v, I_s = white */
    double cc[3];
    {
        /* camera centre c = -W^T t_wc */
        for (int i = 0; i < 3; ++i)
            cc[i] = -(W[0 * 3 + i] * cam->t[0] + W[1 * 3 + i] * cam->t[1] + W[2 * 3 + i] * cam->t[2]);
    }
    cplx v[3];
    cplx vd[3] = {cc[0] - mu[0], cc[1] - mu[1], cc[2] - mu[2]};
    cplx vn = csqrt_pos(vd[0] * vd[0] + vd[1] * vd[1] + vd[2] * vd[2]);
    for (int k = 0; k < 3; ++k) v[k] = vd[k] / vn;
    cplx l[3];
    int32_t head;
    memcpy(&head, &light[15], sizeof(head));
    if (head) {
        for (int k = 0; k < 3; ++k) l[k] = v[k];
    } else if (ldir) {
        cplx ln = csqrt_pos(ldir[0] * ldir[0] + ldir[1] * ldir[1] + ldir[2] * ldir[2]);
        for (int k = 0; k < 3; ++k) l[k] = ldir[k] / ln;
    } else {
        double ln = sqrt((double)light[12] * light[12] + (double)light[13] * light[13] +
                         (double)light[14] * light[14]);
        for (int k = 0; k < 3; ++k) l[k] = (double)light[12 + k] / ln;
    }
    cplx nn = csqrt_pos(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
    cplx nu[3];
    for (int k = 0; k < 3; ++k) nu[k] = nrm[k] / nn;
    cplx nl = nu[0] * l[0] + nu[1] * l[1] + nu[2] * l[2];
    cplx hv[3] = {v[0] + l[0], v[1] + l[1], v[2] + l[2]};
    cplx hn = csqrt_pos(hv[0] * hv[0] + hv[1] * hv[1] + hv[2] * hv[2]);
    cplx spec = 0.0;
    cplx nh = 0.0;
    if (creal(hn) > 0.0) {
        for (int k = 0; k < 3; ++k) nh += nu[k] * (hv[k] / hn);
        cplx a = cabs_cs(nh);
        if (creal(cabs_cs(nl)) > 0.0 && creal(a) > 0.0)
            spec = shd[2] * cexp(shd[3] * clog(a));
    }
    cplx anl = cabs_cs(nl);
    cplx rgb[3];
    for (int c = 0; c < 3; ++c) rgb[c] = shd[0] * col[c] + shd[1] * col[c] * anl + spec;

    rec[R_MX] = mx; rec[R_MY] = my;
    rec[R_Q00] = Q00; rec[R_Q01] = Q01; rec[R_Q11] = Q11;
    rec[R_O] = op[0];
    rec[R_CR] = rgb[0]; rec[R_CG] = rgb[1]; rec[R_CB] = rgb[2];

    for (int k = 0; k < R_N; ++k)
        if (!isfinite(creal(rec[k]))) valid = 0;

    if (aux) {
        aux[P_VALID] = valid;
        aux[P_Z32] = (double)z32;
        aux[P_MX] = creal(mx); aux[P_MY] = creal(my);
        aux[P_COV00] = creal(S2[0]); aux[P_COV01] = creal(S2[1]); aux[P_COV11] = creal(S2[3]);
        aux[P_Q00] = creal(Q00); aux[P_Q01] = creal(Q01); aux[P_Q11] = creal(Q11);
        aux[P_O] = creal(op[0]);
        aux[P_R] = creal(rgb[0]); aux[P_G] = creal(rgb[1]); aux[P_B] = creal(rgb[2]);
        /* conservative pixel half-extent of {alpha >= alpha_min}:
         * o G >= alpha_min  <=>  d^T Q d <= 2 ln(o / alpha_min); the
         * axis-aligned box of that ellipse has half-widths k sqrt(Sigma'_aa). */
        double o = creal(op[0]);
        if (valid && o >= prm->alpha_min) {
            double k2 = 2.0 * log(o / prm->alpha_min);
            if (k2 < 0.0) k2 = 0.0;
            aux[P_EXTX] = sqrt(k2 * creal(S2[0])) + 2.0;
            aux[P_EXTY] = sqrt(k2 * creal(S2[3])) + 2.0;
        } else {
            aux[P_EXTX] = -1.0;
            aux[P_EXTY] = -1.0;
        }
        aux[P_TX] = creal(t[0]); aux[P_TY] = creal(t[1]); aux[P_TZ] = creal(t[2]);
        aux[P_NL] = creal(nl); aux[P_NH] = creal(nh);
        /* FP32 error model inputs of a kernel that computes in single
         * precision: the screen mean carries about one unit in the last place
         * of the larger coordinate; kappa is the condition number of Sigma'. */
        {
            float big = (float)fmax(fabs(creal(mx)), fabs(creal(my)));
            aux[P_DM] = (double)(nextafterf(big, INFINITY) - big) + 1e-6;
            double a2 = creal(S2[0]), b2 = creal(S2[1]), c2 = creal(S2[3]);
            double mid = 0.5 * (a2 + c2), rad = sqrt(0.25 * (a2 - c2) * (a2 - c2) + b2 * b2);
            aux[P_KAPPA] = (mid - rad) > 0.0 ? (mid + rad) / (mid - rad) : 1e30;
        }
        /* Bound on the FP32 error of the colour: about 1e-6 relative, plus the
         * specular lobe's sensitivity k_s beta |n.h|^(beta-1) times a 4e-7
         * error in n.h, plus the whole lobe when |n.l| is too close to 0 for
         * the [|n.l| > 0] gate to be decided in FP32. */
        {
            double ahv = fabs(creal(nh)), anlv = fabs(creal(nl));
            double ks = creal(shd[2]), be = creal(shd[3]);
            double big = fmax(fabs(creal(rgb[0])), fmax(fabs(creal(rgb[1])), fabs(creal(rgb[2]))));
            double e = 1e-6 * (big + 1.0);
            if (creal(spec) != 0.0 && ahv > 0.0) e += ks * be * pow(ahv, be - 1.0) * 4e-7;
            if (anlv < 1e-6 && ahv > 0.0) e += fabs(ks) * pow(ahv, be);
            aux[P_ERGB] = e;
        }
    }
    return valid;
}

static const float *light_row(const og_gauss *g, const float *edits, int n_models, int64_t i)
{
    int m = g->model_id ? g->model_id[i] : 0;
    if (m < 0 || m >= n_models) m = 0;
    return edits + 16 * (int64_t)m;
}

static int project_real(const og_gauss *g, const float *edits, int n_models,
                        const og_camera *cam, const og_params *prm, int64_t i,
                        double *aux)
{
    double pr[N_PARAM];
    cplx p[N_PARAM], rec[R_N];
    gather_params(g, i, pr);
    for (int k = 0; k < N_PARAM; ++k) p[k] = pr[k];
    float z32 = depth_key(cam, g->mean[i], g->mean[g->n + i], g->mean[2 * g->n + i]);
    for (int k = 0; k < N_PARAM; ++k)
        if (!isfinite(pr[k])) {
            memset(aux, 0, sizeof(double) * P_WIDTH);
            aux[P_EXTX] = aux[P_EXTY] = -1.0;
            return 0;
        }
    return project_one(p, z32, cam, light_row(g, edits, n_models, i), NULL, prm, rec, aux);
}

/* Exported: per-Gaussian projection diagnostics, out[n][P_WIDTH]. */
int og_project(const og_gauss *g, const float *edits, int n_models, const og_camera *cam,
               const og_params *prm, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < g->n; ++i) project_real(g, edits, n_models, cam, prm, i, out + i * P_WIDTH);
    return 0;
}

/* Exported: the 9x21 Jacobian d(record)/d(params) of one Gaussian by the
 * complex step, jac[9][21].  Returns the valid flag. */
int og_jacobian(const og_gauss *g, const float *edits, int n_models, const og_camera *cam,
                const og_params *prm, int64_t i, double *jac)
{
    double pr[N_PARAM];
    gather_params(g, i, pr);
    float z32 = depth_key(cam, g->mean[i], g->mean[g->n + i], g->mean[2 * g->n + i]);
    const float *lr = light_row(g, edits, n_models, i);
    int valid = 1;
    for (int k = 0; k < N_PARAM; ++k) {
        cplx p[N_PARAM], rec[R_N];
        double h = 1e-30 * (fabs(pr[k]) > 1.0 ? fabs(pr[k]) : 1.0);
        for (int j = 0; j < N_PARAM; ++j) p[j] = pr[j];
        p[k] = pr[k] + I * h;
        valid = project_one(p, z32, cam, lr, NULL, prm, rec, NULL);
        for (int r = 0; r < R_N; ++r) jac[r * N_PARAM + k] = cimag(rec[r]) / h;
    }
    return valid;
}

/* ------------------------------------------------------------- rendering */
typedef struct { float z; int64_t idx; } key_t_;

static int cmp_key(const void *a, const void *b)
{
    const key_t_ *x = a, *y = b;
    if (x->z < y->z) return -1;
    if (x->z > y->z) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

/* Kept Gaussians sorted by (depth key, index), ascending. */
static int64_t sorted_order(const double *proj, int64_t n, int64_t *order)
{
    key_t_ *keys = malloc(sizeof(key_t_) * (n > 0 ? n : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i)
        if (proj[i * P_WIDTH + P_VALID] != 0.0) {
            keys[m].z = (float)proj[i * P_WIDTH + P_Z32];
            keys[m].idx = i;
            ++m;
        }
    qsort(keys, m, sizeof(key_t_), cmp_key);
    for (int64_t k = 0; k < m; ++k) order[k] = keys[k].idx;
    free(keys);
    return m;
}

/* Decision flags of a pixel (bit set = the FP32 result may take the other
 * branch, by the error model below). */
enum { AMB_ALPHA_MIN = 1, AMB_T_MIN = 2, AMB_ALPHA_MAX = 4, AMB_SHADE = 8, AMB_MANY = 16 };
enum { GATE_ALPHA = 1, GATE_T = 2 };
#define MAX_AMB 8

typedef struct {
    int64_t k;   /* position in the sorted order */
    int gate;    /* GATE_ALPHA or GATE_T */
} dec_t;

typedef struct {
    int64_t idx;
    double alpha, raw, G, T, dx, dy;
} hit_t;

static int flipped(const dec_t *flips, int nflips, int64_t k, int gate)
{
    for (int i = 0; i < nflips; ++i)
        if (flips[i].k == k && flips[i].gate == gate) return 1;
    return 0;
}

/*
 * Composite one pixel front to back.  Fills hits (the composited list) when
 * non-NULL (capacity m).  flips: decisions to take the other way.  amb (when
 * non-NULL, capacity MAX_AMB): receives the decisions that an FP32
 * evaluation could take the other way, by the error model
 *   |ln alpha error| <= 2e-6 + (3e-7 kappa + 2e-6) |power| + |Q d|_1 dm
 * (dm, kappa per Gaussian), and for the transmittance the running sum of
 * alpha/(1-alpha) times those bounds.  Returns the number composited.
 */
static int64_t composite_pixel(const double *proj, const int64_t *order, int64_t m,
                               const og_params *prm, double px, double py, int use_box,
                               const dec_t *flips, int nflips, double rgba[4], double *T_final,
                               int *flags, hit_t *hits, int64_t *evaluated, dec_t *amb, int *namb)
{
    double T = 1.0, C[3] = {0, 0, 0}, A = 0.0, eT = 0.0, eshade = 0.0;
    int64_t nh = 0, ev = 0;
    int fl = 0, na = 0;
    for (int64_t k = 0; k < m; ++k) {
        const double *g = proj + order[k] * P_WIDTH;
        double dx = px - g[P_MX], dy = py - g[P_MY];
        if (use_box && (fabs(dx) > g[P_EXTX] || fabs(dy) > g[P_EXTY])) continue;
        ++ev;
        double power = -0.5 * (g[P_Q00] * dx * dx + 2.0 * g[P_Q01] * dx * dy + g[P_Q11] * dy * dy);
        double G = exp(power);
        double raw = g[P_O] * G;
        double alpha = raw < prm->alpha_max ? raw : prm->alpha_max;
        double qdx = g[P_Q00] * dx + g[P_Q01] * dy, qdy = g[P_Q01] * dx + g[P_Q11] * dy;
        double ea = 2e-6 + (3e-7 * g[P_KAPPA] + 2e-6) * fabs(power) + (fabs(qdx) + fabs(qdy)) * g[P_DM];
        int pass = alpha >= prm->alpha_min;
        if (alpha > 0.0 && fabs(log(alpha / prm->alpha_min)) <= ea) {
            fl |= AMB_ALPHA_MIN;
            if (amb && na < MAX_AMB) amb[na] = (dec_t){k, GATE_ALPHA};
            ++na;
        }
        if (flips && flipped(flips, nflips, k, GATE_ALPHA)) pass = !pass;
        if (!pass) continue;
        if (raw > 0.0 && fabs(log(raw / prm->alpha_max)) <= ea) fl |= AMB_ALPHA_MAX;
        double Tn = T * (1.0 - alpha);
        double eTn = eT + alpha / (1.0 - alpha) * ea + 2e-7;
        int stop = Tn < prm->T_min;
        if (fabs(log(Tn / prm->T_min)) <= eTn) {
            fl |= AMB_T_MIN;
            if (amb && na < MAX_AMB) amb[na] = (dec_t){k, GATE_T};
            ++na;
        }
        if (flips && flipped(flips, nflips, k, GATE_T)) stop = !stop;
        if (stop) break;
        double w = T * alpha;
        eshade += w * g[P_ERGB];
        C[0] += w * g[P_R];
        C[1] += w * g[P_G];
        C[2] += w * g[P_B];
        A += w;
        if (hits) {
            hits[nh].idx = order[k];
            hits[nh].alpha = alpha;
            hits[nh].raw = raw;
            hits[nh].G = G;
            hits[nh].T = T;
            hits[nh].dx = dx;
            hits[nh].dy = dy;
        }
        ++nh;
        T = Tn;
        eT = eTn;
    }
    if (eshade > 2e-5) fl |= AMB_SHADE;
    rgba[0] = C[0] + T * prm->bg[0];
    rgba[1] = C[1] + T * prm->bg[1];
    rgba[2] = C[2] + T * prm->bg[2];
    rgba[3] = A;
    if (T_final) *T_final = T;
    if (flags) *flags = fl;
    if (evaluated) *evaluated = ev;
    if (namb) *namb = na;
    return nh;
}

static void pixel_coords(const og_params *prm, const int32_t *pix, int64_t p, double *px, double *py)
{
    int64_t x, y;
    if (pix) { x = pix[2 * p]; y = pix[2 * p + 1]; }
    else { x = p % prm->width; y = p / prm->width; }
    *px = (double)x + 0.5;
    *py = (double)y + 0.5;
}

/*
 * Exported: render npix pixels (pix = [npix][2] of (x, y), or NULL for the
 * whole image in row-major order).  rgba: [npix][4].  flags: [npix] or NULL.
 * alt: [npix][3][4] or NULL, with n_alt [npix]: for a pixel with one or two
 * ambiguous decisions, the images obtained by flipping each non-empty subset
 * of them (1 or 3 alternatives); a pixel with more gets AMB_MANY and none.
 * maxw: [n] or NULL, the largest T*alpha each Gaussian reaches over the
 * rendered pixels.  stats[0] = composited pairs, stats[1] = Gaussians kept,
 * stats[2] = evaluated (in-box) pairs.  use_box = 0 evaluates every kept
 * Gaussian at every pixel.  proj_out: [n][P_WIDTH] or NULL.
 */
int og_render(const og_gauss *g, const float *edits, int n_models, const og_camera *cam,
              const og_params *prm, int64_t npix, const int32_t *pix, int use_box,
              double *rgba, int32_t *flags, double *alt, int32_t *n_alt, double *maxw,
              int64_t *stats, double *proj_out)
{
    int64_t n = g->n;
    double *proj = proj_out ? proj_out : malloc(sizeof(double) * P_WIDTH * (n > 0 ? n : 1));
    int64_t *order = malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    og_project(g, edits, n_models, cam, prm, proj);
    int64_t m = sorted_order(proj, n, order);
    if (maxw) for (int64_t i = 0; i < n; ++i) maxw[i] = 0.0;
    int64_t comp = 0, evald = 0;
#pragma omp parallel reduction(+ : comp, evald)
    {
        hit_t *hits = maxw ? malloc(sizeof(hit_t) * (m > 0 ? m : 1)) : NULL;
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < npix; ++p) {
            double px, py, Tf;
            int fl, na;
            int64_t ev;
            dec_t amb[MAX_AMB];
            pixel_coords(prm, pix, p, &px, &py);
            int64_t nh = composite_pixel(proj, order, m, prm, px, py, use_box, NULL, 0, rgba + 4 * p,
                                         &Tf, &fl, hits, &ev, amb, &na);
            comp += nh;
            evald += ev;
            int nalt = 0;
            if (na > 2) fl |= AMB_MANY;
            if (alt && na >= 1 && na <= 2) {
                for (int mask = 1; mask < (1 << na); ++mask) {
                    dec_t fl_set[2];
                    int nf = 0;
                    for (int b = 0; b < na; ++b)
                        if (mask & (1 << b)) fl_set[nf++] = amb[b];
                    composite_pixel(proj, order, m, prm, px, py, use_box, fl_set, nf,
                                    alt + (p * 3 + nalt) * 4, NULL, NULL, NULL, NULL, NULL, NULL);
                    ++nalt;
                }
            }
            if (n_alt) n_alt[p] = nalt;
            if (flags) flags[p] = fl;
            if (maxw)
                for (int64_t k = 0; k < nh; ++k) {
                    double w = hits[k].T * hits[k].alpha;
                    int64_t gi = hits[k].idx;
#pragma omp critical(og_maxw)
                    if (w > maxw[gi]) maxw[gi] = w;
                }
        }
        free(hits);
    }
    if (stats) { stats[0] = comp; stats[1] = m; stats[2] = evald; }
    free(order);
    if (!proj_out) free(proj);
    return 0;
}

/*
 * Exported: gradient of L = sum_p sum_c dl[p][c] * RGBA[p][c] over the given
 * pixels.  grad_rec: [n][9] gradient w.r.t. the record values (mx, my, Q00,
 * Q01, Q11, o, r, g, b), or NULL.  grad: [21][n] gradient w.r.t. the Gaussian
 * parameters (mean 3, log_scale 3, quat 4, opacity 1, normal 3, color 3,
 * shade 4), or NULL.
 *
 * Per pixel, with hits i = 1..K front to back, T_f the final transmittance
 * and bg the background:
 *   dC/dc_i     = T_i alpha_i
 *   dC/dalpha_i = T_i c_i - B_i / (1 - alpha_i),   B_i = sum_{j>i} T_j alpha_j c_j + T_f bg
 *   dA/dalpha_i = T_i     - D_i / (1 - alpha_i),   D_i = sum_{j>i} T_j alpha_j
 * (differentiate T_j = prod_{k<j}(1 - alpha_k) in Eq. 2).  No gradient flows
 * through alpha where the alpha_max cap is active.
 */
int og_backward(const og_gauss *g, const float *edits, int n_models, const og_camera *cam,
                const og_params *prm, int64_t npix, const int32_t *pix, const double *dl,
                double *grad_rec, double *grad)
{
    int64_t n = g->n;
    double *proj = malloc(sizeof(double) * P_WIDTH * (n > 0 ? n : 1));
    int64_t *order = malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    double *gr = calloc((size_t)(n > 0 ? n : 1) * R_N, sizeof(double));
    og_project(g, edits, n_models, cam, prm, proj);
    int64_t m = sorted_order(proj, n, order);
#pragma omp parallel
    {
        hit_t *hits = malloc(sizeof(hit_t) * (m > 0 ? m : 1));
#pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < npix; ++p) {
            const double *u = dl + 4 * p;
            if (u[0] == 0.0 && u[1] == 0.0 && u[2] == 0.0 && u[3] == 0.0) continue;
            double px, py, Tf, rgba[4];
            pixel_coords(prm, pix, p, &px, &py);
            int64_t nh = composite_pixel(proj, order, m, prm, px, py, 1, NULL, 0, rgba, &Tf, NULL, hits,
                                         NULL, NULL, NULL);
            double B[3] = {Tf * prm->bg[0], Tf * prm->bg[1], Tf * prm->bg[2]};
            double D = 0.0;
            for (int64_t k = nh - 1; k >= 0; --k) {
                const hit_t *h = &hits[k];
                const double *gp = proj + h->idx * P_WIDTH;
                double c[3] = {gp[P_R], gp[P_G], gp[P_B]};
                double w = h->T * h->alpha;
                double one_m = 1.0 - h->alpha;
                double dLda = 0.0;
                for (int ch = 0; ch < 3; ++ch) dLda += u[ch] * (h->T * c[ch] - B[ch] / one_m);
                dLda += u[3] * (h->T - D / one_m);
                double loc[R_N] = {0};
                for (int ch = 0; ch < 3; ++ch) loc[R_CR + ch] = u[ch] * w;
                if (h->raw <= prm->alpha_max) {
                    double o = gp[P_O];
                    double dLdG = dLda * o;
                    double dLdpow = dLdG * h->G;
                    loc[R_O] = dLda * h->G;
                    loc[R_Q00] = dLdpow * (-0.5 * h->dx * h->dx);
                    loc[R_Q01] = dLdpow * (-h->dx * h->dy);
                    loc[R_Q11] = dLdpow * (-0.5 * h->dy * h->dy);
                    loc[R_MX] = dLdpow * (gp[P_Q00] * h->dx + gp[P_Q01] * h->dy);
                    loc[R_MY] = dLdpow * (gp[P_Q01] * h->dx + gp[P_Q11] * h->dy);
                }
                for (int r = 0; r < R_N; ++r) {
#pragma omp atomic
                    gr[h->idx * R_N + r] += loc[r];
                }
                for (int ch = 0; ch < 3; ++ch) B[ch] += w * c[ch];
                D += w;
            }
        }
        free(hits);
    }
    if (grad_rec) memcpy(grad_rec, gr, sizeof(double) * R_N * n);
    if (grad) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            double jac[R_N * N_PARAM];
            int any = 0;
            for (int r = 0; r < R_N; ++r) any |= gr[i * R_N + r] != 0.0;
            for (int k = 0; k < N_PARAM; ++k) grad[k * n + i] = 0.0;
            if (!any || proj[i * P_WIDTH + P_VALID] == 0.0) continue;
            og_jacobian(g, edits, n_models, cam, prm, i, jac);
            for (int k = 0; k < N_PARAM; ++k) {
                double acc = 0.0;
                for (int r = 0; r < R_N; ++r) acc += jac[r * N_PARAM + k] * gr[i * R_N + r];
                grad[k * n + i] = acc;
            }
        }
    }
    free(gr);
    free(order);
    free(proj);
    return 0;
}

/* Exported: gradient of L with respect to each model's orbital light
 * direction (the unnormalised vector of its edit row; Sec. 4.6 learns the
 * light direction of the composed scene), given the record gradients
 * grad_rec[n][9] of og_backward: out[m][3] = sum over the kept Gaussians i of
 * model m of grad_rec[i] . d rec_i / d dir_m, the derivative by the complex
 * step of the same projection code.  Headlight models (l = v) get 0. */
int og_light_grad(const og_gauss *g, const float *edits, int n_models, const og_camera *cam,
                  const og_params *prm, const double *grad_rec, double *out)
{
    int64_t n = g->n;
    for (int k = 0; k < 3 * n_models; ++k) out[k] = 0.0;
#pragma omp parallel
    {
        double *acc = calloc((size_t)(3 * n_models), sizeof(double));
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            const double *gr = grad_rec + i * R_N;
            int any = 0;
            for (int r = 0; r < R_N; ++r) any |= gr[r] != 0.0;
            if (!any) continue;
            int m = g->model_id ? g->model_id[i] : 0;
            if (m < 0 || m >= n_models) m = 0;
            const float *lr = edits + 16 * (int64_t)m;
            int32_t head;
            memcpy(&head, &lr[15], sizeof(head));
            if (head) continue;
            double pr[N_PARAM];
            cplx p[N_PARAM], rec[R_N];
            gather_params(g, i, pr);
            for (int k = 0; k < N_PARAM; ++k) p[k] = pr[k];
            float z32 = depth_key(cam, g->mean[i], g->mean[g->n + i], g->mean[2 * g->n + i]);
            for (int k = 0; k < 3; ++k) {
                cplx ld[3] = {lr[12], lr[13], lr[14]};
                double h = 1e-30 * (fabs((double)lr[12 + k]) > 1.0 ? fabs((double)lr[12 + k]) : 1.0);
                ld[k] += I * h;
                if (!project_one(p, z32, cam, lr, ld, prm, rec, NULL)) break;
                double d = 0.0;
                for (int r = 0; r < R_N; ++r) d += gr[r] * (cimag(rec[r]) / h);
                acc[3 * m + k] += d;
            }
        }
#pragma omp critical
        for (int k = 0; k < 3 * n_models; ++k) out[k] += acc[k];
        free(acc);
    }
    return 0;
}

int og_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
