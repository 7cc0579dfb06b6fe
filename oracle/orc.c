/*
 * orc.c -- CPU ORACLE for the hybrid beamline hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, serial, FP64 C written from the paper
 * (Sandberg et al., PASC '24) and textbook linear beam optics, used to check
 * the GPU library.  Only the tests, the smoke check and the benchmark's CPU
 * baseline leg may load it; the product path never does.  No blocking, no
 * fusion, no reordering beyond what each definition below states.
 *
 * Readings of the paper that fix what is computed (the paper itself gives no
 * element maps or stage physics; it treats every element as a per-particle
 * map f: R^6 -> R^6 without collective effects, §1):
 *  - coordinates relative to a reference particle, s independent (§1);
 *  - drift / thick quad / sector bend / thin lens are first-order
 *    (linear) transfer maps of the linearised equations of motion;
 *  - the plasma stage is linear ion-channel focusing with a linear
 *    energy ramp, integrated by kick-drift-kick, each particle focused
 *    according to its own energy (chromatic);
 *  - the surrogate is the feed-forward network of §3 Eq. (3) with tanh,
 *    trained on the MSE of §3 Eq. (4) with Adam, on coordinates normalised
 *    per direction by mean and standard deviation (§3);
 *  - beam moments and emittance as defined in §4 (unweighted, centred).
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* CODATA 2018 (exact where defined in SI). */
#define ORC_QE 1.602176634e-19
#define ORC_EPS0 8.8541878128e-12
#define ORC_ME_KG 9.1093837015e-31
#define ORC_CLIGHT 299792458.0

#define ROW(z, j, ld) ((z) + (int64_t)(j) * (ld))

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers:
 * as easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with
 * a Weyl-sequence key schedule.                                        */
/* ------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Box-Muller transform (Box & Muller 1958) of two 53-bit uniforms taken from
 * one Philox block.  Coordinate pair q of particle g uses counter
 * (g_lo, g_hi, q, 'GAUS'); pairs are (x,y), (t,px), (py,pt). */
int orc_fill_gaussian(double* z, int64_t n, int64_t ld, uint64_t seed,
                      const double mean[6], const double sigma[6],
                      int64_t i0, const int64_t* idx)
{
    if (!z || n < 0 || ld < n) return -1;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    const double two53inv = 1.0 / 9007199254740992.0;
    for (int64_t i = 0; i < n; i++) {
        int64_t g = idx ? idx[i] : i0 + i;
        for (uint32_t q = 0; q < 3; q++) {
            uint32_t ctr[4] = {(uint32_t)g, (uint32_t)((uint64_t)g >> 32), q, 0x47415553u};
            uint32_t o[4];
            orc_philox4x32_10(ctr, key, o);
            uint64_t a = ((uint64_t)(o[0] >> 5) << 26) | (o[1] >> 6);
            uint64_t b = ((uint64_t)(o[2] >> 5) << 26) | (o[3] >> 6);
            double u1 = ((double)a + 1.0) * two53inv;    /* (0, 1] */
            double u2 = (double)b * two53inv;            /* [0, 1) */
            double r = sqrt(-2.0 * log(u1));
            double ang = 2.0 * M_PI * u2;
            ROW(z, 2 * q, ld)[i] = mean[2 * q] + sigma[2 * q] * (r * cos(ang));
            ROW(z, 2 * q + 1, ld)[i] = mean[2 * q + 1] + sigma[2 * q + 1] * (r * sin(ang));
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Linear element maps.  Each is the exact solution over the element of
 * the linearised equations of motion in (x,px,y,py,t,pt):
 *   drift:  x' = px, y' = py, t' = pt/(beta gamma)^2
 *   quad:   px' = -k x, py' = +k y (plus the drift terms)
 *   sbend:  px' = -x/rho^2 - pt/(rho beta), t' = x/(rho beta) + pt/(beta gamma)^2
 *   lens:   px -= x/f, py -= y/f (thin, axisymmetric)
 * ------------------------------------------------------------------ */
static void ref_kin(const orc_ref* ref, double* bg, double* beta)
{
    double g = ref->gamma;
    *bg = sqrt(g * g - 1.0);
    *beta = *bg / g;
}

/* sin(w L)/w and the hyperbolic analogue, finite as w -> 0 */
static double sin_over(double w, double L) { return w == 0.0 ? L : sin(w * L) / w; }
static double sinh_over(double w, double L) { return w == 0.0 ? L : sinh(w * L) / w; }

static void apply_drift(double* z, int64_t n, int64_t ld, double L, double bg)
{
    double* x = ROW(z, 0, ld); double* y = ROW(z, 1, ld); double* t = ROW(z, 2, ld);
    double* px = ROW(z, 3, ld); double* py = ROW(z, 4, ld); double* pt = ROW(z, 5, ld);
    double r56 = L / (bg * bg);
    for (int64_t i = 0; i < n; i++) {
        x[i] = x[i] + L * px[i];
        y[i] = y[i] + L * py[i];
        t[i] = t[i] + r56 * pt[i];
    }
}

/* Chromatic focusing: a particle with relative momentum deviation delta
 * (to first order delta = -pt / beta) sees the strength k / (1 + delta)
 * ~ k (1 - delta).  With w = sqrt|k| the plane matrix [[a, b], [c, a]] then
 * changes, to first order in delta, by delta * [[a', b'], [c', a']], the
 * derivative of the matrix along dw/ddelta = -w/2:
 *   focusing (cos):     a' = (wL/2) sin wL,  b' = (sin wL / w - L cos wL)/2,
 *                       c' = (w/2)(sin wL + wL cos wL)
 *   defocusing (cosh):  a' = -(wL/2) sinh wL, b' = (sinh wL / w - L cosh wL)/2,
 *                       c' = -(w/2)(sinh wL + wL cosh wL)
 * (the w -> 0 limits vanish).  Drifts and the px = dx/ds relation stay
 * those of the reference momentum, as in the achromatic maps. */
static void chrom_plane(int focusing, double w, double L, double* da, double* db, double* dc)
{
    if (w == 0.0) { *da = *db = *dc = 0.0; return; }
    double wl = w * L;
    if (focusing) {
        *da = 0.5 * wl * sin(wl);
        *db = 0.5 * (sin(wl) / w - L * cos(wl));
        *dc = 0.5 * w * (sin(wl) + wl * cos(wl));
    } else {
        *da = -0.5 * wl * sinh(wl);
        *db = 0.5 * (sinh(wl) / w - L * cosh(wl));
        *dc = -0.5 * w * (sinh(wl) + wl * cosh(wl));
    }
}

static void apply_quad(double* z, int64_t n, int64_t ld, double L, double k, double bg, double beta,
                       int chromatic)
{
    if (k == 0.0) { apply_drift(z, n, ld, L, bg); return; }
    double w = sqrt(fabs(k));
    /* focusing-plane and defocusing-plane 2x2 matrices */
    double fc = cos(w * L), fs = sin_over(w, L), fm = -w * sin(w * L);
    double dc = cosh(w * L), ds = sinh_over(w, L), dm = w * sinh(w * L);
    double ax, bx, cx, ay, by, cy;   /* [[a, b], [c, a]] per plane */
    if (k > 0) { ax = fc; bx = fs; cx = fm; ay = dc; by = ds; cy = dm; }
    else       { ax = dc; bx = ds; cx = dm; ay = fc; by = fs; cy = fm; }
    /* chromatic derivatives per plane, zero when achromatic */
    double dax = 0, dbx = 0, dcx = 0, day = 0, dby = 0, dcy = 0;
    if (chromatic) {
        chrom_plane(k > 0, w, L, &dax, &dbx, &dcx);
        chrom_plane(k < 0, w, L, &day, &dby, &dcy);
    }
    double r56 = L / (bg * bg);
    double* x = ROW(z, 0, ld); double* y = ROW(z, 1, ld); double* t = ROW(z, 2, ld);
    double* px = ROW(z, 3, ld); double* py = ROW(z, 4, ld); double* pt = ROW(z, 5, ld);
    for (int64_t i = 0; i < n; i++) {
        double x0 = x[i], px0 = px[i], y0 = y[i], py0 = py[i];
        double d = -pt[i] / beta;
        x[i] = ax * x0 + bx * px0 + d * (dax * x0 + dbx * px0);
        px[i] = cx * x0 + ax * px0 + d * (dcx * x0 + dax * px0);
        y[i] = ay * y0 + by * py0 + d * (day * y0 + dby * py0);
        py[i] = cy * y0 + ay * py0 + d * (dcy * y0 + day * py0);
        t[i] = t[i] + r56 * pt[i];
    }
}

/* theta - sin(theta), accurate for small theta (series below 0.1 rad). */
static double theta_minus_sin(double th)
{
    double a = fabs(th);
    if (a >= 0.1) return th - sin(th);
    /* th^3/3! - th^5/5! + th^7/7! - ... ; terms fall by >= 1e-2 each */
    double t2 = th * th, term = th * t2 / 6.0, s = 0.0;
    for (int k = 1; k < 12; k++) {
        s += term;
        term *= -t2 / ((2.0 * k + 2.0) * (2.0 * k + 3.0));
    }
    return s;
}

static void apply_sbend(double* z, int64_t n, int64_t ld, double L, double th, double bg, double beta)
{
    if (th == 0.0) { apply_drift(z, n, ld, L, bg); return; }
    double C = cos(th), S = sin(th);
    double rho = L / th;
    double one_m_c = 2.0 * sin(0.5 * th) * sin(0.5 * th);     /* 1 - cos */
    double m11 = C, m12 = rho * S, m16 = -rho * one_m_c / beta;
    double m21 = -S / rho, m22 = C, m26 = -S / beta;
    double m51 = S / beta, m52 = rho * one_m_c / beta;
    double path = rho * theta_minus_sin(th);                  /* L - rho S */
    double m56 = L / (bg * bg) - path / (beta * beta);
    double* x = ROW(z, 0, ld); double* y = ROW(z, 1, ld); double* t = ROW(z, 2, ld);
    double* px = ROW(z, 3, ld); double* py = ROW(z, 4, ld); double* pt = ROW(z, 5, ld);
    for (int64_t i = 0; i < n; i++) {
        double x0 = x[i], px0 = px[i], pt0 = pt[i];
        x[i] = m11 * x0 + m12 * px0 + m16 * pt0;
        px[i] = m21 * x0 + m22 * px0 + m26 * pt0;
        y[i] = y[i] + L * py[i];
        t[i] = t[i] + m51 * x0 + m52 * px0 + m56 * pt0;
    }
}

/* Thin lens; chromatic: focal length f (1 + delta), first order in delta. */
static void apply_lens(double* z, int64_t n, int64_t ld, double f, double beta, int chromatic)
{
    double* x = ROW(z, 0, ld); double* y = ROW(z, 1, ld);
    double* px = ROW(z, 3, ld); double* py = ROW(z, 4, ld); double* pt = ROW(z, 5, ld);
    for (int64_t i = 0; i < n; i++) {
        double s = chromatic ? 1.0 + pt[i] / beta : 1.0;     /* 1 - delta */
        px[i] = px[i] - x[i] * s / f;
        py[i] = py[i] - y[i] * s / f;
    }
}

/* ------------------------------------------------------------------ */
/* Fine-step plasma stage: linear ion-channel focusing du/ds = -kappa x,
 * kappa = k_p^2/2, drift dx/ds = u/gamma_i(s) with u = p_x/(m c), the
 * particle's own gamma_i(s) = gamma_ref(s) + dgamma_i, the reference ramping
 * linearly from gamma_in to gamma_out over L; symmetric kick-drift-kick. */
/* ------------------------------------------------------------------ */
static int apply_stage(double* z, int64_t n, int64_t ld, const orc_elem* st, orc_ref* ref)
{
    if (st->nsub < 1 || !(st->L > 0.0) || !(st->n0_m3 >= 0.0)) return -1;
    const double g_in = ref->gamma;
    const double g_out = g_in + st->dE_MeV / ref->mass_MeV;
    if (!(g_out > 1.0)) return -1;
    const double bg_in = sqrt(g_in * g_in - 1.0), bg_out = sqrt(g_out * g_out - 1.0);
    const double L = st->L;
    const int64_t N = st->nsub;
    const double h = L / (double)N;
    const double gp = (g_out - g_in) / L;
    const double kp2 = st->n0_m3 * ORC_QE * ORC_QE / (ORC_EPS0 * ORC_ME_KG * ORC_CLIGHT * ORC_CLIGHT);
    const double kappa = 0.5 * kp2;
    /* first-order flight-time term, G -> 0 limit is the drift's */
    const double r56 = (gp == 0.0) ? bg_in * L / (g_in * g_in * g_in)
                                   : bg_in * (1.0 / (g_in * g_in) - 1.0 / (g_out * g_out)) / (2.0 * gp);
    double* x = ROW(z, 0, ld); double* y = ROW(z, 1, ld); double* t = ROW(z, 2, ld);
    double* px = ROW(z, 3, ld); double* py = ROW(z, 4, ld); double* pt = ROW(z, 5, ld);
    /* Energy-correlated gain: particle i gains dE (1 + chirp t_i), t_i its
     * entry t, so its own gradient is gp (1 + chirp t_i).  Its flight time
     * then carries -chirp t_i gp * integral s / gamma_ref(s)^3 ds
     * = -chirp t_i gp L^2 / (2 gamma_in gamma_out^2). */
    const double chirp = st->chirp;
    const double t_chirp = gp * L * L / (2.0 * g_in * g_out * g_out);
    for (int64_t i = 0; i < n; i++) {
        double pt_in = pt[i], t_in = t[i];
        double dg = -pt_in * bg_in;
        double gpi = gp * (1.0 + chirp * t_in);
        double xi = x[i], yi = y[i];
        double ux = px[i] * bg_in, uy = py[i] * bg_in;
        for (int64_t s = 0; s < N; s++) {
            ux = ux - 0.5 * h * kappa * xi;
            uy = uy - 0.5 * h * kappa * yi;
            double gam = g_in + gpi * (((double)s + 0.5) * h) + dg;
            xi = xi + h * ux / gam;
            yi = yi + h * uy / gam;
            ux = ux - 0.5 * h * kappa * xi;
            uy = uy - 0.5 * h * kappa * yi;
        }
        x[i] = xi; y[i] = yi;
        px[i] = ux / bg_out; py[i] = uy / bg_out;
        t[i] = t_in + r56 * pt_in - chirp * t_in * t_chirp;
        /* E_i,out - E_ref,out = -pt_in bg_in + chirp t_in (g_out - g_in)  (units m c^2) */
        pt[i] = (pt_in * bg_in - chirp * t_in * (g_out - g_in)) / bg_out;
    }
    ref->gamma = g_out;
    ref->s += L;
    return 0;
}

int orc_push(double* z, int64_t n, int64_t ld, const orc_elem* e, int32_t n_elem, orc_ref* ref)
{
    if (!z || n < 0 || ld < n || (n_elem > 0 && !e) || !ref || !(ref->gamma > 1.0)) return -1;
    for (int32_t j = 0; j < n_elem; j++) {
        double bg, beta;
        ref_kin(ref, &bg, &beta);
        switch (e[j].kind) {
        case ORC_DRIFT: apply_drift(z, n, ld, e[j].L, bg); ref->s += e[j].L; break;
        case ORC_QUAD: apply_quad(z, n, ld, e[j].L, e[j].k, bg, beta, e[j].chromatic); ref->s += e[j].L; break;
        case ORC_SBEND: apply_sbend(z, n, ld, e[j].L, e[j].angle, bg, beta); ref->s += e[j].L; break;
        case ORC_THIN_LENS:
            if (e[j].f == 0.0) return -1;
            apply_lens(z, n, ld, e[j].f, beta, e[j].chromatic);
            break;
        case ORC_STAGE:
            if (apply_stage(z, n, ld, &e[j], ref)) return -1;
            break;
        default: return -1;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Exact sums: non-overlapping expansions grown one double at a time
 * (Shewchuk, "Adaptive precision floating-point arithmetic", 1997, grow-
 * expansion with zero elimination).  Products enter exactly through the
 * FMA two-product (a*b = hi + lo).                                    */
/* ------------------------------------------------------------------ */
typedef struct { double* p; int n, cap; } xsum;

static void xs_init(xsum* s) { s->n = 0; s->cap = 32; s->p = (double*)malloc(32 * sizeof(double)); }
static void xs_free(xsum* s) { free(s->p); s->p = NULL; s->n = s->cap = 0; }
static void xs_add(xsum* s, double x)
{
    int j = 0;
    for (int i = 0; i < s->n; i++) {
        double y = s->p[i];
        double a = x, b = y;
        if (fabs(a) < fabs(b)) { a = y; b = x; }
        double hi = a + b;
        double lo = b - (hi - a);
        if (lo != 0.0) s->p[j++] = lo;
        x = hi;
    }
    if (j + 1 > s->cap) { s->cap *= 2; s->p = (double*)realloc(s->p, s->cap * sizeof(double)); }
    s->p[j++] = x;
    s->n = j;
}
static void xs_add_prod(xsum* s, double a, double b)
{
    double hi = a * b;
    double lo = fma(a, b, -hi);
    xs_add(s, hi);
    xs_add(s, lo);
}
static double xs_value(const xsum* s)
{
    double v = 0.0;
    for (int i = 0; i < s->n; i++) v += s->p[i];
    return v;
}

static int upper_index(int j, int k) { return j * 6 - j * (j - 1) / 2 + (k - j); }

int orc_moments(const double* z, int64_t n, int64_t ld, double mean6[6], double cov21[21])
{
    if (!z || n <= 0 || ld < n) return -1;
    xsum S[6], P[21];
    for (int j = 0; j < 6; j++) xs_init(&S[j]);
    for (int q = 0; q < 21; q++) xs_init(&P[q]);
    for (int64_t i = 0; i < n; i++) {
        double v[6];
        for (int j = 0; j < 6; j++) { v[j] = ROW(z, j, ld)[i]; xs_add(&S[j], v[j]); }
        for (int j = 0; j < 6; j++)
            for (int k = j; k < 6; k++) xs_add_prod(&P[upper_index(j, k)], v[j], v[k]);
    }
    const double nd = (double)n;
    for (int j = 0; j < 6; j++) mean6[j] = xs_value(&S[j]) / nd;
    /* cov_jk = (n * sum x_j x_k - sum x_j * sum x_k) / n^2, numerator exact */
    for (int j = 0; j < 6; j++)
        for (int k = j; k < 6; k++) {
            xsum E; xs_init(&E);
            xsum* Pjk = &P[upper_index(j, k)];
            for (int a = 0; a < Pjk->n; a++) xs_add_prod(&E, nd, Pjk->p[a]);
            for (int a = 0; a < S[j].n; a++)
                for (int b = 0; b < S[k].n; b++) xs_add_prod(&E, -S[j].p[a], S[k].p[b]);
            cov21[upper_index(j, k)] = xs_value(&E) / (nd * nd);
            xs_free(&E);
        }
    for (int j = 0; j < 6; j++) xs_free(&S[j]);
    for (int q = 0; q < 21; q++) xs_free(&P[q]);
    return 0;
}

/* eps = sqrt(<dx^2><dpx^2> - <dx dpx>^2) per plane (§4), determinant exact */
int orc_emittances(const double cov21[21], double eps3[3])
{
    static const int pos[3] = {0, 1, 2}, mom[3] = {3, 4, 5};
    for (int p = 0; p < 3; p++) {
        double a = cov21[upper_index(pos[p], pos[p])];
        double b = cov21[upper_index(pos[p], mom[p])];
        double d = cov21[upper_index(mom[p], mom[p])];
        xsum E; xs_init(&E);
        xs_add_prod(&E, a, d);
        xs_add_prod(&E, -b, b);
        double det = xs_value(&E);
        xs_free(&E);
        eps3[p] = det > 0.0 ? sqrt(det) : 0.0;
    }
    return 0;
}

int orc_compare(const double* s, const double* f, int64_t n, int64_t ld,
                double rms6[6], double centroid6[6], double eps_rel3[3])
{
    if (!s || !f || n <= 0 || ld < n) return -1;
    double ms[6], cs[21], mf[6], cf[21], es[3], ef[3];
    orc_moments(s, n, ld, ms, cs);
    orc_moments(f, n, ld, mf, cf);
    orc_emittances(cs, es);
    orc_emittances(cf, ef);
    for (int j = 0; j < 6; j++) {
        xsum D; xs_init(&D);
        const double* sj = ROW(s, j, ld);
        const double* fj = ROW(f, j, ld);
        for (int64_t i = 0; i < n; i++) { double d = sj[i] - fj[i]; xs_add_prod(&D, d, d); }
        double sig = sqrt(cf[upper_index(j, j)]);
        rms6[j] = sqrt(xs_value(&D) / (double)n) / sig;
        centroid6[j] = (ms[j] - mf[j]) / sig;
        xs_free(&D);
    }
    for (int p = 0; p < 3; p++) eps_rel3[p] = es[p] / ef[p] - 1.0;
    return 0;
}

/* ------------------------------------------------------------------ */
/* bfloat16: keep the top 16 bits of the FP32 pattern, round to nearest,
 * ties to even; NaN stays NaN.                                         */
/* ------------------------------------------------------------------ */
float orc_bf16(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) {
        if (u & 0x007fffffu) u |= 0x00400000u;
        u &= 0xffff0000u;
    } else {
        uint32_t lsb = (u >> 16) & 1u;
        u = (u + 0x7fffu + lsb) & 0xffff0000u;
    }
    memcpy(&x, &u, 4);
    return x;
}

/* ------------------------------------------------------------------ */
/* MLP surrogate.  Layers l = 0..H (H = hidden layers): a_l = A_l h_l + b_l,
 * h_{l+1} = tanh(a_l) for l < H, output = a_H (§3 Eq. 3).  Parameters are
 * stored flat: A_0 (out x in, row-major), b_0, A_1, b_1, ..., A_H, b_H.  */
/* ------------------------------------------------------------------ */
static int layer_in(const orc_shape* sh, int l) { return l == 0 ? sh->n_in : sh->width; }
static int layer_out(const orc_shape* sh, int l) { return l == sh->hidden ? sh->n_out : sh->width; }

int64_t orc_mlp_nparams(const orc_shape* sh)
{
    int64_t np = 0;
    for (int l = 0; l <= sh->hidden; l++) np += (int64_t)layer_out(sh, l) * (layer_in(sh, l) + 1);
    return np;
}

static int64_t layer_offset(const orc_shape* sh, int l)
{
    int64_t off = 0;
    for (int q = 0; q < l; q++) off += (int64_t)layer_out(sh, q) * (layer_in(sh, q) + 1);
    return off;
}

/* U(-1/sqrt(fan_in), 1/sqrt(fan_in)) for weights and biases; parameter p
 * draws word 0 of Philox block (p, 0, 0, 'MLPI'). */
int orc_mlp_init(const orc_shape* sh, uint64_t seed, float* params)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int l = 0; l <= sh->hidden; l++) {
        int64_t off = layer_offset(sh, l);
        int64_t cnt = (int64_t)layer_out(sh, l) * (layer_in(sh, l) + 1);
        double bound = 1.0 / sqrt((double)layer_in(sh, l));
        for (int64_t q = 0; q < cnt; q++) {
            int64_t p = off + q;
            uint32_t ctr[4] = {(uint32_t)p, (uint32_t)((uint64_t)p >> 32), 0u, 0x4D4C5049u};
            uint32_t o[4];
            orc_philox4x32_10(ctr, key, o);
            double u = (double)(o[0] >> 8) * (1.0 / 16777216.0);
            params[p] = (float)((2.0 * u - 1.0) * bound);
        }
    }
    return 0;
}

#define MAXW 1024

/* Forward pass of one sample.  xin: raw input (6 doubles).  Stores the
 * network input actually used (act[0]), each hidden activation act[l] and the
 * normalised output yhat.  Mode 0 is the network of Eq. (3) in FP64 and is
 * the parity reference.  Mode 1 FOLLOWS THE LIBRARY KERNEL (a secondary,
 * kernel-specific check, not a statement of the method): it applies the
 * kernel's own rounding points:
 *   hidden layers form the pre-activation scaled by c = 2/ln 2 (FP32 c),
 *   from FP32 c*w and c*b, and take tanh(ln2/2 * that);
 *   input: FP32 value split into bf16 hi + lo, first-layer (scaled) weights
 *   split the same way, product keeps hi*hi + hi*lo + lo*hi; other hidden
 *   weights and activations bf16; output layer unscaled, result FP32. */
#define ORC_TANH_SCALE 2.8853900817779268f
typedef struct { double act[8][MAXW]; double yhat[MAXW]; } fwd_state;

static void forward_one(const orc_shape* sh, const float* prm, const double* norm, int mode,
                        const double* xin, fwd_state* st)
{
    const int H = sh->hidden;
    for (int j = 0; j < sh->n_in; j++) {
        double xh = (xin[j] - norm[j]) / norm[6 + j];
        st->act[0][j] = mode ? (double)(float)xh : xh;
    }
    for (int l = 0; l <= H; l++) {
        const int ni = layer_in(sh, l), no = layer_out(sh, l);
        const float* A = prm + layer_offset(sh, l);
        const float* b = A + (int64_t)no * ni;
        const double* in = st->act[l];
        double* out = (l == H) ? st->yhat : st->act[l + 1];
        const float cs = (mode && l < H) ? ORC_TANH_SCALE : 1.0f;
        for (int o = 0; o < no; o++) {
            double acc = mode ? (double)(b[o] * cs) : (double)b[o];
            for (int i = 0; i < ni; i++) {
                float w = A[(int64_t)o * ni + i];
                if (!mode) {
                    acc += (double)w * in[i];
                } else if (l == 0) {
                    float xs = (float)in[i];
                    float xhi = orc_bf16(xs), xlo = orc_bf16(xs - xhi);
                    float wc = w * cs;
                    float whi = orc_bf16(wc), wlo = orc_bf16(wc - whi);
                    acc += (double)whi * xhi + (double)whi * xlo + (double)wlo * xhi;
                } else {
                    acc += (double)orc_bf16(w * cs) * in[i];
                }
            }
            if (l == H) {
                out[o] = mode ? (double)(float)acc : acc;
            } else if (!mode) {
                out[o] = tanh(acc);
            } else {
                out[o] = (double)orc_bf16((float)tanh((double)(float)acc * (0.5 * M_LN2)));
            }
        }
    }
}

int orc_mlp_apply(const orc_shape* sh, const float* params, const double* norm, int mode,
                  const double* zin, double* zout, int64_t n, int64_t ld)
{
    if (sh->width > MAXW || sh->hidden > 6 || sh->n_in != 6 || sh->n_out != 6) return -1;
    fwd_state* st = (fwd_state*)malloc(sizeof(fwd_state));
    for (int64_t i = 0; i < n; i++) {
        double x[6];
        for (int j = 0; j < 6; j++) x[j] = ROW(zin, j, ld)[i];
        forward_one(sh, params, norm, mode, x, st);
        for (int j = 0; j < 6; j++) ROW(zout, j, ld)[i] = norm[12 + j] + norm[18 + j] * st->yhat[j];
    }
    free(st);
    return 0;
}

/* MSE (Eq. 4) over b pairs x 6 outputs in normalised coordinates, and its
 * gradient by reverse-mode differentiation.  Mode 1 rounds the back-
 * propagated error to bf16 where the GPU feeds it to bf16 products, and
 * uses bf16 weights, as the forward. */
int orc_mlp_loss_grad(const orc_shape* sh, const float* params, const double* norm, int mode,
                      const double* zin, const double* zout, int64_t ld,
                      const int64_t* idx, int64_t b, double* grad, double* loss)
{
    if (sh->width > MAXW || sh->hidden > 6 || b <= 0) return -1;
    const int H = sh->hidden;
    const int64_t np = orc_mlp_nparams(sh);
    memset(grad, 0, np * sizeof(double));
    fwd_state* st = (fwd_state*)malloc(sizeof(fwd_state));
    double* dl = (double*)malloc(MAXW * sizeof(double));
    double* dprev = (double*)malloc(MAXW * sizeof(double));
    double lsum = 0.0;
    const double scale = 2.0 / ((double)b * sh->n_out);
    for (int64_t q = 0; q < b; q++) {
        const int64_t i = idx[q];
        double x[6];
        for (int j = 0; j < 6; j++) x[j] = ROW(zin, j, ld)[i];
        forward_one(sh, params, norm, mode, x, st);
        for (int o = 0; o < sh->n_out; o++) {
            double yt = (ROW(zout, o, ld)[i] - norm[12 + o]) / norm[18 + o];
            double d;
            if (mode) {
                float d32 = (float)st->yhat[o] - (float)yt;
                d = (double)d32;
                dl[o] = (double)(float)(d * scale);
            } else {
                d = st->yhat[o] - yt;
                dl[o] = d * scale;
            }
            lsum += d * d;
        }
        for (int l = H; l >= 0; l--) {
            const int ni = layer_in(sh, l), no = layer_out(sh, l);
            const float* A = params + layer_offset(sh, l);
            double* gA = grad + layer_offset(sh, l);
            double* gb = gA + (int64_t)no * ni;
            const double* in = st->act[l];
            for (int o = 0; o < no; o++) {
                double dq = (mode && l > 0) ? (double)orc_bf16((float)dl[o]) : dl[o];
                for (int ii = 0; ii < ni; ii++) gA[(int64_t)o * ni + ii] += dq * in[ii];
                gb[o] += dl[o];
            }
            if (l > 0) {
                for (int ii = 0; ii < ni; ii++) {
                    double e = 0.0;
                    for (int o = 0; o < no; o++) {
                        float w = A[(int64_t)o * ni + ii];
                        if (mode) e += (double)orc_bf16(w) * (double)orc_bf16((float)dl[o]);
                        else e += (double)w * dl[o];
                    }
                    double h = in[ii];
                    double dd = e * (1.0 - h * h);
                    dprev[ii] = mode ? (double)(float)dd : dd;
                }
                memcpy(dl, dprev, ni * sizeof(double));
            }
        }
    }
    *loss = lsum / ((double)b * sh->n_out);
    free(dprev); free(dl); free(st);
    return 0;
}

/* Adam (Kingma & Ba 2015) with bias correction, step t >= 1. */
int orc_adam_step(int64_t np, float* params, double* m, double* v, const double* grad,
                  int64_t t, double lr, double b1, double b2, double eps)
{
    if (t < 1) return -1;
    const double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t p = 0; p < np; p++) {
        m[p] = b1 * m[p] + (1.0 - b1) * grad[p];
        v[p] = b2 * v[p] + (1.0 - b2) * grad[p] * grad[p];
        double mh = m[p] / c1, vh = v[p] / c2;
        params[p] = (float)((double)params[p] - lr * mh / (sqrt(vh) + eps));
    }
    return 0;
}

/* mean and population standard deviation per direction (§3), exact sums */
int orc_norm_stats(const double* zin, const double* zout, int64_t n_train, int64_t ld, double* norm)
{
    double m[6], c[21];
    if (orc_moments(zin, n_train, ld, m, c)) return -1;
    for (int j = 0; j < 6; j++) { norm[j] = m[j]; norm[6 + j] = sqrt(c[upper_index(j, j)]); }
    if (orc_moments(zout, n_train, ld, m, c)) return -1;
    for (int j = 0; j < 6; j++) { norm[12 + j] = m[j]; norm[18 + j] = sqrt(c[upper_index(j, j)]); }
    return 0;
}

/* Fisher-Yates from the identity each epoch: for i = n-1 .. 1, swap i with
 * j = floor(r (i+1) / 2^32), r = word (i mod 4) of Philox block
 * (i/4 lo, i/4 hi, epoch, 'SHUF'). */
int orc_epoch_perm(int64_t n, uint64_t seed, int64_t epoch, int64_t* perm)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t i = 0; i < n; i++) perm[i] = i;
    for (int64_t i = n - 1; i >= 1; i--) {
        uint64_t blk = (uint64_t)i >> 2;
        uint32_t ctr[4] = {(uint32_t)blk, (uint32_t)(blk >> 32), (uint32_t)epoch, 0x53485546u};
        uint32_t o[4];
        orc_philox4x32_10(ctr, key, o);
        uint64_t j = ((uint64_t)o[i & 3] * (uint64_t)(i + 1)) >> 32;
        int64_t tmp = perm[i]; perm[i] = perm[j]; perm[j] = tmp;
    }
    return 0;
}

/* Learning rate of optimizer step t (1-based) of `planned`: a half cosine
 * from lr at the first step to lr_final at the last (constant when they are
 * equal).  The paper and the benchmark definition name a rate but no
 * schedule; the anneal is this build's reading. */
double orc_lr_at(int64_t t, int64_t planned, double lr, double lr_final)
{
    if (planned <= 1 || lr_final == lr) return lr;
    return lr_final + 0.5 * (lr - lr_final) * (1.0 + cos(M_PI * (double)(t - 1) / (double)(planned - 1)));
}

int orc_mlp_train(const orc_shape* sh, float* params, double* norm, int mode,
                  const double* zin, const double* zout, int64_t n_pairs, int64_t ld,
                  int64_t batch, int64_t epochs, int64_t max_steps, double lr, double lr_final,
                  double b1, double b2, double eps, double train_frac, uint64_t shuffle_seed,
                  double* loss_log)
{
    const int64_t n_train = (int64_t)llround(train_frac * (double)n_pairs);
    const int64_t n_test = n_pairs - n_train;
    if (n_train < batch || batch <= 0) return -1;
    if (orc_norm_stats(zin, zout, n_train, ld, norm)) return -1;
    const int64_t np = orc_mlp_nparams(sh);
    double* m = (double*)calloc(np, sizeof(double));
    double* v = (double*)calloc(np, sizeof(double));
    double* g = (double*)malloc(np * sizeof(double));
    int64_t* perm = (int64_t*)malloc(n_train * sizeof(int64_t));
    int64_t* tidx = (int64_t*)malloc((n_test > 0 ? n_test : 1) * sizeof(int64_t));
    for (int64_t i = 0; i < n_test; i++) tidx[i] = n_train + i;
    const int64_t steps_per_epoch = n_train / batch;
    /* learning rate: half-cosine anneal from lr to lr_final over the planned steps */
    int64_t planned = epochs * steps_per_epoch;
    if (max_steps >= 0 && max_steps < planned) planned = max_steps;
    int64_t t = 0;
    for (int64_t e = 0; e < epochs; e++) {
        orc_epoch_perm(n_train, shuffle_seed, e, perm);
        double lsum = 0.0;
        int64_t done = 0;
        for (int64_t s = 0; s < steps_per_epoch; s++) {
            if (max_steps >= 0 && t >= max_steps) break;
            double loss;
            orc_mlp_loss_grad(sh, params, norm, mode, zin, zout, ld, perm + s * batch, batch, g, &loss);
            t++;
            orc_adam_step(np, params, m, v, g, t, orc_lr_at(t, planned, lr, lr_final), b1, b2, eps);
            lsum += loss;
            done++;
        }
        double tl = 0.0;
        if (n_test > 0) orc_mlp_loss_grad(sh, params, norm, mode, zin, zout, ld, tidx, n_test, g, &tl);
        if (loss_log) { loss_log[2 * e] = done ? lsum / done : 0.0; loss_log[2 * e + 1] = tl; }
    }
    free(tidx); free(perm); free(g); free(v); free(m);
    return 0;
}

/* ------------------------------------------------------------------ */
/* PReLU network, the shape the paper trains (§3 Eq. 2 and 3; §4.2: several
 * hidden layers of equal width).  Hidden layer l < H:
 *   v = A_l h_l + b_l,   h_{l+1} = prelu(v) = v if v > 0, a_l v otherwise,
 * with ONE learned slope a_l per hidden layer; output A_H h_H + b_H.  Flat
 * parameters: A_0 (out x in, row-major), b_0, a_0, A_1, b_1, a_1, ...,
 * A_{H-1}, b_{H-1}, a_{H-1}, A_H, b_H.  Weights and biases draw like the
 * tanh network's (parameter p: Philox block (p, 0, 0, 'MLPI')); slopes start
 * at 0.25 and draw nothing.
 * Mode 1 applies the GPU rounding points: network input FP32; first layer
 * FP32 weights, pre-activation rounded to FP32; other layers bf16 weights
 * and bf16 activations with the pre-activation rounded to FP32; the slope
 * product in FP32; each hidden activation rounded to bf16; output FP32.    */
/* ------------------------------------------------------------------ */
static int64_t prelu_layer_offset(const orc_shape* sh, int l)
{
    int64_t off = 0;
    for (int q = 0; q < l; q++) off += (int64_t)layer_out(sh, q) * (layer_in(sh, q) + 1) + 1;
    return off;
}

int64_t orc_prelu_nparams(const orc_shape* sh)
{
    return prelu_layer_offset(sh, sh->hidden) + (int64_t)sh->n_out * (sh->width + 1);
}

int orc_prelu_init(const orc_shape* sh, uint64_t seed, float* params)
{
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int l = 0; l <= sh->hidden; l++) {
        const int64_t off = prelu_layer_offset(sh, l);
        const int64_t cnt = (int64_t)layer_out(sh, l) * (layer_in(sh, l) + 1);
        const double bound = 1.0 / sqrt((double)layer_in(sh, l));
        for (int64_t q = 0; q < cnt; q++) {
            const int64_t p = off + q;
            uint32_t ctr[4] = {(uint32_t)p, (uint32_t)((uint64_t)p >> 32), 0u, 0x4D4C5049u};
            uint32_t o[4];
            orc_philox4x32_10(ctr, key, o);
            const double u = (double)(o[0] >> 8) * (1.0 / 16777216.0);
            params[p] = (float)((2.0 * u - 1.0) * bound);
        }
        if (l < sh->hidden) params[off + cnt] = 0.25f;
    }
    return 0;
}

/* pre[l][o]: pre-activation of hidden layer l (as used by the slope). */
typedef struct { double act[8][MAXW]; double pre[8][MAXW]; double yhat[MAXW]; } prelu_state;

static void prelu_forward_one(const orc_shape* sh, const float* prm, const double* norm, int mode,
                              const double* xin, prelu_state* st)
{
    const int H = sh->hidden;
    for (int j = 0; j < sh->n_in; j++) {
        const double xh = (xin[j] - norm[j]) / norm[6 + j];
        st->act[0][j] = mode ? (double)(float)xh : xh;
    }
    for (int l = 0; l <= H; l++) {
        const int ni = layer_in(sh, l), no = layer_out(sh, l);
        const float* A = prm + prelu_layer_offset(sh, l);
        const float* b = A + (int64_t)no * ni;
        const float slope = (l < H) ? b[no] : 0.0f;
        const double* in = st->act[l];
        for (int o = 0; o < no; o++) {
            double acc = (double)b[o];
            for (int i = 0; i < ni; i++) {
                const float w = A[(int64_t)o * ni + i];
                acc += (double)((mode && l > 0) ? orc_bf16(w) : w) * in[i];
            }
            if (l == H) {
                st->yhat[o] = mode ? (double)(float)acc : acc;
                continue;
            }
            double v;
            if (mode) {
                const float v32 = (float)acc;
                v = (double)orc_bf16(v32 > 0.0f ? v32 : slope * v32);
                st->pre[l][o] = (double)v32;
            } else {
                v = acc > 0.0 ? acc : (double)slope * acc;
                st->pre[l][o] = acc;
            }
            st->act[l + 1][o] = v;
        }
    }
}

int orc_prelu_apply(const orc_shape* sh, const float* params, const double* norm, int mode,
                    const double* zin, double* zout, int64_t n, int64_t ld)
{
    if (sh->width > MAXW || sh->hidden < 1 || sh->hidden > 7 || sh->n_in != 6 || sh->n_out != 6) return -1;
    prelu_state* st = (prelu_state*)malloc(sizeof(prelu_state));
    for (int64_t i = 0; i < n; i++) {
        double x[6];
        for (int j = 0; j < 6; j++) x[j] = ROW(zin, j, ld)[i];
        prelu_forward_one(sh, params, norm, mode, x, st);
        for (int j = 0; j < 6; j++) ROW(zout, j, ld)[i] = norm[12 + j] + norm[18 + j] * st->yhat[j];
    }
    free(st);
    return 0;
}

/* MSE (Eq. 4) over b pairs x 6 outputs in normalised coordinates and its
 * exact FP64 gradient by reverse-mode differentiation (mode 0 only).  The
 * slope gradient collects the error times the pre-activation wherever the
 * pre-activation is not positive. */
int orc_prelu_loss_grad(const orc_shape* sh, const float* params, const double* norm,
                        const double* zin, const double* zout, int64_t ld,
                        const int64_t* idx, int64_t b, double* grad, double* loss)
{
    if (sh->width > MAXW || sh->hidden < 1 || sh->hidden > 7 || b <= 0) return -1;
    const int H = sh->hidden;
    const int64_t np = orc_prelu_nparams(sh);
    memset(grad, 0, np * sizeof(double));
    prelu_state* st = (prelu_state*)malloc(sizeof(prelu_state));
    double* dl = (double*)malloc(MAXW * sizeof(double));
    double* dprev = (double*)malloc(MAXW * sizeof(double));
    double lsum = 0.0;
    const double scale = 2.0 / ((double)b * sh->n_out);
    for (int64_t q = 0; q < b; q++) {
        const int64_t i = idx[q];
        double x[6];
        for (int j = 0; j < 6; j++) x[j] = ROW(zin, j, ld)[i];
        prelu_forward_one(sh, params, norm, 0, x, st);
        for (int o = 0; o < sh->n_out; o++) {
            const double d = st->yhat[o] - (ROW(zout, o, ld)[i] - norm[12 + o]) / norm[18 + o];
            dl[o] = d * scale;              /* dL/d(output) */
            lsum += d * d;
        }
        for (int l = H; l >= 0; l--) {
            const int ni = layer_in(sh, l), no = layer_out(sh, l);
            const float* A = params + prelu_layer_offset(sh, l);
            double* gA = grad + prelu_layer_offset(sh, l);
            double* gb = gA + (int64_t)no * ni;
            const double* in = st->act[l];
            /* dl holds dL/dv for this layer's pre-activations v */
            for (int o = 0; o < no; o++) {
                for (int ii = 0; ii < ni; ii++) gA[(int64_t)o * ni + ii] += dl[o] * in[ii];
                gb[o] += dl[o];
            }
            if (l == 0) break;
            /* back through layer l-1's PReLU: h = prelu(u), u = pre[l-1] */
            const float* Ap = params + prelu_layer_offset(sh, l - 1);
            const double slope = (double)Ap[(int64_t)ni * (layer_in(sh, l - 1) + 1)];
            double* gslope = grad + prelu_layer_offset(sh, l - 1) + (int64_t)ni * (layer_in(sh, l - 1) + 1);
            for (int ii = 0; ii < ni; ii++) {
                double e = 0.0;
                for (int o = 0; o < no; o++) e += (double)A[(int64_t)o * ni + ii] * dl[o];
                const double u = st->pre[l - 1][ii];
                if (u > 0.0) {
                    dprev[ii] = e;
                } else {
                    dprev[ii] = slope * e;
                    *gslope += e * u;
                }
            }
            memcpy(dl, dprev, ni * sizeof(double));
        }
    }
    *loss = lsum / ((double)b * sh->n_out);
    free(dprev); free(dl); free(st);
    return 0;
}
