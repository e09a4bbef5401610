/*
 * FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see hd_oracle.h).
 *
 * Plain loops, one system at a time, no blocking or fusion: each function
 * follows the definition it cites so that it can be checked against the
 * paper by eye.  Built with -O2 -ffp-contract=off so that every product and
 * sum is rounded exactly as written.
 */
#include "hd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { MOBILE = 0, FIXED = 1, RIGID = 2 };

struct orc_sys {
    orc_params p;
    int dim, n;
    double *x, *v, *rO;      /* SoA [dim][n] */
    uint8_t *type, *role;
    double *cofs;            /* rigid atoms: offset from the rigid-body COM */
    int n_rigid, first_rigid;
    double XR[3], VR[3], XR0[3];
    double *ftot;            /* total force at the current positions */
    double *tuu;             /* T[u,u] of the last evaluation */
    /* eigenvalue variable: the mode estimate q (atom layout, rigid atoms
     * the body's component), its normalised spread w = P q/|q|, H w and
     * T[w,w] of the last evaluation */
    double *qm, *wn, *hw, *tww;
    double xi[4], eta[4];    /* Nose-Hoover chain velocities and positions */
    double FR[3];            /* total force on the rigid body */
    int64_t step;
    double t_md, t_hyper;
    orc_scalars last;
    int brute;
    int have_force;
};

static double nhc_energy(const orc_sys *s);

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from the definition in Salmon et al. (SC'11): ten rounds of
 * two 32x32->64 multiplies with the round keys bumped by the Weyl constants. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * c0;
        uint64_t p1 = (uint64_t)M1 * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Counter = (step low, step high, particle, tag); key = (seed low, seed high).
 * Uniforms u = (w + 1/2) 2^-32 lie strictly inside (0, 1); Box-Muller maps
 * (u0, u1) -> (z0, z1) and (u2, u3) -> (z2, z3). */
void orc_normals(uint64_t seed, int64_t step, uint32_t particle, uint32_t tag, double z[4])
{
    uint32_t ctr[4] = {(uint32_t)((uint64_t)step & 0xffffffffu),
                       (uint32_t)((uint64_t)step >> 32), particle, tag};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t w[4];
    orc_philox4x32_10(ctr, key, w);
    const double two_m32 = 2.3283064365386963e-10; /* 2^-32 */
    double u[4];
    for (int k = 0; k < 4; ++k) u[k] = ((double)w[k] + 0.5) * two_m32;
    const double two_pi = 6.283185307179586;
    double r0 = sqrt(-2.0 * log(u[0]));
    double r1 = sqrt(-2.0 * log(u[2]));
    z[0] = r0 * cos(two_pi * u[1]);
    z[1] = r0 * sin(two_pi * u[1]);
    z[2] = r1 * cos(two_pi * u[3]);
    z[3] = r1 * sin(two_pi * u[3]);
}

/* ------------------------------------------------------------------------ */
/* Minimum image along one axis: strict comparisons with half the box. */
static double minimg(double dx, double L, int periodic)
{
    if (!periodic) return dx;
    if (dx > 0.5 * L) dx -= L;
    else if (dx < -0.5 * L) dx += L;
    return dx;
}

static double wrap(double x, double L, int periodic)
{
    if (!periodic) return x;
    if (x >= L) x -= L;
    else if (x < 0.0) x += L;
    return x;
}

/* r^2 between atoms i and j with displacement dx_k = x_j - x_i, summed as
 * (dx*dx + dy*dy) + dz*dz. */
static double pair_r2(const orc_params *p, const double *x, int n, int i, int j)
{
    double r2 = 0.0;
    for (int k = 0; k < p->dim; ++k) {
        double d = minimg(x[k * n + j] - x[k * n + i], p->box[k], p->periodic[k]);
        r2 = r2 + d * d;
    }
    return r2;
}

static int excluded(const uint8_t *role, int i, int j)
{
    return (role[i] == FIXED && role[j] == FIXED) || (role[i] == RIGID && role[j] == RIGID);
}

int64_t orc_pairs_brute(const orc_params *p, const double *x, const uint8_t *role,
                        double rl, int exclude, int32_t *ij, int64_t cap)
{
    const int n = p->n;
    const double rl2 = rl * rl;
    int64_t cnt = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            if (exclude && excluded(role, i, j)) continue;
            if (pair_r2(p, x, n, i, j) < rl2) {
                if (cnt < cap) { ij[2 * cnt] = i; ij[2 * cnt + 1] = j; }
                ++cnt;
            }
        }
    return cnt;
}

/* Cell list: per axis nc cells of edge >= rl (a single cell when fewer than
 * three would fit on a periodic axis); open axes span the current extent. */
typedef struct {
    int nc[3];
    double lo[3], h[3];
    int *head, *next;
} cells_t;

static int cell_coord(const cells_t *c, int k, double xk)
{
    int ci = (int)floor((xk - c->lo[k]) / c->h[k]);
    if (ci < 0) ci = 0;
    if (ci >= c->nc[k]) ci = c->nc[k] - 1;
    return ci;
}

static void cells_build(cells_t *c, const orc_params *p, const double *x, double rl)
{
    const int n = p->n;
    for (int k = 0; k < 3; ++k) { c->nc[k] = 1; c->lo[k] = 0.0; c->h[k] = 1.0; }
    for (int k = 0; k < p->dim; ++k) {
        if (p->periodic[k]) {
            int m = (int)floor(p->box[k] / rl);
            if (m < 3) m = 1;
            c->nc[k] = m;
            c->lo[k] = 0.0;
            c->h[k] = p->box[k] / m;
        } else {
            double mn = x[k * n], mx = x[k * n];
            for (int i = 1; i < n; ++i) {
                if (x[k * n + i] < mn) mn = x[k * n + i];
                if (x[k * n + i] > mx) mx = x[k * n + i];
            }
            int m = (int)floor((mx - mn) / rl);
            if (m < 1) m = 1;
            c->nc[k] = m;
            c->lo[k] = mn;
            c->h[k] = (mx - mn) / m;
            if (c->h[k] < rl) c->h[k] = rl;
        }
    }
    int ncell = c->nc[0] * c->nc[1] * c->nc[2];
    c->head = (int *)malloc(sizeof(int) * ncell);
    c->next = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
    for (int q = 0; q < ncell; ++q) c->head[q] = -1;
    for (int i = n - 1; i >= 0; --i) {
        int cc[3] = {0, 0, 0};
        for (int k = 0; k < p->dim; ++k) cc[k] = cell_coord(c, k, x[k * n + i]);
        int q = (cc[2] * c->nc[1] + cc[1]) * c->nc[0] + cc[0];
        c->next[i] = c->head[q];
        c->head[q] = i;
    }
}

static void cells_free(cells_t *c) { free(c->head); free(c->next); }

/* Visit every pair i<j in neighbouring cells once and apply fn to those with
 * r^2 < rl^2 (and not excluded when exclude != 0). */
typedef void (*pair_fn)(void *ctx, int i, int j);

static void for_pairs_cells(const orc_params *p, const double *x, const uint8_t *role,
                            double rl, int exclude, pair_fn fn, void *ctx)
{
    const int n = p->n;
    cells_t c;
    cells_build(&c, p, x, rl);
    const double rl2 = rl * rl;
    int lo[3], hi[3];
    for (int i = 0; i < n; ++i) {
        int cc[3] = {0, 0, 0};
        for (int k = 0; k < p->dim; ++k) cc[k] = cell_coord(&c, k, x[k * n + i]);
        for (int k = 0; k < 3; ++k) {
            if (c.nc[k] == 1) { lo[k] = 0; hi[k] = 0; }
            else { lo[k] = -1; hi[k] = 1; }
        }
        for (int oz = lo[2]; oz <= hi[2]; ++oz)
            for (int oy = lo[1]; oy <= hi[1]; ++oy)
                for (int ox = lo[0]; ox <= hi[0]; ++ox) {
                    int q3[3] = {cc[0] + ox, cc[1] + oy, cc[2] + oz};
                    int skip = 0;
                    for (int k = 0; k < 3; ++k) {
                        if (q3[k] < 0 || q3[k] >= c.nc[k]) {
                            if (k < p->dim && p->periodic[k]) q3[k] = (q3[k] + c.nc[k]) % c.nc[k];
                            else skip = 1;
                        }
                    }
                    if (skip) continue;
                    int q = (q3[2] * c.nc[1] + q3[1]) * c.nc[0] + q3[0];
                    for (int j = c.head[q]; j >= 0; j = c.next[j]) {
                        if (j <= i) continue;
                        if (exclude && excluded(role, i, j)) continue;
                        if (pair_r2(p, x, n, i, j) < rl2) fn(ctx, i, j);
                    }
                }
    }
    cells_free(&c);
}

typedef struct { int32_t *ij; int64_t cap, cnt; } collect_ctx;
static void collect_pair(void *vctx, int i, int j)
{
    collect_ctx *c = (collect_ctx *)vctx;
    if (c->cnt < c->cap) { c->ij[2 * c->cnt] = i; c->ij[2 * c->cnt + 1] = j; }
    c->cnt++;
}

int64_t orc_pairs_cells(const orc_params *p, const double *x, const uint8_t *role,
                        double rl, int exclude, int32_t *ij, int64_t cap)
{
    collect_ctx c = {ij, cap, 0};
    for_pairs_cells(p, x, role, rl, exclude, collect_pair, &c);
    return c.cnt;
}

/* ------------------------------------------------------------------------ */
/* System state */

static void place_rigid(orc_sys *s)
{
    const int n = s->n;
    for (int i = 0; i < n; ++i) {
        if (s->role[i] != RIGID) continue;
        for (int k = 0; k < s->dim; ++k)
            s->x[k * n + i] = wrap(s->XR[k] + s->cofs[k * n + i], s->p.box[k], s->p.periodic[k]);
    }
}

/* Rigid-body centre of mass from the current rigid atom positions, unwrapped
 * about the first rigid atom; offsets c_i = x_i - X_R. */
static void init_rigid(orc_sys *s)
{
    const int n = s->n;
    s->n_rigid = 0;
    s->first_rigid = -1;
    for (int i = 0; i < n; ++i)
        if (s->role[i] == RIGID) { if (s->first_rigid < 0) s->first_rigid = i; s->n_rigid++; }
    for (int k = 0; k < 3; ++k) { s->XR[k] = 0.0; s->VR[k] = 0.0; s->XR0[k] = 0.0; }
    if (s->n_rigid == 0) return;
    const int f = s->first_rigid;
    for (int k = 0; k < s->dim; ++k) {
        double xf = s->x[k * n + f];
        double sum = 0.0;
        for (int i = 0; i < n; ++i)
            if (s->role[i] == RIGID)
                sum += xf + minimg(s->x[k * n + i] - xf, s->p.box[k], s->p.periodic[k]);
        s->XR[k] = sum / s->n_rigid;
        for (int i = 0; i < n; ++i)
            if (s->role[i] == RIGID)
                s->cofs[k * n + i] = (xf + minimg(s->x[k * n + i] - xf, s->p.box[k], s->p.periodic[k])) - s->XR[k];
        s->XR0[k] = s->XR[k];
    }
    place_rigid(s);
}

orc_sys *orc_create(const orc_params *p, const double *x, const uint8_t *type,
                    const uint8_t *role, const double *rO)
{
    orc_sys *s = (orc_sys *)calloc(1, sizeof(orc_sys));
    s->p = *p;
    s->dim = p->dim;
    s->n = p->n;
    size_t nd = (size_t)p->dim * p->n;
    s->x = (double *)malloc(sizeof(double) * nd);
    s->v = (double *)calloc(nd, sizeof(double));
    s->rO = (double *)malloc(sizeof(double) * nd);
    s->cofs = (double *)calloc(nd, sizeof(double));
    s->ftot = (double *)calloc(nd, sizeof(double));
    s->tuu = (double *)calloc(nd, sizeof(double));
    s->qm = (double *)calloc(nd, sizeof(double));
    s->wn = (double *)calloc(nd, sizeof(double));
    s->hw = (double *)calloc(nd, sizeof(double));
    s->tww = (double *)calloc(nd, sizeof(double));
    s->type = (uint8_t *)malloc(p->n);
    s->role = (uint8_t *)malloc(p->n);
    memcpy(s->x, x, sizeof(double) * nd);
    memcpy(s->rO, rO ? rO : x, sizeof(double) * nd);
    memcpy(s->type, type, p->n);
    memcpy(s->role, role, p->n);
    init_rigid(s);
    return s;
}

void orc_destroy(orc_sys *s)
{
    if (!s) return;
    free(s->x); free(s->v); free(s->rO); free(s->cofs); free(s->ftot); free(s->tuu);
    free(s->qm); free(s->wn); free(s->hw); free(s->tww);
    free(s->type); free(s->role);
    free(s);
}

void orc_set_params(orc_sys *s, const orc_params *p)
{
    s->p = *p;
    s->have_force = 0;
}

/* New positions: mobile and fixed atoms are copied; the rigid body moves by
 * the minimum-image displacement of its first atom and the rigid atoms are
 * re-placed at X_R + c_i. */
void orc_set_positions(orc_sys *s, const double *x)
{
    const int n = s->n;
    if (s->n_rigid > 0) {
        const int f = s->first_rigid;
        for (int k = 0; k < s->dim; ++k)
            s->XR[k] = s->XR[k] + minimg(x[k * n + f] - s->x[k * n + f], s->p.box[k], s->p.periodic[k]);
    }
    for (int i = 0; i < n; ++i)
        if (s->role[i] != RIGID)
            for (int k = 0; k < s->dim; ++k) s->x[k * n + i] = x[k * n + i];
    place_rigid(s);
    s->have_force = 0;
}

/* New velocities: mobile atoms copied; fixed atoms zero; the rigid body takes
 * the mean velocity of its atoms. */
void orc_set_velocities(orc_sys *s, const double *v)
{
    const int n = s->n;
    for (int k = 0; k < s->dim; ++k) {
        double sum = 0.0;
        for (int i = 0; i < n; ++i) {
            if (s->role[i] == MOBILE) s->v[k * n + i] = v[k * n + i];
            else if (s->role[i] == FIXED) s->v[k * n + i] = 0.0;
            else sum += v[k * n + i];
        }
        if (s->n_rigid > 0) s->VR[k] = sum / s->n_rigid;
        for (int i = 0; i < n; ++i)
            if (s->role[i] == RIGID) s->v[k * n + i] = s->VR[k];
    }
}

void orc_set_reference(orc_sys *s, const double *rO)
{
    memcpy(s->rO, rO, sizeof(double) * (size_t)s->dim * s->n);
    s->have_force = 0;
}

void orc_set_pair_method(orc_sys *s, int brute) { s->brute = brute; }

/* Maxwell-Boltzmann draw: v = sqrt(kT/m) z with tag 1 at step 0; the rigid
 * body (particle index n) with its total mass. */
void orc_init_velocities(orc_sys *s)
{
    const int n = s->n;
    double z[4];
    for (int i = 0; i < n; ++i) {
        for (int k = 0; k < s->dim; ++k) s->v[k * n + i] = 0.0;
        if (s->role[i] != MOBILE) continue;
        orc_normals(s->p.seed, 0, (uint32_t)i, 1u, z);
        double sc = sqrt(s->p.kT / s->p.mass);
        for (int k = 0; k < s->dim; ++k) s->v[k * n + i] = sc * z[k];
    }
    if (s->n_rigid > 0) {
        orc_normals(s->p.seed, 0, (uint32_t)n, 1u, z);
        double M = s->p.mass * s->n_rigid;
        double sc = sqrt(s->p.kT / M);
        for (int k = 0; k < s->dim; ++k) s->VR[k] = sc * z[k];
        for (int i = 0; i < n; ++i)
            if (s->role[i] == RIGID)
                for (int k = 0; k < s->dim; ++k) s->v[k * n + i] = s->VR[k];
    }
}

/* ------------------------------------------------------------------------ */
/* Energy, forces and the Hessian-vector product */

typedef struct {
    const orc_sys *s;
    const double *u;
    double *f, *hu, *e_atom, *tuu;
    double e_lj;
    double shift[2][2];
} pair_ctx;

/* One Lennard-Jones pair (eq. 9), energy-shifted at rc, or a harmonic tip
 * bond (eq. 12) between tip atoms when the model has them.  Delta = x_i - x_j
 * (minimum image).  f = -phi'(r)/r so that F_i += f Delta; the pair Hessian
 * block is B I + C Delta Delta^T with B = phi'/r = -f and
 * C = (phi'' - phi'/r)/r^2; (Hu)_i += B w + C (Delta.w) Delta, w = u_i - u_j,
 * with the opposite sign on j.  The pair's share of u.Hu is
 * B |w|^2 + C (Delta.w)^2; its gradient in x_i at fixed u, with dB/dr = r C
 * and Dc = (dC/dr)/r, is (C |w|^2 + Dc (Delta.w)^2) Delta + 2 C (Delta.w) w,
 * the pair's share of T[u,u] (opposite sign on j). */
static void lj_pair(void *vctx, int i, int j)
{
    pair_ctx *c = (pair_ctx *)vctx;
    const orc_sys *s = c->s;
    const orc_params *p = &s->p;
    const int n = s->n, dim = s->dim;
    double D[3] = {0, 0, 0}, w[3] = {0, 0, 0};
    double r2 = 0.0;
    for (int k = 0; k < dim; ++k) {
        D[k] = -minimg(s->x[k * n + j] - s->x[k * n + i], p->box[k], p->periodic[k]);
        r2 = r2 + D[k] * D[k];
    }
    int a = s->type[i], b = s->type[j];
    double phi, f, C, Dc;
    if (p->tip_bonds && a == 1 && b == 1) {
        /* harmonic tip bond (eq. 12): phi = k (r - r0)^2 / 2, so
         * f = -phi'/r = -k (r - r0)/r and C = (phi'' - phi'/r)/r^2
         * = k r0 / r^3 */
        if (!(r2 < p->r_bond_cut * p->r_bond_cut)) return;
        double r = sqrt(r2), dr = r - p->r_bond;
        phi = 0.5 * p->k_bond * dr * dr;
        f = -p->k_bond * dr / r;
        C = p->k_bond * p->r_bond / (r * r2);
        Dc = -3.0 * p->k_bond * p->r_bond / (r * r2 * r2);
    } else {
        if (!(r2 < p->rc * p->rc)) return;
        double eps = p->eps[a][b];
        double s2 = p->sig[a][b] * p->sig[a][b];
        double r2i = 1.0 / r2;
        double sr2 = s2 * r2i;
        double sr6 = sr2 * sr2 * sr2;
        phi = 4.0 * eps * (sr6 * sr6 - sr6) - c->shift[a][b];
        f = eps * r2i * sr6 * (48.0 * sr6 - 24.0);
        C = eps * r2i * r2i * sr6 * (672.0 * sr6 - 192.0);
        /* C = eps (672 s^12 r^-16 - 192 s^6 r^-10); (dC/dr)/r: */
        Dc = eps * r2i * r2i * r2i * sr6 * (-10752.0 * sr6 + 1920.0);
    }
    double B = -f;
    double Dw = 0.0;
    for (int k = 0; k < dim; ++k) {
        w[k] = c->u[k * n + i] - c->u[k * n + j];
        Dw = Dw + D[k] * w[k];
    }
    double w2 = 0.0;
    for (int k = 0; k < dim; ++k) w2 = w2 + w[k] * w[k];
    for (int k = 0; k < dim; ++k) {
        c->f[k * n + i] += f * D[k];
        c->f[k * n + j] -= f * D[k];
        double h = B * w[k] + C * Dw * D[k];
        c->hu[k * n + i] += h;
        c->hu[k * n + j] -= h;
        double t = (C * w2 + Dc * Dw * Dw) * D[k] + 2.0 * C * Dw * w[k];
        c->tuu[k * n + i] += t;
        c->tuu[k * n + j] -= t;
    }
    c->e_atom[i] += 0.5 * phi;
    c->e_atom[j] += 0.5 * phi;
    c->e_lj += phi;
}

/* The switch of eq. 14 (eq. 15 has the same form) of a bias variable v with
 * critical values lo ("lower") and hi ("upper"), and its derivative d dV/dv:
 * dV_max at or beyond hi, zero at or beyond lo, dV_max (1 - xi^m)^2 with
 * xi = (v - hi)/(lo - hi) between them.  With lo < hi (slope, curvature) the
 * bias is full for large values; with lo > hi (the distance, which grows
 * towards the dividing surface) for small ones. */
static void bias_switch(const orc_params *p, double v, double lo, double hi, double *dv, double *dvp)
{
    const int up = lo < hi;
    if (up ? v >= hi : v <= hi) { *dv = p->dv_max; *dvp = 0.0; return; }
    if (up ? v <= lo : v >= lo) { *dv = 0.0; *dvp = 0.0; return; }
    double xi = (v - hi) / (lo - hi);
    double xm1 = 1.0;
    for (int q = 0; q < p->m_b - 1; ++q) xm1 *= xi;  /* xi^(m-1) */
    double xm = xm1 * xi;                            /* xi^m */
    double one = 1.0 - xm;
    *dv = p->dv_max * one * one;
    *dvp = -2.0 * p->m_b * p->dv_max * one * xm1 / (lo - hi);
}

static double slider_at(const orc_params *p, int64_t step)
{
    return p->x_slider + p->v_slider * ((double)step * p->dt);
}

/* Full evaluation at the current positions.  Writes the scalars into *sc. */
static void evaluate(orc_sys *s, double *f, double *hu, double *fb, double *ftot,
                     double *e_atom, orc_scalars *sc)
{
    const orc_params *p = &s->p;
    const int n = s->n, dim = s->dim;
    const size_t nd = (size_t)dim * n;
    double *u = (double *)calloc(nd, sizeof(double));
    memset(f, 0, sizeof(double) * nd);
    memset(hu, 0, sizeof(double) * nd);
    memset(e_atom, 0, sizeof(double) * n);

    /* u = r - r_O (eq. 7), minimum image; fixed atoms are not degrees of
     * freedom and carry u = 0. */
    for (int i = 0; i < n; ++i) {
        if (s->role[i] == FIXED) continue;
        for (int k = 0; k < dim; ++k)
            u[k * n + i] = minimg(s->x[k * n + i] - s->rO[k * n + i], p->box[k], p->periodic[k]);
    }

    pair_ctx c;
    memset(s->tuu, 0, sizeof(double) * nd);
    c.s = s; c.u = u; c.f = f; c.hu = hu; c.e_atom = e_atom; c.tuu = s->tuu; c.e_lj = 0.0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double s2 = p->sig[a][b] * p->sig[a][b];
            double sr2 = s2 / (p->rc * p->rc);
            double sr6 = sr2 * sr2 * sr2;
            c.shift[a][b] = 4.0 * p->eps[a][b] * (sr6 * sr6 - sr6);
        }
    if (s->brute) {
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) {
                if (excluded(s->role, i, j)) continue;
                lj_pair(&c, i, j);
            }
    } else {
        for_pairs_cells(p, s->x, s->role, p->rc, 1, lj_pair, &c);
    }

    /* Slider drive on the rigid layer (Sec. 3.1.1): spring k along x to the
     * slider, a y anchor of the same stiffness in 3D, and the normal load F_N
     * pushing down along the last axis.  Each rigid atom carries 1/n_R of the
     * drive force; the drive Hessian couples all rigid atoms with k/n_R^2. */
    double v_drive = 0.0, xs = slider_at(p, s->step), x_tip = 0.0, f_lat = 0.0;
    if (s->n_rigid > 0) {
        const int nR = s->n_rigid;
        const int perp = dim - 1;
        double Fd[3] = {0, 0, 0};
        x_tip = s->XR[0] - s->XR0[0];
        f_lat = p->k_spring * (xs - x_tip);
        v_drive = 0.5 * p->k_spring * (xs - x_tip) * (xs - x_tip);
        Fd[0] = p->k_spring * (xs - x_tip);
        if (dim == 3) {
            double dy = s->XR[1] - s->XR0[1];
            v_drive += 0.5 * p->k_spring * dy * dy;
            Fd[1] = -p->k_spring * dy;
        }
        v_drive += p->f_normal * (s->XR[perp] - s->XR0[perp]);
        Fd[perp] += -p->f_normal;
        double UR[3] = {0, 0, 0};
        for (int i = 0; i < n; ++i)
            if (s->role[i] == RIGID)
                for (int k = 0; k < dim; ++k) UR[k] += u[k * n + i];
        int nspring = (dim == 3) ? 2 : 1;   /* axes with a spring */
        for (int i = 0; i < n; ++i) {
            if (s->role[i] != RIGID) continue;
            for (int k = 0; k < dim; ++k) f[k * n + i] += Fd[k] / nR;
            for (int k = 0; k < nspring; ++k)
                hu[k * n + i] += p->k_spring / ((double)nR * nR) * UR[k];
        }
    }

    /* d (eq. 7), slope g = grad V . s = -F.u/d (eq. 5), curvature
     * kappa = s.H s = u.Hu/d^2 (eq. 6). */
    double d2 = 0.0, G = 0.0, uHu = 0.0;
    for (int i = 0; i < n; ++i) {
        if (s->role[i] == FIXED) continue;
        for (int k = 0; k < dim; ++k) {
            d2 += u[k * n + i] * u[k * n + i];
            G += f[k * n + i] * u[k * n + i];
            uHu += u[k * n + i] * hu[k * n + i];
        }
    }
    double d = sqrt(d2);
    const int has_d = d >= 1e-12;
    double g = has_d ? -G / d : 0.0;
    double kappa = has_d ? uHu / d2 : 0.0;

    /* The eigenvalue variable (eq. 15): lambda = w.Hw, the Rayleigh quotient
     * of the reduced Hessian along the mode estimate, with w = P q/|q| the
     * mode spread over the atoms (each rigid atom moves with the rigid body,
     * fixed atoms do not move) and |q| taken over the degrees of freedom.
     * A second pass of the pair terms with u replaced by w gives H w and
     * T[w,w], the gradient of lambda at fixed q; the drive's Hessian adds
     * its share on the rigid atoms as for H u. */
    const int eig = (p->bias_var1 == 3 || p->bias_var2 == 3);
    double lam = 0.0;
    int have_q = 0;
    memset(s->wn, 0, sizeof(double) * nd);
    memset(s->hw, 0, sizeof(double) * nd);
    memset(s->tww, 0, sizeof(double) * nd);
    if (eig) {
        double q2 = 0.0;
        for (int i = 0; i < n; ++i)
            if (s->role[i] == MOBILE)
                for (int k = 0; k < dim; ++k) q2 += s->qm[k * n + i] * s->qm[k * n + i];
        if (s->n_rigid > 0)
            for (int k = 0; k < dim; ++k)
                q2 += s->qm[k * n + s->first_rigid] * s->qm[k * n + s->first_rigid];
        have_q = q2 > 0.0;
        if (have_q) {
            const double inv = 1.0 / sqrt(q2);
            for (int i = 0; i < n; ++i) {
                if (s->role[i] == FIXED) continue;
                const int src = s->role[i] == RIGID ? s->first_rigid : i;
                for (int k = 0; k < dim; ++k) s->wn[k * n + i] = s->qm[k * n + src] * inv;
            }
            double *f2 = (double *)calloc(nd, sizeof(double));
            double *e2 = (double *)calloc((size_t)n, sizeof(double));
            pair_ctx c2 = c;
            c2.u = s->wn; c2.f = f2; c2.hu = s->hw; c2.e_atom = e2; c2.tuu = s->tww; c2.e_lj = 0.0;
            if (s->brute) {
                for (int i = 0; i < n; ++i)
                    for (int j = i + 1; j < n; ++j) {
                        if (excluded(s->role, i, j)) continue;
                        lj_pair(&c2, i, j);
                    }
            } else {
                for_pairs_cells(p, s->x, s->role, p->rc, 1, lj_pair, &c2);
            }
            free(f2);
            free(e2);
            if (s->n_rigid > 0) {
                const int nR = s->n_rigid, nspring = (dim == 3) ? 2 : 1;
                double WR[3] = {0, 0, 0};
                for (int i = 0; i < n; ++i)
                    if (s->role[i] == RIGID)
                        for (int k = 0; k < dim; ++k) WR[k] += s->wn[k * n + i];
                for (int i = 0; i < n; ++i) {
                    if (s->role[i] != RIGID) continue;
                    for (int k = 0; k < nspring; ++k)
                        s->hw[k * n + i] += p->k_spring / ((double)nR * nR) * WR[k];
                }
            }
            for (int i = 0; i < n; ++i) {
                if (s->role[i] == FIXED) continue;
                for (int k = 0; k < dim; ++k) lam += s->wn[k * n + i] * s->hw[k * n + i];
            }
        }
    }

    /* Bias (eq. 13): dV = dV1(v1) + dV2(v2) - dV1 dV2 / dV_max, each dVi the
     * switch of eq. 14 in its variable (no second variable: dV2 = 0, and
     * eq. 13 reduces to dV1).  Its force is -grad dV, by the chain rule
     * -(1 - dV2/dV_max) dV1' grad v1 - (1 - dV1/dV_max) dV2' grad v2. */
    const double val[4] = {g, kappa, d, lam};
    double dv1 = 0.0, dvp1 = 0.0, dv2 = 0.0, dvp2 = 0.0;
    const int v1 = p->bias_var1, v2 = p->bias_var2;
    if (p->bias_on) {
        bias_switch(p, val[v1], p->g_lo, p->g_hi, &dv1, &dvp1);
        if (v2 >= 0) bias_switch(p, val[v2], p->b2_lo, p->b2_hi, &dv2, &dvp2);
    }
    double dv = dv1, w1 = dvp1, w2 = 0.0;
    if (p->bias_on && v2 >= 0) {
        dv = dv1 + dv2 - dv1 * dv2 / p->dv_max;
        w1 = dvp1 * (1.0 - dv2 / p->dv_max);   /* d dV / d v1 */
        w2 = dvp2 * (1.0 - dv1 / p->dv_max);   /* d dV / d v2 */
    }
    double dvp = w1;
    for (size_t q = 0; q < nd; ++q) fb[q] = 0.0;
    if (p->bias_on && has_d && (w1 != 0.0 || w2 != 0.0)) {
        for (int i = 0; i < n; ++i) {
            if (s->role[i] == FIXED) continue;
            for (int k = 0; k < dim; ++k) {
                const size_t q = (size_t)k * n + i;
                double grad[4];
                grad[0] = (hu[q] - f[q] - g * u[q] / d) / d;
                grad[1] = (2.0 * hu[q] + s->tuu[q]) / d2 - 2.0 * kappa * u[q] / d2;
                grad[2] = u[q] / d;
                grad[3] = s->tww[q];
                double gr = w1 * grad[v1];
                if (v2 >= 0) gr += w2 * grad[v2];
                fb[q] = -gr;
            }
        }
    }
    for (size_t q = 0; q < nd; ++q) ftot[q] = f[q] + fb[q];
    for (int k = 0; k < 3; ++k) s->FR[k] = 0.0;
    for (int i = 0; i < n; ++i)
        if (s->role[i] == RIGID)
            for (int k = 0; k < dim; ++k) s->FR[k] += ftot[k * n + i];

    /* kinetic energy: mobile atoms plus the rigid body */
    double ek = 0.0;
    for (int i = 0; i < n; ++i)
        if (s->role[i] == MOBILE)
            for (int k = 0; k < dim; ++k) ek += 0.5 * p->mass * s->v[k * n + i] * s->v[k * n + i];
    if (s->n_rigid > 0)
        for (int k = 0; k < dim; ++k) ek += 0.5 * p->mass * s->n_rigid * s->VR[k] * s->VR[k];

    sc->e_lj = c.e_lj;
    sc->v_drive = v_drive;
    sc->e_pot = c.e_lj + v_drive;
    sc->e_kin = ek;
    sc->d = d;
    sc->g = g;
    sc->dv = dv;
    sc->dvp = dvp;
    sc->kappa = kappa;
    sc->lambda = lam;
    sc->dv1 = dv1;
    sc->dv2 = dv2;
    sc->e_nhc = nhc_energy(s);
    sc->x_slider = xs;
    sc->x_tip = x_tip;
    sc->f_lat = f_lat;
    sc->t_md = s->t_md;
    sc->t_hyper = s->t_hyper;
    sc->step = s->step;
    sc->flags = isfinite(sc->e_pot) ? 0 : 1;
    free(u);
}

void orc_compute(orc_sys *s, double *f_lj, double *hu, double *f_b, double *f_tot,
                 double *e_atom, orc_scalars *out)
{
    const size_t nd = (size_t)s->dim * s->n;
    double *F = (double *)malloc(sizeof(double) * nd);
    double *H = (double *)malloc(sizeof(double) * nd);
    double *B = (double *)malloc(sizeof(double) * nd);
    double *E = (double *)malloc(sizeof(double) * s->n);
    orc_scalars sc;
    evaluate(s, F, H, B, s->ftot, E, &sc);
    s->have_force = 1;
    s->last = sc;
    if (f_lj) memcpy(f_lj, F, sizeof(double) * nd);
    if (hu) memcpy(hu, H, sizeof(double) * nd);
    if (f_b) memcpy(f_b, B, sizeof(double) * nd);
    if (f_tot) memcpy(f_tot, s->ftot, sizeof(double) * nd);
    if (e_atom) memcpy(e_atom, E, sizeof(double) * s->n);
    if (out) *out = sc;
    free(F); free(H); free(B); free(E);
}

/* One rotation step of the eigenvalue variable's mode estimate after an
 * evaluation: q <- w - alpha (P^T H w - lambda w) over the degrees of
 * freedom (w the unit mode of that evaluation, P^T H w's rigid-body row the
 * sum over its atoms), a gradient step on the Rayleigh quotient that turns
 * w towards the lowest mode; normalised at the next evaluation. */
static void rotate_mode(orc_sys *s)
{
    const orc_params *p = &s->p;
    const int n = s->n, dim = s->dim;
    if (!(p->bias_var1 == 3 || p->bias_var2 == 3)) return;
    const double lam = s->last.lambda, a = p->mode_alpha;
    int any = 0;
    for (int i = 0; i < n && !any; ++i)
        for (int k = 0; k < dim; ++k) any = any || s->wn[k * n + i] != 0.0;
    if (!any) return;
    for (int i = 0; i < n; ++i) {
        if (s->role[i] != MOBILE) continue;
        for (int k = 0; k < dim; ++k) {
            const size_t q = (size_t)k * n + i;
            s->qm[q] = s->wn[q] - a * (s->hw[q] - lam * s->wn[q]);
        }
    }
    if (s->n_rigid > 0) {
        const int f = s->first_rigid;
        for (int k = 0; k < dim; ++k) {
            double HR = 0.0;
            for (int i = 0; i < n; ++i)
                if (s->role[i] == RIGID) HR += s->hw[k * n + i];
            const double qR = s->wn[k * n + f] - a * (HR - lam * s->wn[k * n + f]);
            for (int i = 0; i < n; ++i)
                if (s->role[i] == RIGID) s->qm[k * n + i] = qR;
        }
    }
}

void orc_set_mode(orc_sys *s, const double *q)
{
    const int n = s->n;
    for (int i = 0; i < n; ++i) {
        const int src = s->role[i] == RIGID ? s->first_rigid : i;
        for (int k = 0; k < s->dim; ++k)
            s->qm[k * n + i] = s->role[i] == FIXED ? 0.0 : q[k * n + src];
    }
    s->have_force = 0;
}

void orc_get_mode(const orc_sys *s, double *q)
{
    const int n = s->n, dim = s->dim;
    double q2 = 0.0;
    for (int i = 0; i < n; ++i)
        if (s->role[i] == MOBILE)
            for (int k = 0; k < dim; ++k) q2 += s->qm[k * n + i] * s->qm[k * n + i];
    if (s->n_rigid > 0)
        for (int k = 0; k < dim; ++k) q2 += s->qm[k * n + s->first_rigid] * s->qm[k * n + s->first_rigid];
    const double inv = q2 > 0.0 ? 1.0 / sqrt(q2) : 0.0;
    for (size_t k = 0; k < (size_t)dim * n; ++k) q[k] = s->qm[k] * inv;
}

void orc_rotate_mode(orc_sys *s)
{
    const size_t nd = (size_t)s->dim * s->n;
    double *F = (double *)malloc(sizeof(double) * nd);
    double *H = (double *)malloc(sizeof(double) * nd);
    double *B = (double *)malloc(sizeof(double) * nd);
    double *E = (double *)malloc(sizeof(double) * s->n);
    evaluate(s, F, H, B, s->ftot, E, &s->last);
    s->have_force = 1;
    rotate_mode(s);
    s->have_force = 0;
    free(F); free(H); free(B); free(E);
}

/* ------------------------------------------------------------------------ */
/* Langevin BAOAB (Leimkuhler & Matthews 2013) per integrated degree of
 * freedom -- each mobile atom and the rigid body as one particle of mass
 * n_R m:  B: v += dt/2 F/m;  A: x += dt/2 v;  O: v = c1 v + c2 xi;
 * A: x += dt/2 v;  new forces;  B: v += dt/2 F/m.  Fixed atoms never move.
 * The noise xi for step n uses Philox counter (n, particle, tag 0). */
/* ------------------------------------------------------------------------ */
/* Nose-Hoover chain (Martyna, Klein, Tuckerman 1992) */

static int nhc_dof(const orc_sys *s)
{
    int nm = 0;
    for (int i = 0; i < s->n; ++i) nm += s->role[i] == MOBILE;
    return s->dim * (nm + (s->n_rigid > 0 ? 1 : 0));
}

/* Twice the kinetic energy of the integrated degrees of freedom. */
static double twice_kinetic(const orc_sys *s)
{
    const int n = s->n, dim = s->dim;
    double k2 = 0.0;
    for (int i = 0; i < n; ++i)
        if (s->role[i] == MOBILE)
            for (int k = 0; k < dim; ++k) k2 += s->p.mass * s->v[k * n + i] * s->v[k * n + i];
    if (s->n_rigid > 0)
        for (int k = 0; k < dim; ++k) k2 += s->p.mass * s->n_rigid * s->VR[k] * s->VR[k];
    return k2;
}

/* The force on chain thermostat j (0-based) given twice the kinetic
 * energy k2 of the particles. */
static double nhc_G(const orc_sys *s, int j, double k2, const double Q[4])
{
    const double kT = s->p.kT;
    if (j == 0) return (k2 - nhc_dof(s) * kT) / Q[0];
    return (Q[j - 1] * s->xi[j - 1] * s->xi[j - 1] - kT) / Q[j];
}

/* Propagate the chain over a time h (half a step): the thermostat
 * velocities from the chain's end inwards over h/2, the particle velocities
 * scaled by exp(-xi_1 h) and the thermostat positions advanced by h, then the
 * thermostat velocities outwards over h/2; each inner update is wrapped in
 * exp(-xi_{j+1} h/4) factors.  Returns the velocity scale factor. */
static double nhc_propagate(orc_sys *s, double h)
{
    const int M = s->p.nhc_len;
    const double kT = s->p.kT, t2 = s->p.nhc_tau * s->p.nhc_tau;
    double Q[4];
    Q[0] = nhc_dof(s) * kT * t2;
    for (int j = 1; j < 4; ++j) Q[j] = kT * t2;
    double k2 = twice_kinetic(s);
    s->xi[M - 1] += 0.5 * h * nhc_G(s, M - 1, k2, Q);
    for (int j = M - 2; j >= 0; --j) {
        const double e = exp(-0.25 * h * s->xi[j + 1]);
        s->xi[j] *= e;
        s->xi[j] += 0.5 * h * nhc_G(s, j, k2, Q);
        s->xi[j] *= e;
    }
    const double scale = exp(-h * s->xi[0]);
    k2 *= scale * scale;
    for (int j = 0; j < M; ++j) s->eta[j] += h * s->xi[j];
    for (int j = 0; j < M - 1; ++j) {
        const double e = exp(-0.25 * h * s->xi[j + 1]);
        s->xi[j] *= e;
        s->xi[j] += 0.5 * h * nhc_G(s, j, k2, Q);
        s->xi[j] *= e;
    }
    s->xi[M - 1] += 0.5 * h * nhc_G(s, M - 1, k2, Q);
    return scale;
}

static void scale_velocities(orc_sys *s, double c)
{
    const int n = s->n, dim = s->dim;
    for (int i = 0; i < n; ++i)
        if (s->role[i] != FIXED)
            for (int k = 0; k < dim; ++k) s->v[k * n + i] *= c;
    for (int k = 0; k < dim; ++k) s->VR[k] *= c;
}

static double nhc_energy(const orc_sys *s)
{
    if (s->p.thermostat != 1) return 0.0;
    const double kT = s->p.kT, t2 = s->p.nhc_tau * s->p.nhc_tau;
    double e = nhc_dof(s) * kT * s->eta[0];
    for (int j = 0; j < s->p.nhc_len; ++j) {
        const double Q = (j == 0 ? nhc_dof(s) * kT : kT) * t2;
        e += 0.5 * Q * s->xi[j] * s->xi[j];
        if (j > 0) e += kT * s->eta[j];
    }
    return e;
}

void orc_get_nhc(const orc_sys *s, double xi[4], double eta[4])
{
    for (int j = 0; j < 4; ++j) { xi[j] = s->xi[j]; eta[j] = s->eta[j]; }
}

void orc_set_nhc(orc_sys *s, const double xi[4], const double eta[4])
{
    for (int j = 0; j < 4; ++j) { s->xi[j] = xi[j]; s->eta[j] = eta[j]; }
}

/* One step of velocity Verlet inside the chain's half steps:
 * chain(dt/2); v += dt/2 F/m; x += dt v; forces; v += dt/2 F/m; chain(dt/2). */
static void nhc_vv_step(orc_sys *s, double *F, double *H, double *B, double *E)
{
    const orc_params *p = &s->p;
    const int n = s->n, dim = s->dim;
    const double dt = p->dt, hdt = 0.5 * p->dt;
    const double M = p->mass * s->n_rigid;
    scale_velocities(s, nhc_propagate(s, hdt));
    for (int i = 0; i < n; ++i) {
        if (s->role[i] != MOBILE) continue;
        for (int k = 0; k < dim; ++k) {
            double v = s->v[k * n + i] + hdt * s->ftot[k * n + i] / p->mass;
            s->v[k * n + i] = v;
            s->x[k * n + i] = wrap(s->x[k * n + i] + dt * v, p->box[k], p->periodic[k]);
        }
    }
    if (s->n_rigid > 0) {
        for (int k = 0; k < dim; ++k) {
            s->VR[k] = s->VR[k] + hdt * s->FR[k] / M;
            s->XR[k] = s->XR[k] + dt * s->VR[k];
        }
        place_rigid(s);
    }
    s->step = s->step + 1;
    evaluate(s, F, H, B, s->ftot, E, &s->last);
    rotate_mode(s);
    for (int i = 0; i < n; ++i) {
        if (s->role[i] != MOBILE) continue;
        for (int k = 0; k < dim; ++k) s->v[k * n + i] = s->v[k * n + i] + hdt * s->ftot[k * n + i] / p->mass;
    }
    if (s->n_rigid > 0)
        for (int k = 0; k < dim; ++k) s->VR[k] = s->VR[k] + hdt * s->FR[k] / M;
    scale_velocities(s, nhc_propagate(s, hdt));
    for (int i = 0; i < n; ++i)
        if (s->role[i] == RIGID)
            for (int k = 0; k < dim; ++k) s->v[k * n + i] = s->VR[k];
}

void orc_step(orc_sys *s, int64_t nsteps)
{
    const orc_params *p = &s->p;
    const int n = s->n, dim = s->dim;
    const size_t nd = (size_t)dim * n;
    double *F = (double *)malloc(sizeof(double) * nd);
    double *H = (double *)malloc(sizeof(double) * nd);
    double *B = (double *)malloc(sizeof(double) * nd);
    double *E = (double *)malloc(sizeof(double) * n);
    if (!s->have_force) {
        evaluate(s, F, H, B, s->ftot, E, &s->last);
        s->have_force = 1;
    }
    const double dt = p->dt, hdt = 0.5 * p->dt;
    const double c1 = exp(-p->gamma * dt);
    const double c2 = sqrt((1.0 - c1 * c1) * p->kT / p->mass);
    const double M = p->mass * s->n_rigid;
    const double c2R = s->n_rigid > 0 ? sqrt((1.0 - c1 * c1) * p->kT / M) : 0.0;
    double z[4];
    for (int64_t it = 0; it < nsteps; ++it) {
        const int64_t step = s->step;
        if (p->thermostat == 1) {
            nhc_vv_step(s, F, H, B, E);
            goto clock;
        }
        for (int i = 0; i < n; ++i) {
            if (s->role[i] != MOBILE) continue;
            orc_normals(p->seed, step, (uint32_t)i, 0u, z);
            for (int k = 0; k < dim; ++k) {
                double v = s->v[k * n + i];
                double x = s->x[k * n + i];
                v = v + hdt * s->ftot[k * n + i] / p->mass;
                x = x + hdt * v;
                v = c1 * v + c2 * z[k];
                x = x + hdt * v;
                s->x[k * n + i] = wrap(x, p->box[k], p->periodic[k]);
                s->v[k * n + i] = v;
            }
        }
        if (s->n_rigid > 0) {
            orc_normals(p->seed, step, (uint32_t)n, 0u, z);
            for (int k = 0; k < dim; ++k) {
                double v = s->VR[k];
                double x = s->XR[k];
                v = v + hdt * s->FR[k] / M;
                x = x + hdt * v;
                v = c1 * v + c2R * z[k];
                x = x + hdt * v;
                s->XR[k] = x;
                s->VR[k] = v;
            }
            place_rigid(s);
        }
        s->step = step + 1;
        evaluate(s, F, H, B, s->ftot, E, &s->last);
        rotate_mode(s);
        for (int i = 0; i < n; ++i) {
            if (s->role[i] != MOBILE) continue;
            for (int k = 0; k < dim; ++k)
                s->v[k * n + i] = s->v[k * n + i] + hdt * s->ftot[k * n + i] / p->mass;
        }
        if (s->n_rigid > 0) {
            for (int k = 0; k < dim; ++k) s->VR[k] = s->VR[k] + hdt * s->FR[k] / M;
            for (int i = 0; i < n; ++i)
                if (s->role[i] == RIGID)
                    for (int k = 0; k < dim; ++k) s->v[k * n + i] = s->VR[k];
        }
    clock:
        /* boosted clock, right Riemann sum: dV at the post-step positions */
        s->t_md += dt;
        s->t_hyper += dt * exp(s->last.dv / p->kT);
        /* refresh kinetic energy and clock in the reported scalars */
        double ek = 0.0;
        for (int i = 0; i < n; ++i)
            if (s->role[i] == MOBILE)
                for (int k = 0; k < dim; ++k) ek += 0.5 * p->mass * s->v[k * n + i] * s->v[k * n + i];
        for (int k = 0; k < dim; ++k) ek += 0.5 * M * s->VR[k] * s->VR[k];
        s->last.e_kin = ek;
        s->last.e_nhc = nhc_energy(s);
        s->last.t_md = s->t_md;
        s->last.t_hyper = s->t_hyper;
    }
    free(F); free(H); free(B); free(E);
}

void orc_get_positions(const orc_sys *s, double *x)
{
    memcpy(x, s->x, sizeof(double) * (size_t)s->dim * s->n);
}

void orc_get_velocities(const orc_sys *s, double *v)
{
    memcpy(v, s->v, sizeof(double) * (size_t)s->dim * s->n);
}

void orc_get_scalars(const orc_sys *s, orc_scalars *out) { *out = s->last; }

void orc_get_rigid(const orc_sys *s, double XR[3], double VR[3], double XR0[3])
{
    for (int k = 0; k < 3; ++k) { XR[k] = s->XR[k]; VR[k] = s->VR[k]; XR0[k] = s->XR0[k]; }
}

/* ------------------------------------------------------------------------ */
/* FIRE (Bitzek et al., PRL 97, 170201, 2006) on the unbiased potential:
 * mobile atoms and the rigid body are the degrees of freedom; MD with
 * velocity mixing v <- (1-a) v + a |v| F/|F| while P = F.v > 0, restart with a
 * smaller step when P <= 0. */
int64_t orc_fire(orc_sys *s, double ftol, int64_t maxit)
{
    orc_params saved = s->p;
    s->p.bias_on = 0;
    const int n = s->n, dim = s->dim;
    const size_t nd = (size_t)dim * n;
    double *F = (double *)malloc(sizeof(double) * nd);
    double *H = (double *)malloc(sizeof(double) * nd);
    double *B = (double *)malloc(sizeof(double) * nd);
    double *E = (double *)malloc(sizeof(double) * n);
    double *v = (double *)calloc(nd, sizeof(double));
    double VR[3] = {0, 0, 0};
    const double M = s->p.mass * (s->n_rigid > 0 ? s->n_rigid : 1);
    double dt = s->p.dt, dtmax = 10.0 * s->p.dt, alpha = 0.1;
    const double alpha0 = 0.1, finc = 1.1, fdec = 0.5, falpha = 0.99;
    const int nmin = 5;
    int since_neg = 0;
    int64_t it;
    orc_scalars sc;
    evaluate(s, F, H, B, s->ftot, E, &sc);
    for (it = 0; it < maxit; ++it) {
        /* convergence on max |F| over degrees of freedom */
        double fmax2 = 0.0;
        for (int i = 0; i < n; ++i) {
            if (s->role[i] != MOBILE) continue;
            double a = 0.0;
            for (int k = 0; k < dim; ++k) a += F[k * n + i] * F[k * n + i];
            if (a > fmax2) fmax2 = a;
        }
        if (s->n_rigid > 0) {
            double a = 0.0;
            for (int k = 0; k < dim; ++k) a += s->FR[k] * s->FR[k];
            if (a > fmax2) fmax2 = a;
        }
        if (sqrt(fmax2) < ftol) break;
        /* power and norms */
        double P = 0.0, vv = 0.0, ff = 0.0;
        for (int i = 0; i < n; ++i) {
            if (s->role[i] != MOBILE) continue;
            for (int k = 0; k < dim; ++k) {
                P += F[k * n + i] * v[k * n + i];
                vv += v[k * n + i] * v[k * n + i];
                ff += F[k * n + i] * F[k * n + i];
            }
        }
        for (int k = 0; k < dim && s->n_rigid > 0; ++k) {
            P += s->FR[k] * VR[k];
            vv += VR[k] * VR[k];
            ff += s->FR[k] * s->FR[k];
        }
        double vn = sqrt(vv), fn = sqrt(ff);
        if (P > 0.0) {
            double mixv = 1.0 - alpha, mixf = (fn > 0.0) ? alpha * vn / fn : 0.0;
            for (int i = 0; i < n; ++i) {
                if (s->role[i] != MOBILE) continue;
                for (int k = 0; k < dim; ++k) v[k * n + i] = mixv * v[k * n + i] + mixf * F[k * n + i];
            }
            for (int k = 0; k < dim; ++k) VR[k] = mixv * VR[k] + mixf * s->FR[k];
            if (since_neg > nmin) {
                dt = dt * finc; if (dt > dtmax) dt = dtmax;
                alpha *= falpha;
            }
            since_neg++;
        } else {
            dt *= fdec;
            alpha = alpha0;
            since_neg = 0;
            for (size_t q = 0; q < nd; ++q) v[q] = 0.0;
            for (int k = 0; k < 3; ++k) VR[k] = 0.0;
        }
        /* semi-implicit Euler step */
        for (int i = 0; i < n; ++i) {
            if (s->role[i] != MOBILE) continue;
            for (int k = 0; k < dim; ++k) {
                v[k * n + i] += dt * F[k * n + i] / s->p.mass;
                s->x[k * n + i] = wrap(s->x[k * n + i] + dt * v[k * n + i], s->p.box[k], s->p.periodic[k]);
            }
        }
        if (s->n_rigid > 0) {
            for (int k = 0; k < dim; ++k) {
                VR[k] += dt * s->FR[k] / M;
                s->XR[k] += dt * VR[k];
            }
            place_rigid(s);
        }
        evaluate(s, F, H, B, s->ftot, E, &sc);
    }
    free(F); free(H); free(B); free(E); free(v);
    s->p = saved;
    s->have_force = 0;
    return it < maxit ? it : -it;
}

void orc_get_tuu(const orc_sys *s, double *t)
{
    const int eig = (s->p.bias_var1 == 3 || s->p.bias_var2 == 3);
    memcpy(t, eig ? s->tww : s->tuu, sizeof(double) * (size_t)s->dim * s->n);
}
