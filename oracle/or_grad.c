/*
 * Forward-mode derivative of the stopping depth with respect to the
 * electronic-stopping scale k and the ZBL screening-length scale s.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * The same track algorithm as or_track.c (domain following, ZBL forces with
 * recoil, local friction, adaptive velocity Verlet, interpolated stop), run
 * on dual numbers that carry d/dk and d/ds along with every value.  Branches
 * (the active term of the time-step minimum, the domain update, the events)
 * are taken on the values; newly created atoms are constants (their positions
 * come from the crystal description, not from k or s); the starting position
 * and velocity are constants.  The derivative of the mean projected range is
 * the mean of the per-track derivatives over stopped tracks.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "or_internal.h"

typedef struct {
    double v, dk, ds;
} dn;

static dn D(double v) { dn r = {v, 0.0, 0.0}; return r; }
static dn dadd(dn a, dn b) { dn r = {a.v + b.v, a.dk + b.dk, a.ds + b.ds}; return r; }
static dn dsub(dn a, dn b) { dn r = {a.v - b.v, a.dk - b.dk, a.ds - b.ds}; return r; }
static dn dmul(dn a, dn b) { dn r = {a.v * b.v, a.dk * b.v + a.v * b.dk, a.ds * b.v + a.v * b.ds}; return r; }
static dn dscale(dn a, double c) { dn r = {a.v * c, a.dk * c, a.ds * c}; return r; }
static dn ddiv(dn a, dn b)
{
    double q = a.v / b.v;
    dn r = {q, (a.dk - q * b.dk) / b.v, (a.ds - q * b.ds) / b.v};
    return r;
}
static dn dexp(dn a)
{
    double e = exp(a.v);
    dn r = {e, e * a.dk, e * a.ds};
    return r;
}
static dn dsqrt(dn a)
{
    double q = sqrt(a.v);
    dn r = {q, a.dk / (2.0 * q), a.ds / (2.0 * q)};
    return r;
}

typedef struct {
    dn x[3], v[3], f[3];
    int64_t cell[3];
    int32_t basis, exists;
} gatom;

typedef struct {
    dn x[3], v[3], F[3], rho;
    int64_t center[3];
    uint64_t key;
    int64_t steps;
    int32_t species, status;
    gatom atom[OR_NSLOT];
} gtrack;

static const double gc[4] = {0.18175, 0.50986, 0.28022, 0.02817};
static const double gd[4] = {3.19980, 0.94229, 0.40290, 0.20162};

/* ZBL pair term on duals: the screening length a = s a_U carries d/ds = a_U. */
static void gpair(const or_params* p, int species, const dn d[3], dn* coef, dn* wr)
{
    double aU = or_unscaled_screening_length(p, species, 0);
    dn a = {p->s * aU, 0.0, aU};
    double zz = (p->pot_mode == OR_POT_NONE) ? 0.0 : (double)p->Z1[species] * (double)p->Z2 * OR_COULOMB;
    dn r2 = dadd(dadd(dmul(d[0], d[0]), dmul(d[1], d[1])), dmul(d[2], d[2]));
    dn r = dsqrt(r2);
    dn x = ddiv(r, a);
    dn phi = D(0.0), dphi = D(0.0);
    for (int i = 0; i < 4; ++i) {
        dn e = dexp(dscale(x, -gd[i]));
        phi = dadd(phi, dscale(e, gc[i]));
        dphi = dsub(dphi, dscale(e, gc[i] * gd[i]));
    }
    /* V'(r) = zz (phi'/(a r) - phi/r^2); coef = -V'(r)/r */
    dn t1 = ddiv(dphi, dmul(a, r));
    dn t2 = ddiv(phi, r2);
    dn dV = dscale(dsub(t1, t2), zz);
    *coef = dscale(ddiv(dV, r), -1.0);
    double lambda = aU / 0.3;
    *wr = dscale(dexp(dscale(r, -1.0 / lambda)), 1.0 / (8.0 * OR_PI * lambda * lambda * lambda));
}

static void gforces(const or_params* p, gtrack* t)
{
    for (int k = 0; k < 3; ++k) t->F[k] = D(0.0);
    t->rho = D(0.0);
    for (int j = 0; j < OR_NSLOT; ++j) {
        gatom* at = &t->atom[j];
        if (!at->exists) continue;
        dn d[3];
        for (int k = 0; k < 3; ++k) d[k] = dsub(t->x[k], at->x[k]);
        dn coef, wr;
        gpair(p, t->species, d, &coef, &wr);
        for (int k = 0; k < 3; ++k) {
            dn fk = dmul(coef, d[k]);
            t->F[k] = dadd(t->F[k], fk);
            at->f[k] = dscale(fk, -1.0);
        }
        t->rho = dadd(t->rho, wr);
    }
}

static void gcreate(const or_params* p, const gtrack* t, const int64_t c[3], int b, gatom* at)
{
    double f[3], g[3];
    int type;
    or_site(p, b, f, &type);
    or_gauss3(t->key, p->seed, c[0], c[1], c[2], b, g);
    for (int d = 0; d < 3; ++d) {
        at->x[d] = D(p->a * ((double)c[d] + f[d]) + p->sigma * g[d]);
        at->v[d] = D(0.0);
        at->f[d] = D(0.0);
        at->cell[d] = c[d];
    }
    at->basis = b;
    at->exists = 1;
}

static void gdomain(const or_params* p, gtrack* t, int fresh)
{
    int64_t nc[3];
    for (int d = 0; d < 3; ++d) nc[d] = (int64_t)floor(t->x[d].v / p->a);
    if (!fresh && nc[0] == t->center[0] && nc[1] == t->center[1] && nc[2] == t->center[2]) return;
    gatom* old = (gatom*)malloc(sizeof(gatom) * OR_NSLOT);
    memcpy(old, t->atom, sizeof(gatom) * OR_NSLOT);
    int slot = 0;
    for (int i = -1; i <= 1; ++i)
        for (int j = -1; j <= 1; ++j)
            for (int k = -1; k <= 1; ++k) {
                int64_t c[3] = {nc[0] + i, nc[1] + j, nc[2] + k};
                for (int b = 0; b < OR_NBASIS; ++b, ++slot) {
                    gatom* at = &t->atom[slot];
                    int found = -1;
                    if (!fresh)
                        for (int q = 0; q < OR_NSLOT; ++q)
                            if (old[q].exists && old[q].basis == b && old[q].cell[0] == c[0] &&
                                old[q].cell[1] == c[1] && old[q].cell[2] == c[2]) {
                                found = q;
                                break;
                            }
                    if (found >= 0) {
                        *at = old[found];
                    } else if (c[2] >= 0) {
                        gcreate(p, t, c, b, at);
                    } else {
                        memset(at, 0, sizeof(*at));
                        at->exists = 0;
                    }
                }
            }
    for (int d = 0; d < 3; ++d) t->center[d] = nc[d];
    free(old);
}

/* One step on duals (same order as or_track_step). */
static void gstep(const or_params* p, gtrack* t)
{
    double M1 = p->M1[t->species], M2 = p->M2;
    /* time step from the state at the start of the step; the active term of the
     * minimum carries the derivative */
    dn v2 = dadd(dadd(dmul(t->v[0], t->v[0]), dmul(t->v[1], t->v[1])), dmul(t->v[2], t->v[2]));
    dn a2 = dscale(dadd(dadd(dmul(t->F[0], t->F[0]), dmul(t->F[1], t->F[1])), dmul(t->F[2], t->F[2])),
                   1.0 / (M1 * M1));
    dn vmax2 = v2, amax2 = a2;
    for (int j = 0; j < OR_NSLOT; ++j) {
        gatom* at = &t->atom[j];
        if (!at->exists) continue;
        dn av2 = dadd(dadd(dmul(at->v[0], at->v[0]), dmul(at->v[1], at->v[1])), dmul(at->v[2], at->v[2]));
        dn af2 = dscale(dadd(dadd(dmul(at->f[0], at->f[0]), dmul(at->f[1], at->f[1])), dmul(at->f[2], at->f[2])),
                        1.0 / (M2 * M2));
        if (av2.v > vmax2.v) vmax2 = av2;
        if (af2.v > amax2.v) amax2 = af2;
    }
    dn dt = D(p->dt_max);
    if (vmax2.v > 0.0) {
        dn dv = ddiv(D(p->dx_max), dsqrt(vmax2));
        if (dv.v < dt.v) dt = dv;
    }
    if (amax2.v > 0.0) {
        dn da = dsqrt(ddiv(D(2.0 * p->dx_max), dsqrt(amax2)));
        if (da.v < dt.v) dt = da;
    }
    /* friction coefficient: gamma = k * gamma0 * rho / N (local) or k * gamma0 (uniform) */
    double N = (double)OR_NBASIS / (p->a * p->a * p->a);
    double gamma0 = N * or_lss_kL(p, t->species, 0) * sqrt(M1 / 2.0);
    dn kk = {p->k, 1.0, 0.0};
    dn g1;
    if (p->stop_mode == OR_STOP_OFF) g1 = D(0.0);
    else if (p->stop_mode == OR_STOP_UNIFORM) g1 = dscale(kk, gamma0);
    else g1 = dscale(dmul(kk, t->rho), gamma0 / N);
    dn h1 = dscale(dt, 1.0 / (2.0 * M1));
    dn fr1 = dexp(dscale(dmul(g1, h1), -1.0));
    for (int k = 0; k < 3; ++k) t->v[k] = dmul(t->v[k], fr1);
    for (int k = 0; k < 3; ++k) t->v[k] = dadd(t->v[k], dmul(t->F[k], h1));
    dn h2 = dscale(dt, 1.0 / (2.0 * M2));
    for (int j = 0; j < OR_NSLOT; ++j) {
        gatom* at = &t->atom[j];
        if (!at->exists) continue;
        for (int k = 0; k < 3; ++k) at->v[k] = dadd(at->v[k], dmul(at->f[k], h2));
    }
    for (int k = 0; k < 3; ++k) t->x[k] = dadd(t->x[k], dmul(t->v[k], dt));
    for (int j = 0; j < OR_NSLOT; ++j) {
        gatom* at = &t->atom[j];
        if (!at->exists) continue;
        for (int k = 0; k < 3; ++k) at->x[k] = dadd(at->x[k], dmul(at->v[k], dt));
    }
    gdomain(p, t, 0);
    gforces(p, t);
    for (int k = 0; k < 3; ++k) t->v[k] = dadd(t->v[k], dmul(t->F[k], h1));
    for (int j = 0; j < OR_NSLOT; ++j) {
        gatom* at = &t->atom[j];
        if (!at->exists) continue;
        for (int k = 0; k < 3; ++k) at->v[k] = dadd(at->v[k], dmul(at->f[k], h2));
    }
    dn g2;
    if (p->stop_mode == OR_STOP_OFF) g2 = D(0.0);
    else if (p->stop_mode == OR_STOP_UNIFORM) g2 = dscale(kk, gamma0);
    else g2 = dscale(dmul(kk, t->rho), gamma0 / N);
    dn fr2 = dexp(dscale(dmul(g2, h1), -1.0));
    for (int k = 0; k < 3; ++k) t->v[k] = dmul(t->v[k], fr2);
    t->steps += 1;
}

/* Runs one primary (no cloning) to termination on duals.  out[0..2] = stopping
 * depth and its derivatives with respect to k and s; returns the status. */
int32_t or_grad_track(const or_params* p, int32_t species, double E0, const double pos[3],
                      const double dir[3], uint64_t key, int64_t max_steps, double out[3],
                      int64_t* steps_out)
{
    /* diamond, depth range and no vacancy only (the adjoint's domain) */
    if (p->structure != OR_DIAMOND || p->range_mode != OR_RANGE_DEPTH || p->vacancy) return -3;
    if (p->stop_mode == OR_STOP_FKBK || p->r_cut > 0.0) return -3;   /* derivatives cover the local LS model, 27 cells */
    gtrack* t = (gtrack*)calloc(1, sizeof(gtrack));
    if (!t) return -1;
    double M1 = p->M1[species];
    double dn_ = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    double speed = sqrt(2.0 * E0 / M1);
    for (int k = 0; k < 3; ++k) {
        t->x[k] = D(pos[k]);
        t->v[k] = D(speed * dir[k] / dn_);
    }
    t->key = key;
    t->species = species;
    gdomain(p, t, 1);
    gforces(p, t);
    int32_t status = OR_ACTIVE;
    out[0] = out[1] = out[2] = 0.0;
    for (;;) {
        dn ke0 = dscale(dadd(dadd(dmul(t->v[0], t->v[0]), dmul(t->v[1], t->v[1])), dmul(t->v[2], t->v[2])),
                        0.5 * M1);
        dn z0 = t->x[2];
        gstep(p, t);
        int finite = 1;
        for (int k = 0; k < 3; ++k)
            if (!isfinite(t->x[k].v) || !isfinite(t->v[k].v)) finite = 0;
        if (!finite) { status = OR_NONFINITE; break; }
        dn ke = dscale(dadd(dadd(dmul(t->v[0], t->v[0]), dmul(t->v[1], t->v[1])), dmul(t->v[2], t->v[2])),
                       0.5 * M1);
        if (ke.v < p->E_stop) {
            dn zs;
            if (ke0.v > p->E_stop) {
                /* z_stop = z0 + (z1 - z0) (ke0 - E) / (ke0 - ke1) */
                dn th = ddiv(dsub(ke0, D(p->E_stop)), dsub(ke0, ke));
                zs = dadd(z0, dmul(dsub(t->x[2], z0), th));
            } else {
                zs = z0;
            }
            out[0] = zs.v; out[1] = zs.dk; out[2] = zs.ds;
            status = OR_STOPPED;
            break;
        }
        if (t->x[2].v < p->z_start && t->v[2].v < 0.0) { status = OR_BACKSCATTERED; break; }
        if (max_steps > 0 && t->steps >= max_steps) { status = OR_STEPCAP; break; }
    }
    if (steps_out) *steps_out = t->steps;
    free(t);
    return status;
}
