/*
 * Primary sampling and the whole run (every primary with all its clones) for
 * the oracle.  TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
#include <math.h>
#include <pthread.h>
#include <stdatomic.h>
#include <stdlib.h>
#include <string.h>
#include "or_internal.h"

/* Primaries all start with the same statistical description (Sec. 3):
 * entry point uniform over one surface unit cell at height z_start,
 * species drawn uniformly from the list, energy log-uniform in
 * [E_min, E_max] (fixed when equal), direction either a fixed polar tilt
 * with uniform azimuth, or uniform on a cone of half-angle alpha about an
 * axis, or the cone for ids below n_cone and the tilt for the rest, or
 * uniform over the sphere (a recoil, Sec. 4: random direction).  With
 * start_mode OR_START_SITE the start point is the lattice point (0, 0,
 * z_start) instead (an on-lattice recoil, Sec. 4).  The threshold table is
 * chosen by species and by equal log-energy band. */
void or_sample_primaries(const or_sampler* s, uint64_t seed, int64_t id0, int64_t n,
                         int32_t* species, double* E0, double* pos, double* dir,
                         uint64_t* key, int32_t* table)
{
    for (int64_t q = 0; q < n; ++q) {
        int64_t id = id0 + q;
        uint64_t kk[2] = {seed, 0};
        uint64_t c0[4] = {OR_TAG_SAMPLE, (uint64_t)id, 0, 0};
        uint64_t c1[4] = {OR_TAG_SAMPLE, (uint64_t)id, 1, 0};
        uint64_t r0[4], r1[4];
        or_philox4x64(c0, kk, r0);
        or_philox4x64(c1, kk, r1);
        double u[8];
        for (int i = 0; i < 4; ++i) {
            u[i] = or_u01(r0[i]);
            u[4 + i] = or_u01(r1[i]);
        }
        if (s->start_mode == OR_START_SITE) {
            pos[q] = 0.0;
            pos[n + q] = 0.0;
        } else {
            pos[q] = s->a * u[0];
            pos[n + q] = s->a * u[1];
        }
        pos[2 * n + q] = s->z_start;

        int ci = (int)floor((double)s->n_choice * u[2]);
        if (ci > s->n_choice - 1) ci = s->n_choice - 1;
        species[q] = s->choice[ci];

        if (s->E_min == s->E_max)
            E0[q] = s->E_min;
        else
            E0[q] = s->E_min * exp(u[3] * log(s->E_max / s->E_min));
        int band = 0;
        if (s->n_energy_tables > 1) {
            band = (int)floor((double)s->n_energy_tables * u[3]);
            if (band > s->n_energy_tables - 1) band = s->n_energy_tables - 1;
        }
        table[q] = ci * (s->n_energy_tables > 1 ? s->n_energy_tables : 1) + band;

        int cone = s->dir_mode == OR_DIR_CONE || (s->dir_mode == OR_DIR_MIXED && id < s->n_cone);
        double phi = 2.0 * OR_PI * u[4];
        if (s->dir_mode == OR_DIR_ISOTROPIC) {
            /* uniform on the sphere: cos(theta) uniform in [-1, 1] */
            double ct = 1.0 - 2.0 * u[5];
            double st = sqrt(fmax(0.0, 1.0 - ct * ct));
            dir[q] = st * cos(phi);
            dir[n + q] = st * sin(phi);
            dir[2 * n + q] = ct;
        } else if (!cone) {
            dir[q] = sin(s->tilt) * cos(phi);
            dir[n + q] = sin(s->tilt) * sin(phi);
            dir[2 * n + q] = cos(s->tilt);
        } else {
            /* uniform on the spherical cap: cos(theta) uniform in [cos(alpha), 1] */
            double ct = 1.0 - u[5] * (1.0 - cos(s->half_angle));
            double st = sqrt(fmax(0.0, 1.0 - ct * ct));
            const double* A = s->axis;
            double h[3] = {1.0, 0.0, 0.0};
            if (fabs(A[0]) >= 0.9) { h[0] = 0.0; h[1] = 1.0; }
            /* e1 = normalise(A x h), e2 = A x e1 */
            double e1[3] = {A[1] * h[2] - A[2] * h[1], A[2] * h[0] - A[0] * h[2], A[0] * h[1] - A[1] * h[0]};
            double n1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
            for (int d = 0; d < 3; ++d) e1[d] /= n1;
            double e2[3] = {A[1] * e1[2] - A[2] * e1[1], A[2] * e1[0] - A[0] * e1[2], A[0] * e1[1] - A[1] * e1[0]};
            for (int d = 0; d < 3; ++d)
                dir[d * n + q] = st * (cos(phi) * e1[d] + sin(phi) * e2[d]) + ct * A[d];
        }
        key[q] = or_primary_key(seed, id);
    }
}

/* ---- run ---------------------------------------------------------------- */

typedef struct {
    const or_params* p;
    int64_t n;
    const int32_t *species, *table;
    const double *E0, *pos, *dir;
    const uint64_t* key;
    const int64_t* lineage;
    atomic_llong next;
    /* per-primary partial moments, summed in primary order at the end */
    double* sum_wz;
    double* sum_wz2;
    or_result* log;
    int64_t log_cap;
    atomic_llong log_count;
    int32_t error;
} run_shared;

typedef struct {
    run_shared* sh;
    double* hist;
    or_stats st;
} run_local;

static void record_finished(run_local* L, const or_track* t, int64_t q)
{
    const or_params* p = L->sh->p;
    L->st.finished += 1;
    if (t->status == OR_STOPPED) {
        L->st.n_stopped += 1;
        L->st.w_stopped += t->w;
        double z = t->z_stop;
        if (z < 0.0) {
            L->st.w_underflow += t->w;
        } else {
            double fb = floor(z / p->bin_width);
            if (fb >= (double)p->n_bins) L->st.w_overflow += t->w;
            else L->hist[(int64_t)fb] += t->w;
        }
        L->sh->sum_wz[q] += t->w * z;
        L->sh->sum_wz2[q] += t->w * z * z;
    } else if (t->status == OR_BACKSCATTERED) {
        L->st.n_backscattered += 1;
        L->st.w_backscattered += t->w;
    } else {
        if (t->status == OR_NONFINITE) L->st.n_nonfinite += 1;
        else L->st.n_stepcap += 1;
        L->st.w_quarantined += t->w;
    }
    if (L->sh->log) {
        int64_t i = atomic_fetch_add(&L->sh->log_count, 1);
        if (i < L->sh->log_cap) {
            or_result* r = &L->sh->log[i];
            r->lineage = t->lineage;
            r->status = t->status;
            r->next_k = t->next_k;
            r->z_stop = t->z_stop;
            r->w = t->w;
            r->steps = t->steps;
        }
    }
}

static int64_t domain_atoms(const or_track* t)
{
    int64_t c = 0;
    for (int j = 0; j < t->n_atoms; ++j) c += t->atom[j].exists;
    return c;
}

/* Runs primary q and, depth first, every clone it produces (Sec. 2: a
 * system is cloned when its ion reaches a cloning depth and the statistical
 * weight of each copy is halved; the paper's clients likewise finish every
 * clone of an ion before taking the next, Sec. 3). */
static void run_primary(run_local* L, int64_t q)
{
    run_shared* sh = L->sh;
    const or_params* p = sh->p;
    int cap = p->n_thresh * (p->n_clones > 1 ? p->n_clones - 1 : 1) + 4;
    or_track* stack = (or_track*)malloc(sizeof(or_track) * (size_t)cap);
    or_track* t = (or_track*)malloc(sizeof(or_track));
    if (!stack || !t) {
        sh->error = 1;
        free(stack);
        free(t);
        return;
    }
    int top = 0;
    double pos[3] = {sh->pos[q], sh->pos[sh->n + q], sh->pos[2 * sh->n + q]};
    double dir[3] = {sh->dir[q], sh->dir[sh->n + q], sh->dir[2 * sh->n + q]};
    or_track_init(p, sh->species[q], sh->E0[q], pos, dir, sh->key[q], sh->table[q],
                  sh->lineage ? sh->lineage[q] : q, &stack[top++]);
    L->st.primaries += 1;
    L->st.pair_evals += domain_atoms(&stack[0]);

    while (top > 0) {
        *t = stack[--top];
        while (t->status == OR_ACTIVE) {
            double M1 = p->M1[t->species];
            double ke = 0.5 * M1 * (t->v[0] * t->v[0] + t->v[1] * t->v[1] + t->v[2] * t->v[2]);
            double z = or_range_coord(p, t);
            or_track_step(p, t);
            L->st.track_steps += 1;
            L->st.pair_evals += domain_atoms(t);
            int32_t st = or_track_events(p, t, ke, z);
            if (st != OR_ACTIVE) break;
            const double* thr = p->thresholds + (int64_t)t->table * p->n_thresh;
            const double zr = or_range_coord(p, t);
            while (t->next_k < p->n_thresh && zr >= thr[t->next_k]) {
                int32_t k = t->next_k;
                uint64_t parent = t->key;
                t->w = t->w / (double)p->n_clones;
                t->next_k = k + 1;
                for (int i = p->n_clones - 1; i >= 1; --i) {
                    if (top >= cap) {
                        sh->error = 2;
                        break;
                    }
                    stack[top] = *t;
                    stack[top].key = or_child_key(parent, p->seed, k, i);
                    top++;
                    L->st.clones += 1;
                }
                t->key = or_child_key(parent, p->seed, k, 0);
            }
        }
        record_finished(L, t, q);
    }
    free(stack);
    free(t);
}

static void* worker(void* arg)
{
    run_local* L = (run_local*)arg;
    run_shared* sh = L->sh;
    for (;;) {
        int64_t q = atomic_fetch_add(&sh->next, 1);
        if (q >= sh->n) break;
        run_primary(L, q);
    }
    return NULL;
}

static void add_stats(or_stats* a, const or_stats* b)
{
    a->primaries += b->primaries;
    a->finished += b->finished;
    a->clones += b->clones;
    a->track_steps += b->track_steps;
    a->pair_evals += b->pair_evals;
    a->n_stopped += b->n_stopped;
    a->n_backscattered += b->n_backscattered;
    a->n_nonfinite += b->n_nonfinite;
    a->n_stepcap += b->n_stepcap;
    a->w_stopped += b->w_stopped;
    a->w_backscattered += b->w_backscattered;
    a->w_underflow += b->w_underflow;
    a->w_overflow += b->w_overflow;
    a->w_quarantined += b->w_quarantined;
}

int32_t or_run(const or_params* p, int64_t n, const int32_t* species, const double* E0,
               const double* pos, const double* dir, const uint64_t* key,
               const int32_t* table, const int64_t* lineage, int32_t nthreads,
               double* hist, or_stats* stats, or_result* log, int64_t log_cap,
               int64_t* log_count)
{
    if (nthreads < 1) nthreads = 1;
    run_shared sh;
    memset(&sh, 0, sizeof(sh));
    sh.p = p;
    sh.n = n;
    sh.species = species;
    sh.table = table;
    sh.E0 = E0;
    sh.pos = pos;
    sh.dir = dir;
    sh.key = key;
    sh.lineage = lineage;
    atomic_init(&sh.next, 0);
    atomic_init(&sh.log_count, 0);
    sh.log = log;
    sh.log_cap = log_cap;
    sh.sum_wz = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    sh.sum_wz2 = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    run_local* L = (run_local*)calloc((size_t)nthreads, sizeof(run_local));
    pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!sh.sum_wz || !sh.sum_wz2 || !L || !th) {
        free(sh.sum_wz); free(sh.sum_wz2); free(L); free(th);
        return -2;
    }
    for (int i = 0; i < nthreads; ++i) {
        L[i].sh = &sh;
        L[i].hist = (double*)calloc((size_t)p->n_bins, sizeof(double));
    }
    for (int i = 1; i < nthreads; ++i) pthread_create(&th[i], NULL, worker, &L[i]);
    worker(&L[0]);
    for (int i = 1; i < nthreads; ++i) pthread_join(th[i], NULL);

    /* every bin is a sum of powers of two far above 2^-53 of the total, so
     * the merge order does not change the histogram */
    for (int i = 0; i < nthreads; ++i) {
        for (int32_t b = 0; b < p->n_bins; ++b) hist[b] += L[i].hist[b];
        add_stats(stats, &L[i].st);
        free(L[i].hist);
    }
    for (int64_t q = 0; q < n; ++q) {
        stats->sum_wz += sh.sum_wz[q];
        stats->sum_wz2 += sh.sum_wz2[q];
    }
    if (log_count) *log_count = atomic_load(&sh.log_count);
    free(sh.sum_wz); free(sh.sum_wz2); free(L); free(th);
    return sh.error ? -sh.error : 0;
}
