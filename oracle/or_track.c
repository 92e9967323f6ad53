/*
 * One ion track: domain following, forces, one integration step, events.
 * TEST INFRASTRUCTURE ONLY (see oracle.h).
 */
#include <math.h>
#include <string.h>
#include "or_internal.h"

/* Site b of the cubic cell (in units of the cell) and its target species.
 * Diamond: the fcc sites and the same sites shifted by (1/4,1/4,1/4), one
 * species.  Fluorite (UO2, Sec. 2 and Sec. 4): cations (species 0) on the
 * fcc sites b = 0..3, anions (species 1) on the eight sites with every
 * coordinate 1/4 or 3/4, b = 4..11. */
void or_site(const or_params* p, int b, double f[3], int* type)
{
    static const double fcc[4][3] = {{0, 0, 0}, {0, 0.5, 0.5}, {0.5, 0, 0.5}, {0.5, 0.5, 0}};
    if (p->structure == OR_FLUORITE) {
        if (b < 4) {
            for (int d = 0; d < 3; ++d) f[d] = fcc[b][d];
            *type = 0;
        } else {
            int j = b - 4;
            f[0] = 0.25 + 0.5 * (double)((j >> 2) & 1);
            f[1] = 0.25 + 0.5 * (double)((j >> 1) & 1);
            f[2] = 0.25 + 0.5 * (double)(j & 1);
            *type = 1;
        }
        return;
    }
    for (int d = 0; d < 3; ++d) f[d] = fcc[b & 3][d] + (b >= 4 ? 0.25 : 0.0);
    *type = 0;
}

int or_nbasis(const or_params* p) { return p->structure == OR_FLUORITE ? OR_MAX_BASIS : OR_NBASIS; }
double or_type_mass(const or_params* p, int type) { return type ? p->M2b : p->M2; }

/* The vacant site of a recoil track (Sec. 4: the primary is a lattice atom
 * set in motion, so its own site is empty). */
static int is_vacant(const or_track* t, const int64_t c[3], int b)
{
    return t->vac_basis == b && c[0] == t->vac_cell[0] && c[1] == t->vac_cell[1] && c[2] == t->vac_cell[2];
}

/* Creates basis atom b of cell c for the crystal realisation of the track:
 * ideal site plus an independent Gaussian displacement per axis with the rms
 * of its species, at rest (Sec. 2: thermal structure drawn from its
 * statistical description; the temperature is represented by Gaussian
 * lattice displacements, Sec. 4). */
static void create_atom(const or_params* p, const or_track* t, const int64_t c[3], int b, or_atom* at)
{
    double f[3], g[3];
    int type;
    or_site(p, b, f, &type);
    double sigma = type ? p->sigma_b : p->sigma;
    or_gauss3(t->key, p->seed, c[0], c[1], c[2], b, g);
    for (int d = 0; d < 3; ++d) {
        at->x[d] = p->a * ((double)c[d] + f[d]) + sigma * g[d];
        at->v[d] = 0.0;
        at->f[d] = 0.0;
        at->cell[d] = c[d];
    }
    at->basis = b;
    at->type = type;
    at->exists = 1;
}

static int64_t cell_index(double x, double a)
{
    return (int64_t)floor(x / a);
}

static double ion_atom_distance(const or_track* t, const or_atom* at, double d[3])
{
    for (int k = 0; k < 3; ++k) d[k] = t->x[k] - at->x[k];
    return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

/* Builds or rebuilds the 27-cell domain around the cell holding the ion
 * (Sec. 2 and Fig. 1: when the ion breaches a neighbouring cell the main
 * cell moves there, cells that are no longer neighbours are removed and the
 * new neighbouring cells are produced).  Cells exist only in the half space
 * z >= 0 (the crystal surface is the plane z = 0).  Returns 1 if the domain
 * changed. */
static int maintain_domain(const or_params* p, or_track* t, int fresh)
{
    if (p->structure == OR_ISOLATED) return 0;
    int64_t nc[3];
    for (int d = 0; d < 3; ++d) nc[d] = cell_index(t->x[d], p->a);
    if (!fresh && nc[0] == t->center[0] && nc[1] == t->center[1] && nc[2] == t->center[2])
        return 0;

    const int nb = or_nbasis(p), na = t->n_atoms;
    or_atom old[OR_MAX_ATOMS];
    memcpy(old, t->atom, sizeof(old));
    int kept[OR_MAX_ATOMS];
    for (int j = 0; j < OR_MAX_ATOMS; ++j) kept[j] = 0;

    int slot = 0;
    for (int i = -1; i <= 1; ++i)
        for (int j = -1; j <= 1; ++j)
            for (int k = -1; k <= 1; ++k) {
                int64_t c[3] = {nc[0] + i, nc[1] + j, nc[2] + k};
                for (int b = 0; b < nb; ++b, ++slot) {
                    or_atom* at = &t->atom[slot];
                    int found = -1;
                    if (!fresh) {
                        for (int q = 0; q < na; ++q)
                            if (old[q].exists && old[q].basis == b && old[q].cell[0] == c[0] &&
                                old[q].cell[1] == c[1] && old[q].cell[2] == c[2]) {
                                found = q;
                                break;
                            }
                    }
                    if (found >= 0) {
                        *at = old[found];
                        kept[found] = 1;
                    } else if (c[2] >= 0 && !is_vacant(t, c, b)) {
                        create_atom(p, t, c, b, at);
                        double d[3];
                        double r = ion_atom_distance(t, at, d);
                        t->e_in += or_pair_potential(p, t->species, at->type, r);
                    } else {
                        double f[3];
                        memset(at, 0, sizeof(*at));
                        at->cell[0] = c[0]; at->cell[1] = c[1]; at->cell[2] = c[2];
                        at->basis = b;
                        or_site(p, b, f, &at->type);
                        at->exists = 0;
                    }
                }
            }
    if (!fresh) {
        /* atoms that left the domain take their energy and momentum with them */
        for (int q = 0; q < na; ++q) {
            if (!old[q].exists || kept[q]) continue;
            double d[3];
            double r = ion_atom_distance(t, &old[q], d);
            double v2 = old[q].v[0] * old[q].v[0] + old[q].v[1] * old[q].v[1] + old[q].v[2] * old[q].v[2];
            double M2 = or_type_mass(p, old[q].type);
            t->e_out += 0.5 * M2 * v2 + or_pair_potential(p, t->species, old[q].type, r);
            for (int k = 0; k < 3; ++k) t->p_out[k] += M2 * old[q].v[k];
        }
    }
    for (int d = 0; d < 3; ++d) t->center[d] = nc[d];
    return 1;
}

/* Ion-atom forces and the local density at the ion.  Every atom of the
 * domain interacts with the ion (Sec. 2: the 27 cells); atoms do not interact
 * with each other, and each feels the reaction of its own pair force.  With a
 * cut-off r_cut > 0 (an interaction set smaller than the paper's 27 cells, a
 * variant to be checked against it), atoms farther than r_cut from the ion
 * are skipped: no force on either side and no density. */
void or_compute_forces(const or_params* p, or_track* t)
{
    or_pair_consts pcs[2];
    or_pair_constants(p, t->species, 0, &pcs[0]);
    or_pair_constants(p, t->species, p->structure == OR_FLUORITE ? 1 : 0, &pcs[1]);
    for (int k = 0; k < 3; ++k) t->F[k] = 0.0;
    t->rho = 0.0;
    for (int j = 0; j < t->n_atoms; ++j) {
        or_atom* at = &t->atom[j];
        if (!at->exists) continue;
        double d[3];
        double r = ion_atom_distance(t, at, d);
        if (p->r_cut > 0.0 && r > p->r_cut) {
            for (int k = 0; k < 3; ++k) at->f[k] = 0.0;
            continue;
        }
        const or_pair_consts* pc = &pcs[at->type];
        double V, dVdr;
        or_zbl_c(pc, r, &V, &dVdr);
        for (int k = 0; k < 3; ++k) {
            double fk = -dVdr * d[k] / r;   /* force on the ion from atom j */
            t->F[k] += fk;
            at->f[k] = -fk;
        }
        t->rho += pc->firsov ? or_firsov_weight_c(pc, r) : or_density_weight_c(pc, r);
    }
}

void or_track_init(const or_params* p, int32_t species, double E0, const double pos[3],
                   const double dir[3], uint64_t key, int32_t table, int64_t lineage, or_track* t)
{
    memset(t, 0, sizeof(*t));
    double M1 = p->M1[species];
    double dn = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    double speed = sqrt(2.0 * E0 / M1);
    for (int k = 0; k < 3; ++k) {
        t->x[k] = pos[k];
        t->v[k] = speed * dir[k] / dn;
    }
    t->w = 1.0;
    t->key = key;
    t->species = species;
    t->table = table;
    t->lineage = lineage;
    t->status = OR_ACTIVE;
    t->vac_basis = -1;
    for (int k = 0; k < 3; ++k) t->x0[k] = pos[k];
    if (p->structure == OR_ISOLATED) {
        t->n_atoms = 1;
        t->atom[0].exists = 1;
    } else {
        if (p->vacancy) {
            /* the basis-0 site of the cell whose origin is nearest the start point */
            for (int k = 0; k < 3; ++k) t->vac_cell[k] = (int64_t)floor(pos[k] / p->a + 0.25);
            t->vac_basis = 0;
        }
        t->n_atoms = 27 * or_nbasis(p);
        maintain_domain(p, t, 1);
        t->e_in = 0.0;   /* the initial crystal is part of the system, not an inflow */
    }
    or_compute_forces(p, t);
}

/* Adaptive time step.  Sec. 2 (and Fig. 2) only says the step follows the
 * kinetic and the collisional energy scale; the reading used: no particle
 * (ion or domain atom) moves more than dx_max in one step, either from its
 * current velocity or from its current acceleration, and dt <= dt_max. */
static double time_step(const or_params* p, const or_track* t)
{
    double M1 = p->M1[t->species];
    double v2 = t->v[0] * t->v[0] + t->v[1] * t->v[1] + t->v[2] * t->v[2];
    double f2 = t->F[0] * t->F[0] + t->F[1] * t->F[1] + t->F[2] * t->F[2];
    double vmax2 = v2;
    double amax2 = f2 / (M1 * M1);
    for (int j = 0; j < t->n_atoms; ++j) {
        const or_atom* at = &t->atom[j];
        if (!at->exists) continue;
        double av2 = at->v[0] * at->v[0] + at->v[1] * at->v[1] + at->v[2] * at->v[2];
        double M2 = or_type_mass(p, at->type);
        double af2 = (at->f[0] * at->f[0] + at->f[1] * at->f[1] + at->f[2] * at->f[2]) / (M2 * M2);
        if (av2 > vmax2) vmax2 = av2;
        if (af2 > amax2) amax2 = af2;
    }
    double dt = p->dt_max;
    if (vmax2 > 0.0) {
        double dv = p->dx_max / sqrt(vmax2);
        if (dv < dt) dt = dv;
    }
    if (amax2 > 0.0) {
        double da = sqrt(2.0 * p->dx_max / sqrt(amax2));
        if (da < dt) dt = da;
    }
    return dt;
}

/* One step: velocity Verlet on the ion and the domain atoms (Sec. 2,
 * "standard Verlet-type" integrator), with the velocity-dependent stopping
 * force split off symmetrically (half a step of exact friction before the
 * first and after the second half kick), and the domain rebuilt after the
 * drift. */
double or_track_step(const or_params* p, or_track* t)
{
    double M1 = p->M1[t->species];
    double dt = time_step(p, t);

    double v2 = t->v[0] * t->v[0] + t->v[1] * t->v[1] + t->v[2] * t->v[2];
    double fr1 = exp(-or_stopping_gamma(p, t->species, t->rho, v2) * dt / (2.0 * M1));
    for (int k = 0; k < 3; ++k) t->v[k] *= fr1;

    for (int k = 0; k < 3; ++k) t->v[k] += t->F[k] * dt / (2.0 * M1);
    for (int j = 0; j < t->n_atoms; ++j) {
        or_atom* at = &t->atom[j];
        if (!at->exists) continue;
        for (int k = 0; k < 3; ++k) at->v[k] += at->f[k] * dt / (2.0 * or_type_mass(p, at->type));
    }

    for (int k = 0; k < 3; ++k) t->x[k] += t->v[k] * dt;
    for (int j = 0; j < t->n_atoms; ++j) {
        or_atom* at = &t->atom[j];
        if (!at->exists) continue;
        for (int k = 0; k < 3; ++k) at->x[k] += at->v[k] * dt;
    }

    maintain_domain(p, t, 0);
    or_compute_forces(p, t);

    for (int k = 0; k < 3; ++k) t->v[k] += t->F[k] * dt / (2.0 * M1);
    for (int j = 0; j < t->n_atoms; ++j) {
        or_atom* at = &t->atom[j];
        if (!at->exists) continue;
        for (int k = 0; k < 3; ++k) at->v[k] += at->f[k] * dt / (2.0 * or_type_mass(p, at->type));
    }

    v2 = t->v[0] * t->v[0] + t->v[1] * t->v[1] + t->v[2] * t->v[2];
    double fr2 = exp(-or_stopping_gamma(p, t->species, t->rho, v2) * dt / (2.0 * M1));
    for (int k = 0; k < 3; ++k) t->v[k] *= fr2;

    t->steps += 1;
    return dt;
}

/* The range coordinate: the depth z, or with a radial range the distance
 * from the primary's start point (a recoil inside the crystal, Sec. 4). */
double or_range_coord(const or_params* p, const or_track* t)
{
    if (p->range_mode != OR_RANGE_RADIAL) return t->x[2];
    double d[3];
    for (int k = 0; k < 3; ++k) d[k] = t->x[k] - t->x0[k];
    return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

static double ion_ke(const or_params* p, const or_track* t)
{
    return 0.5 * p->M1[t->species] * (t->v[0] * t->v[0] + t->v[1] * t->v[1] + t->v[2] * t->v[2]);
}

/* Termination events after a step, in the order: non-finite state, stop,
 * backscatter, step cap.  The stopping depth (range coordinate) is
 * interpolated linearly in kinetic energy within the last step; z_before is
 * its value before the step.  Splitting is handled by the caller. */
int32_t or_track_events(const or_params* p, or_track* t, double ke_before, double z_before)
{
    int finite = 1;
    for (int k = 0; k < 3; ++k)
        if (!isfinite(t->x[k]) || !isfinite(t->v[k])) finite = 0;
    if (!finite) {
        t->status = OR_NONFINITE;
        return t->status;
    }
    double ke = ion_ke(p, t);
    if (ke < p->E_stop) {
        if (ke_before > p->E_stop)
            t->z_stop = z_before + (or_range_coord(p, t) - z_before) * (ke_before - p->E_stop) / (ke_before - ke);
        else
            t->z_stop = z_before;
        t->status = OR_STOPPED;
        return t->status;
    }
    if (t->x[2] < p->z_start && t->v[2] < 0.0) {
        t->status = OR_BACKSCATTERED;
        return t->status;
    }
    if (p->max_steps > 0 && t->steps >= p->max_steps) {
        t->status = OR_STEPCAP;
        return t->status;
    }
    return OR_ACTIVE;
}

void or_track_advance(const or_params* p, or_track* t, int64_t nsteps, int32_t with_events)
{
    for (int64_t n = 0; n < nsteps; ++n) {
        double ke = ion_ke(p, t), z = or_range_coord(p, t);
        or_track_step(p, t);
        if (with_events && or_track_events(p, t, ke, z) != OR_ACTIVE) return;
    }
}

/* Conserved totals with stopping off: kinetic energy of the ion and atoms,
 * ion-atom potential energy, plus what dropped atoms carried away, minus the
 * potential energy created atoms brought in; and total momentum. */
void or_track_ledger(const or_params* p, const or_track* t, double* energy, double momentum[3])
{
    double M1 = p->M1[t->species];
    double e = ion_ke(p, t);
    for (int k = 0; k < 3; ++k) momentum[k] = M1 * t->v[k] + t->p_out[k];
    for (int j = 0; j < t->n_atoms; ++j) {
        const or_atom* at = &t->atom[j];
        if (!at->exists) continue;
        double d[3];
        double r = ion_atom_distance(t, at, d);
        double v2 = at->v[0] * at->v[0] + at->v[1] * at->v[1] + at->v[2] * at->v[2];
        double M2 = or_type_mass(p, at->type);
        e += 0.5 * M2 * v2 + or_pair_potential(p, t->species, at->type, r);
        for (int k = 0; k < 3; ++k) momentum[k] += M2 * at->v[k];
    }
    *energy = e + t->e_out - t->e_in;
}

/* ---- exchange record --------------------------------------------------
 * Flat array of 64-bit words: a 32-word header then nine atom fields (x, y,
 * z, vx, vy, vz, fx, fy, fz) of NS entries each (NS = 216 for diamond, 344
 * for fluorite).  With r = (c_x mod 3)*9 + (c_y mod 3)*3 + (c_z mod 3), the
 * slot of basis atom b of cell c is r*8 + b (diamond); r*4 + b for the
 * fluorite cations and 128 + r*8 + (b - 4) for its anions (slots 108..127
 * stay empty).  Header words 25-27: cell of the vacant site, 28: its basis
 * index (-1: none), 29-31: the start point. */
enum { REC_HDR = 32 };

static int rec_nslot(const or_params* p) { return p->structure == OR_FLUORITE ? OR_NSLOT_FLUORITE : OR_NSLOT; }
int64_t or_record_words(const or_params* p) { return REC_HDR + 9 * (int64_t)rec_nslot(p); }
int64_t or_track_size(void) { return (int64_t)sizeof(or_track); }

static int mod3(int64_t c) { return (int)(((c % 3) + 3) % 3); }

static int slot_of(const or_params* p, const int64_t c[3], int b)
{
    int r = mod3(c[0]) * 9 + mod3(c[1]) * 3 + mod3(c[2]);
    if (p->structure == OR_FLUORITE) return b < 4 ? r * 4 + b : OR_ANION_SLOT0 + r * 8 + (b - 4);
    return r * OR_NBASIS + b;
}

void or_track_export(const or_params* p, const or_track* t, double* rec)
{
    const int NS = rec_nslot(p);
    memset(rec, 0, sizeof(double) * (size_t)or_record_words(p));
    int64_t* irec = (int64_t*)rec;
    for (int k = 0; k < 3; ++k) {
        rec[k] = t->x[k];
        rec[3 + k] = t->v[k];
        rec[6 + k] = t->F[k];
        irec[12 + k] = t->center[k];
        irec[25 + k] = t->vac_basis >= 0 ? t->vac_cell[k] : 0;
        rec[29 + k] = t->x0[k];
    }
    rec[9] = t->rho;
    rec[10] = t->w;
    rec[11] = t->z_stop;
    irec[15] = (int64_t)t->key;
    irec[16] = t->steps;
    irec[17] = t->lineage;
    irec[18] = t->species;
    irec[19] = t->next_k;
    irec[20] = t->table;
    irec[21] = t->status;
    irec[28] = t->vac_basis;
    for (int j = 0; j < t->n_atoms; ++j) {
        const or_atom* at = &t->atom[j];
        if (!at->exists) continue;
        int s = (p->structure == OR_ISOLATED) ? 0 : slot_of(p, at->cell, at->basis);
        for (int k = 0; k < 3; ++k) {
            rec[REC_HDR + (0 + k) * NS + s] = at->x[k];
            rec[REC_HDR + (3 + k) * NS + s] = at->v[k];
            rec[REC_HDR + (6 + k) * NS + s] = at->f[k];
        }
    }
}

void or_track_import(const or_params* p, const double* rec, or_track* t)
{
    const int NS = rec_nslot(p);
    memset(t, 0, sizeof(*t));
    const int64_t* irec = (const int64_t*)rec;
    for (int k = 0; k < 3; ++k) {
        t->x[k] = rec[k];
        t->v[k] = rec[3 + k];
        t->F[k] = rec[6 + k];
        t->center[k] = irec[12 + k];
        t->vac_cell[k] = irec[25 + k];
        t->x0[k] = rec[29 + k];
    }
    t->rho = rec[9];
    t->w = rec[10];
    t->z_stop = rec[11];
    t->key = (uint64_t)irec[15];
    t->steps = irec[16];
    t->lineage = irec[17];
    t->species = (int32_t)irec[18];
    t->next_k = (int32_t)irec[19];
    t->table = (int32_t)irec[20];
    t->status = (int32_t)irec[21];
    t->vac_basis = (int32_t)irec[28];
    if (p->structure == OR_ISOLATED) {
        t->n_atoms = 1;
        or_atom* at = &t->atom[0];
        at->exists = 1;
        for (int k = 0; k < 3; ++k) {
            at->x[k] = rec[REC_HDR + (0 + k) * NS];
            at->v[k] = rec[REC_HDR + (3 + k) * NS];
            at->f[k] = rec[REC_HDR + (6 + k) * NS];
        }
        return;
    }
    const int nb = or_nbasis(p);
    t->n_atoms = 27 * nb;
    int slot = 0;
    for (int i = -1; i <= 1; ++i)
        for (int j = -1; j <= 1; ++j)
            for (int k = -1; k <= 1; ++k) {
                int64_t c[3] = {t->center[0] + i, t->center[1] + j, t->center[2] + k};
                for (int b = 0; b < nb; ++b, ++slot) {
                    or_atom* at = &t->atom[slot];
                    double f[3];
                    for (int d = 0; d < 3; ++d) at->cell[d] = c[d];
                    at->basis = b;
                    or_site(p, b, f, &at->type);
                    at->exists = c[2] >= 0 && !is_vacant(t, c, b);
                    if (!at->exists) continue;
                    int s = slot_of(p, c, b);
                    for (int d = 0; d < 3; ++d) {
                        at->x[d] = rec[REC_HDR + (0 + d) * NS + s];
                        at->v[d] = rec[REC_HDR + (3 + d) * NS + s];
                        at->f[d] = rec[REC_HDR + (6 + d) * NS + s];
                    }
                }
            }
}
