/*
 * REED-MD reference oracle: plain, serial-per-track FP64 CPU implementation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this code; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no source, header, constant or
 * helper with the HIP library: every physical constant and every step below
 * is written out here on its own.
 *
 * What it computes (Jeon & Gronbech-Jensen, "Efficient Parallel Algorithm for
 * Statistical Ion Track Simulations in Crystalline Materials", Sec. 2 "Review
 * of the REED-MD Algorithm", and Figs. 1-3):
 *   - domain following: only the 27 unit cells around the ion exist; the
 *     ion sits in the centre cell; when it enters a neighbouring cell the
 *     centre moves, wake cells are discarded and new front cells are created
 *     from the statistical (thermal) description of the crystal (Sec. 2,
 *     Fig. 1);
 *   - nuclear interactions by the ZBL universal screened Coulomb potential
 *     only (Sec. 2, "First" and "Second");
 *   - local electronic stopping (Sec. 2, "Third"; the configured Local
 *     Lindhard-Scharff reading, or the paper's Firsov local loss plus a
 *     Brandt-Kitagawa loss in the interstitial electron density, read from the
 *     works it cites, see or_physics.c);
 *   - Verlet-type integration with an adaptive time step derived from the
 *     kinetic and the collisional energy scale (Sec. 2, Fig. 2);
 *   - rare-event enhancement: the system is cloned at cloning depths and the
 *     statistical weight is halved per cloning (Sec. 2, Fig. 3);
 *   - a weighted range (stopping depth) histogram (Sec. 2).
 * Where the paper is silent (formulas are deferred to its references) the
 * readings listed in the design notes are followed; each is named in the
 * function that implements it.
 *
 * Units: length in Angstrom, energy in eV, mass in amu; time in
 * tau = sqrt(amu * A^2 / eV) = 10.18 fs (the unit quoted with Fig. 2).
 *
 * Pins (tests/test_oracle_pins.py, each against something other than this
 * code): Philox against numpy's generator; the ZBL potential, its derivative,
 * screening length and nuclear stopping against closed forms and published
 * fits; the stopping constant against Lindhard's reduced form; pure friction
 * and the collision-free stopping depth and its k-derivative against closed
 * forms; the time step's speed, acceleration (ion and atom masses) and dt_max
 * branches against their closed forms; the backscatter rule on free ions
 * crossing z_start in both directions; head-on turning points and scattering
 * angles against root finding and quadrature; energy, momentum and weight ledgers; splitting against brute
 * force; the forward-mode derivative against finite differences of the
 * oracle's own stopping depth.  Fluorite (tests/test_oracle_fluorite.py):
 * textbook geometry and coordination, the anion pair and stopping constants
 * against the Coulomb limit, the printed reduced energy and Lindhard's form,
 * compound friction paths in closed form, the stopping-weighted mean density,
 * the recoil vacancy, the isotropic on-site sampler, the radial range of a
 * free ion, energy and momentum ledgers with two masses, exact record round
 * trips.  Firsov + Brandt-Kitagawa stopping (tests/test_oracle_fkbk.py): Firsov's
 * cross-section as the impact-parameter integral of his collision loss, the
 * kernel's volume integral, flybys past one atom against the kernel's line
 * integral (closed form head on, quadrature off axis) and their speed
 * independence, the effective-charge limits, the atomic velocity unit, a free
 * ion's exponential decay under the Brandt-Kitagawa friction, k = 0 against
 * stopping off; the slow-proton friction of the electron gas is parity
 * unpinned.  The absolute range profile of a full run is
 * parity unpinned against the paper (it prints no profile values and its
 * figures are not available); it is only compared with the GPU library.
 */
#ifndef REEDMD_ORACLE_H
#define REEDMD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_MAX_SPECIES = 8, OR_NCELL = 27, OR_NBASIS = 8, OR_NSLOT = 216 };
/* Fluorite (UO2, Sec. 2 and Sec. 4: 27 cells of the 12-atom fluorite cell):
 * 4 cation and 8 anion sites per cell, 324 domain atoms; the record keeps the
 * 108 cation slots first, padded to 128, then the 216 anion slots. */
enum { OR_MAX_BASIS = 12, OR_MAX_ATOMS = 324, OR_NSLOT_FLUORITE = 344, OR_ANION_SLOT0 = 128 };

/* structures */
enum { OR_DIAMOND = 0, OR_ISOLATED = 1, OR_FLUORITE = 2 };
/* range coordinate (cloning distances and the histogram) */
enum { OR_RANGE_DEPTH = 0, OR_RANGE_RADIAL = 1 };
/* potential modes */
enum { OR_POT_ZBL = 0, OR_POT_NONE = 1 };
/* stopping modes */
enum { OR_STOP_OFF = 0, OR_STOP_UNIFORM = 1, OR_STOP_LOCAL = 2, OR_STOP_FKBK = 3 };
/* track status */
enum { OR_ACTIVE = 0, OR_STOPPED = 1, OR_BACKSCATTERED = 2, OR_NONFINITE = 3,
       OR_STEPCAP = 4 };

typedef struct {
    /* crystal */
    double a;            /* cubic lattice constant (A) */
    double M2;           /* target atom mass (amu) */
    double sigma;        /* thermal rms displacement per axis (A) */
    int32_t Z2;          /* target atomic number */
    int32_t structure;   /* OR_DIAMOND, or OR_ISOLATED (one atom at the origin, no domain following) */
    /* interaction */
    int32_t pot_mode;    /* OR_POT_ZBL / OR_POT_NONE */
    int32_t stop_mode;   /* OR_STOP_* */
    double s;            /* ZBL screening-length scale */
    double k;            /* electronic stopping scale */
    /* integration and events */
    double dx_max;       /* max displacement per step (A) */
    double dt_max;       /* max time step (tau) */
    double E_stop;       /* stop below this kinetic energy (eV) */
    double z_start;      /* start plane; backscatter when z < z_start moving outward */
    int64_t max_steps;   /* per-track step cap (<=0: none) */
    uint64_t seed;       /* crystal realisation seed */
    /* splitting */
    int32_t n_thresh;    /* thresholds per table */
    int32_t n_tables;
    const double* thresholds; /* [n_tables][n_thresh], ascending */
    int32_t n_clones;    /* copies per cloning (2) */
    int32_t n_bins;
    double bin_width;    /* histogram bin width (A), bins cover [0, n_bins*bin_width) */
    /* species */
    int32_t n_species;
    int32_t Z1[OR_MAX_SPECIES];
    double M1[OR_MAX_SPECIES];
    /* second target species: the anion sites of fluorite (the fields above
     * describe target species 0, the only one of diamond) */
    double M2b, sigma_b;
    int32_t Z2b;
    int32_t range_mode;  /* OR_RANGE_DEPTH: z; OR_RANGE_RADIAL: distance from the start point */
    int32_t vacancy;     /* 1: the primary is the recoil of the basis-0 atom of the cell whose
                            origin is nearest its start point; that site stays empty */
    int32_t pad_;
    double r_cut;        /* interaction cut-off (A): domain atoms farther than r_cut from the ion
                            exert no force and add no density; 0: every atom of the 27 cells */
    double n_e;          /* OR_STOP_FKBK: interstitial electron density (electrons per A^3) of the
                            Brandt-Kitagawa term; 0: the local Firsov term alone */
} or_params;

/* One domain atom. */
typedef struct {
    double x[3], v[3], f[3];
    int64_t cell[3];
    int32_t basis;
    int32_t type;        /* target species */
    int32_t exists;
    int32_t pad_;
} or_atom;

/* One ion track with its 27-cell domain (atoms in canonical offset order:
 * offset (i,j,k) in {-1,0,1}^3 with i slowest, then basis b). */
typedef struct {
    double x[3], v[3], F[3];    /* ion position, velocity, ZBL force */
    double rho;                 /* local electron-density weight at the ion */
    double w;                   /* statistical weight */
    int64_t center[3];          /* centre cell */
    uint64_t key;               /* crystal-realisation key of this track */
    int64_t steps;
    int64_t lineage;            /* primary id */
    int32_t species, next_k, table, status;
    double z_stop;
    int32_t n_atoms;            /* 216 (diamond) or 324 (fluorite), 1 for OR_ISOLATED */
    int32_t vac_basis;          /* basis index of the vacant site, -1: none */
    int64_t vac_cell[3];        /* cell of the vacant site */
    double x0[3];               /* start point of the primary (radial range) */
    or_atom atom[OR_MAX_ATOMS];
    /* conservation ledger (stopping off): energy and momentum carried out of
     * the domain by dropped atoms, and potential energy brought in by created atoms */
    double e_out, e_in, p_out[3];
} or_track;

typedef struct {
    int64_t primaries, finished, clones, track_steps, pair_evals;
    int64_t n_stopped, n_backscattered, n_nonfinite, n_stepcap, reserved0;
    double w_stopped, w_backscattered, w_underflow, w_overflow, w_quarantined;
    double sum_wz, sum_wz2, reserved1;
} or_stats;

/* Finished-track log entry. */
typedef struct {
    int64_t lineage;
    int32_t status, next_k;
    double z_stop;
    double w;
    int64_t steps;
} or_result;

/* Primary sampler description. */
enum { OR_DIR_TILT = 0, OR_DIR_CONE = 1, OR_DIR_MIXED = 2, OR_DIR_ISOTROPIC = 3 };
enum { OR_START_SURFACE = 0, OR_START_SITE = 1 };
typedef struct {
    int32_t n_choice;         /* species drawn uniformly from choice[0..n_choice) */
    int32_t choice[OR_MAX_SPECIES];
    int32_t dir_mode;         /* OR_DIR_* */
    int32_t n_energy_tables;  /* threshold tables per species (equal log-energy bands) */
    double E_min, E_max;      /* log-uniform energy; E_min == E_max gives a fixed energy */
    double tilt;              /* polar tilt from +z (rad), azimuth uniform */
    double axis[3];           /* cone axis (unit) */
    double half_angle;        /* cone half angle (rad) */
    int64_t n_cone;           /* DIR_MIXED: ids below this use the cone */
    double a;                 /* entry area is [0,a)^2 */
    double z_start;
    int32_t start_mode;       /* OR_START_SURFACE: uniform over [0,a)^2 at z_start;
                                 OR_START_SITE: the lattice point (0, 0, z_start) */
    int32_t pad_;
} or_sampler;

/* RNG (counter-based Philox4x64-10) */
void or_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
double or_u01(uint64_t w);
/* crystal-realisation keys: of primary `id`, and of clone i made when a track
 * with key `key` crosses cloning depth k (copy 0 continues the parent) */
uint64_t or_primary_key(uint64_t seed, int64_t id);
uint64_t or_child_key(uint64_t key, uint64_t seed, int32_t k, int32_t i);
void or_child_keys(const uint64_t* in, int64_t n, uint64_t seed, int32_t k, int32_t n_clones, uint64_t* out);

/* physics primitives */
/* `type` is the target species (0, or 1 for the fluorite anions) */
double or_screening_length(const or_params* p, int species, int type);
double or_unscaled_screening_length(const or_params* p, int species, int type);
void or_zbl(const or_params* p, int species, int type, double r, double* V, double* dVdr);
double or_lss_kL(const or_params* p, int species, int type);
double or_density_weight(const or_params* p, int species, int type, double r);
double or_gamma(const or_params* p, int species, double rho);
double or_stopping_gamma(const or_params* p, int species, double rho, double v2);
double or_firsov_b(const or_params* p, int species, int type);
double or_firsov_norm(const or_params* p, int species, int type);
double or_firsov_weight(const or_params* p, int species, int type, double r);
double or_bk_zeta(const or_params* p, int species, double v);
double or_bk_proton_friction(const or_params* p);
double or_bk_gamma(const or_params* p, int species, double v);
void or_site(const or_params* p, int b, double f[3], int* type);

/* sampler */
void or_sample_primaries(const or_sampler* s, uint64_t seed, int64_t id0, int64_t n,
                         int32_t* species, double* E0, double* pos, double* dir,
                         uint64_t* key, int32_t* table);

/* single-track interface */
int64_t or_track_size(void);
void or_track_init(const or_params* p, int32_t species, double E0, const double pos[3],
                   const double dir[3], uint64_t key, int32_t table, int64_t lineage,
                   or_track* t);
double or_track_step(const or_params* p, or_track* t);      /* returns dt */
int32_t or_track_events(const or_params* p, or_track* t, double ke_before, double z_before);
double or_range_coord(const or_params* p, const or_track* t);
void or_track_advance(const or_params* p, or_track* t, int64_t nsteps, int32_t with_events);
void or_track_ledger(const or_params* p, const or_track* t, double* energy, double momentum[3]);
void or_track_export(const or_params* p, const or_track* t, double* record);
void or_track_import(const or_params* p, const double* record, or_track* t);
int64_t or_record_words(const or_params* p);

/* whole run: every primary with all of its clones, weighted histogram out */
int32_t or_run(const or_params* p, int64_t n, const int32_t* species, const double* E0,
               const double* pos, const double* dir, const uint64_t* key,
               const int32_t* table, const int64_t* lineage, int32_t nthreads,
               double* hist, or_stats* stats, or_result* log, int64_t log_cap,
               int64_t* log_count);

/* forward-mode derivative of one primary's stopping depth w.r.t. (k, s); no cloning */
int32_t or_grad_track(const or_params* p, int32_t species, double E0, const double pos[3],
                      const double dir[3], uint64_t key, int64_t max_steps, double out[3],
                      int64_t* steps_out);

#ifdef __cplusplus
}
#endif
#endif
