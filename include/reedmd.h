/*
 * reedmd — MI355X (gfx950) REED-MD ion-track engine, C ABI.
 *
 * Rare Event Enhanced Domain-following Molecular Dynamics (Jeon and
 * Gronbech-Jensen, "Efficient Parallel Algorithm for Statistical Ion Track
 * Simulations in Crystalline Materials", Sec. 2): many independent ion tracks
 * are advanced through a thermally disordered crystal.  Each track carries
 * its own 27-unit-cell domain of target atoms that follows the ion (Sec. 2,
 * Fig. 1); ions feel ZBL screened-Coulomb forces from every domain atom and a
 * local electronic friction; the equations of motion are integrated with an
 * adaptive-step velocity Verlet scheme (Sec. 2, Fig. 2); tracks are cloned
 * with halved statistical weights when they reach cloning depths (Sec. 2,
 * Fig. 3); stopped ions are collected in a weighted depth histogram.
 *
 * Units: length A, energy eV, mass amu, time tau = sqrt(amu A^2 / eV) = 10.18 fs.
 *
 * Conventions for every entry point:
 *   - Pointers documented as "device" point to device memory owned by the
 *     caller (e.g. torch tensors); "host" pointers are read or written before
 *     the call returns.  The context owns its own scratch memory (clone stacks,
 *     the clone queue, counters) and frees it in reedmd_destroy.
 *   - Work is enqueued on the caller's HIP stream and the call returns without
 *     waiting, except where a function says it synchronises.
 *   - Errors are status codes, never exceptions; arguments are checked before
 *     anything is launched.  reedmd_last_error() describes the last failure.
 *   - A context is not thread safe: use one context per host thread.
 */
#ifndef REEDMD_H
#define REEDMD_H
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define REEDMD_NSLOT 216                 /* 27 cells x 8 diamond basis atoms */
#define REEDMD_RECORD_WORDS (32 + 9 * 216)
#define REEDMD_NSLOT_FLUORITE 344        /* 27 x 4 cation slots padded to 128, then 27 x 8 anion slots */
#define REEDMD_RECORD_WORDS_FLUORITE (32 + 9 * 344)
#define REEDMD_MAX_SPECIES 8

typedef struct reedmd_ctx reedmd_ctx;

typedef enum {
    REEDMD_OK = 0,
    REEDMD_EINVAL = -1,        /* invalid argument (nothing was launched) */
    REEDMD_ENOMEM = -2,        /* device allocation failed */
    REEDMD_EHIP = -3,          /* HIP runtime error (message in reedmd_last_error) */
    REEDMD_EUNSUPPORTED = -5   /* valid but not implemented combination */
} reedmd_status;

enum { REEDMD_DIAMOND = 0, REEDMD_FLUORITE = 1 };
/* range coordinate used for the cloning depths and the histogram */
enum { REEDMD_RANGE_DEPTH = 0, REEDMD_RANGE_RADIAL = 1 };
enum { REEDMD_POT_ZBL = 0, REEDMD_POT_NONE = 1 };
enum { REEDMD_STOP_OFF = 0, REEDMD_STOP_UNIFORM = 1, REEDMD_STOP_LOCAL = 2, REEDMD_STOP_FKBK = 3 };
enum { REEDMD_FORM_PLAIN = 0, REEDMD_FORM_PERSISTENT = 1 };
/* Precision of the ion-atom pair term (distance, screening exponentials, force
 * coefficient, density weight).  Positions, velocities, force components and
 * sums, kicks, drifts and the step size are FP64 in both. */
enum { REEDMD_FORCE_FP64 = 0, REEDMD_FORCE_FP32 = 1 };
enum { REEDMD_DIR_TILT = 0, REEDMD_DIR_CONE = 1, REEDMD_DIR_MIXED = 2, REEDMD_DIR_ISOTROPIC = 3 };
enum { REEDMD_START_SURFACE = 0, REEDMD_START_SITE = 1 };
/* track status (record word 21, result log) */
enum { REEDMD_ACTIVE = 0, REEDMD_STOPPED = 1, REEDMD_BACKSCATTERED = 2, REEDMD_NONFINITE = 3,
       REEDMD_STEPCAP = 4, REEDMD_CANCELLED = 5, REEDMD_LOST = 6 };

/* Target crystal (Sec. 2: the domain is made of unit cells of the target
 * structure; Sec. 4: temperature as Gaussian displacements of lattice atoms).
 * Cubic cell of constant a; every created atom sits at its ideal site plus an
 * independent N(0, sigma^2) displacement per axis (sigma of its species), at
 * rest.  The crystal occupies z >= 0 (cells with c_z >= 0).
 *   REEDMD_DIAMOND: 8 atoms per cell of one species (Z2, M2, sigma).
 *   REEDMD_FLUORITE (UO2, Sec. 4: 27 cells of the 12-atom cell): cations
 *   (Z2, M2, sigma) on the 4 fcc sites, anions (Z2b, M2b, sigma_b) on the 8
 *   sites with every coordinate 1/4 or 3/4.  Local stopping adds over the two
 *   species (Bragg's rule). */
typedef struct {
    double a;            /* cubic lattice constant (A), > 0 */
    double M2;           /* target (cation) mass (amu), > 0 */
    double sigma;        /* thermal rms displacement per axis (A), >= 0 */
    int32_t Z2;          /* target (cation) atomic number, > 0 */
    int32_t structure;   /* REEDMD_DIAMOND or REEDMD_FLUORITE */
    double M2b;          /* fluorite anion mass (amu), > 0 for fluorite */
    double sigma_b;      /* fluorite anion rms displacement (A), >= 0 */
    int32_t Z2b;         /* fluorite anion atomic number, > 0 for fluorite */
    int32_t reserved;
} reedmd_lattice;

/* Ion-atom interaction (Sec. 2, "First"): ZBL universal screened Coulomb,
 * V(r) = Z1 Z2 e^2 / r * sum_i c_i exp(-d_i r / a), a = s * 0.8854 a0 / (Z1^0.23 + Z2^0.23). */
typedef struct {
    int32_t mode;        /* REEDMD_POT_ZBL, or REEDMD_POT_NONE (no nuclear force; tests) */
    int32_t reserved;
    double s;            /* screening-length scale in [0.01, 100] (1 = ZBL); REEDMD_EINVAL outside */
} reedmd_potential;

/* Electronic stopping (Sec. 2, "Third"), read as a local Lindhard-Scharff
 * friction F = -gamma(x) v with gamma = k N kL sqrt(M1/2) rho(x)/N, where
 * rho(x) = sum_j exp(-r_j/lambda)/(8 pi lambda^3), lambda = a_U/0.3 (unscaled a_U),
 * kL = 1.212 Z1^(7/6) Z2 / ((Z1^(2/3)+Z2^(2/3))^(3/2) sqrt(M1)).  UNIFORM uses rho = N.
 * FKBK is the paper's model (Sec. 2, "Third"; parameters not printed there), read
 * from the works it cites: gamma = k (sum_j C 3 b^3 / (pi (1 + b r_j)^5) + (zeta Z1)^2 gamma_p),
 * a local Firsov loss over the domain atoms (b = 0.31 (Z1+Z2)^(1/3) per A,
 * C = 0.3254 (Z1+Z2) / sqrt(2): Firsov's stopping cross-section over the speed in
 * sqrt(eV/amu)) plus the Brandt-Kitagawa loss of the ion's effective charge zeta Z1
 * (zeta from the Brandt-Kitagawa formula with the Ziegler-Biersack-Littmark
 * ionisation fit) in the interstitial electron gas of density n_e, gamma_p being
 * the slow-proton friction of that gas (Ritchie).  FKBK runs with FP64 pair terms
 * and the 27-cell interaction set (REEDMD_EUNSUPPORTED otherwise); reedmd_grad
 * covers OFF, UNIFORM and LOCAL. */
typedef struct {
    int32_t mode;        /* REEDMD_STOP_OFF / _UNIFORM / _LOCAL / _FKBK */
    int32_t reserved;
    double k;            /* stopping scale, >= 0 */
    double n_e;          /* FKBK: interstitial (muffin-tin residual) electron density, electrons per
                            A^3, finite and >= 0 (0: the Firsov part alone); ignored otherwise */
} reedmd_stopping;

/* Ion species table (host struct, passed by pointer, copied at the call). */
typedef struct {
    int32_t n_species;               /* 1..REEDMD_MAX_SPECIES */
    int32_t reserved;
    int32_t Z1[REEDMD_MAX_SPECIES];  /* > 0 */
    double M1[REEDMD_MAX_SPECIES];   /* amu, > 0 */
} reedmd_species;

/* A batch of primary ions (Sec. 3: all primaries share one statistical
 * description).  Every array is device memory owned by the caller, of length
 * n (pos and dir: [3][n], component major).  Entry i gets lineage id0 + i. */
typedef struct {
    int64_t n;
    int64_t id0;
    int32_t* species;    /* index into the species table */
    double* energy;      /* initial kinetic energy (eV), > E_stop */
    double* pos;         /* start position (A) */
    double* dir;         /* direction (normalised by the library) */
    uint64_t* key;       /* crystal-realisation key of the primary */
    int32_t* table;      /* cloning-depth table index, < n_tables */
} reedmd_batch;

/* Primary sampler (counter-based, seed + lineage id): entry point uniform in
 * [0,a)^2 at z = z_start, or the lattice point (0, 0, z_start) (START_SITE: an
 * on-lattice recoil, Sec. 4); species uniform over choice[]; energy log-uniform
 * in [E_min, E_max] (fixed if equal); direction a polar tilt with uniform
 * azimuth, or uniform in a cone of half angle about axis, or the cone for
 * ids < n_cone and the tilt otherwise, or uniform over the sphere (ISOTROPIC).
 * table = choice index * n_energy_tables + energy band. */
typedef struct {
    int32_t n_choice;
    int32_t choice[REEDMD_MAX_SPECIES];
    int32_t dir_mode;                 /* REEDMD_DIR_* */
    int32_t n_energy_tables;          /* >= 1 */
    int32_t start_mode;               /* REEDMD_START_SURFACE or REEDMD_START_SITE */
    double E_min, E_max;
    double tilt;                      /* rad */
    double axis[3];                   /* unit vector */
    double half_angle;                /* rad */
    int64_t n_cone;
    double a;
    double z_start;
} reedmd_sampler;

/* Run parameters (host struct; the pointers inside are device memory). */
typedef struct {
    double dx_max;       /* max displacement of any particle per step (A), > 0 */
    double dt_max;       /* max step (tau), > 0 */
    double E_stop;       /* stop when the ion's kinetic energy falls below (eV), > 0 */
    double z_start;      /* backscatter when z < z_start and v_z < 0 */
    int64_t max_steps;   /* per-track step cap (capped tracks are quarantined); <= 0: 2,000,000 */
    uint64_t seed;       /* crystal seed shared by every track */
    int32_t n_thresh;    /* cloning depths per table (0 = no splitting) */
    int32_t n_tables;    /* >= 1 when n_thresh > 0 */
    const double* thresholds;  /* device [n_tables][n_thresh], ascending, spaced > 2 dx_max */
    int32_t n_clones;    /* copies per cloning, >= 2 (each gets weight / n_clones) */
    int32_t n_bins;      /* histogram bins, > 0 */
    double bin_width;    /* bins cover [0, n_bins * bin_width) (A) */
    int32_t form;        /* REEDMD_FORM_PLAIN or REEDMD_FORM_PERSISTENT */
    int32_t lanes_per_track;   /* 64, 32 or 16; 0 = from the autotune cache (default 64) */
    int32_t waves_per_cu;      /* persistent form: resident waves per CU (0 = default) */
    int32_t queue_capacity;    /* persistent form: clone-queue records (0 = default: 4 per primary of the
                                  batch, at least 4,096 and at most 65,536) */
    const int32_t* cancel;     /* device word polled by the kernel, non-zero = cancel; may be NULL */
    void* track_log;           /* optional device array of reedmd_result, may be NULL */
    int64_t track_log_cap;
    int32_t force_precision;   /* REEDMD_FORCE_FP64 (0) or REEDMD_FORCE_FP32 (1; run, track_init,
                                  debug_step, autotune; reedmd_grad is FP64 only) */
    int32_t range_mode;        /* REEDMD_RANGE_DEPTH: cloning depths and histogram in z;
                                  REEDMD_RANGE_RADIAL: in the distance from the primary's start
                                  point (recoils inside the crystal, Sec. 4); fluorite only
                                  (diamond: REEDMD_EUNSUPPORTED) */
    int32_t vacancy;           /* 1: each primary is the recoil of the basis-0 atom of the cell
                                  whose origin is nearest its start point (floor(x/a + 1/4) per
                                  axis); that site stays empty for the whole track and its clones;
                                  fluorite only (diamond: REEDMD_EUNSUPPORTED) */
    int32_t no_tail_handoff;   /* persistent form with 16 or 32 lanes per track: 0 (default) hands the
                                  tail to a 64-lane launch of the track kernel in the same pipeline
                                  once every primary is claimed and no more tracks are live than that
                                  launch has segments (running tracks move through the clone queue,
                                  exactly: results are the same bit for bit); 1: no handoff */
    double r_cut;              /* interaction set of the domain (Sec. 2 builds it from the 27 cells
                                  around the ion): 0 (default) = every atom of the 27 cells; > 0 =
                                  only atoms within r_cut (A) of the ion exert force on it, are
                                  pushed by it and add to the electron density (all atoms still
                                  move; the in-range atoms are compacted so the pair work shrinks
                                  with the set); diamond target with FP64 forces only, else
                                  REEDMD_EUNSUPPORTED; < 0 = the set reedmd_autotune_domain recorded
                                  for this configuration and batch size (27 cells if none),
                                  resolved by reedmd_run, reedmd_run_noalloc, reedmd_run_refined
                                  and reedmd_autotune (REEDMD_EINVAL for reedmd_track_init and
                                  reedmd_debug_step); reedmd_grad: 0 only (REEDMD_EUNSUPPORTED) */
} reedmd_run_params;

/* Finished-track entry of the optional log (48 bytes). */
typedef struct {
    int64_t lineage;
    int32_t status;
    int32_t next_k;      /* cloning depths crossed: weight = n_clones^-next_k */
    double z_stop;
    double w;
    int64_t steps;
    uint64_t key;        /* crystal-realisation key the track ended with: the primary's key,
                            re-derived at every cloning depth k as the key of copy i (copy 0
                            continues the parent; Sec. 2, clones differ only in material
                            created after the cloning) */
} reedmd_result;

/* Run statistics (device struct owned by the caller; reedmd_run adds to it). */
typedef struct {
    int64_t primaries, finished, clones, track_steps, pair_evals;
    int64_t n_stopped, n_backscattered, n_nonfinite, n_stepcap, n_cancelled;
    double w_stopped, w_backscattered, w_underflow, w_overflow, w_quarantined;
    double sum_wz, sum_wz2, w_cancelled;
    int64_t max_queue, stack_overflow, log_count, error_flags;
    int64_t handed_off;  /* tracks moved to the 64-lane tail launch (see no_tail_handoff) */
} reedmd_stats;

/* Library version, e.g. 100 for 0.1.0. */
int32_t reedmd_version(void);

/* Creates a context for one target crystal and interaction model on the
 * current HIP device.  out receives the context (host).  EINVAL on bad
 * values, EHIP if no device is usable. */
reedmd_status reedmd_create(const reedmd_lattice* lattice, const reedmd_potential* potential,
                            const reedmd_stopping* stopping, reedmd_ctx** out);

/* Frees the context and all memory it owns; NULL is ignored.  Synchronises
 * the device first. */
void reedmd_destroy(reedmd_ctx* ctx);

/* Number of persistent-form pipelines (queue reset, track kernel, statistics)
 * the context keeps as instantiated HIP graphs: one per launch shape (lanes per
 * track, precision, target, workgroups, queue capacity), at most 16 (the cache
 * is emptied when a 17th shape arrives or the scratch memory grows).  Every call
 * writes its own arguments into the graph's kernel nodes, so fresh buffers do
 * not add entries.  Host call; 0 for NULL. */
int32_t reedmd_cached_graphs(const reedmd_ctx* ctx);

/* Message for the last non-OK status returned on this context (never NULL;
 * ctx may be NULL for errors of reedmd_create). */
const char* reedmd_last_error(const reedmd_ctx* ctx);

/* Fills out's device arrays (n = out->n entries, lineage ids id0 .. id0+n-1)
 * from the counter-based sampler keyed by seed (Sec. 3: every primary starts
 * from the same statistical description).  Enqueued on stream. */
reedmd_status reedmd_sample_primaries(reedmd_ctx* ctx, const reedmd_sampler* sampler,
                                      uint64_t seed, const reedmd_batch* out, hipStream_t stream);

/* Runs every primary of the batch to termination together with every clone
 * it produces (Sec. 2), and adds the weights of stopped ions to d_hist
 * (device, n_bins doubles, bin = floor(z_stop / bin_width)) and the run totals
 * to d_stats (device).  PLAIN form: a static assignment of primaries to
 * wavefronts, each finishing its own clones depth first.  PERSISTENT form:
 * resident wavefronts take primaries and clones from a device work queue
 * until no track is live (replacing the paper's host-client polling, Sec. 3).
 * Enqueued on stream; the results are valid once the stream reaches this
 * point.  A non-zero *cancel drains the run: live and unstarted tracks end
 * with status CANCELLED and their weight goes to w_cancelled. */
reedmd_status reedmd_run(reedmd_ctx* ctx, const reedmd_species* species, const reedmd_batch* batch,
                         const reedmd_run_params* params, double* d_hist, reedmd_stats* d_stats,
                         hipStream_t stream);

/* The plain form of reedmd_run for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): it calls no hipMalloc, hipFree or allocating library routine.
 * Its scratch memory (queue state, claim order, clone stacks) is one static
 * device array of 128 MiB that the library defines and every GPU it runs on
 * holds until the process ends; the caller still passes the inputs and the
 * outputs (d_hist, d_stats, the optional track log), with the meanings of
 * reedmd_run.  params->form must be REEDMD_FORM_PLAIN (EUNSUPPORTED
 * otherwise).  The number of track segments is cut to what fits the array
 * (results do not depend on it); EINVAL when a batch's claim order (4 bytes
 * per primary) or one segment's clone stack (n_thresh * (n_clones - 1) + 1
 * records) does not fit.  Every call on a GPU uses that GPU's one array and
 * leaves its contents behind (each call clears what must start at zero), so
 * calls that overlap on one GPU race: run them in order on one stream.
 * Enqueued on stream. */
reedmd_status reedmd_run_noalloc(reedmd_ctx* ctx, const reedmd_species* species, const reedmd_batch* batch,
                                 const reedmd_run_params* params, double* d_hist, reedmd_stats* d_stats,
                                 hipStream_t stream);

/* Adaptive cloning depths (Sec. 2: the depths are placed from the statistics
 * gathered so far; Sec. 3: criteria are updated between complete tracks). */
typedef struct {
    int32_t n_epochs;       /* the batch runs in n_epochs epochs, 1..4096 */
    int32_t in_launch;      /* 0: one launch per epoch; 1: all epochs in one persistent launch */
    const double* probs;    /* host, n_thresh target survival probabilities, strictly decreasing in (0,1) */
    double min_gap;         /* minimum spacing of successive depths (A), >= 0 */
    double* snapshots;      /* in_launch only: optional device [n_epochs][n_tables][n_bins + 2] */
    double min_weight;      /* a target k is placed only if probs[k] x booked weight >= min_weight
                               (primaries' worth; 1 is a good default), finite, >= 0 */
} reedmd_refine;

/* Like reedmd_run, with the cloning depths refined between epochs.  Epoch e
 * runs batch entries [n e / E, n (e+1) / E) with the depth tables in force;
 * params->thresholds (device, n_tables x n_thresh) are those of epoch 0.
 * Before epoch e > 0 every table is re-placed from all tracks of that table
 * booked so far: with S(z) = (weight stopped at z_stop >= z) / (all weight
 * booked for the table) on the histogram's bin edges, depth k is where S falls
 * to probs[k] (linear in S within the bin); the targets placed so are the
 * leading ones, and the rest (S does not reach them within the histogram, or
 * the statistics are too thin for them: probs[k] times the booked weight
 * below min_weight) keep their previous depths shifted by the move of the last
 * placed depth (unshifted when none is placed); the depths are then made
 * increasing by at least min_gap.  New depths apply only to primaries started
 * later, so every primary family keeps one depth table and the estimator stays
 * unbiased.  d_hist, d_stats and the optional track log accumulate over all
 * epochs as in reedmd_run; d_depths (device, optional, n_epochs x n_tables x
 * n_thresh doubles) receives the tables each epoch ran with; params->thresholds
 * is not modified.
 *
 * in_launch = 1 runs every epoch inside one launch of the persistent form
 * (params->form must be REEDMD_FORM_PERSISTENT, else EINVAL): epoch e is the
 * claim positions [ceil(n e / E), ceil(n (e+1) / E)) of the primaries (claimed
 * in the launch's longest-expected-first order), and the segment that claims
 * the first position of epoch e > 0 re-places every table from the tracks
 * booked by then (the same rule applied to the depths of epoch 0, so a target
 * not placed keeps its epoch-0 depth shifted by the last placed one's move)
 * while the other segments go on running; the epoch's other primaries start
 * once its tables are published.
 * No launch boundary drains the GPU between epochs; which tracks a table's
 * statistics hold depends on timing, so the depths are not reproducible run
 * to run (each family still keeps one table and the estimator stays unbiased).
 * The statistics each table was placed from (per table: stopped weight of each
 * bin, stopped weight beyond the last bin, all booked weight; zeros for epoch
 * 0) go to snapshots when it is non-NULL.
 *
 * Allocates its work buffers, synchronises the stream.  EINVAL for invalid
 * settings (n_thresh >= 1 is required). */
reedmd_status reedmd_run_refined(reedmd_ctx* ctx, const reedmd_species* species, const reedmd_batch* batch,
                                 const reedmd_run_params* params, const reedmd_refine* rf, double* d_hist,
                                 reedmd_stats* d_stats, double* d_depths, hipStream_t stream);

/* Builds the starting record (ion, its full domain and the forces at the
 * start point) of each batch entry into d_records (device, n *
 * REEDMD_RECORD_WORDS 64-bit words; REEDMD_RECORD_WORDS_FLUORITE for a
 * fluorite context).  Record layout: words 0-2 ion position,
 * 3-5 velocity, 6-8 ZBL force, 9 local (stopping-weighted) density, 10 weight,
 * 11 stopping depth (range coordinate), 12-14 centre cell (int64), 15 key
 * (uint64), 16 steps, 17 lineage, 18 species, 19 crossed thresholds, 20 table,
 * 21 status, 22-23 largest atom |v|^2 and |f/M|^2 (valid when word 24 == 1;
 * records made elsewhere may leave 22-24 zero and the library then recomputes
 * them), 25-27 cell of the vacant site (int64), 28 its basis index (-1: none),
 * 29-31 start point of the primary; then nine fields x, y, z, vx, vy, vz, fx,
 * fy, fz of the domain atoms with NS = 216 (diamond) or 344 (fluorite) entries
 * each.  With r = (c_x mod 3)*9 + (c_y mod 3)*3 + (c_z mod 3), the slot of
 * basis atom b of cell c is r*8 + b (diamond); r*4 + b for the fluorite
 * cations (b < 4) and 128 + r*8 + b - 4 for its anions.  Slots of cells with
 * c_z < 0, the vacant site and fluorite slots 108..127 hold no atom (zeros).
 * Fluorite runs on 64 or 32 lanes per track (16: REEDMD_EUNSUPPORTED). */
reedmd_status reedmd_track_init(reedmd_ctx* ctx, const reedmd_species* species,
                                const reedmd_batch* batch, const reedmd_run_params* params,
                                double* d_records, hipStream_t stream);

/* Advances each of the n records in d_records (device, in place) by nsteps
 * integration steps (Sec. 2), without termination events or cloning.  For
 * per-step parity checks.  lanes_per_track in params selects the kernel.
 * Records are laid out as for reedmd_track_init (REEDMD_RECORD_WORDS, or
 * REEDMD_RECORD_WORDS_FLUORITE for a fluorite context). */
reedmd_status reedmd_debug_step(reedmd_ctx* ctx, const reedmd_species* species,
                                const reedmd_run_params* params, double* d_records, int64_t n,
                                int32_t nsteps, hipStream_t stream);

/* Derivative of the mean projected range (mean stopping depth over the tracks
 * of the batch that stop; backscattered and capped tracks are excluded) with
 * respect to the electronic-stopping scale k and the ZBL screening-length
 * scale s, evaluated at (k, s) (they replace the context's values for this
 * call; k >= 0 and s in [0.01, 100], EINVAL otherwise).  Reverse mode: every
 * track runs forward with a checkpoint of its full state every 64 steps, a log
 * of each step's size and starting ion state, and a log of the atoms each
 * domain move drops; the reverse sweep then rebuilds each step's starting
 * state from the state after it (domain atoms run backwards, the ion from the
 * log, dropped atoms from their log; re-anchored to the checkpoint every 64
 * steps) and applies the adjoint of the steps from last to first.  A track
 * that moves its domain more than 2 (max_steps/64 + 1) times ends as capped.
 * The
 * derivative is pathwise: branches (active step-size term, domain updates,
 * which step stops the ion) are held fixed, created atoms are constants.
 * Requires params->n_thresh == 0, FP64 pair terms, a diamond context, the
 * depth range and no vacancy (EUNSUPPORTED otherwise); params->max_steps
 * bounds the track length and the checkpoint memory (<= 0: 16,384 steps).
 * d_track_out (device, optional, n x 5 doubles) receives per track: stopping
 * depth, d/dk, d/ds, status, steps.  h_result (host, 4 doubles) receives the
 * mean range, its two derivatives and the number of stopped tracks.
 * Synchronises the stream. */
reedmd_status reedmd_grad(reedmd_ctx* ctx, const reedmd_species* species, const reedmd_batch* batch,
                          const reedmd_run_params* params, double k, double s, double* d_track_out,
                          double* h_result, hipStream_t stream);

/* Evaluates, for finite 0 <= y[i] < 1e9 (device, n doubles), the library's
 * exp(-y) into out (device); outside that range the value is unspecified.
 * reedmd_eval_exp_neg: the friction factors' exponential (Cody-Waite reduction
 * to |r| <= ln2/2, degree-10 minimax polynomial, ldexp; relative error 3e-16).
 * reedmd_eval_exp_neg_pair: the exponential of the ion-atom pair terms (same
 * reduction, degree-8 minimax polynomial; relative error 1.08e-12, inside the
 * per-step tolerance of 1e-10 of the FP64 path).  For accuracy tests.
 * Enqueued on stream; EINVAL for n < 0 or NULL arrays. */
reedmd_status reedmd_eval_exp_neg(const double* d_y, double* d_out, int64_t n, hipStream_t stream);
reedmd_status reedmd_eval_exp_neg_pair(const double* d_y, double* d_out, int64_t n, hipStream_t stream);

/* Evaluates the library's natural logarithm (used by the Brandt-Kitagawa
 * stopping, Sec. 2 "Third": its powers y^0.3 and (1-q)^(2/3) are taken as
 * exponentials of logarithms, and ln(1 + x)) into out (device, n doubles):
 * one_plus = 0: ln x for normal finite x > 0 (x = m 2^k, ln m = 2 atanh((m-1)/(m+1))
 * from its series); one_plus = 1: ln(1 + x) for finite x >= 0, with its
 * relative accuracy kept for small x.  Other inputs give unspecified values.
 * For accuracy tests.  Enqueued on stream; EINVAL for n < 0, NULL arrays or
 * one_plus not 0 or 1. */
reedmd_status reedmd_eval_log(const double* d_x, double* d_out, int64_t n, int32_t one_plus, hipStream_t stream);

/* Chooses the launch shape for runs like this one.  Each candidate (lanes per
 * track 64, 32, 16; for the persistent form also one workgroup per CU fewer
 * than the occupancy allows) runs on the first `pilot` primaries of the batch
 * and is cancelled through a pinned host word 400 ms after it starts (unless
 * it ends earlier); the candidate with the most pair evaluations per second
 * (steady-state throughput, not the tail of a small pilot) is recorded in the
 * context's cache under this configuration and batch size class, and
 * *best_lanes and *best_waves (host) receive the choice.  The caller's
 * histogram and statistics are not touched.  Synchronises the stream. */
reedmd_status reedmd_autotune(reedmd_ctx* ctx, const reedmd_species* species,
                              const reedmd_batch* batch, const reedmd_run_params* params,
                              int64_t pilot, hipStream_t stream, int32_t* best_lanes,
                              int32_t* best_waves);

/* Interaction-set autotuner (Sec. 2: the ion interacts with the atoms of
 * the 27 cells around it; a cut-off keeps those within r_cut, fewer pair
 * terms, which must leave the range distribution unchanged).
 * candidates (host, n_candidates values, 1..8): 0 = the 27 cells, > 0 = a
 * cut-off radius (A).  The first `pilot` primaries of the batch run to the
 * end (params as given, finished-track log kept internally) once with the 27
 * cells, the reference, and once per cut-off candidate.  A candidate passes
 * its gate when the weighted two-sample Kolmogorov-Smirnov test of its
 * stopping depths against the reference's (effective sizes (sum w)^2 /
 * sum w^2, asymptotic Kolmogorov distribution) gives p > gate_p and its
 * weighted mean and standard deviation of the depth differ from the
 * reference's by at most gate_rel relative, or by at most three standard
 * errors of the difference where those exceed gate_rel (a pilot too small
 * to resolve gate_rel cannot fail on noise; use a pilot whose standard
 * errors are below gate_rel / 3 for a strict gate).  Of the passing
 * candidates (the 27 cells always pass) the one whose pilot run took the
 * least GPU time is recorded in the context's cache under this
 * configuration and batch size class (the lanes and waves entry of
 * reedmd_autotune is kept) and written to *best_r_cut (host).  report
 * (host, may be NULL): 5 values per candidate in input order, the pilot
 * run's GPU milliseconds, the KS p value, the relative difference of the
 * mean, of the standard deviation, and 1 if the gate passed else 0.  Caller
 * histogram and statistics are not touched; synchronises the stream.
 * EINVAL: NULL arguments, n_candidates outside 1..8, a negative or
 * non-finite candidate, pilot <= 0, gate_p outside [0, 1), gate_rel < 0. */
reedmd_status reedmd_autotune_domain(reedmd_ctx* ctx, const reedmd_species* species,
                                     const reedmd_batch* batch, const reedmd_run_params* params,
                                     const double* candidates, int32_t n_candidates, int64_t pilot,
                                     double gate_p, double gate_rel, hipStream_t stream,
                                     double* best_r_cut, double* report);

/* The launch shape reedmd_run would use for this batch size and these
 * parameters (after the autotune cache), written to out (host, 5 values):
 * lanes per track, workgroups (256 threads each), track segments, workgroups
 * of the track kernel that fit on one CU, clone-queue capacity (0 for the
 * plain form).  Host call; nothing is enqueued.  EINVAL for NULL arguments or
 * invalid parameters. */
reedmd_status reedmd_launch_shape(reedmd_ctx* ctx, const reedmd_batch* batch,
                                  const reedmd_run_params* params, int64_t* out);

#ifdef __cplusplus
}
#endif
#endif
