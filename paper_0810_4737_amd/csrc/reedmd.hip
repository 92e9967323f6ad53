// reedmd C ABI: context, argument checks, scratch memory, launches, hipGraph
// capture of the persistent pipeline and the launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/reedmd.h"
#include "adjoint_kernels.hpp"
#include "track_kernels.hpp"

// Scratch memory of the allocation-free entry point (reedmd_run_noalloc): one
// static device array of this size, which every GPU the library runs on holds
// (its own copy) until the process ends.
constexpr unsigned long long kNoAllocBytes = 128ull << 20;   // 128 MiB

using namespace reedmd;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr double kCoulomb = 14.3996454784;   // e^2 / (4 pi eps0), eV A (CODATA 2018)
constexpr double kBohr = 0.529177210903;     // A
constexpr double kHartree = 27.211386245988;  // eV (CODATA 2018)
constexpr double kAuVelocity = 2.18769126364e6;   // atomic unit of velocity, m/s (CODATA 2018)
// The velocity unit of the library, sqrt(eV/amu), in m/s (eV and amu of CODATA 2018).
const double kVelocityUnit = std::sqrt(1.602176634e-19 / 1.66053906660e-27);

// Friction coefficient of a slow proton in an electron gas of density n_e (electrons
// per A^3), Ritchie (1959): 2 / (3 pi) [ln(1 + pi / (alpha rs)) - 1 / (1 + alpha rs / pi)]
// in atomic units, alpha = (4 / (9 pi))^(1/3), rs the Wigner-Seitz radius in bohr;
// returned in eV / A per sqrt(eV/amu).
double bk_proton_friction(double n_e)
{
    const double rs = std::cbrt(3.0 / (4.0 * M_PI * n_e * kBohr * kBohr * kBohr));
    const double alpha = std::cbrt(4.0 / (9.0 * M_PI));
    const double g_au = 2.0 / (3.0 * M_PI) * (std::log(1.0 + M_PI / (alpha * rs)) - 1.0 / (1.0 + alpha * rs / M_PI));
    return g_au * (kHartree / kBohr) / (kAuVelocity / kVelocityUnit);
}
constexpr int kBlock = 256;                  // 4 wavefronts per workgroup
constexpr long long kDefaultMaxSteps = 2000000;   // step cap when the caller sets none
constexpr double kMinScreening = 0.01;         // accepted range of the screening-length scale s:
constexpr double kMaxScreening = 100.0;        // keeps every exponent argument below 1e9
constexpr long long kDefaultGradSteps = 16384;    // gradient step cap when the caller sets none
constexpr int kTuneBoxMs = 400;                   // autotuner: time box of each candidate launch
constexpr size_t kGradScratchBytes = size_t(48) << 30;   // checkpoint memory per launch chunk
constexpr size_t kMaxGraphs = 16;
constexpr long long kMaxQueue = 65536;            // default clone-queue capacity cap (1.0 GB of diamond records)                 // instantiated persistent pipelines kept per context

thread_local std::string g_create_error;

// Host code never uses the name of the allocation-free entry point's scratch
// array as an address: its device address is taken once per device with
// hipGetSymbolAddress at context creation and kept here.
constexpr int kMaxDevices = 64;
void* g_noalloc_ptr[kMaxDevices] = {};

}  // namespace

struct reedmd_ctx {
    int device = 0;
    int cu_count = 0;
    reedmd_lattice lat{};
    reedmd_potential pot{};
    reedmd_stopping stop{};
    std::string err;
    // scratch
    void* scratch = nullptr;       // QueueState + qseq + qrec
    size_t scratch_bytes = 0;
    double* stack = nullptr;
    size_t stack_bytes = 0;
    int* ordbuf = nullptr;         // claim order: bucket counts, offsets, order of the batch
    size_t ordbuf_bytes = 0;
    double* gscratch = nullptr;    // adjoint checkpoints, segment states, outputs
    size_t gscratch_bytes = 0;
    // autotune cache: config hash -> (lanes, waves per CU)
    struct Tuned {
        int lanes, waves;
        double r_cut;   // interaction set: 0 = the 27 cells, > 0 = cut-off radius (A)
    };
    std::map<unsigned long long, Tuned> tune;
    // persistent pipelines (reset -> claim order -> track kernel -> statistics) as instantiated graphs,
    // one per launch shape; the kernel arguments of every call are written into the nodes
    struct Graph {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipGraphNode_t node[7] = {};   // reset, order count, scan, scatter, track kernel, [64-lane tail], statistics
    };
    std::map<std::vector<long long>, Graph> graphs;
};

namespace {

reedmd_status fail(reedmd_ctx* ctx, reedmd_status st, const std::string& msg)
{
    if (ctx) ctx->err = msg;
    else g_create_error = msg;
    return st;
}

reedmd_status hip_fail(reedmd_ctx* ctx, hipError_t e, const char* what)
{
    return fail(ctx, REEDMD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(ctx, call)                                   \
    do {                                                     \
        hipError_t e__ = (call);                             \
        if (e__ != hipSuccess) return hip_fail(ctx, e__, #call); \
    } while (0)

// Per-species constants for the kernels (ZBL screening length and Coulomb
// prefactor, density kernel, Lindhard-Scharff friction coefficient).  With two
// target species (fluorite) the second gets its own pair constants, its density
// weight carries k_L(species 1) / k_L(species 0) (Bragg additivity), and the
// friction uses the stopping-weighted uniform density N_0 + N_1 k_L1 / k_L0.
void prepare_species(const reedmd_ctx* ctx, const reedmd_species* sp, KernelArgs& A)
{
    const bool fl = ctx->lat.structure == REEDMD_FLUORITE;
    const double a3 = ctx->lat.a * ctx->lat.a * ctx->lat.a;
    const double N0 = (fl ? 4.0 : 8.0) / a3, N1 = fl ? 8.0 / a3 : 0.0;
    double min_rate = HUGE_VAL;
    const double zc[4] = {kZc0, kZc1, kZc2, kZc3}, zd[4] = {kZd0, kZd1, kZd2, kZd3};
    struct Target {
        double inv_a, zz, inv_lambda, wnorm, kL;
    };
    auto target = [&](double Z1, double M1, double Z2) {
        Target t;
        const double aU = 0.8854 * kBohr / (std::pow(Z1, 0.23) + std::pow(Z2, 0.23));
        const double lambda = aU / 0.3;
        const double z23 = std::pow(Z1, 2.0 / 3.0) + std::pow(Z2, 2.0 / 3.0);
        t.kL = 1.212 * std::pow(Z1, 7.0 / 6.0) * Z2 / (std::pow(z23, 1.5) * std::sqrt(M1));
        t.inv_a = 1.0 / (ctx->pot.s * aU);
        t.zz = (ctx->pot.mode == REEDMD_POT_ZBL) ? Z1 * Z2 * kCoulomb : 0.0;
        t.inv_lambda = 1.0 / lambda;
        t.wnorm = 1.0 / (8.0 * M_PI * lambda * lambda * lambda);
        return t;
    };
    for (int i = 0; i < kMaxSpecies; ++i) {
        SpeciesConst& c = A.sp[i];
        PairConst& c2 = A.pc2[i];
        if (i >= sp->n_species) {
            c = SpeciesConst{1.0, 0.5, 1.0, 0.0, 1.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0};
            c2 = PairConst{};
            c2.lam2 = 1.0;
            c.lam2 = 1.0;
            continue;
        }
        const double Z1 = sp->Z1[i], M1 = sp->M1[i];
        const Target t0 = target(Z1, M1, ctx->lat.Z2);
        const double N = fl ? N0 + N1 * target(Z1, M1, ctx->lat.Z2b).kL / t0.kL : N0;
        const double gamma0 = N * t0.kL * std::sqrt(M1 / 2.0);
        c.M1 = M1;
        c.half_inv_M1 = 1.0 / (2.0 * M1);
        c.inv_M1sq = 1.0 / (M1 * M1);
        c.inv_a = t0.inv_a;
        c.zz = t0.zz;
        c.inv_lambda = t0.inv_lambda;
        c.wnorm = t0.wnorm;
        for (int j = 0; j < 4; ++j) {
            c.rate[j] = zd[j] * c.inv_a * M_LOG2E;
            c.amp[j] = c.zz * zc[j];
            c.damp[j] = c.zz * zc[j] * zd[j] * c.inv_a;
            c.rate2f[j] = static_cast<float>(c.rate[j]);
            c.amp_f[j] = static_cast<float>(c.amp[j]);
            c.damp_f[j] = static_cast<float>(c.damp[j]);
        }
        c.lam2 = c.inv_lambda * M_LOG2E;
        c.lam2f = static_cast<float>(c.lam2);
        min_rate = std::min(min_rate, std::min(zd[3] * c.inv_a, c.inv_lambda));
        c2 = PairConst{};
        c2.lam2 = 1.0;
        if (fl) {
            const Target t1 = target(Z1, M1, ctx->lat.Z2b);
            c2.lam2 = t1.inv_lambda * M_LOG2E;
            c2.wnorm = t1.wnorm * (t1.kL / t0.kL);
            for (int j = 0; j < 4; ++j) {
                c2.rate[j] = zd[j] * t1.inv_a * M_LOG2E;
                c2.amp[j] = t1.zz * zc[j];
                c2.damp[j] = t1.zz * zc[j] * zd[j] * t1.inv_a;
                c2.rate2f[j] = static_cast<float>(c2.rate[j]);
                c2.amp_f[j] = static_cast<float>(c2.amp[j]);
                c2.damp_f[j] = static_cast<float>(c2.damp[j]);
            }
            c2.lam2f = static_cast<float>(c2.lam2);
            min_rate = std::min(min_rate, std::min(zd[3] * t1.inv_a, t1.inv_lambda));
        }
        c.g_const = 0.0;
        c.g_rho = 0.0;
        c.dg_const = 0.0;
        c.dg_rho = 0.0;
        if (ctx->stop.mode == REEDMD_STOP_UNIFORM) {
            c.g_const = ctx->stop.k * gamma0;
            c.dg_const = gamma0;
        }
        if (ctx->stop.mode == REEDMD_STOP_LOCAL) {
            c.g_rho = ctx->stop.k * gamma0 / N;
            c.dg_rho = gamma0 / N;
        }
        if (ctx->stop.mode == REEDMD_STOP_FKBK) {
            // Firsov: the density weight becomes the kernel C 3 b^3 / (pi (1 + b r)^5) with
            // C = 0.3254 (Z1+Z2) / sqrt(2) (Firsov's cross-section over the speed); b rides in lam2
            auto firsov = [&](double Z2, double& b, double& norm) {
                b = 0.31 * std::cbrt(Z1 + Z2);
                norm = 0.3254 * (Z1 + Z2) / std::sqrt(2.0) * 3.0 * b * b * b / M_PI;
            };
            firsov(ctx->lat.Z2, c.lam2, c.wnorm);
            if (fl) firsov(ctx->lat.Z2b, c2.lam2, c2.wnorm);
            c.g_rho = ctx->stop.k;
            c.dg_rho = 1.0;
            // Brandt-Kitagawa: k Z1^2 gamma_p, gamma_p the slow-proton friction of the electron gas
            A.bk_z13[i] = std::cbrt(Z1);
            A.bk_pref[i] = ctx->stop.n_e > 0.0 ? ctx->stop.k * Z1 * Z1 * bk_proton_friction(ctx->stop.n_e) : 0.0;
        }
    }
    if (ctx->stop.mode == REEDMD_STOP_FKBK && ctx->stop.n_e > 0.0) {
        const double n_au = ctx->stop.n_e * kBohr * kBohr * kBohr;
        A.bk_vF = std::cbrt(9.0 * M_PI / 4.0) / std::cbrt(3.0 / (4.0 * M_PI * n_au));
        A.bk_inv_vunit = kVelocityUnit / kAuVelocity;
    }
    // Empty slots are parked where the slowest exponential of every species in use
    // is below e^-1000, so their pair terms are exactly zero (at least 1 um away).
    A.park = std::max(1.0e4, 1.0e3 / min_rate);
}

int lattice_of(const reedmd_ctx* ctx) { return ctx->lat.structure == REEDMD_FLUORITE ? kFluorite : kDiamond; }

// Pass variant of the track kernels for an interaction set (resolved r_cut) and the
// context's stopping model.
int pass_variant(const reedmd_ctx* ctx, double r_cut)
{
    return (r_cut > 0.0 ? kVarCut : 0) | (ctx->stop.mode == REEDMD_STOP_FKBK ? kVarFirsov : 0);
}
size_t record_words(const reedmd_ctx* ctx)
{
    return lattice_of(ctx) == kFluorite ? Lattice<kFluorite>::kRecWords : Lattice<kDiamond>::kRecWords;
}

reedmd_status check_species(reedmd_ctx* ctx, const reedmd_species* sp)
{
    if (!sp) return fail(ctx, REEDMD_EINVAL, "species table is NULL");
    if (sp->n_species < 1 || sp->n_species > REEDMD_MAX_SPECIES)
        return fail(ctx, REEDMD_EINVAL, "n_species must be in 1..8");
    for (int i = 0; i < sp->n_species; ++i)
        if (sp->Z1[i] <= 0 || !(sp->M1[i] > 0.0)) return fail(ctx, REEDMD_EINVAL, "species Z1 and M1 must be positive");
    return REEDMD_OK;
}

reedmd_status check_params(reedmd_ctx* ctx, const reedmd_run_params* p, bool need_hist, bool cached_rcut = true)
{
    if (!p) return fail(ctx, REEDMD_EINVAL, "params is NULL");
    if (!std::isfinite(p->r_cut)) return fail(ctx, REEDMD_EINVAL, "r_cut must be finite");
    if (p->r_cut < 0.0 && !cached_rcut)
        return fail(ctx, REEDMD_EINVAL, "r_cut < 0 (the domain autotuner's choice) is resolved by the run entry points only");
    if (p->r_cut > 0.0 && (lattice_of(ctx) != kDiamond || p->force_precision != REEDMD_FORCE_FP64))
        return fail(ctx, REEDMD_EUNSUPPORTED, "the interaction cut-off is built for the diamond target with FP64 forces");
    if (ctx->stop.mode == REEDMD_STOP_FKBK && (p->force_precision != REEDMD_FORCE_FP64 || p->r_cut > 0.0))
        return fail(ctx, REEDMD_EUNSUPPORTED, "the Firsov + Brandt-Kitagawa stopping runs with FP64 pair terms and the 27 cells");
    if (p->range_mode != REEDMD_RANGE_DEPTH && p->range_mode != REEDMD_RANGE_RADIAL)
        return fail(ctx, REEDMD_EINVAL, "range_mode must be REEDMD_RANGE_DEPTH or REEDMD_RANGE_RADIAL");
    if (p->vacancy != 0 && p->vacancy != 1) return fail(ctx, REEDMD_EINVAL, "vacancy must be 0 or 1");
    if (lattice_of(ctx) != kFluorite && (p->range_mode != REEDMD_RANGE_DEPTH || p->vacancy != 0))
        return fail(ctx, REEDMD_EUNSUPPORTED, "the radial range and the recoil vacancy are built for the fluorite target");
    if (lattice_of(ctx) == kFluorite && p->lanes_per_track == 16)
        return fail(ctx, REEDMD_EUNSUPPORTED, "the fluorite domain (344 slots) runs on 32 or 64 lanes per track");
    if (!(p->dx_max > 0.0) || !(p->dt_max > 0.0) || !(p->E_stop > 0.0) || !std::isfinite(p->z_start))
        return fail(ctx, REEDMD_EINVAL, "dx_max, dt_max and E_stop must be positive, z_start finite");
    if (p->n_thresh < 0 || p->n_thresh > 64) return fail(ctx, REEDMD_EINVAL, "n_thresh must be in 0..64");
    if (p->n_thresh > 0) {
        if (p->n_tables < 1 || !p->thresholds) return fail(ctx, REEDMD_EINVAL, "thresholds need n_tables >= 1 and a pointer");
        if (p->n_clones < 2 || p->n_clones > 16) return fail(ctx, REEDMD_EINVAL, "n_clones must be in 2..16");
    }
    if (need_hist) {
        if (p->n_bins <= 0 || !(p->bin_width > 0.0)) return fail(ctx, REEDMD_EINVAL, "n_bins and bin_width must be positive");
        if (p->form != REEDMD_FORM_PLAIN && p->form != REEDMD_FORM_PERSISTENT)
            return fail(ctx, REEDMD_EINVAL, "unknown form");
    }
    if (p->lanes_per_track != 0 && p->lanes_per_track != 64 && p->lanes_per_track != 32 && p->lanes_per_track != 16)
        return fail(ctx, REEDMD_EINVAL, "lanes_per_track must be 0, 16, 32 or 64");
    if (p->waves_per_cu < 0 || p->waves_per_cu > 32) return fail(ctx, REEDMD_EINVAL, "waves_per_cu must be in 0..32");
    if (p->queue_capacity < 0) return fail(ctx, REEDMD_EINVAL, "queue_capacity must be >= 0");
    if (p->track_log && p->track_log_cap < 0) return fail(ctx, REEDMD_EINVAL, "track_log_cap must be >= 0");
    if (p->no_tail_handoff != 0 && p->no_tail_handoff != 1) return fail(ctx, REEDMD_EINVAL, "no_tail_handoff must be 0 or 1");
    if (p->force_precision != REEDMD_FORCE_FP64 && p->force_precision != REEDMD_FORCE_FP32)
        return fail(ctx, REEDMD_EINVAL, "force_precision must be REEDMD_FORCE_FP64 or REEDMD_FORCE_FP32");
    return REEDMD_OK;
}

reedmd_status check_batch(reedmd_ctx* ctx, const reedmd_batch* b)
{
    if (!b) return fail(ctx, REEDMD_EINVAL, "batch is NULL");
    if (b->n < 0) return fail(ctx, REEDMD_EINVAL, "batch n must be >= 0");
    if (b->n > 0 && (!b->species || !b->energy || !b->pos || !b->dir || !b->key || !b->table))
        return fail(ctx, REEDMD_EINVAL, "batch arrays must be non-NULL");
    return REEDMD_OK;
}

void fill_common(const reedmd_ctx* ctx, const reedmd_species* sp, const reedmd_run_params* p, KernelArgs& A)
{
    std::memset(&A, 0, sizeof(A));
    prepare_species(ctx, sp, A);
    A.n_species = sp->n_species;
    A.a = ctx->lat.a;
    A.inv_a = 1.0 / ctx->lat.a;
    A.M2 = ctx->lat.M2;
    A.sigma = ctx->lat.sigma;
    A.inv_M2sq = 1.0 / (ctx->lat.M2 * ctx->lat.M2);
    A.half_inv_M2 = 1.0 / (2.0 * ctx->lat.M2);
    const bool fl = lattice_of(ctx) == kFluorite;
    A.M2b = fl ? ctx->lat.M2b : ctx->lat.M2;
    A.sigma_b = fl ? ctx->lat.sigma_b : ctx->lat.sigma;
    A.inv_M2bsq = 1.0 / (A.M2b * A.M2b);
    A.half_inv_M2b = 1.0 / (2.0 * A.M2b);
    A.structure = lattice_of(ctx);
    A.range_mode = p->range_mode;
    A.vacancy = p->vacancy;
    A.dx_max = p->dx_max;
    A.dt_max = p->dt_max;
    A.E_stop = p->E_stop;
    A.z_start = p->z_start;
    A.max_steps = p->max_steps > 0 ? p->max_steps : kDefaultMaxSteps;
    A.seed = p->seed;
    A.thr = p->thresholds;
    A.n_thresh = p->n_thresh;
    A.n_tables = p->n_tables;
    A.n_clones = p->n_clones < 2 ? 2 : p->n_clones;
    A.n_bins = p->n_bins;
    A.bin_width = p->bin_width;
    A.rc2 = p->r_cut > 0.0 ? p->r_cut * p->r_cut : 0.0;
}

void fill_batch(const reedmd_batch* b, KernelArgs& A)
{
    A.n = b->n;
    A.id0 = b->id0;
    A.species = b->species;
    A.energy = b->energy;
    A.pos = b->pos;
    A.dir = b->dir;
    A.key = reinterpret_cast<const unsigned long long*>(b->key);
    A.table = b->table;
}

// Kernel variants: lanes per track (64, 32, 16; fluorite 64, 32) x form x
// pair-term precision x target structure x pass variant (kVarCut: diamond with
// FP64 pair terms; kVarFirsov: FP64 pair terms).
template <int MODE, bool F32, int LAT, int VAR>
const void* track_ptr_l(int L)
{
    if (L == 64) return reinterpret_cast<const void*>(&track_kernel<64, MODE, F32, LAT, VAR>);
    if constexpr (LAT == kFluorite) {
        return reinterpret_cast<const void*>(&track_kernel<32, MODE, F32, LAT, VAR>);
    } else {
        if (L == 32) return reinterpret_cast<const void*>(&track_kernel<32, MODE, F32, LAT, VAR>);
        return reinterpret_cast<const void*>(&track_kernel<16, MODE, F32, LAT, VAR>);
    }
}

template <int MODE>
const void* track_ptr_m(int L, bool f32, int lat, int var)
{
    if (var == kVarCut) return track_ptr_l<MODE, false, kDiamond, kVarCut>(L);
    if (var == kVarFirsov)
        return lat == kFluorite ? track_ptr_l<MODE, false, kFluorite, kVarFirsov>(L)
                                : track_ptr_l<MODE, false, kDiamond, kVarFirsov>(L);
    if (lat == kFluorite)
        return f32 ? track_ptr_l<MODE, true, kFluorite, 0>(L) : track_ptr_l<MODE, false, kFluorite, 0>(L);
    return f32 ? track_ptr_l<MODE, true, kDiamond, 0>(L) : track_ptr_l<MODE, false, kDiamond, 0>(L);
}

// The track kernel of a launch shape (launches and graph nodes take the function itself).
const void* track_kernel_ptr(int L, int mode, bool f32, int lat, int var)
{
    return mode == kModePlain ? track_ptr_m<kModePlain>(L, f32, lat, var) : track_ptr_m<kModePersistent>(L, f32, lat, var);
}

int resident_blocks_per_cu(int L, int mode, bool f32, int lat, int var)
{
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, track_kernel_ptr(L, mode, f32, lat, var), kBlock, 0);
    return (e != hipSuccess || nb < 1) ? 1 : nb;
}

// The debug kernels (starting records, steps without events) of a variant.
template <bool INIT, bool F32, int LAT, int VAR>
const void* aux_ptr_l(int L)
{
    if (L == 64)
        return INIT ? reinterpret_cast<const void*>(&init_kernel<64, F32, LAT, VAR>)
                    : reinterpret_cast<const void*>(&step_kernel<64, F32, LAT, VAR>);
    if constexpr (LAT == kFluorite) {
        return INIT ? reinterpret_cast<const void*>(&init_kernel<32, F32, LAT, VAR>)
                    : reinterpret_cast<const void*>(&step_kernel<32, F32, LAT, VAR>);
    } else {
        if (L == 32)
            return INIT ? reinterpret_cast<const void*>(&init_kernel<32, F32, LAT, VAR>)
                        : reinterpret_cast<const void*>(&step_kernel<32, F32, LAT, VAR>);
        return INIT ? reinterpret_cast<const void*>(&init_kernel<16, F32, LAT, VAR>)
                    : reinterpret_cast<const void*>(&step_kernel<16, F32, LAT, VAR>);
    }
}

template <bool INIT>
const void* aux_ptr(int L, bool f32, int lat, int var)
{
    if (var == kVarCut) return aux_ptr_l<INIT, false, kDiamond, kVarCut>(L);
    if (var == kVarFirsov)
        return lat == kFluorite ? aux_ptr_l<INIT, false, kFluorite, kVarFirsov>(L)
                                : aux_ptr_l<INIT, false, kDiamond, kVarFirsov>(L);
    if (lat == kFluorite) return f32 ? aux_ptr_l<INIT, true, kFluorite, 0>(L) : aux_ptr_l<INIT, false, kFluorite, 0>(L);
    return f32 ? aux_ptr_l<INIT, true, kDiamond, 0>(L) : aux_ptr_l<INIT, false, kDiamond, 0>(L);
}

hipError_t launch_aux(bool init, int L, bool f32, int lat, int var, const KernelArgs& A, long long blocks, hipStream_t s)
{
    void* args[] = {const_cast<KernelArgs*>(&A)};
    const void* f = init ? aux_ptr<true>(L, f32, lat, var) : aux_ptr<false>(L, f32, lat, var);
    return hipLaunchKernel(f, dim3(static_cast<unsigned>(blocks)), dim3(kBlock), args, 0, s);
}

constexpr int kOrderBuckets = 512;
constexpr int kOrderBlocks = 256;   // grid of the order kernels (grid-stride over the batch)

// Queue state reset (a kernel, not a memset, so the pipeline can be kept as a graph).
__global__ void queue_reset_kernel(QueueState* q, unsigned long long* seq, int cap, long long n)
{
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i == 0) {
        q->head = 0;
        q->tail = 0;
        q->live = n;
        q->prim_next = 0;
        q->depth_max = 0;
        q->log_next = 0;
        q->handoff = 0;
        q->tail_left = 0;
    }
    if (i < cap) seq[i] = static_cast<unsigned long long>(i);
}

// Claim order of the primaries: longest expected tracks first, so that the
// long clone families of a batch start early instead of ending it.  The cost
// proxy is E0 / M1 (the ion's speed squared sets the number of steps of a
// track, dx_max per step, and with it the number of cloning depths it
// crosses); a counting sort into 16 buckets per octave of E0 / M1, largest
// first.  Every
// primary family is computed the same way wherever and whenever it runs, so
// the order changes no result.  The sort is stable, so primaries of one bucket
// keep the batch order.
struct OrderArgs {
    long long n;
    const int* species;
    const double* energy;
    double inv_M1[kMaxSpecies];
    int n_species;
    int pad;
    int* counts;    // [kOrderBuckets][kOrderBlocks]
    int* offsets;   // [kOrderBuckets][kOrderBlocks]
    int* order;     // [n]
};

__device__ __forceinline__ int order_bucket(const OrderArgs& O, long long q)
{
    const int sp = O.species[q];
    const double r = O.energy[q] * ((sp >= 0 && sp < O.n_species) ? O.inv_M1[sp] : 1.0);
    double b = (r > 0.0) ? floor(16.0 * log2(r)) + 128.0 : 0.0;
    b = fmin(fmax(b, 0.0), static_cast<double>(kOrderBuckets - 1));   // NaN goes to bucket 0
    return kOrderBuckets - 1 - static_cast<int>(b);
}

// The sort is stable (batch order inside a bucket): block g owns the contiguous
// chunk [g c, (g+1) c) of the batch, c = ceil(n / kOrderBlocks).
__device__ __forceinline__ void order_chunk(const OrderArgs& O, long long& lo, long long& hi)
{
    const long long c = (O.n + kOrderBlocks - 1) / kOrderBlocks;
    lo = static_cast<long long>(blockIdx.x) * c;
    hi = lo + c < O.n ? lo + c : O.n;
}

// Counts of every bucket in every chunk: counts[bucket * kOrderBlocks + block].
__global__ void __launch_bounds__(256) order_count_kernel(const OrderArgs O)
{
    __shared__ int c[kOrderBuckets];
    for (int i = threadIdx.x; i < kOrderBuckets; i += blockDim.x) c[i] = 0;
    __syncthreads();
    long long lo, hi;
    order_chunk(O, lo, hi);
    for (long long q = lo + threadIdx.x; q < hi; q += blockDim.x) atomicAdd(&c[order_bucket(O, q)], 1);
    __syncthreads();
    for (int i = threadIdx.x; i < kOrderBuckets; i += blockDim.x) O.counts[i * kOrderBlocks + blockIdx.x] = c[i];
}

// Exclusive prefix over (bucket, block) in that order: the start of every
// chunk's run of every bucket.  One thread per bucket sums its chunks, the
// bucket totals are scanned in LDS.
__global__ void __launch_bounds__(kOrderBuckets) order_scan_kernel(const OrderArgs O)
{
    __shared__ int tot[kOrderBuckets];
    const int b = threadIdx.x;
    int run = 0;
    for (int g = 0; g < kOrderBlocks; ++g) {
        const int c = O.counts[b * kOrderBlocks + g];
        O.offsets[b * kOrderBlocks + g] = run;
        run += c;
    }
    tot[b] = run;
    __syncthreads();
    if (b == 0) {
        int acc = 0;
        for (int i = 0; i < kOrderBuckets; ++i) {
            const int t = tot[i];
            tot[i] = acc;
            acc += t;
        }
    }
    __syncthreads();
    for (int g = 0; g < kOrderBlocks; ++g) O.offsets[b * kOrderBlocks + g] += tot[b];
}

// One thread per chunk places its primaries in batch order (the chunk's bucket
// offsets staged in LDS).
__global__ void __launch_bounds__(64) order_scatter_kernel(const OrderArgs O)
{
    __shared__ int off[kOrderBuckets];
    for (int i = threadIdx.x; i < kOrderBuckets; i += blockDim.x) off[i] = O.offsets[i * kOrderBlocks + blockIdx.x];
    __syncthreads();
    if (threadIdx.x != 0) return;
    long long lo, hi;
    order_chunk(O, lo, hi);
    for (long long q = lo; q < hi; ++q) O.order[off[order_bucket(O, q)]++] = static_cast<int>(q);
}

// Copies the number of logged results into the caller's stats at the end.
__global__ void stats_finalize_kernel(const QueueState* q, reedmd_stats* st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) st->log_count += q->log_next;
}

void drop_graphs(reedmd_ctx* ctx)
{
    for (auto& g : ctx->graphs) {
        (void)hipGraphExecDestroy(g.second.exec);
        (void)hipGraphDestroy(g.second.graph);
    }
    ctx->graphs.clear();
}

reedmd_status ensure_scratch(reedmd_ctx* ctx, int qcap, size_t stack_records)
{
    const size_t qbytes = 256 + static_cast<size_t>(qcap) * 8 + static_cast<size_t>(qcap) * record_words(ctx) * 8;
    const size_t need_q = ((qbytes + 4095) / 4096) * 4096;
    if (need_q > ctx->scratch_bytes) {
        HIP_TRY(ctx, hipDeviceSynchronize());
        if (ctx->scratch) (void)hipFree(ctx->scratch);
        ctx->scratch = nullptr;
        ctx->scratch_bytes = 0;
        drop_graphs(ctx);
        if (hipMalloc(&ctx->scratch, need_q) != hipSuccess) {
            ctx->scratch = nullptr;
            return fail(ctx, REEDMD_ENOMEM, "cannot allocate the clone queue");
        }
        ctx->scratch_bytes = need_q;
    }
    const size_t need_s = std::max<size_t>(stack_records, 1) * record_words(ctx) * 8;
    if (need_s > ctx->stack_bytes) {
        HIP_TRY(ctx, hipDeviceSynchronize());
        if (ctx->stack) (void)hipFree(ctx->stack);
        ctx->stack = nullptr;
        ctx->stack_bytes = 0;
        drop_graphs(ctx);
        if (hipMalloc(reinterpret_cast<void**>(&ctx->stack), need_s) != hipSuccess) {
            ctx->stack = nullptr;
            return fail(ctx, REEDMD_ENOMEM, "cannot allocate clone stacks");
        }
        ctx->stack_bytes = need_s;
    }
    return REEDMD_OK;
}

reedmd_status ensure_order(reedmd_ctx* ctx, long long n)
{
    const size_t need = (2 * static_cast<size_t>(kOrderBuckets) * kOrderBlocks + static_cast<size_t>(std::max<long long>(n, 1))) *
                        sizeof(int);
    if (need <= ctx->ordbuf_bytes) return REEDMD_OK;
    HIP_TRY(ctx, hipDeviceSynchronize());
    if (ctx->ordbuf) (void)hipFree(ctx->ordbuf);
    ctx->ordbuf = nullptr;
    ctx->ordbuf_bytes = 0;
    const size_t grow = std::max(need, need + need / 4);
    if (hipMalloc(reinterpret_cast<void**>(&ctx->ordbuf), grow) != hipSuccess) {
        ctx->ordbuf = nullptr;
        return fail(ctx, REEDMD_ENOMEM, "cannot allocate the claim order");
    }
    ctx->ordbuf_bytes = grow;
    return REEDMD_OK;
}

// Gate statistics of the interaction-set autotuner, from finished-track logs.
struct DepthSample {
    std::vector<std::pair<double, double>> zw;   // (stopping depth, weight) of stopped tracks, sorted
    double mean = 0.0, sd = 0.0, se_mean = 0.0, se_sd = 0.0, n_eff = 0.0;
};

// Weighted mean and standard deviation of the stopping depth, with standard errors
// that take each primary's family (the primary and its clones, which share the early
// path) as one independent unit: first-order expansion of the two ratio estimators.
DepthSample depth_sample(const std::vector<reedmd_result>& log)
{
    DepthSample d;
    std::map<int64_t, std::array<double, 3>> fam;
    double W = 0.0, S = 0.0, Q = 0.0, W2 = 0.0;
    for (const reedmd_result& r : log) {
        if (r.status != REEDMD_STOPPED) continue;
        d.zw.emplace_back(r.z_stop, r.w);
        auto& f = fam[r.lineage];
        f[0] += r.w;
        f[1] += r.w * r.z_stop;
        f[2] += r.w * r.z_stop * r.z_stop;
        W += r.w;
        S += r.w * r.z_stop;
        Q += r.w * r.z_stop * r.z_stop;
        W2 += r.w * r.w;
    }
    std::sort(d.zw.begin(), d.zw.end());
    if (!(W > 0.0)) return d;
    d.n_eff = W * W / W2;
    d.mean = S / W;
    const double e2 = Q / W;
    d.sd = std::sqrt(std::max(e2 - d.mean * d.mean, 0.0));
    double vm = 0.0, vs = 0.0;
    for (const auto& kv : fam) {
        const double a = kv.second[1] - d.mean * kv.second[0];
        const double b = (kv.second[2] - e2 * kv.second[0]) - 2.0 * d.mean * a;
        vm += a * a;
        vs += b * b;
    }
    d.se_mean = std::sqrt(vm) / W;
    d.se_sd = d.sd > 0.0 ? std::sqrt(vs) / (2.0 * d.sd * W) : 0.0;
    return d;
}

// Survival function of the Kolmogorov distribution, P(K > x): the alternating series
// 2 sum_k (-1)^(k-1) exp(-2 k^2 x^2) for x >= 1, the complement of the theta-function
// series sqrt(2 pi) / x sum_k exp(-(2k-1)^2 pi^2 / (8 x^2)) below (both converge fast there).
double kolmogorov_sf(double x)
{
    if (x <= 0.0) return 1.0;
    if (x >= 1.0) {
        double s = 0.0;
        for (int k = 1; k <= 100; ++k) {
            const double t = std::exp(-2.0 * k * k * x * x);
            s += (k & 1) ? t : -t;
            if (t < 1e-18) break;
        }
        return std::min(1.0, std::max(0.0, 2.0 * s));
    }
    const double pi = 3.14159265358979323846;
    double c = 0.0;
    for (int k = 1; k <= 100; ++k) {
        const double m = 2.0 * k - 1.0;
        const double t = std::exp(-m * m * pi * pi / (8.0 * x * x));
        c += t;
        if (t < 1e-18) break;
    }
    return std::min(1.0, std::max(0.0, 1.0 - std::sqrt(2.0 * pi) / x * c));
}

// Two-sample Kolmogorov-Smirnov test of weighted samples: the largest distance of
// the two weighted empirical distribution functions, and its p value at the
// effective sample sizes (sum w)^2 / sum w^2.
double weighted_ks_p(const DepthSample& a, const DepthSample& b, double* D_out)
{
    if (a.zw.empty() || b.zw.empty()) {
        if (D_out) *D_out = 1.0;
        return 0.0;
    }
    double Wa = 0.0, Wb = 0.0;
    for (const auto& e : a.zw) Wa += e.second;
    for (const auto& e : b.zw) Wb += e.second;
    size_t i = 0, j = 0;
    double Fa = 0.0, Fb = 0.0, D = 0.0;
    while (i < a.zw.size() || j < b.zw.size()) {
        const double z = (j >= b.zw.size() || (i < a.zw.size() && a.zw[i].first <= b.zw[j].first)) ? a.zw[i].first
                                                                                                   : b.zw[j].first;
        while (i < a.zw.size() && a.zw[i].first == z) Fa += a.zw[i++].second;
        while (j < b.zw.size() && b.zw[j].first == z) Fb += b.zw[j++].second;
        D = std::max(D, std::fabs(Fa / Wa - Fb / Wb));
    }
    if (D_out) *D_out = D;
    const double ne = a.n_eff * b.n_eff / (a.n_eff + b.n_eff);
    return kolmogorov_sf(D * std::sqrt(ne));
}

unsigned long long hash_mix(unsigned long long h, unsigned long long v)
{
    h ^= v + 0x9E3779B97F4A7C15ULL + (h << 6) + (h >> 2);
    return h;
}

unsigned long long tune_key(const reedmd_run_params* p, const reedmd_batch* b)
{
    unsigned long long h = 1469598103934665603ULL;
    h = hash_mix(h, static_cast<unsigned long long>(p->form));
    h = hash_mix(h, static_cast<unsigned long long>(p->n_thresh));
    h = hash_mix(h, static_cast<unsigned long long>(p->force_precision));
    h = hash_mix(h, static_cast<unsigned long long>(b->n > 0 ? 63 - __builtin_clzll(static_cast<unsigned long long>(b->n)) : 0));
    return h;
}

// Launch shape for a run.
struct Shape {
    int L;
    int mode;
    bool f32;
    long long seg_total;
    long long blocks;
    int stack_cap;
    int qcap;
    // tail handoff to a 64-lane launch (persistent form with fewer lanes): its workgroups
    // and segments; 0 when off
    long long tail_blocks;
    long long tail_segs;
    double r_cut;   // interaction set after the autotune cache: 0 = the 27 cells
    int var;        // pass variant of the track kernel (kVarCut, kVarFirsov)
};

Shape choose_shape(reedmd_ctx* ctx, const reedmd_run_params* p, const reedmd_batch* b)
{
    Shape s{};
    s.mode = p->form == REEDMD_FORM_PERSISTENT ? kModePersistent : kModePlain;
    s.f32 = p->force_precision == REEDMD_FORCE_FP32;
    int L = p->lanes_per_track;
    int waves = p->waves_per_cu;
    if (L == 0 || (s.mode == kModePersistent && waves == 0)) {
        auto it = ctx->tune.find(tune_key(p, b));
        if (it != ctx->tune.end()) {
            if (L == 0) L = it->second.lanes;
            if (waves == 0) waves = it->second.waves;
        }
    }
    if (L == 0) L = 64;
    if (lattice_of(ctx) == kFluorite && L == 16) L = 32;
    s.L = L;
    s.r_cut = p->r_cut > 0.0 ? p->r_cut : 0.0;
    if (p->r_cut < 0.0) {
        auto it = ctx->tune.find(tune_key(p, b));
        if (it != ctx->tune.end()) s.r_cut = it->second.r_cut;
    }
    s.var = pass_variant(ctx, s.r_cut);
    const int T = 64 / L;
    const int per_wave_block = kBlock / 64;
    s.stack_cap = p->n_thresh > 0 ? p->n_thresh * (std::max(p->n_clones, 2) - 1) + 1 : 0;
    if (s.mode == kModePlain) {
        const long long max_segs = 1ll << 16;
        s.seg_total = std::max<long long>(1, std::min<long long>(b->n, max_segs * T));
        const long long waves_needed = (s.seg_total + T - 1) / T;
        s.blocks = (waves_needed + per_wave_block - 1) / per_wave_block;
        s.qcap = 0;
    } else {
        int bpc = resident_blocks_per_cu(L, s.mode, s.f32, lattice_of(ctx), s.var);
        if (waves > 0) bpc = std::max(1, std::min(bpc, (waves + per_wave_block - 1) / per_wave_block));
        s.blocks = static_cast<long long>(bpc) * ctx->cu_count;
        s.seg_total = s.blocks * per_wave_block * T;
        // default: room for every clone a burst of long families can have pending (a full
        // queue sends clones to the creating segment's stack, where they run one after another)
        s.qcap = p->queue_capacity > 0 ? p->queue_capacity
                                       : static_cast<int>(std::min<long long>(kMaxQueue, std::max<long long>(4096, 4 * b->n)));
        if (L < 64 && p->no_tail_handoff == 0) {
            s.tail_blocks = static_cast<long long>(resident_blocks_per_cu(64, s.mode, s.f32, lattice_of(ctx), s.var)) * ctx->cu_count;
            s.tail_segs = s.tail_blocks * per_wave_block;
        }
        if (p->n_thresh == 0 && s.tail_blocks == 0) s.qcap = 1;
    }
    return s;
}

// Depth refinement inside one persistent launch: E epochs of claim positions,
// targets and spacing, the per-epoch statistics snapshots and publish flags.
struct RefineLaunch {
    int E;
    const double* probs;
    double min_gap, min_weight;
    double* snap;
    int* ready;
};

reedmd_status run_impl(reedmd_ctx* ctx, const reedmd_species* sp, const reedmd_batch* b,
                       const reedmd_run_params* p, double* d_hist, reedmd_stats* d_stats, hipStream_t stream,
                       const Shape* forced, double* d_tstat = nullptr, hipEvent_t ev_start = nullptr,
                       const RefineLaunch* rl = nullptr)
{
    Shape s = forced ? *forced : choose_shape(ctx, p, b);
    const int qcap = s.qcap > 0 ? s.qcap : 1;
    const size_t stack_records = static_cast<size_t>(std::max(s.seg_total, s.tail_segs)) * static_cast<size_t>(std::max(s.stack_cap, 0));
    reedmd_status st = ensure_scratch(ctx, qcap, stack_records);
    if (st != REEDMD_OK) return st;

    KernelArgs A;
    fill_common(ctx, sp, p, A);
    fill_batch(b, A);
    A.rc2 = s.r_cut * s.r_cut;
    A.hist = d_hist;
    A.stats = d_stats;
    A.tstat = d_tstat;
    A.log = static_cast<reedmd_result*>(p->track_log);
    A.log_cap = p->track_log ? p->track_log_cap : 0;
    A.stack = ctx->stack;
    A.stack_cap = s.stack_cap;
    A.q = static_cast<QueueState*>(ctx->scratch);
    A.qseq = reinterpret_cast<unsigned long long*>(static_cast<char*>(ctx->scratch) + 256);
    A.qrec = reinterpret_cast<double*>(static_cast<char*>(ctx->scratch) + 256 + static_cast<size_t>(qcap) * 8);
    A.qcap = (s.mode == kModePersistent && (p->n_thresh > 0 || s.tail_blocks > 0)) ? qcap : 0;
    A.handoff_live = s.tail_segs;
    A.cancel = p->cancel;
    A.seg_total = s.seg_total;
    if (rl != nullptr) {
        A.refine_E = rl->E;
        A.r_probs = rl->probs;
        A.r_min_gap = rl->min_gap;
        A.r_min_weight = rl->min_weight;
        A.r_snap = rl->snap;
        A.r_ready = rl->ready;
    }

    if (b->n == 0) return REEDMD_OK;
    st = ensure_order(ctx, b->n);
    if (st != REEDMD_OK) return st;

    // The pipeline of a run: queue and counter reset, claim order (count, scan,
    // scatter), the track kernel, statistics.  Each call fills one argument set;
    // the persistent form keeps the pipeline as an instantiated graph per launch
    // shape and writes this call's arguments into its nodes, the other forms (and
    // calls made inside a caller's stream capture) launch the kernels directly.
    OrderArgs O{};
    O.n = b->n;
    O.species = b->species;
    O.energy = b->energy;
    for (int i = 0; i < kMaxSpecies; ++i) O.inv_M1[i] = 1.0 / A.sp[i].M1;
    O.n_species = sp->n_species;
    O.counts = ctx->ordbuf;
    O.offsets = ctx->ordbuf + kOrderBuckets * kOrderBlocks;
    O.order = ctx->ordbuf + 2 * kOrderBuckets * kOrderBlocks;
    A.order = O.order;
    QueueState* q = A.q;
    unsigned long long* seq = A.qseq;
    int cap = qcap;
    long long nq = b->n;
    reedmd_stats* st_out = d_stats;
    KernelArgs T = A;   // the 64-lane tail launch: queue only, no handoff of its own
    T.seg_total = s.tail_segs;
    T.handoff_live = 0;
    T.tail = 1;
    void* reset_args[] = {&q, &seq, &cap, &nq};
    void* order_args[] = {&O};
    void* track_args[] = {&A};
    void* tail_args[] = {&T};
    void* fin_args[] = {&q, &st_out};
    const bool tail = s.tail_blocks > 0;
    const int kNodes = tail ? 7 : 6;
    hipKernelNodeParams np[7] = {};
    const void* funcs[7] = {reinterpret_cast<const void*>(queue_reset_kernel),
                            reinterpret_cast<const void*>(order_count_kernel),
                            reinterpret_cast<const void*>(order_scan_kernel),
                            reinterpret_cast<const void*>(order_scatter_kernel),
                            track_kernel_ptr(s.L, s.mode, s.f32, lattice_of(ctx), s.var),
                            track_kernel_ptr(64, s.mode, s.f32, lattice_of(ctx), s.var),
                            reinterpret_cast<const void*>(stats_finalize_kernel)};
    dim3 grids[7] = {dim3((qcap + 255) / 256), dim3(kOrderBlocks), dim3(1), dim3(kOrderBlocks),
                     dim3(static_cast<unsigned>(s.blocks)), dim3(static_cast<unsigned>(std::max(s.tail_blocks, 1ll))), dim3(1)};
    dim3 blocks[7] = {dim3(256), dim3(256), dim3(kOrderBuckets), dim3(64), dim3(kBlock), dim3(kBlock), dim3(64)};
    void** args[7] = {reset_args, order_args, order_args, order_args, track_args, tail_args, fin_args};
    if (!tail) {   // no tail launch: the statistics node follows the track kernel
        funcs[5] = funcs[6];
        grids[5] = grids[6];
        blocks[5] = blocks[6];
        args[5] = args[6];
    }
    for (int k = 0; k < kNodes; ++k) {
        np[k].func = const_cast<void*>(funcs[k]);
        np[k].gridDim = grids[k];
        np[k].blockDim = blocks[k];
        np[k].kernelParams = args[k];
    }

    bool as_graph = s.mode == kModePersistent && !forced;
    if (as_graph) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        HIP_TRY(ctx, hipStreamIsCapturing(stream, &cs));
        as_graph = cs == hipStreamCaptureStatusNone;
    }
    if (!as_graph) {
        if (ev_start) HIP_TRY(ctx, hipEventRecord(ev_start, stream));
        for (int k = 0; k < kNodes; ++k)
            HIP_TRY(ctx, hipLaunchKernel(np[k].func, np[k].gridDim, np[k].blockDim, np[k].kernelParams, 0, stream));
        return REEDMD_OK;
    }
    const std::vector<long long> key = {s.L, s.f32 ? 1 : 0, lattice_of(ctx), s.blocks, qcap, s.tail_blocks, s.var};
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        if (ctx->graphs.size() >= kMaxGraphs) drop_graphs(ctx);
        reedmd_ctx::Graph g;
        hipError_t e = hipGraphCreate(&g.graph, 0);
        for (int k = 0; k < kNodes && e == hipSuccess; ++k) {
            hipGraphNode_t* prev = k > 0 ? &g.node[k - 1] : nullptr;
            e = hipGraphAddKernelNode(&g.node[k], g.graph, prev, k > 0 ? 1 : 0, &np[k]);
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
            if (g.graph) (void)hipGraphDestroy(g.graph);
            return hip_fail(ctx, e, "building the persistent pipeline graph");
        }
        it = ctx->graphs.emplace(key, g).first;
    } else {
        for (int k = 0; k < kNodes; ++k)
            HIP_TRY(ctx, hipGraphExecKernelNodeSetParams(it->second.exec, it->second.node[k], &np[k]));
    }
    if (ev_start) HIP_TRY(ctx, hipEventRecord(ev_start, stream));
    HIP_TRY(ctx, hipGraphLaunch(it->second.exec, stream));
    return REEDMD_OK;
}

// ---------------------------------------------------------------------------
// Adaptive cloning depths between launches (Sec. 2: depths placed from the
// statistics gathered so far; Sec. 3: criteria updated between complete
// tracks): every table re-placed from its statistics by refine_table, starting
// from its current depths; a row holds each booked track's weight in one entry (its
// depth bin, beyond the last bin, or not stopped in the crystal), so its sum is
// all weight booked.  One thread per table.
__global__ void refine_kernel(const double* tstat, int n_bins, double bin_width, int n_tables, int n_thresh,
                              const double* probs, double min_gap, double min_weight, double* thr)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tables) return;
    const double* h = tstat + static_cast<size_t>(t) * (n_bins + 2);
    double total = 0.0;
    for (int i = 0; i < n_bins + 2; ++i) total += h[i];
    refine_table(h, total, n_bins, bin_width, n_thresh, probs, min_gap, min_weight,
                 thr + static_cast<size_t>(t) * n_thresh);
}

// ---------------------------------------------------------------------------
// Primary sampler: mirrors the batch contract of reedmd_sample_primaries.
struct SamplerArgs {
    reedmd_sampler s;
    unsigned long long seed;
    long long id0, n;
    int* species;
    double* energy;
    double* pos;
    double* dir;
    unsigned long long* key;
    int* table;
};

__global__ void sample_kernel(const SamplerArgs S)
{
    const long long q = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= S.n) return;
    const long long id = S.id0 + q;
    const U64x4 r0 = philox4x64_10(kTagSample, static_cast<uint64_t>(id), 0, 0, S.seed, 0);
    const U64x4 r1 = philox4x64_10(kTagSample, static_cast<uint64_t>(id), 1, 0, S.seed, 0);
    double u[8];
    for (int i = 0; i < 4; ++i) {
        u[i] = open_unit(r0.w[i]);
        u[4 + i] = open_unit(r1.w[i]);
    }
    const reedmd_sampler& s = S.s;
    const bool site = s.start_mode == REEDMD_START_SITE;
    S.pos[q] = site ? 0.0 : s.a * u[0];
    S.pos[S.n + q] = site ? 0.0 : s.a * u[1];
    S.pos[2 * S.n + q] = s.z_start;
    int ci = static_cast<int>(floor(static_cast<double>(s.n_choice) * u[2]));
    if (ci > s.n_choice - 1) ci = s.n_choice - 1;
    S.species[q] = s.choice[ci];
    S.energy[q] = (s.E_min == s.E_max) ? s.E_min : s.E_min * exp(u[3] * log(s.E_max / s.E_min));
    const int net = s.n_energy_tables > 1 ? s.n_energy_tables : 1;
    int band = 0;
    if (net > 1) {
        band = static_cast<int>(floor(static_cast<double>(net) * u[3]));
        if (band > net - 1) band = net - 1;
    }
    S.table[q] = ci * net + band;
    const bool cone = s.dir_mode == REEDMD_DIR_CONE || (s.dir_mode == REEDMD_DIR_MIXED && id < s.n_cone);
    constexpr double kTwoPi = 6.283185307179586476925286766559;
    const double phi = kTwoPi * u[4];
    double sp, cp;
    sincos(phi, &sp, &cp);
    if (s.dir_mode == REEDMD_DIR_ISOTROPIC) {
        // uniform on the sphere: cos(theta) uniform in [-1, 1]
        const double ct = 1.0 - 2.0 * u[5];
        const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
        S.dir[q] = st * cp;
        S.dir[S.n + q] = st * sp;
        S.dir[2 * S.n + q] = ct;
    } else if (!cone) {
        double st, ct;
        sincos(s.tilt, &st, &ct);
        S.dir[q] = st * cp;
        S.dir[S.n + q] = st * sp;
        S.dir[2 * S.n + q] = ct;
    } else {
        const double ct = 1.0 - u[5] * (1.0 - cos(s.half_angle));
        const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
        const double* A = s.axis;
        double hx = 1.0, hy = 0.0;
        if (fabs(A[0]) >= 0.9) { hx = 0.0; hy = 1.0; }
        // e1 = normalise(A x h) with h = (hx, hy, 0); e2 = A x e1
        double e1x = -A[2] * hy, e1y = A[2] * hx, e1z = A[0] * hy - A[1] * hx;
        const double n1 = sqrt(e1x * e1x + e1y * e1y + e1z * e1z);
        e1x /= n1; e1y /= n1; e1z /= n1;
        const double e2x = A[1] * e1z - A[2] * e1y, e2y = A[2] * e1x - A[0] * e1z, e2z = A[0] * e1y - A[1] * e1x;
        S.dir[q] = st * (cp * e1x + sp * e2x) + ct * A[0];
        S.dir[S.n + q] = st * (cp * e1y + sp * e2y) + ct * A[1];
        S.dir[2 * S.n + q] = st * (cp * e1z + sp * e2z) + ct * A[2];
    }
    S.key[q] = primary_key(S.seed, id);
}

__global__ void exp_neg_kernel(const double* y, double* out, long long n, int pair)
{
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = pair ? exp_neg_pair(y[i]) : exp_neg(y[i]);
}

__global__ void log_kernel(const double* x, double* out, long long n, int one_plus)
{
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) out[i] = one_plus ? log1p_pos(x[i]) : log_pos(x[i]);
}

}  // namespace

// ===========================================================================
extern "C" {

int32_t reedmd_version(void) { return 100; }

reedmd_status reedmd_create(const reedmd_lattice* lattice, const reedmd_potential* potential,
                            const reedmd_stopping* stopping, reedmd_ctx** out)
{
    if (!out) return fail(nullptr, REEDMD_EINVAL, "out is NULL");
    *out = nullptr;
    if (!lattice || !potential || !stopping) return fail(nullptr, REEDMD_EINVAL, "NULL model description");
    if (!(lattice->a > 0.0) || !(lattice->M2 > 0.0) || !(lattice->sigma >= 0.0) || lattice->Z2 <= 0)
        return fail(nullptr, REEDMD_EINVAL, "lattice a, M2, Z2 must be positive and sigma >= 0");
    if (lattice->structure != REEDMD_DIAMOND && lattice->structure != REEDMD_FLUORITE)
        return fail(nullptr, REEDMD_EUNSUPPORTED, "structure must be REEDMD_DIAMOND or REEDMD_FLUORITE");
    if (lattice->structure == REEDMD_FLUORITE &&
        (!(lattice->M2b > 0.0) || !(lattice->sigma_b >= 0.0) || lattice->Z2b <= 0))
        return fail(nullptr, REEDMD_EINVAL, "fluorite needs M2b, Z2b > 0 and sigma_b >= 0");
    if (potential->mode != REEDMD_POT_ZBL && potential->mode != REEDMD_POT_NONE)
        return fail(nullptr, REEDMD_EINVAL, "unknown potential mode");
    if (!(potential->s >= kMinScreening && potential->s <= kMaxScreening))
        return fail(nullptr, REEDMD_EINVAL, "screening scale s must be in [0.01, 100]");
    if (stopping->mode < REEDMD_STOP_OFF || stopping->mode > REEDMD_STOP_FKBK || !(stopping->k >= 0.0))
        return fail(nullptr, REEDMD_EINVAL, "unknown stopping mode or negative k");
    if (!(stopping->n_e >= 0.0) || !std::isfinite(stopping->n_e))
        return fail(nullptr, REEDMD_EINVAL, "the electron density n_e must be finite and >= 0");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(nullptr, REEDMD_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return fail(nullptr, REEDMD_EHIP, std::string("device attribute: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, REEDMD_EUNSUPPORTED, "device index beyond the supported range");
    if (g_noalloc_ptr[dev] == nullptr) {
        // once per device, with that device current: the device address of the
        // allocation-free entry point's scratch array
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr)
            return fail(nullptr, REEDMD_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_noalloc_ptr[dev] = ptr;
    }
    reedmd_ctx* ctx = new reedmd_ctx();
    ctx->device = dev;
    ctx->cu_count = cus;
    ctx->lat = *lattice;
    ctx->pot = *potential;
    ctx->stop = *stopping;
    *out = ctx;
    return REEDMD_OK;
}

int32_t reedmd_cached_graphs(const reedmd_ctx* ctx)
{
    return ctx ? static_cast<int32_t>(ctx->graphs.size()) : 0;
}

void reedmd_destroy(reedmd_ctx* ctx)
{
    if (!ctx) return;
    (void)hipDeviceSynchronize();
    drop_graphs(ctx);
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->stack) (void)hipFree(ctx->stack);
    if (ctx->gscratch) (void)hipFree(ctx->gscratch);
    if (ctx->ordbuf) (void)hipFree(ctx->ordbuf);
    delete ctx;
}

const char* reedmd_last_error(const reedmd_ctx* ctx)
{
    if (!ctx) return g_create_error.c_str();
    return ctx->err.c_str();
}

reedmd_status reedmd_sample_primaries(reedmd_ctx* ctx, const reedmd_sampler* sampler, uint64_t seed,
                                      const reedmd_batch* out, hipStream_t stream)
{
    if (!ctx) return fail(nullptr, REEDMD_EINVAL, "ctx is NULL");
    if (!sampler) return fail(ctx, REEDMD_EINVAL, "sampler is NULL");
    reedmd_status st = check_batch(ctx, out);
    if (st != REEDMD_OK) return st;
    if (sampler->n_choice < 1 || sampler->n_choice > REEDMD_MAX_SPECIES)
        return fail(ctx, REEDMD_EINVAL, "n_choice must be in 1..8");
    if (sampler->n_energy_tables < 1) return fail(ctx, REEDMD_EINVAL, "n_energy_tables must be >= 1");
    if (!(sampler->E_min > 0.0) || !(sampler->E_max >= sampler->E_min))
        return fail(ctx, REEDMD_EINVAL, "need 0 < E_min <= E_max");
    if (sampler->dir_mode < REEDMD_DIR_TILT || sampler->dir_mode > REEDMD_DIR_ISOTROPIC)
        return fail(ctx, REEDMD_EINVAL, "unknown direction mode");
    if (sampler->start_mode != REEDMD_START_SURFACE && sampler->start_mode != REEDMD_START_SITE)
        return fail(ctx, REEDMD_EINVAL, "unknown start mode");
    if (sampler->dir_mode == REEDMD_DIR_CONE || sampler->dir_mode == REEDMD_DIR_MIXED) {
        const double n2 = sampler->axis[0] * sampler->axis[0] + sampler->axis[1] * sampler->axis[1] +
                          sampler->axis[2] * sampler->axis[2];
        if (std::fabs(n2 - 1.0) > 1e-12) return fail(ctx, REEDMD_EINVAL, "cone axis must be a unit vector");
    }
    if (out->n == 0) return REEDMD_OK;
    SamplerArgs S;
    std::memset(&S, 0, sizeof(S));
    S.s = *sampler;
    S.seed = seed;
    S.id0 = out->id0;
    S.n = out->n;
    S.species = out->species;
    S.energy = out->energy;
    S.pos = out->pos;
    S.dir = out->dir;
    S.key = reinterpret_cast<unsigned long long*>(out->key);
    S.table = out->table;
    const long long blocks = (out->n + 255) / 256;
    hipLaunchKernelGGL(sample_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, S);
    HIP_TRY(ctx, hipGetLastError());
    return REEDMD_OK;
}

reedmd_status reedmd_run(reedmd_ctx* ctx, const reedmd_species* species, const reedmd_batch* batch,
                         const reedmd_run_params* params, double* d_hist, reedmd_stats* d_stats,
                         hipStream_t stream)
{
    if (!ctx) return fail(nullptr, REEDMD_EINVAL, "ctx is NULL");
    reedmd_status st;
    if ((st = check_species(ctx, species)) != REEDMD_OK) return st;
    if ((st = check_batch(ctx, batch)) != REEDMD_OK) return st;
    if ((st = check_params(ctx, params, true)) != REEDMD_OK) return st;
    if (!d_hist || !d_stats) return fail(ctx, REEDMD_EINVAL, "d_hist and d_stats must be non-NULL");
    return run_impl(ctx, species, batch, params, d_hist, d_stats, stream, nullptr);
}

reedmd_status reedmd_run_noalloc(reedmd_ctx* ctx, const reedmd_species* species, const reedmd_batch* batch,
                                 const reedmd_run_params* params, double* d_hist, reedmd_stats* d_stats,
                                 hipStream_t stream)
{
    if (!ctx) return fail(nullptr, REEDMD_EINVAL, "ctx is NULL");
    reedmd_status st;
    if ((st = check_species(ctx, species)) != REEDMD_OK) return st;
    if ((st = check_batch(ctx, batch)) != REEDMD_OK) return st;
    if ((st = check_params(ctx, params, true)) != REEDMD_OK) return st;
    if (!d_hist || !d_stats) return fail(ctx, REEDMD_EINVAL, "d_hist and d_stats must be non-NULL");
    if (params->form != REEDMD_FORM_PLAIN)
        return fail(ctx, REEDMD_EUNSUPPORTED, "the allocation-free run is the plain form (form = REEDMD_FORM_PLAIN)");
    if (batch->n == 0) return REEDMD_OK;
    char* base = static_cast<char*>(g_noalloc_ptr[ctx->device]);
    if (base == nullptr) return fail(ctx, REEDMD_EHIP, "the scratch array has no device address");
    // layout of the scratch array: queue state and its one sequence word, the claim
    // order's counters and offsets, the claim order, then the clone stacks
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t off_seq = 256;
    const size_t off_counts = 512;
    const size_t off_offsets = off_counts + sizeof(int) * kOrderBuckets * kOrderBlocks;
    const size_t off_order = off_offsets + sizeof(int) * kOrderBuckets * kOrderBlocks;
    const size_t off_stack = up(off_order + sizeof(int) * static_cast<size_t>(batch->n));
    if (off_stack > kNoAllocBytes)
        return fail(ctx, REEDMD_EINVAL, "batch too large for the allocation-free run: its claim order needs more than the "
                                        "128 MiB scratch array (at most about 33 million primaries)");
    Shape s = choose_shape(ctx, params, batch);
    const size_t per_seg = static_cast<size_t>(std::max(s.stack_cap, 0)) * record_words(ctx) * sizeof(double);
    const long long fit = per_seg > 0 ? static_cast<long long>((kNoAllocBytes - off_stack) / per_seg) : s.seg_total;
    if (fit < 1)
        return fail(ctx, REEDMD_EINVAL, "one segment's clone stack (n_thresh * (n_clones - 1) + 1 records) does not fit "
                                        "the 128 MiB scratch array of the allocation-free run");
    s.seg_total = std::min(s.seg_total, fit);   // fewer segments, same results (plain static assignment)
    const int T = 64 / s.L;
    s.blocks = (s.seg_total + static_cast<long long>(T) * (kBlock / 64) - 1) / (static_cast<long long>(T) * (kBlock / 64));

    KernelArgs A;
    fill_common(ctx, species, params, A);
    fill_batch(batch, A);
    A.rc2 = s.r_cut * s.r_cut;
    A.hist = d_hist;
    A.stats = d_stats;
    A.log = static_cast<reedmd_result*>(params->track_log);
    A.log_cap = params->track_log ? params->track_log_cap : 0;
    A.q = reinterpret_cast<QueueState*>(base);
    A.qseq = reinterpret_cast<unsigned long long*>(base + off_seq);
    A.qrec = nullptr;
    A.qcap = 0;
    A.stack = reinterpret_cast<double*>(base + off_stack);
    A.stack_cap = s.stack_cap;
    A.cancel = params->cancel;
    A.seg_total = s.seg_total;
    OrderArgs O{};
    O.n = batch->n;
    O.species = batch->species;
    O.energy = batch->energy;
    for (int i = 0; i < kMaxSpecies; ++i) O.inv_M1[i] = 1.0 / A.sp[i].M1;
    O.n_species = species->n_species;
    O.counts = reinterpret_cast<int*>(base + off_counts);
    O.offsets = reinterpret_cast<int*>(base + off_offsets);
    O.order = reinterpret_cast<int*>(base + off_order);
    A.order = O.order;
    // the same kernels as reedmd_run's plain form, launched directly (the queue reset
    // kernel clears the state that must start at zero: no memset)
    hipLaunchKernelGGL(queue_reset_kernel, dim3(1), dim3(256), 0, stream, A.q, A.qseq, 1, batch->n);
    HIP_TRY(ctx, hipGetLastError());
    hipLaunchKernelGGL(order_count_kernel, dim3(kOrderBlocks), dim3(256), 0, stream, O);
    hipLaunchKernelGGL(order_scan_kernel, dim3(1), dim3(kOrderBuckets), 0, stream, O);
    hipLaunchKernelGGL(order_scatter_kernel, dim3(kOrderBlocks), dim3(64), 0, stream, O);
    HIP_TRY(ctx, hipGetLastError());
    void* track_args[] = {&A};
    HIP_TRY(ctx, hipLaunchKernel(track_kernel_ptr(s.L, s.mode, s.f32, lattice_of(ctx), s.var), dim3(static_cast<unsigned>(s.blocks)),
                                 dim3(kBlock), track_args, 0, stream));
    hipLaunchKernelGGL(stats_finalize_kernel, dim3(1), dim3(64), 0, stream, A.q, d_stats);
    HIP_TRY(ctx, hipGetLastError());
    return REEDMD_OK;
}

reedmd_status reedmd_track_init(reedmd_ctx* ctx, const reedmd_species* species, const reedmd_batch* batch,
                                const reedmd_run_params* params, double* d_records, hipStream_t stream)
{
    if (!ctx) return fail(nullptr, REEDMD_EINVAL, "ctx is NULL");
    reedmd_status st;
    if ((st = check_species(ctx, species)) != REEDMD_OK) return st;
    if ((st = check_batch(ctx, batch)) != REEDMD_OK) return st;
    if ((st = check_params(ctx, params, false, false)) != REEDMD_OK) return st;
    if (!d_records && batch->n > 0) return fail(ctx, REEDMD_EINVAL, "d_records is NULL");
    if (batch->n == 0) return REEDMD_OK;
    KernelArgs A;
    fill_common(ctx, species, params, A);
    fill_batch(batch, A);
    A.records = d_records;
    const int L = params->lanes_per_track ? params->lanes_per_track : 64;
    const long long waves = (batch->n + (64 / L) - 1) / (64 / L);
    const long long blocks = (waves + 3) / 4;
    HIP_TRY(ctx, launch_aux(true, L, params->force_precision == REEDMD_FORCE_FP32, lattice_of(ctx),
                            pass_variant(ctx, params->r_cut), A, blocks, stream));
    HIP_TRY(ctx, hipGetLastError());
    return REEDMD_OK;
}

reedmd_status reedmd_debug_step(reedmd_ctx* ctx, const reedmd_species* species, const reedmd_run_params* params,
                                double* d_records, int64_t n, int32_t nsteps, hipStream_t stream)
{
    if (!ctx) return fail(nullptr, REEDMD_EINVAL, "ctx is NULL");
    reedmd_status st;
    if ((st = check_species(ctx, species)) != REEDMD_OK) return st;
    if ((st = check_params(ctx, params, false, false)) != REEDMD_OK) return st;
    if (n < 0 || nsteps < 0) return fail(ctx, REEDMD_EINVAL, "n and nsteps must be >= 0");
    if (!d_records && n > 0) return fail(ctx, REEDMD_EINVAL, "d_records is NULL");
    if (n == 0) return REEDMD_OK;
    KernelArgs A;
    fill_common(ctx, species, params, A);
    A.n = n;
    A.records = d_records;
    A.nsteps = nsteps;
    const int L = params->lanes_per_track ? params->lanes_per_track : 64;
    const long long waves = (n + (64 / L) - 1) / (64 / L);
    const long long blocks = (waves + 3) / 4;
    HIP_TRY(ctx, launch_aux(false, L, params->force_precision == REEDMD_FORCE_FP32, lattice_of(ctx),
                            pass_variant(ctx, params->r_cut), A, blocks, stream));
    HIP_TRY(ctx, hipGetLastError());
    return REEDMD_OK;
}

reedmd_status reedmd_grad(reedmd_ctx* ctx, const reedmd_species* species, const reedmd_batch* batch,
                          const reedmd_run_params* params, double k, double s, double* d_track_out,
                          double* h_result, hipStream_t stream)
{
    if (!ctx) return fail(nullptr, REEDMD_EINVAL, "ctx is NULL");
    reedmd_status st;
    if ((st = check_species(ctx, species)) != REEDMD_OK) return st;
    if ((st = check_batch(ctx, batch)) != REEDMD_OK) return st;
    if ((st = check_params(ctx, params, false)) != REEDMD_OK) return st;
    if (!h_result) return fail(ctx, REEDMD_EINVAL, "h_result is NULL");
    if (params->n_thresh != 0) return fail(ctx, REEDMD_EUNSUPPORTED, "the gradient is defined without cloning (n_thresh = 0)");
    if (params->r_cut != 0.0) return fail(ctx, REEDMD_EUNSUPPORTED, "the adjoint covers the 27-cell interaction set (r_cut = 0)");
    if (ctx->stop.mode == REEDMD_STOP_FKBK)
        return fail(ctx, REEDMD_EUNSUPPORTED, "the adjoint covers the OFF, UNIFORM and LOCAL stopping models");
    if (params->force_precision != REEDMD_FORCE_FP64)
        return fail(ctx, REEDMD_EUNSUPPORTED, "the adjoint is FP64 only (force_precision = REEDMD_FORCE_FP64)");
    if (lattice_of(ctx) != kDiamond || params->range_mode != REEDMD_RANGE_DEPTH || params->vacancy != 0)
        return fail(ctx, REEDMD_EUNSUPPORTED, "the adjoint covers the diamond target, depth range, no vacancy");
    if (!(k >= 0.0) || !(s >= kMinScreening && s <= kMaxScreening))
        return fail(ctx, REEDMD_EINVAL, "need k >= 0 and s in [0.01, 100]");
    for (int i = 0; i < 4; ++i) h_result[i] = 0.0;
    const long long n = batch->n;
    if (n == 0) return REEDMD_OK;
    const long long max_steps = params->max_steps > 0 ? params->max_steps : kDefaultGradSteps;
    const int ckpt_cap = static_cast<int>(max_steps / 64 + 1);
    // checkpoints, the step log, and the drop log (up to one domain move per 32 steps)
    const int drop_cap = 2 * ckpt_cap;
    const size_t per_track = (static_cast<size_t>(ckpt_cap) * kRecWords + static_cast<size_t>(ckpt_cap) * 64 * kLogWords +
                              static_cast<size_t>(drop_cap) * kDropWords) * sizeof(double);
    const long long chunk = std::max<long long>(1, std::min<long long>(n, static_cast<long long>(kGradScratchBytes / per_track)));
    const size_t out_bytes = static_cast<size_t>(n) * 5 * sizeof(double) + 64;
    const size_t need = static_cast<size_t>(chunk) * per_track + out_bytes;
    if (need > ctx->gscratch_bytes) {
        HIP_TRY(ctx, hipDeviceSynchronize());
        if (ctx->gscratch) (void)hipFree(ctx->gscratch);
        ctx->gscratch = nullptr;
        ctx->gscratch_bytes = 0;
        if (hipMalloc(reinterpret_cast<void**>(&ctx->gscratch), need) != hipSuccess) {
            ctx->gscratch = nullptr;
            return fail(ctx, REEDMD_ENOMEM, "cannot allocate adjoint checkpoints");
        }
        ctx->gscratch_bytes = need;
    }
    // species constants at the requested (k, s)
    reedmd_ctx at = *ctx;
    at.pot.s = s;
    at.stop.k = k;
    KernelArgs A;
    fill_common(&at, species, params, A);
    fill_batch(batch, A);
    A.max_steps = max_steps;
    A.n_thresh = 0;
    A.inv_s = 1.0 / s;
    A.ckpt_cap = ckpt_cap;
    double* base = ctx->gscratch;
    A.ckpt = base;
    A.steplog = base + static_cast<size_t>(chunk) * ckpt_cap * kRecWords;
    A.droplog = A.steplog + static_cast<size_t>(chunk) * ckpt_cap * 64 * kLogWords;
    A.drop_cap = drop_cap;
    double* own_out = A.droplog + static_cast<size_t>(chunk) * drop_cap * kDropWords;
    double* res = own_out + static_cast<size_t>(n) * 5;
    A.gout = d_track_out ? d_track_out : own_out;
    for (long long q0 = 0; q0 < n; q0 += chunk) {
        A.q0 = q0;
        A.q_end = std::min(n, q0 + chunk);
        const long long waves = A.q_end - q0;
        hipLaunchKernelGGL(grad_kernel, dim3(static_cast<unsigned>(waves)), dim3(64), 0, stream, A);
        HIP_TRY(ctx, hipGetLastError());
    }
    hipLaunchKernelGGL(grad_reduce_kernel, dim3(1), dim3(256), 0, stream, A.gout, n, res);
    HIP_TRY(ctx, hipGetLastError());
    double h[4];
    HIP_TRY(ctx, hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, stream));
    HIP_TRY(ctx, hipStreamSynchronize(stream));
    if (h[0] > 0.0) {
        h_result[0] = h[1] / h[0];
        h_result[1] = h[2] / h[0];
        h_result[2] = h[3] / h[0];
    }
    h_result[3] = h[0];
    return REEDMD_OK;
}

static reedmd_status eval_exp(const double* d_y, double* d_out, int64_t n, int pair, hipStream_t stream)
{
    if (n < 0 || (n > 0 && (!d_y || !d_out))) return fail(nullptr, REEDMD_EINVAL, "bad arguments");
    if (n == 0) return REEDMD_OK;
    hipLaunchKernelGGL(exp_neg_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, stream, d_y,
                       d_out, static_cast<long long>(n), pair);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(nullptr, REEDMD_EHIP, hipGetErrorString(e));
    return REEDMD_OK;
}

reedmd_status reedmd_eval_exp_neg(const double* d_y, double* d_out, int64_t n, hipStream_t stream)
{
    return eval_exp(d_y, d_out, n, 0, stream);
}

reedmd_status reedmd_eval_exp_neg_pair(const double* d_y, double* d_out, int64_t n, hipStream_t stream)
{
    return eval_exp(d_y, d_out, n, 1, stream);
}

reedmd_status reedmd_eval_log(const double* d_x, double* d_out, int64_t n, int32_t one_plus, hipStream_t stream)
{
    if (n < 0 || (n > 0 && (!d_x || !d_out)) || (one_plus != 0 && one_plus != 1))
        return fail(nullptr, REEDMD_EINVAL, "bad arguments");
    if (n == 0) return REEDMD_OK;
    hipLaunchKernelGGL(log_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, stream, d_x, d_out,
                       static_cast<long long>(n), static_cast<int>(one_plus));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(nullptr, REEDMD_EHIP, hipGetErrorString(e));
    return REEDMD_OK;
}

reedmd_status reedmd_autotune(reedmd_ctx* ctx, const reedmd_species* species, const reedmd_batch* batch,
                              const reedmd_run_params* params, int64_t pilot, hipStream_t stream,
                              int32_t* best_lanes, int32_t* best_waves)
{
    if (!ctx) return fail(nullptr, REEDMD_EINVAL, "ctx is NULL");
    reedmd_status st;
    if ((st = check_species(ctx, species)) != REEDMD_OK) return st;
    if ((st = check_batch(ctx, batch)) != REEDMD_OK) return st;
    if ((st = check_params(ctx, params, true)) != REEDMD_OK) return st;
    if (pilot <= 0) return fail(ctx, REEDMD_EINVAL, "pilot must be positive");
    reedmd_batch pb = *batch;
    pb.n = std::min<int64_t>(pilot, batch->n);
    double* hist = nullptr;
    reedmd_stats* stats = nullptr;
    int* cancel = nullptr;   // pinned, fine-grained host word polled by the kernel
    HIP_TRY(ctx, hipMalloc(reinterpret_cast<void**>(&hist), sizeof(double) * params->n_bins));
    HIP_TRY(ctx, hipMalloc(reinterpret_cast<void**>(&stats), sizeof(reedmd_stats)));
    HIP_TRY(ctx, hipHostMalloc(reinterpret_cast<void**>(&cancel), sizeof(int), hipHostMallocCoherent));
    reedmd_run_params p = *params;
    p.track_log = nullptr;
    p.track_log_cap = 0;
    p.cancel = cancel;
    p.r_cut = choose_shape(ctx, params, batch).r_cut;   // the full batch's interaction set
    hipEvent_t e0, e1;
    HIP_TRY(ctx, hipEventCreate(&e0));
    HIP_TRY(ctx, hipEventCreate(&e1));
    double best = -1.0;
    int bl = 64, bw = 0;
    const int lanes[3] = {64, 32, 16};
    const bool persistent = params->form == REEDMD_FORM_PERSISTENT;
    for (int li = 0; li < 3 && st == REEDMD_OK; ++li) {
        // persistent form: the occupancy-sized grid and one workgroup per CU fewer
        if (lattice_of(ctx) == kFluorite && lanes[li] == 16) continue;
        const int var = pass_variant(ctx, p.r_cut);
        const int occ = resident_blocks_per_cu(lanes[li], persistent ? kModePersistent : kModePlain,
                                               params->force_precision == REEDMD_FORCE_FP32, lattice_of(ctx), var);
        const int nw = (persistent && occ > 1) ? 2 : 1;
        for (int wi = 0; wi < nw && st == REEDMD_OK; ++wi) {
            p.lanes_per_track = lanes[li];
            p.waves_per_cu = wi == 0 ? 0 : (occ - 1) * (kBlock / 64);
            Shape s = choose_shape(ctx, &p, &pb);
            reedmd_stats h{};
            HIP_TRY(ctx, hipMemsetAsync(stats, 0, sizeof(reedmd_stats), stream));
            __atomic_store_n(cancel, 0, __ATOMIC_SEQ_CST);
            HIP_TRY(ctx, hipEventRecord(e0, stream));
            st = run_impl(ctx, species, &pb, &p, hist, stats, stream, &s);
            if (st != REEDMD_OK) break;
            HIP_TRY(ctx, hipEventRecord(e1, stream));
            // Steady-state throughput: the run is cancelled (drained with its ledger
            // intact) after a fixed time box from its start, unless it ends earlier.
            const auto t0 = std::chrono::steady_clock::now();
            while (hipEventQuery(e0) == hipErrorNotReady &&
                   std::chrono::steady_clock::now() - t0 < std::chrono::seconds(30)) {
            }
            const auto t1 = std::chrono::steady_clock::now();
            while (hipEventQuery(e1) == hipErrorNotReady &&
                   std::chrono::steady_clock::now() - t1 < std::chrono::milliseconds(kTuneBoxMs)) {
            }
            __atomic_store_n(cancel, 1, __ATOMIC_SEQ_CST);
            HIP_TRY(ctx, hipEventSynchronize(e1));
            float ms = 0.f;
            HIP_TRY(ctx, hipEventElapsedTime(&ms, e0, e1));
            HIP_TRY(ctx, hipMemcpy(&h, stats, sizeof(h), hipMemcpyDeviceToHost));
            const double rate = ms > 0.f ? static_cast<double>(h.pair_evals) / ms : 0.0;
            if (rate > best) {
                best = rate;
                bl = lanes[li];
                bw = p.waves_per_cu;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(hist);
    (void)hipFree(stats);
    (void)hipHostFree(cancel);
    if (st != REEDMD_OK) return st;
    // the lanes and waves entry of this configuration; a recorded interaction set stays
    auto prev = ctx->tune.find(tune_key(params, batch));
    const double rc = prev != ctx->tune.end() ? prev->second.r_cut : 0.0;
    ctx->tune[tune_key(params, batch)] = reedmd_ctx::Tuned{bl, bw, rc};
    if (best_lanes) *best_lanes = bl;
    if (best_waves) *best_waves = bw;
    return REEDMD_OK;
}

reedmd_status reedmd_autotune_domain(reedmd_ctx* ctx, const reedmd_species* species, const reedmd_batch* batch,
                                     const reedmd_run_params* params, const double* candidates, int32_t n_candidates,
                                     int64_t pilot, double gate_p, double gate_rel, hipStream_t stream,
                                     double* best_r_cut, double* report)
{
    if (!ctx) return fail(nullptr, REEDMD_EINVAL, "ctx is NULL");
    reedmd_status st;
    if ((st = check_species(ctx, species)) != REEDMD_OK) return st;
    if ((st = check_batch(ctx, batch)) != REEDMD_OK) return st;
    if ((st = check_params(ctx, params, true)) != REEDMD_OK) return st;
    if (!candidates || !best_r_cut) return fail(ctx, REEDMD_EINVAL, "candidates and best_r_cut must be non-NULL");
    if (n_candidates < 1 || n_candidates > 8) return fail(ctx, REEDMD_EINVAL, "n_candidates must be in 1..8");
    bool any_cut = false;
    for (int c = 0; c < n_candidates; ++c) {
        if (!(candidates[c] >= 0.0) || !std::isfinite(candidates[c]))
            return fail(ctx, REEDMD_EINVAL, "candidates must be finite and >= 0 (0 = the 27 cells)");
        any_cut |= candidates[c] > 0.0;
    }
    if (any_cut && (lattice_of(ctx) != kDiamond || params->force_precision != REEDMD_FORCE_FP64 ||
                    ctx->stop.mode == REEDMD_STOP_FKBK))
        return fail(ctx, REEDMD_EUNSUPPORTED, "the interaction cut-off is built for the diamond target with FP64 forces "
                                              "and the Lindhard-Scharff stopping");
    if (pilot <= 0) return fail(ctx, REEDMD_EINVAL, "pilot must be positive");
    if (!(gate_p >= 0.0 && gate_p < 1.0) || !(gate_rel >= 0.0) || !std::isfinite(gate_rel))
        return fail(ctx, REEDMD_EINVAL, "need gate_p in [0, 1) and gate_rel >= 0");
    reedmd_batch pb = *batch;
    pb.n = std::min<int64_t>(pilot, batch->n);
    if (pb.n == 0) {
        *best_r_cut = 0.0;
        return REEDMD_OK;
    }
    double* hist = nullptr;
    reedmd_stats* stats = nullptr;
    reedmd_result* log = nullptr;
    int64_t cap = 16 * pb.n;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto release = [&]() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipFree(hist);
        (void)hipFree(stats);
        (void)hipFree(log);
    };
    // one pilot run of an interaction set to its end: GPU time and the finished-track log
    auto pilot_run = [&](double rc, float* ms, std::vector<reedmd_result>& out) -> reedmd_status {
        for (int attempt = 0; attempt < 2; ++attempt) {
            reedmd_run_params p = *params;
            p.r_cut = rc;
            p.track_log = log;
            p.track_log_cap = cap;
            reedmd_stats h{};
            HIP_TRY(ctx, hipMemsetAsync(hist, 0, sizeof(double) * params->n_bins, stream));
            HIP_TRY(ctx, hipMemsetAsync(stats, 0, sizeof(reedmd_stats), stream));
            reedmd_status rs = run_impl(ctx, species, &pb, &p, hist, stats, stream, nullptr, nullptr, e0);
            if (rs != REEDMD_OK) return rs;
            HIP_TRY(ctx, hipEventRecord(e1, stream));
            HIP_TRY(ctx, hipEventSynchronize(e1));
            HIP_TRY(ctx, hipEventElapsedTime(ms, e0, e1));
            HIP_TRY(ctx, hipMemcpy(&h, stats, sizeof(h), hipMemcpyDeviceToHost));
            if (h.log_count <= cap) {
                out.resize(static_cast<size_t>(h.log_count));
                if (h.log_count > 0)
                    HIP_TRY(ctx, hipMemcpy(out.data(), log, sizeof(reedmd_result) * h.log_count, hipMemcpyDeviceToHost));
                return REEDMD_OK;
            }
            // more finished tracks than the log holds: grow it and run again
            (void)hipFree(log);
            log = nullptr;
            cap = h.log_count + h.log_count / 4;
            HIP_TRY(ctx, hipMalloc(reinterpret_cast<void**>(&log), sizeof(reedmd_result) * cap));
        }
        return fail(ctx, REEDMD_EHIP, "the pilot run's finished-track count changed between its two runs");
    };
    st = [&]() -> reedmd_status {
        HIP_TRY(ctx, hipMalloc(reinterpret_cast<void**>(&hist), sizeof(double) * params->n_bins));
        HIP_TRY(ctx, hipMalloc(reinterpret_cast<void**>(&stats), sizeof(reedmd_stats)));
        HIP_TRY(ctx, hipMalloc(reinterpret_cast<void**>(&log), sizeof(reedmd_result) * cap));
        HIP_TRY(ctx, hipEventCreate(&e0));
        HIP_TRY(ctx, hipEventCreate(&e1));
        std::vector<reedmd_result> lg;
        float ms_ref = 0.f;
        reedmd_status rs = pilot_run(0.0, &ms_ref, lg);
        if (rs != REEDMD_OK) return rs;
        const DepthSample ref = depth_sample(lg);
        double best_ms = -1.0, best_rc = 0.0;
        for (int c = 0; c < n_candidates; ++c) {
            const double rc = candidates[c];
            float ms = ms_ref;
            double p = 1.0, dm = 0.0, ds = 0.0;
            bool pass = true;
            if (rc > 0.0) {
                rs = pilot_run(rc, &ms, lg);
                if (rs != REEDMD_OK) return rs;
                const DepthSample d = depth_sample(lg);
                p = weighted_ks_p(d, ref, nullptr);
                dm = ref.mean != 0.0 ? std::fabs(d.mean - ref.mean) / std::fabs(ref.mean) : 0.0;
                ds = ref.sd != 0.0 ? std::fabs(d.sd - ref.sd) / ref.sd : 0.0;
                const double bm = std::max(gate_rel, 3.0 * std::hypot(d.se_mean, ref.se_mean) / std::fabs(ref.mean));
                const double bs = std::max(gate_rel, 3.0 * std::hypot(d.se_sd, ref.se_sd) / ref.sd);
                pass = p > gate_p && dm <= bm && ds <= bs;
            }
            if (report) {
                report[5 * c + 0] = ms;
                report[5 * c + 1] = p;
                report[5 * c + 2] = dm;
                report[5 * c + 3] = ds;
                report[5 * c + 4] = pass ? 1.0 : 0.0;
            }
            if (pass && (best_ms < 0.0 || ms < best_ms)) {
                best_ms = ms;
                best_rc = rc;
            }
        }
        if (best_ms < 0.0) best_rc = 0.0;   // only failing cut-offs offered: the 27 cells
        auto prev = ctx->tune.find(tune_key(params, batch));
        reedmd_ctx::Tuned t{0, 0, best_rc};
        if (prev != ctx->tune.end()) {
            t.lanes = prev->second.lanes;
            t.waves = prev->second.waves;
        }
        ctx->tune[tune_key(params, batch)] = t;
        *best_r_cut = best_rc;
        return REEDMD_OK;
    }();
    release();
    return st;
}

// All epochs of a refined run in one persistent launch (settings validated by the caller):
// version e of the depth tables ([E][n_tables][n_thresh], version 0 the caller's) is
// computed and published inside the launch by the first claimer of epoch e.
static reedmd_status run_refined_in_launch(reedmd_ctx* ctx, const reedmd_species* species,
                                           const reedmd_batch* batch, const reedmd_run_params* params,
                                           const reedmd_refine* rf, int E, double* d_hist, reedmd_stats* d_stats,
                                           double* d_depths, hipStream_t stream)
{
    const int nt = params->n_tables, nk = params->n_thresh, nb = params->n_bins;
    const size_t thr_b = sizeof(double) * E * nt * nk, ts_b = sizeof(double) * nt * (nb + 2);
    const size_t snap_b = ts_b * E, pr_b = sizeof(double) * nk, rd_b = sizeof(int) * E;
    char* work = nullptr;
    HIP_TRY(ctx, hipMalloc(reinterpret_cast<void**>(&work), thr_b + ts_b + snap_b + pr_b + rd_b + 256));
    double* thr = reinterpret_cast<double*>(work);
    double* tstat = thr + static_cast<size_t>(E) * nt * nk;
    double* snap = tstat + static_cast<size_t>(nt) * (nb + 2);
    double* probs = snap + static_cast<size_t>(E) * nt * (nb + 2);
    int* ready = reinterpret_cast<int*>(probs + nk);
    auto body = [&]() -> reedmd_status {
        const int one = 1;
        HIP_TRY(ctx, hipMemsetAsync(work, 0, thr_b + ts_b + snap_b + pr_b + rd_b, stream));
        HIP_TRY(ctx, hipMemcpyAsync(thr, params->thresholds, sizeof(double) * nt * nk, hipMemcpyDeviceToDevice, stream));
        HIP_TRY(ctx, hipMemcpyAsync(probs, rf->probs, pr_b, hipMemcpyHostToDevice, stream));
        HIP_TRY(ctx, hipMemcpyAsync(ready, &one, sizeof(int), hipMemcpyHostToDevice, stream));
        reedmd_run_params p = *params;
        p.thresholds = thr;
        p.r_cut = choose_shape(ctx, params, batch).r_cut;
        const Shape shape = choose_shape(ctx, &p, batch);
        const RefineLaunch rl{E, probs, rf->min_gap, rf->min_weight, snap, ready};
        const reedmd_status rs = run_impl(ctx, species, batch, &p, d_hist, d_stats, stream, &shape, tstat, nullptr, &rl);
        if (rs != REEDMD_OK) return rs;
        if (d_depths) HIP_TRY(ctx, hipMemcpyAsync(d_depths, thr, thr_b, hipMemcpyDeviceToDevice, stream));
        if (rf->snapshots) HIP_TRY(ctx, hipMemcpyAsync(rf->snapshots, snap, snap_b, hipMemcpyDeviceToDevice, stream));
        HIP_TRY(ctx, hipStreamSynchronize(stream));
        return REEDMD_OK;
    };
    const reedmd_status rs = body();
    (void)hipStreamSynchronize(stream);
    (void)hipFree(work);
    return rs;
}

reedmd_status reedmd_run_refined(reedmd_ctx* ctx, const reedmd_species* species, const reedmd_batch* batch,
                                 const reedmd_run_params* params, const reedmd_refine* rf, double* d_hist,
                                 reedmd_stats* d_stats, double* d_depths, hipStream_t stream)
{
    if (!ctx) return fail(nullptr, REEDMD_EINVAL, "ctx is NULL");
    reedmd_status st;
    if ((st = check_species(ctx, species)) != REEDMD_OK) return st;
    if ((st = check_batch(ctx, batch)) != REEDMD_OK) return st;
    if ((st = check_params(ctx, params, true)) != REEDMD_OK) return st;
    if (!d_hist || !d_stats) return fail(ctx, REEDMD_EINVAL, "d_hist and d_stats must be non-NULL");
    if (!rf || !rf->probs) return fail(ctx, REEDMD_EINVAL, "refine settings and probs must be non-NULL");
    if (params->n_thresh < 1) return fail(ctx, REEDMD_EINVAL, "adaptive depths need n_thresh >= 1");
    if (rf->n_epochs < 1 || rf->n_epochs > 4096) return fail(ctx, REEDMD_EINVAL, "n_epochs must be in 1..4096");
    if (!(rf->min_gap >= 0.0) || !std::isfinite(rf->min_gap)) return fail(ctx, REEDMD_EINVAL, "min_gap must be >= 0");
    if (!(rf->min_weight >= 0.0) || !std::isfinite(rf->min_weight))
        return fail(ctx, REEDMD_EINVAL, "min_weight must be finite and >= 0");
    for (int k = 0; k < params->n_thresh; ++k) {
        const double pk = rf->probs[k];
        if (!(pk > 0.0 && pk < 1.0) || (k > 0 && !(pk < rf->probs[k - 1])))
            return fail(ctx, REEDMD_EINVAL, "probs must decrease strictly inside (0, 1)");
    }
    if (rf->in_launch != 0 && rf->in_launch != 1) return fail(ctx, REEDMD_EINVAL, "in_launch must be 0 or 1");
    if (rf->in_launch && params->form != REEDMD_FORM_PERSISTENT)
        return fail(ctx, REEDMD_EINVAL, "in-launch refinement needs the persistent form");
    const long long n = batch->n;
    if (n == 0) return REEDMD_OK;
    const int E = static_cast<int>(std::min<long long>(rf->n_epochs, n));
    const int nt = params->n_tables, nk = params->n_thresh, nb = params->n_bins;
    if (rf->in_launch) return run_refined_in_launch(ctx, species, batch, params, rf, E, d_hist, d_stats, d_depths, stream);
    const long long m = (n + E - 1) / E;   // largest epoch
    // work buffers: depth tables, per-table statistics, targets, one epoch of primaries
    const size_t thr_b = sizeof(double) * nt * nk, ts_b = sizeof(double) * nt * (nb + 2), pr_b = sizeof(double) * nk;
    const size_t sub_b = static_cast<size_t>(m) * (sizeof(int) * 2 + sizeof(double) * 7 + sizeof(unsigned long long));
    char* work = nullptr;
    HIP_TRY(ctx, hipMalloc(reinterpret_cast<void**>(&work), thr_b + ts_b + pr_b + sub_b + 256));
    double* thr = reinterpret_cast<double*>(work);
    double* tstat = thr + nt * nk;
    double* probs = tstat + static_cast<size_t>(nt) * (nb + 2);
    double* sub_energy = probs + nk;
    double* sub_pos = sub_energy + m;
    double* sub_dir = sub_pos + 3 * m;
    unsigned long long* sub_key = reinterpret_cast<unsigned long long*>(sub_dir + 3 * m);
    int* sub_species = reinterpret_cast<int*>(sub_key + m);
    int* sub_table = sub_species + m;
    auto body = [&]() -> reedmd_status {
        HIP_TRY(ctx, hipMemcpyAsync(thr, params->thresholds, thr_b, hipMemcpyDeviceToDevice, stream));
        HIP_TRY(ctx, hipMemsetAsync(tstat, 0, ts_b, stream));
        HIP_TRY(ctx, hipMemcpyAsync(probs, rf->probs, pr_b, hipMemcpyHostToDevice, stream));
        reedmd_run_params p = *params;
        p.thresholds = thr;
        p.r_cut = choose_shape(ctx, params, batch).r_cut;   // the whole batch's interaction set
        reedmd_result* log0 = static_cast<reedmd_result*>(params->track_log);
        int64_t log_done = 0;
        reedmd_stats h0{};
        if (log0) {
            HIP_TRY(ctx, hipMemcpyAsync(&h0, d_stats, sizeof(h0), hipMemcpyDeviceToHost, stream));
            HIP_TRY(ctx, hipStreamSynchronize(stream));
        }
        for (int e = 0; e < E; ++e) {
            const long long lo = n * e / E, hi = n * (e + 1) / E, ne = hi - lo;
            if (e > 0)
                hipLaunchKernelGGL(refine_kernel, dim3((nt + 63) / 64), dim3(64), 0, stream, tstat, nb,
                                   params->bin_width, nt, nk, probs, rf->min_gap, rf->min_weight, thr);
            HIP_TRY(ctx, hipGetLastError());
            if (d_depths)
                HIP_TRY(ctx, hipMemcpyAsync(d_depths + static_cast<size_t>(e) * nt * nk, thr, thr_b,
                                            hipMemcpyDeviceToDevice, stream));
            HIP_TRY(ctx, hipMemcpyAsync(sub_species, batch->species + lo, sizeof(int) * ne, hipMemcpyDeviceToDevice, stream));
            HIP_TRY(ctx, hipMemcpyAsync(sub_table, batch->table + lo, sizeof(int) * ne, hipMemcpyDeviceToDevice, stream));
            HIP_TRY(ctx, hipMemcpyAsync(sub_energy, batch->energy + lo, sizeof(double) * ne, hipMemcpyDeviceToDevice, stream));
            HIP_TRY(ctx, hipMemcpyAsync(sub_key, batch->key + lo, sizeof(uint64_t) * ne, hipMemcpyDeviceToDevice, stream));
            for (int c = 0; c < 3; ++c) {
                HIP_TRY(ctx, hipMemcpyAsync(sub_pos + c * ne, batch->pos + c * n + lo, sizeof(double) * ne,
                                            hipMemcpyDeviceToDevice, stream));
                HIP_TRY(ctx, hipMemcpyAsync(sub_dir + c * ne, batch->dir + c * n + lo, sizeof(double) * ne,
                                            hipMemcpyDeviceToDevice, stream));
            }
            reedmd_batch sb{};
            sb.n = ne;
            sb.id0 = batch->id0 + lo;
            sb.species = sub_species;
            sb.energy = sub_energy;
            sb.pos = sub_pos;
            sb.dir = sub_dir;
            sb.key = reinterpret_cast<uint64_t*>(sub_key);
            sb.table = sub_table;
            if (log0) {
                p.track_log = log0 + log_done;
                p.track_log_cap = std::max<int64_t>(0, params->track_log_cap - log_done);
            }
            const Shape shape = choose_shape(ctx, &p, &sb);
            const reedmd_status rs = run_impl(ctx, species, &sb, &p, d_hist, d_stats, stream, &shape, tstat);
            if (rs != REEDMD_OK) return rs;
            if (log0) {
                reedmd_stats h{};
                HIP_TRY(ctx, hipMemcpyAsync(&h, d_stats, sizeof(h), hipMemcpyDeviceToHost, stream));
                HIP_TRY(ctx, hipStreamSynchronize(stream));
                log_done = std::min<int64_t>(params->track_log_cap, h.log_count - h0.log_count);
            }
        }
        HIP_TRY(ctx, hipStreamSynchronize(stream));
        return REEDMD_OK;
    };
    const reedmd_status rs = body();
    (void)hipStreamSynchronize(stream);
    (void)hipFree(work);
    return rs;
}

reedmd_status reedmd_launch_shape(reedmd_ctx* ctx, const reedmd_batch* batch, const reedmd_run_params* params,
                                  int64_t* out)
{
    if (!ctx) return fail(nullptr, REEDMD_EINVAL, "ctx is NULL");
    reedmd_status st;
    if ((st = check_batch(ctx, batch)) != REEDMD_OK) return st;
    if ((st = check_params(ctx, params, true)) != REEDMD_OK) return st;
    if (!out) return fail(ctx, REEDMD_EINVAL, "out is NULL");
    const Shape s = choose_shape(ctx, params, batch);
    out[0] = s.L;
    out[1] = s.blocks;
    out[2] = s.seg_total;
    out[3] = resident_blocks_per_cu(s.L, s.mode, s.f32, lattice_of(ctx), s.var);
    out[4] = s.mode == kModePersistent ? s.qcap : 0;
    return REEDMD_OK;
}

}  // extern "C"
