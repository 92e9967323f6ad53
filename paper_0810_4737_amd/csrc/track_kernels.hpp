// REED-MD track kernels for gfx950.
//
// Mapping: one wavefront holds T = 64 / L track segments of L lanes.  The
// domain atoms of a track (216 for diamond, 324 for fluorite) live in the VGPRs
// of its segment: slot s is held by lane (s mod L) as its register element s / L.  Slots are indexed by cell
// residue (c mod 3 per axis) so that moving the domain never moves data: when
// the centre cell changes, exactly the slots whose cell left the 3x3x3 block
// are re-created in place (Sec. 2, Fig. 1).  Per step, one fused pass over a
// lane's slots does half kick, drift, the ZBL pair term, the reaction force
// and the second half kick; segment reductions (xor shuffles) give the ion
// force, the local density and the largest atom speed and acceleration.
#pragma once
#include "device_physics.hpp"
#include "../../include/reedmd.h"

namespace reedmd {

enum : int { kModePlain = 0, kModePersistent = 1 };

// Minimum resident wavefronts per SIMD asked of the register allocator for the
// track kernels (the unified VGPR/AGPR file holds 512 registers per lane).
#ifndef REEDMD_PAIR_BARRIER
#define REEDMD_PAIR_BARRIER 0
#endif
#ifndef REEDMD_WAVES_PER_SIMD
#define REEDMD_WAVES_PER_SIMD(L, LAT) ((L) >= 32 && (LAT) == kDiamond ? 2 : 1)
#endif



// Clone queue (persistent form): bounded multi-producer multi-consumer ring
// with one sequence word per slot (slot free for ticket t when seq == t, full
// when seq == t + 1).
struct QueueState {
    unsigned long long head;
    unsigned long long tail;
    long long live;         // tracks not yet finished (unclaimed primaries included)
    long long prim_next;    // next unclaimed primary
    long long depth_max;
    long long log_next;     // next free entry of the optional result log
    long long handoff;      // 1: running tracks move to the queue for the wider tail kernel
    long long tail_left;    // segments of the tail launch that have left early (see kTailReserve)
};

// The tail launch keeps at least this many idle segments, and twice the live tracks, waiting
// for clones; the other idle segments leave, so that the compute units are free for other
// work (the next batch on another stream) while the last long tracks finish.
constexpr long long kTailReserve = 64;

struct KernelArgs {
    SpeciesConst sp[kMaxSpecies];
    PairConst pc2[kMaxSpecies];   // against the second target species (fluorite anions)
    // crystal (M2, sigma: target species 0; M2b, sigma_b: species 1)
    double a, inv_a, M2, sigma, inv_M2sq, half_inv_M2;
    double M2b, sigma_b, inv_M2bsq, half_inv_M2b;
    double park;            // empty slots sit this far above the domain centre
    int structure;          // kDiamond / kFluorite
    int range_mode;         // 0: depth z; 1: distance from the start point
    int vacancy;            // 1: the basis-0 site of the start cell is vacant (recoil)
    int pad_lat;
    // integration and events
    double dx_max, dt_max, E_stop, z_start;
    long long max_steps;
    unsigned long long seed;
    // cloning
    const double* thr;
    int n_thresh, n_tables, n_clones, n_bins;
    int n_species;
    double bin_width;
    // batch
    long long n, id0;
    const int* species;
    const double* energy;
    const double* pos;
    const double* dir;
    const unsigned long long* key;
    const int* table;
    // outputs
    double* hist;
    double* tstat;          // optional, per depth table: [n_bins] stopped weight by bin, overflow, total
    reedmd_stats* stats;
    reedmd_result* log;
    long long log_cap;
    // scratch
    double* stack;          // [segments][stack_cap][kRecWords]
    int stack_cap;
    int qcap;               // 0: no shared queue
    QueueState* q;
    unsigned long long* qseq;
    double* qrec;
    const int* cancel;
    double rc2;             // interaction cut-off squared (A^2); 0: every atom of the 27 cells
    // Firsov + Brandt-Kitagawa stopping: per species k Z1^2 gamma_p (0: no Brandt-Kitagawa
    // term) and Z1^(1/3); the electron gas's Fermi speed (atomic units) and the inverse of the
    // atomic velocity unit in sqrt(eV/amu)
    double bk_pref[kMaxSpecies];
    double bk_z13[kMaxSpecies];
    double bk_vF, bk_inv_vunit;
    // cloning depths re-placed inside the launch (0: off): epoch e = claim positions
    // [ceil(n e / E), ceil(n (e+1) / E)); the first claimer of epoch e computes table version e
    // (thr holds [E][n_tables][n_thresh]) from a snapshot of tstat (snap: [E][n_tables][n_bins+2])
    // and sets ready[e]; the epoch's other claims wait for it
    int refine_E;
    int pad_refine;
    const double* r_probs;
    double r_min_gap, r_min_weight;
    double* r_snap;
    int* r_ready;
    const int* order;       // optional: batch entry of the i-th claimed primary (longest expected first)
    long long seg_total;
    // tail handoff (persistent form with fewer than 64 lanes per track): once every primary
    // is claimed and at most handoff_live tracks are live, running tracks are stored in the
    // queue and finished by a 64-lane launch of the same kernel (tail = 1), which takes work
    // from the queue only; 0: no handoff
    long long handoff_live;
    int tail;
    int pad_tail;
    // debug entry points
    double* records;
    int nsteps;
    // gradient entry point
    double inv_s;           // 1 / screening-length scale
    double* ckpt;           // [n][ckpt_cap][kRecWords]  state every 64 steps
    double* steplog;        // [n][ckpt_cap * 64][12]    per step: dt, StepInfo code, ion x, v, F, rho before it
    double* droplog;        // [n][drop_cap][kDropWords] per domain move: the old centre, the dropped atoms
    int drop_cap;
    int ckpt_cap;
    double* gout;           // [n][5]: z_stop, dz/dk, dz/ds, status, steps
    long long q0, q_end;    // batch entries [q0, q_end) handled by this launch
};

// Rarely used kernel arguments are re-read from the kernel-argument segment
// where they are needed (every kernel of this file takes one KernelArgs by
// value, which sits at offset 0 of that segment).  The empty asm makes the
// pointer opaque, so the compiler cannot hoist those scalar loads out of the
// step loop into scalar registers, which otherwise spill into vector-register
// lanes inside the hot loop.
typedef const __attribute__((address_space(4))) unsigned long long KernargWord;
__device__ __forceinline__ KernelArgs cold_args()
{
    static_assert(sizeof(KernelArgs) % 8 == 0, "argument block is copied in 64-bit words");
    KernargWord* p = (KernargWord*)(__builtin_amdgcn_kernarg_segment_ptr());
    asm volatile("" : "+s"(p));
    KernelArgs a;
    unsigned long long* d = reinterpret_cast<unsigned long long*>(&a);
#pragma unroll
    for (int i = 0; i < static_cast<int>(sizeof(KernelArgs) / 8); ++i) d[i] = p[i];
    return a;
}

// Per-track LDS area: [waves per workgroup][tracks per wave] of the atom
// forces [3][SL*L] (the slots padded to whole lane rows, so every lane of a row
// has an entry) followed by kTrackHdr words: the start point (3), the cell of
// the vacant site (3) and its basis index (-1: none), the running track's
// step and pair-term counts not yet booked (two 32-bit words; see track_kernel)
// and the number of atoms in its domain (kept here rather than in a register
// that the track kernel would spill and reload every step).
// With an interaction cut-off (CUT) the header is followed by the list of the
// slots within the cut-off (one int per slot).
constexpr int kTrackHdr = 9;
constexpr int kCountWord = 7;   // header word of the unbooked step and pair-term counts
constexpr int kExistWord = 8;   // header word of the number of atoms in the domain
template <int L, int LAT = kDiamond, bool CUT = false>
struct ForceLds {
    static constexpr int kStride = ((Lattice<LAT>::kSlots + L - 1) / L) * L;
    static constexpr int kTracksPerBlock = 4 * (64 / L);
    static constexpr int kTrackDoubles = 3 * kStride + kTrackHdr + (CUT ? kStride / 2 : 0);
    static constexpr int kDoubles = kTracksPerBlock * kTrackDoubles;
};
template <int L, int LAT = kDiamond, bool CUT = false>
__device__ __forceinline__ double* force_slab(double* s_force)
{
    const int track_in_block = (threadIdx.x >> 6) * (64 / L) + (threadIdx.x & 63) / L;
    return s_force + track_in_block * ForceLds<L, LAT, CUT>::kTrackDoubles;
}

// Species constants are staged in LDS once per workgroup (indexed per lane):
// the SpeciesConst table, followed by the PairConst table of the second target
// species.
constexpr int kSpeciesLdsDoubles = (sizeof(SpeciesConst) + sizeof(PairConst)) * kMaxSpecies / sizeof(double);
__device__ __forceinline__ const SpeciesConst* stage_species(const KernelArgs& A, double* s_sp)
{
    constexpr int kW1 = sizeof(SpeciesConst) * kMaxSpecies / sizeof(double);
    constexpr int kW2 = sizeof(PairConst) * kMaxSpecies / sizeof(double);
    static_assert(kW1 + kW2 == kSpeciesLdsDoubles, "species tables are whole doubles");
    for (int i = threadIdx.x; i < kW1 + kW2; i += blockDim.x)
        s_sp[i] = (i < kW1) ? reinterpret_cast<const double*>(A.sp)[i] : reinterpret_cast<const double*>(A.pc2)[i - kW1];
    __syncthreads();
    return reinterpret_cast<const SpeciesConst*>(s_sp);
}
__device__ __forceinline__ const PairConst* pair_table2(const SpeciesConst* sp)
{
    return reinterpret_cast<const PairConst*>(sp + kMaxSpecies);
}

// ---------------------------------------------------------------------------
// Segment reductions.  Within a 16-lane row: DPP butterflies (quad permutes,
// half-row and row mirrors); across the two rows of a 32-lane half: a
// ds_swizzle xor 16; across the two halves of the wavefront: readlane of
// lanes 0 and 32.  Every stage combines a value with its partner's using a
// commutative operation, so every lane of a segment ends with bitwise the
// same result.
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v)
{
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    return __hiloint2double(dpp_i32<CTRL>(__double2hiint(v)), dpp_i32<CTRL>(__double2loint(v)));
}
__device__ __forceinline__ double swz16_f64(double v)
{
    return __hiloint2double(__builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401F),
                            __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401F));
}
__device__ __forceinline__ double lane_f64(double v, int lane)
{
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}
constexpr int kQuadXor1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kRowHalfMirror = 0x141;
constexpr int kRowMirror = 0x140;

__device__ __forceinline__ double xor32_f64(double v)
{
    const int src = ((threadIdx.x & 63) ^ 32) << 2;
    return __hiloint2double(__builtin_amdgcn_ds_bpermute(src, __double2hiint(v)),
                            __builtin_amdgcn_ds_bpermute(src, __double2loint(v)));
}

// Sums over a track's slots use one fixed order for every lane layout, so that
// results do not depend on the lanes per track (or on anything else the
// autotuner chooses).  Slot s belongs to column q = s mod 64; a lane keeps one
// partial per column it holds (G = 64 / L of them: column q = lane + L m in
// acc[m]), each summed over its slots in increasing order; the 64 column
// partials are then combined as a butterfly over the column index, bit 4
// first, then bit 5, then bits 0 to 3.  Addition is commutative in IEEE
// arithmetic, so both partners of every stage hold the same value and every
// lane ends with bitwise the same sum.
template <int L>
struct SegReduce {
    static constexpr int G = 64 / L;
    __device__ __forceinline__ static double lanes16(double v)
    {
        v += dpp_f64<kQuadXor1>(v);
        v += dpp_f64<kQuadXor2>(v);
        v += dpp_f64<kRowHalfMirror>(v);   // pairs quads: on equal quad values the same as xor 4
        v += dpp_f64<kRowMirror>(v);       // pairs half rows: the same as xor 8
        return v;
    }
    // Plain segment sum of one value per lane (the adjoint's sums, which need no
    // agreement between layouts).
    __device__ __forceinline__ static double sum(double v)
    {
        v = lanes16(v);
        if (L >= 32) v += swz16_f64(v);
        if (L == 64) v = lane_f64(v, 0) + lane_f64(v, 32);
        return v;
    }
    __device__ __forceinline__ static double csum(const double (&acc)[G])
    {
        double v;
        if constexpr (L == 16) {
            v = (acc[0] + acc[1]) + (acc[2] + acc[3]);
        } else if constexpr (L == 32) {
            v = (acc[0] + swz16_f64(acc[0])) + (acc[1] + swz16_f64(acc[1]));
        } else {
            v = acc[0] + swz16_f64(acc[0]);
            v += xor32_f64(v);
        }
        return lanes16(v);
    }
    __device__ __forceinline__ static double max(double v)
    {
        v = fmax(v, dpp_f64<kQuadXor1>(v));
        v = fmax(v, dpp_f64<kQuadXor2>(v));
        v = fmax(v, dpp_f64<kRowHalfMirror>(v));
        v = fmax(v, dpp_f64<kRowMirror>(v));
        if (L >= 32) v = fmax(v, swz16_f64(v));
        if (L == 64) v = fmax(lane_f64(v, 0), lane_f64(v, 32));
        return v;
    }
    __device__ __forceinline__ static int isum(int v)
    {
        v += dpp_i32<kQuadXor1>(v);
        v += dpp_i32<kQuadXor2>(v);
        v += dpp_i32<kRowHalfMirror>(v);
        v += dpp_i32<kRowMirror>(v);
        if (L >= 32) v += __builtin_amdgcn_ds_swizzle(v, 0x401F);
        if (L == 64) v = __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 32);
        return v;
    }
};

// Register-resident state of one track segment.
template <int L, int LAT = kDiamond>
struct TrackRegs {
    static constexpr int SL = (Lattice<LAT>::kSlots + L - 1) / L;
    static constexpr int FS = ForceLds<L, LAT>::kStride;
    double ax[SL], ay[SL], az[SL], avx[SL], avy[SL], avz[SL];
    double* fl;          // LDS: this track's atom forces, [3][FS] (fx, fy, fz by slot), then its header
    unsigned exist;      // bit i: register slot i holds an existing atom
    // ion (segment-uniform)
    double x, y, z, vx, vy, vz, Fx, Fy, Fz, rho, w, zstop;
    double vmax2a, amax2a;   // largest atom |v|^2 and |f/M2|^2 after the last pass
    double thr_next;         // next cloning depth (+inf when none is left)
    int cx, cy, cz;
    unsigned long long key;
    long long steps, lineage;
    int species, next_k, table, status;
    int n_exist;             // atoms in the domain (segment-uniform)
    int n_eval;              // pair terms evaluated by the last pass with a cut-off (without one: n_exist)
};

template <int L, int LAT>
__device__ __forceinline__ void refresh_threshold(TrackRegs<L, LAT>& t, const KernelArgs& A)
{
    t.thr_next = (t.next_k < A.n_thresh) ? A.thr[static_cast<size_t>(t.table) * A.n_thresh + t.next_k]
                                         : __builtin_huge_val();
}

// Empty register slots (cells above the surface, and the lanes past slot 215)
// are parked at rest above the domain centre at the parking distance, where
// every pair exponential underflows to exactly 0: their pair terms vanish and
// the pass over the slots needs no branch.
template <int L, int LAT>
__device__ __forceinline__ void park_slot(TrackRegs<L, LAT>& t, int i, int s, double px, double py, double pz)
{
    constexpr int FS = TrackRegs<L, LAT>::FS;
    t.ax[i] = px; t.ay[i] = py; t.az[i] = pz;
    t.avx[i] = 0.0; t.avy[i] = 0.0; t.avz[i] = 0.0;
    t.fl[0 * FS + s] = 0.0; t.fl[1 * FS + s] = 0.0; t.fl[2 * FS + s] = 0.0;
}

// Position of the k-th set bit (from 0) of m, k < popcount(m).
__device__ __forceinline__ int kth_set_bit(unsigned m, int k)
{
    int pos = 0;
#pragma unroll
    for (int w = 16; w >= 1; w >>= 1) {
        const int c = __popc(m & ((1u << w) - 1u));
        if (k >= c) {
            k -= c;
            m >>= w;
            pos += w;
        }
    }
    return pos;
}

// Bit c set: ring cell c (residues c / 9, c / 3 % 3, c % 3) holds a different
// unit cell around the new centre than around the old one (every cell when
// `all`) and that cell lies in the crystal.  One ballot per 27 cells over the
// segment's lanes; the result is the same in every lane of the segment.
template <int L>
__device__ __forceinline__ unsigned new_cell_mask(int sl, int ncx, int ncy, int ncz, int ocx, int ocy, int ocz,
                                                  bool all)
{
    const int base = (threadIdx.x & 63) - sl;
    unsigned m = 0;
#pragma unroll
    for (int pass = 0; pass * L < 27; ++pass) {
        const int c = pass * L + sl;
        const int rx = c / 9, ry = (c / 3) % 3, rz = c % 3;
        const int nz = cell_of_residue(rz, ncz);
        const bool changed = all || cell_of_residue(rx, ncx) != cell_of_residue(rx, ocx) ||
                             cell_of_residue(ry, ncy) != cell_of_residue(ry, ocy) || nz != cell_of_residue(rz, ocz);
        const unsigned long long b = __ballot(c < 27 && changed && nz >= 0);
        const unsigned long long seg = (L == 64) ? b : ((b >> base) & ((1ull << (L % 64)) - 1ull));
        m |= static_cast<unsigned>(seg) << (pass * L);
    }
    return m;
}

// The track's header words in LDS (after its forces): start point, cell of
// the vacant site and its basis index (negative: none).  Every lane of the
// segment writes the same values.
template <int L, int LAT>
__device__ __forceinline__ double* track_hdr(const TrackRegs<L, LAT>& t)
{
    return t.fl + 3 * TrackRegs<L, LAT>::FS;
}
__device__ __forceinline__ bool vacant_site(const double* h, int cx, int cy, int cz, int b)
{
    return h[6] >= 0.0 && b == static_cast<int>(h[6]) && cx == static_cast<int>(h[3]) &&
           cy == static_cast<int>(h[4]) && cz == static_cast<int>(h[5]);
}

template <int L, int LAT>
__device__ __forceinline__ void regenerate(TrackRegs<L, LAT>& t, const KernelArgs& A, int sl, int ncx,
                                           int ncy, int ncz, bool all, double* drop = nullptr)
{
    using Lat = Lattice<LAT>;
    constexpr int FS = TrackRegs<L, LAT>::FS;
    constexpr int NB = Lat::kCellAtoms;
    const KernelArgs C = cold_args();
    const double* h = track_hdr(t);
    const unsigned newc = new_cell_mask<L>(sl, ncx, ncy, ncz, t.cx, t.cy, t.cz, all);
    // The atoms of every new cell are created spread evenly over the lanes of
    // the segment (a face shift creates a third of the domain), and each
    // position is staged in the force entries of its slot, which the new atom
    // discards.  The vacant site of a recoil is not created.
    const int n_new = NB * __popc(newc);
    for (int idx = sl; idx < n_new; idx += L) {
        const int cell = kth_set_bit(newc, idx / NB), b = idx % NB;
        const int rx = cell / 9, ry = (cell / 3) % 3, rz = cell % 3;
        const int gx = cell_of_residue(rx, ncx), gy = cell_of_residue(ry, ncy), gz = cell_of_residue(rz, ncz);
        if (LAT == kFluorite && vacant_site(h, gx, gy, gz, b)) continue;
        const double3 p = create_atom(t.key, C.seed, gx, gy, gz, b, C.a, C.sigma, C.sigma_b, LAT == kFluorite);
        const int s = Lat::slot(cell, b);
        t.fl[0 * FS + s] = p.x;
        t.fl[1 * FS + s] = p.y;
        t.fl[2 * FS + s] = p.z;
    }
    // positions written by other lanes of this wavefront are read below
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const double parkx = C.a * (static_cast<double>(ncx) + 0.5);
    const double parky = C.a * (static_cast<double>(ncy) + 0.5);
    const double parkz = C.a * (static_cast<double>(ncz) + 0.5) - C.park;
    unsigned ex = 0;
#pragma unroll
    for (int i = 0; i < TrackRegs<L, LAT>::SL; ++i) {
        const int s = sl + L * i;
        const int cell = (s < Lat::kSlots) ? Lat::cell_of_slot(s) : -1;
        if (drop != nullptr && ((t.exist >> i) & 1u)) {
            // the atom leaves the domain when its cell does: its position and velocity
            // go to the drop log, [6][kSlots] by slot (the adjoint restores them)
            const int rx = cell / 9, ry = (cell / 3) % 3, rz = cell % 3;
            if (cell_of_residue(rx, ncx) != cell_of_residue(rx, t.cx) ||
                cell_of_residue(ry, ncy) != cell_of_residue(ry, t.cy) ||
                cell_of_residue(rz, ncz) != cell_of_residue(rz, t.cz)) {
                constexpr int NS = Lat::kSlots;
                drop[0 * NS + s] = t.ax[i]; drop[1 * NS + s] = t.ay[i]; drop[2 * NS + s] = t.az[i];
                drop[3 * NS + s] = t.avx[i]; drop[4 * NS + s] = t.avy[i]; drop[5 * NS + s] = t.avz[i];
            }
        }
        if (cell < 0 || cell_of_residue(cell % 3, ncz) < 0 ||
            (LAT == kFluorite &&
             vacant_site(h, cell_of_residue(cell / 9, ncx), cell_of_residue((cell / 3) % 3, ncy),
                         cell_of_residue(cell % 3, ncz), Lat::basis_of_slot(s)))) {
            park_slot<L, LAT>(t, i, s, parkx, parky, parkz);
            continue;
        }
        ex |= (1u << i);
        if ((newc >> cell) & 1u) {
            t.ax[i] = t.fl[0 * FS + s];
            t.ay[i] = t.fl[1 * FS + s];
            t.az[i] = t.fl[2 * FS + s];
            t.avx[i] = 0.0; t.avy[i] = 0.0; t.avz[i] = 0.0;
            t.fl[0 * FS + s] = 0.0; t.fl[1 * FS + s] = 0.0; t.fl[2 * FS + s] = 0.0;
        }
    }
    t.exist = ex;
    t.cx = ncx; t.cy = ncy; t.cz = ncz;
    t.n_exist = SegReduce<L>::isum(__popc(ex));
    if (sl == 0) reinterpret_cast<volatile int*>(track_hdr(t) + kExistWord)[0] = t.n_exist;
}

// The range coordinate: the depth z, or the distance from the start point
// (recoils; built into the fluorite kernels only, as is the vacant site).
template <int L, int LAT>
__device__ __forceinline__ double range_coord(const TrackRegs<L, LAT>& t, int range_mode)
{
    if (LAT != kFluorite || range_mode == 0) return t.z;
    const double* h = track_hdr(t);
    const double dx = t.x - h[0], dy = t.y - h[1], dz = t.z - h[2];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

// What the reverse sweep of the adjoint needs to know of a step's size: dt,
// and in code which term of the minimum set it (0: dt_max, 1: the speed term,
// 2: the acceleration term) plus whether the ion (rather than an atom) holds
// the largest speed (bit 2) and the largest acceleration (bit 3).
struct StepInfo {
    double dt;
    int code;
};

// One integration step (velocity Verlet with symmetric friction halves); a
// step with fresh == true has dt = 0 and builds the whole domain (start of a
// primary).  Returns the kinetic energy before the step via ke0, and the
// step's size via info when given, and the atoms a domain move drops via drop
// when given (see regenerate).
// Variants of the pair pass: bit 0, the interaction cut-off (compacted list);
// bit 1, the Firsov + Brandt-Kitagawa stopping (Firsov kernel instead of the
// exponential density weight, and the speed-dependent Brandt-Kitagawa friction).
constexpr int kVarCut = 1, kVarFirsov = 2;

template <int L, bool F32 = false, int LAT = kDiamond, int VAR = 0>
__device__ __forceinline__ void track_step(TrackRegs<L, LAT>& t, const KernelArgs& A, const SpeciesConst* sp, int sl,
                                           bool fresh, double& ke0, double& z0, StepInfo* info = nullptr,
                                           double* drop = nullptr)
{
    constexpr int FS = TrackRegs<L, LAT>::FS;
    constexpr bool FL = LAT == kFluorite;
    constexpr bool CUT = (VAR & kVarCut) != 0;
    constexpr bool FK = (VAR & kVarFirsov) != 0;
    static_assert(!(FK && F32), "the Firsov stopping variant has FP64 pair terms");
    // the run's scalar settings re-read from the argument segment at every step (scalar
    // loads), instead of registers held across the persistent loop that the allocator spills
    const KernelArgs C = cold_args();
    const SpeciesConst& c = sp[t.species];
    const PairConst& c1 = pair_table2(sp)[t.species];
    const double M1 = c.M1;
    const double v2 = t.vx * t.vx + t.vy * t.vy + t.vz * t.vz;
    const double f2 = t.Fx * t.Fx + t.Fy * t.Fy + t.Fz * t.Fz;
    const double vmax2 = fmax(v2, t.vmax2a);
    const double amax2 = fmax(f2 * c.inv_M1sq, t.amax2a);
    double dt = C.dt_max;
    if (vmax2 > 0.0) dt = fmin(dt, C.dx_max * rsqrt_pos(vmax2));
    if (amax2 > 0.0) dt = fmin(dt, sqrt(2.0 * C.dx_max * rsqrt_pos(amax2)));
    if (fresh) dt = 0.0;
    if (info != nullptr) {
        const bool by_a = amax2 > 0.0 && dt == sqrt(2.0 * C.dx_max * rsqrt_pos(amax2));
        const bool by_v = vmax2 > 0.0 && dt == C.dx_max * rsqrt_pos(vmax2);
        info->dt = dt;
        info->code = (by_a ? 2 : (by_v ? 1 : 0)) | ((v2 >= t.vmax2a) ? 4 : 0) |
                     ((f2 * c.inv_M1sq >= t.amax2a) ? 8 : 0);
    }
    ke0 = 0.5 * M1 * v2;
    z0 = range_coord(t, C.range_mode);

    const double h1 = dt * c.half_inv_M1;
    double g1 = c.g_const + c.g_rho * t.rho;
    if constexpr (FK) {
        const double pref = A.bk_pref[t.species];
        if (pref != 0.0) g1 += bk_friction(v2, pref, A.bk_z13[t.species], A.bk_vF, A.bk_inv_vunit);
    }
    const double fr1 = exp_neg(g1 * h1);
    t.vx = t.vx * fr1 + t.Fx * h1;
    t.vy = t.vy * fr1 + t.Fy * h1;
    t.vz = t.vz * fr1 + t.Fz * h1;
    t.x += t.vx * dt;
    t.y += t.vy * dt;
    t.z += t.vz * dt;

    if (fresh || !inside_cell(t.x, t.cx, C.a, C.inv_a) || !inside_cell(t.y, t.cy, C.a, C.inv_a) ||
        !inside_cell(t.z, t.cz, C.a, C.inv_a)) {
        const int ncx = floor_cell(t.x, C.a), ncy = floor_cell(t.y, C.a), ncz = floor_cell(t.z, C.a);
        if (fresh || ncx != t.cx || ncy != t.cy || ncz != t.cz) regenerate<L, LAT>(t, A, sl, ncx, ncy, ncz, fresh, drop);
    }

    // fused pass over every register slot (parked slots contribute exact zeros):
    // atom kick and drift, pair term at the new positions, second atom kick
    // (fluorite: register slot i holds anions from slot 128 on, a whole lane row
    // of one target species, so the choice of constants and mass is static)
    const double h2a = dt * C.half_inv_M2;
    const double h2b = FL ? dt * C.half_inv_M2b : h2a;
    constexpr int G = SegReduce<L>::G;
    double Fx[G], Fy[G], Fz[G], rho[G], rho1[G];
#pragma unroll
    for (int m = 0; m < G; ++m) Fx[m] = Fy[m] = Fz[m] = rho[m] = rho1[m] = 0.0;
    double vm = 0.0, fm = 0.0;
    if constexpr (CUT) {
        // Interaction cut-off: pair terms only for the atoms within sqrt(rc2) of the ion,
        // compacted so that the rounds over them take ceil(listed / L) passes instead of one
        // per register slot.
        static_assert(LAT == kDiamond && !F32, "the interaction cut-off is built for the diamond FP64 kernels");
        constexpr int SL = TrackRegs<L, LAT>::SL;
        int* list = reinterpret_cast<int*>(t.fl + 3 * FS + kTrackHdr);
        const int base = (threadIdx.x & 63) - sl;
        int count = 0;   // segment-uniform
        // (a) first half kick and drift of every slot; the new position of a slot within the
        //     cut-off is staged in its force entry (the old force is spent), zero otherwise,
        //     and the slots within are listed in increasing slot order
#pragma unroll
        for (int i = 0; i < SL; ++i) {
            double* f = t.fl + (sl + L * i);
            const double vx = t.avx[i] + f[0 * FS] * h2a;
            const double vy = t.avy[i] + f[1 * FS] * h2a;
            const double vz = t.avz[i] + f[2 * FS] * h2a;
            const double px = t.ax[i] + vx * dt;
            const double py = t.ay[i] + vy * dt;
            const double pz = t.az[i] + vz * dt;
            t.avx[i] = vx; t.avy[i] = vy; t.avz[i] = vz;
            t.ax[i] = px; t.ay[i] = py; t.az[i] = pz;
            const double dx = t.x - px, dy = t.y - py, dz = t.z - pz;
            const bool in = dx * dx + dy * dy + dz * dz <= C.rc2;
            f[0 * FS] = in ? px : 0.0;
            f[1 * FS] = in ? py : 0.0;
            f[2 * FS] = in ? pz : 0.0;
            const unsigned long long b = __ballot(in);
            const unsigned long long seg = (L == 64) ? b : ((b >> base) & ((1ull << (L % 64)) - 1ull));
            if (in) list[count + __popcll(seg & ((1ull << sl) - 1ull))] = sl + L * i;
            count += __popcll(seg);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // (b) pair terms over the list: entry j on lane j mod L in round j / L (empty entries
        //     of the last round take the parking distance, where every term is exactly 0);
        //     the sums follow the same column tree as the full pass, over list entries
#pragma unroll
        for (int k = 0; k < SL; ++k) {
            if (__all(k * L >= count)) break;
            const int m = k % G;
            const int j = k * L + sl;
            const bool valid = j < count;
            const int s = valid ? list[j] : 0;
            double dx = 0.0, dy = 0.0, dz = C.park;
            if (valid) {
                dx = t.x - t.fl[0 * FS + s];
                dy = t.y - t.fl[1 * FS + s];
                dz = t.z - t.fl[2 * FS + s];
            }
            double coef, ew;
            zbl_pair<FK>(c, dx, dy, dz, coef, ew);
            const double fx = -coef * dx, fy = -coef * dy, fz = -coef * dz;   // force on the atom
            Fx[m] -= fx; Fy[m] -= fy; Fz[m] -= fz;
            rho[m] += ew;
            if (valid) {
                t.fl[0 * FS + s] = fx;
                t.fl[1 * FS + s] = fy;
                t.fl[2 * FS + s] = fz;
            }
            fm = fmax(fm, fx * fx + fy * fy + fz * fz);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // (c) second half kick of every slot with its new force (zero beyond the cut-off)
#pragma unroll
        for (int i = 0; i < SL; ++i) {
            const double* f = t.fl + (sl + L * i);
            const double vx = t.avx[i] + f[0 * FS] * h2a;
            const double vy = t.avy[i] + f[1 * FS] * h2a;
            const double vz = t.avz[i] + f[2 * FS] * h2a;
            t.avx[i] = vx; t.avy[i] = vy; t.avz[i] = vz;
            vm = fmax(vm, vx * vx + vy * vy + vz * vz);
        }
        t.n_eval = count;
    } else {
    #pragma unroll
        for (int i = 0; i < TrackRegs<L, LAT>::SL; ++i) {
            const int m = i % G;   // column group of register slot i
            const bool anion = FL && L * i >= Lattice<LAT>::kAnion0;
            const double h2 = anion ? h2b : h2a;
            double* f = t.fl + (sl + L * i);
            double vx = t.avx[i] + f[0 * FS] * h2;
            double vy = t.avy[i] + f[1 * FS] * h2;
            double vz = t.avz[i] + f[2 * FS] * h2;
            const double px = t.ax[i] + vx * dt;
            const double py = t.ay[i] + vy * dt;
            const double pz = t.az[i] + vz * dt;
            const double dx = t.x - px, dy = t.y - py, dz = t.z - pz;
            double coef, ew;
            if (anion) {
                if constexpr (F32) zbl_pair_f32(c1, dx, dy, dz, coef, ew);
                else zbl_pair<FK>(c1, dx, dy, dz, coef, ew);
            } else {
                if constexpr (F32) zbl_pair_f32(c, dx, dy, dz, coef, ew);
                else zbl_pair<FK>(c, dx, dy, dz, coef, ew);
            }
            const double fx = -coef * dx, fy = -coef * dy, fz = -coef * dz;   // force on the atom
            Fx[m] -= fx; Fy[m] -= fy; Fz[m] -= fz;
            if (anion) rho1[m] += ew;
            else rho[m] += ew;
            vx += fx * h2; vy += fy * h2; vz += fz * h2;
            t.ax[i] = px; t.ay[i] = py; t.az[i] = pz;
            t.avx[i] = vx; t.avy[i] = vy; t.avz[i] = vz;
            f[0 * FS] = fx; f[1 * FS] = fy; f[2 * FS] = fz;
            vm = fmax(vm, vx * vx + vy * vy + vz * vz);
            if constexpr (FL) fm = fmax(fm, (fx * fx + fy * fy + fz * fz) * (anion ? C.inv_M2bsq : C.inv_M2sq));
            else fm = fmax(fm, fx * fx + fy * fy + fz * fz);
    #if REEDMD_PAIR_BARRIER
            __builtin_amdgcn_sched_barrier(0);
    #endif
        }
    }
    t.Fx = SegReduce<L>::csum(Fx);
    t.Fy = SegReduce<L>::csum(Fy);
    t.Fz = SegReduce<L>::csum(Fz);
    if constexpr (FL) {
        t.rho = SegReduce<L>::csum(rho) * c.wnorm + SegReduce<L>::csum(rho1) * c1.wnorm;
        t.vmax2a = SegReduce<L>::max(vm);
        t.amax2a = SegReduce<L>::max(fm);
    } else {
        t.rho = SegReduce<L>::csum(rho) * c.wnorm;
        t.vmax2a = SegReduce<L>::max(vm);
        t.amax2a = SegReduce<L>::max(fm) * C.inv_M2sq;
    }

    // second half kick, then the friction at the kicked speed
    const double kx = t.vx + t.Fx * h1, ky = t.vy + t.Fy * h1, kz = t.vz + t.Fz * h1;
    double g2 = c.g_const + c.g_rho * t.rho;
    if constexpr (FK) {
        const double pref = A.bk_pref[t.species];
        if (pref != 0.0) {
            const double w2 = kx * kx + ky * ky + kz * kz;
            g2 += bk_friction(w2, pref, A.bk_z13[t.species], A.bk_vF, A.bk_inv_vunit);
        }
    }
    const double fr2 = exp_neg(g2 * h1);
    t.vx = kx * fr2;
    t.vy = ky * fr2;
    t.vz = kz * fr2;
    if (!fresh) t.steps += 1;
}

// ---------------------------------------------------------------------------
// Record transfer (segment cooperative).  Layout as documented for
// reedmd_track_init; the atom fields have Lattice<LAT>::kSlots entries.
template <int L, int LAT>
__device__ __forceinline__ void store_record(const TrackRegs<L, LAT>& t, double* rec, int sl)
{
    constexpr int NS = Lattice<LAT>::kSlots;
    if (sl == 0) {
        const double* h = track_hdr(t);
        long long* ir = reinterpret_cast<long long*>(rec);
        rec[0] = t.x; rec[1] = t.y; rec[2] = t.z;
        rec[3] = t.vx; rec[4] = t.vy; rec[5] = t.vz;
        rec[6] = t.Fx; rec[7] = t.Fy; rec[8] = t.Fz;
        rec[9] = t.rho; rec[10] = t.w; rec[11] = t.zstop;
        ir[12] = t.cx; ir[13] = t.cy; ir[14] = t.cz;
        ir[15] = static_cast<long long>(t.key);
        ir[16] = t.steps; ir[17] = t.lineage;
        ir[18] = t.species; ir[19] = t.next_k; ir[20] = t.table; ir[21] = t.status;
        rec[22] = t.vmax2a;
        rec[23] = t.amax2a;
        ir[24] = 1;   // words 22-23 hold the atom speed and acceleration maxima
        const bool vac = h[6] >= 0.0;
        ir[25] = vac ? static_cast<long long>(h[3]) : 0;
        ir[26] = vac ? static_cast<long long>(h[4]) : 0;
        ir[27] = vac ? static_cast<long long>(h[5]) : 0;
        ir[28] = vac ? static_cast<long long>(h[6]) : -1;
        rec[29] = h[0]; rec[30] = h[1]; rec[31] = h[2];
    }
    double* at = rec + kHdr;
#pragma unroll
    for (int i = 0; i < TrackRegs<L, LAT>::SL; ++i) {
        const int s = sl + L * i;
        if (s >= NS) continue;
        const bool e = (t.exist >> i) & 1u;
        at[0 * NS + s] = e ? t.ax[i] : 0.0;
        at[1 * NS + s] = e ? t.ay[i] : 0.0;
        at[2 * NS + s] = e ? t.az[i] : 0.0;
        at[3 * NS + s] = e ? t.avx[i] : 0.0;
        at[4 * NS + s] = e ? t.avy[i] : 0.0;
        at[5 * NS + s] = e ? t.avz[i] : 0.0;
        at[6 * NS + s] = e ? t.fl[0 * TrackRegs<L, LAT>::FS + s] : 0.0;
        at[7 * NS + s] = e ? t.fl[1 * TrackRegs<L, LAT>::FS + s] : 0.0;
        at[8 * NS + s] = e ? t.fl[2 * TrackRegs<L, LAT>::FS + s] : 0.0;
    }
}

template <int L, int LAT>
__device__ __forceinline__ void load_record(TrackRegs<L, LAT>& t, const double* rec, int sl, const KernelArgs& A)
{
    using Lat = Lattice<LAT>;
    constexpr int NS = Lat::kSlots;
    const long long* ir = reinterpret_cast<const long long*>(rec);
    t.x = rec[0]; t.y = rec[1]; t.z = rec[2];
    t.vx = rec[3]; t.vy = rec[4]; t.vz = rec[5];
    t.Fx = rec[6]; t.Fy = rec[7]; t.Fz = rec[8];
    t.rho = rec[9]; t.w = rec[10]; t.zstop = rec[11];
    t.cx = static_cast<int>(ir[12]); t.cy = static_cast<int>(ir[13]); t.cz = static_cast<int>(ir[14]);
    t.key = static_cast<unsigned long long>(ir[15]);
    t.steps = ir[16]; t.lineage = ir[17];
    t.species = static_cast<int>(ir[18]); t.next_k = static_cast<int>(ir[19]);
    t.table = static_cast<int>(ir[20]); t.status = static_cast<int>(ir[21]);
    if (t.species < 0 || t.species >= A.n_species) {
        t.species = 0;
        t.status = REEDMD_LOST;
    }
    double* h = track_hdr(t);
    h[0] = rec[29]; h[1] = rec[30]; h[2] = rec[31];
    h[3] = static_cast<double>(ir[25]); h[4] = static_cast<double>(ir[26]); h[5] = static_cast<double>(ir[27]);
    h[6] = (ir[28] >= 0 && ir[28] < Lat::kCellAtoms) ? static_cast<double>(ir[28]) : -1.0;
    const double* at = rec + kHdr;
    constexpr int FS = TrackRegs<L, LAT>::FS;
    const KernelArgs C = cold_args();
    const double parkx = C.a * (static_cast<double>(t.cx) + 0.5);
    const double parky = C.a * (static_cast<double>(t.cy) + 0.5);
    const double parkz = C.a * (static_cast<double>(t.cz) + 0.5) - C.park;
    unsigned ex = 0;
    double vm = 0.0, fm = 0.0;
#pragma unroll
    for (int i = 0; i < TrackRegs<L, LAT>::SL; ++i) {
        const int s = sl + L * i;
        const int cell = (s < NS) ? Lat::cell_of_slot(s) : -1;
        if (cell < 0 || cell_of_residue(cell % 3, t.cz) < 0 ||
            (LAT == kFluorite &&
             vacant_site(h, cell_of_residue(cell / 9, t.cx), cell_of_residue((cell / 3) % 3, t.cy),
                         cell_of_residue(cell % 3, t.cz), Lat::basis_of_slot(s)))) {
            park_slot<L, LAT>(t, i, s, parkx, parky, parkz);
            continue;
        }
        t.ax[i] = at[0 * NS + s]; t.ay[i] = at[1 * NS + s]; t.az[i] = at[2 * NS + s];
        t.avx[i] = at[3 * NS + s]; t.avy[i] = at[4 * NS + s]; t.avz[i] = at[5 * NS + s];
        const double fx = at[6 * NS + s], fy = at[7 * NS + s], fz = at[8 * NS + s];
        t.fl[0 * FS + s] = fx; t.fl[1 * FS + s] = fy; t.fl[2 * FS + s] = fz;
        ex |= (1u << i);
        vm = fmax(vm, t.avx[i] * t.avx[i] + t.avy[i] * t.avy[i] + t.avz[i] * t.avz[i]);
        const bool anion = LAT == kFluorite && L * i >= Lat::kAnion0;
        fm = fmax(fm, (fx * fx + fy * fy + fz * fz) * (anion ? A.inv_M2bsq : A.inv_M2sq));
    }
    t.exist = ex;
    t.n_exist = SegReduce<L>::isum(__popc(ex));
    if (sl == 0) reinterpret_cast<volatile int*>(track_hdr(t) + kExistWord)[0] = t.n_exist;
    if (ir[24] == 1) {
        // maxima stored by this library: reuse them so that a reloaded record continues
        // bitwise like the track that wrote it
        t.vmax2a = rec[22];
        t.amax2a = rec[23];
    } else {
        t.vmax2a = SegReduce<L>::max(vm);
        t.amax2a = SegReduce<L>::max(fm);
    }
}

// Starting state of batch entry q (the fresh step that builds the domain and
// evaluates the first forces is done by the caller).
template <int L, int LAT>
__device__ __forceinline__ void start_primary(TrackRegs<L, LAT>& t, const KernelArgs& A, const SpeciesConst* sp,
                                              long long q)
{
    t.species = A.species[q];
    t.table = A.table[q];
    t.status = REEDMD_ACTIVE;
    if (t.species < 0 || t.species >= A.n_species || (A.n_thresh > 0 && (t.table < 0 || t.table >= A.n_tables))) {
        // invalid batch entry: never stepped, booked as lost (quarantined weight)
        t.status = REEDMD_LOST;
        t.species = 0;
        t.table = 0;
    }
    const SpeciesConst& c = sp[t.species];
    const double dx = A.dir[q], dy = A.dir[A.n + q], dz = A.dir[2 * A.n + q];
    const double dn = sqrt(dx * dx + dy * dy + dz * dz);
    const double speed = sqrt(2.0 * A.energy[q] / c.M1);
    t.x = A.pos[q]; t.y = A.pos[A.n + q]; t.z = A.pos[2 * A.n + q];
    t.vx = speed * dx / dn; t.vy = speed * dy / dn; t.vz = speed * dz / dn;
    {
        // start point; a recoil leaves the basis-0 site of the cell whose origin is
        // nearest its start point empty
        double* h = track_hdr(t);
        const KernelArgs C = cold_args();
        h[0] = t.x; h[1] = t.y; h[2] = t.z;
        h[3] = floor(t.x * C.inv_a + 0.25);
        h[4] = floor(t.y * C.inv_a + 0.25);
        h[5] = floor(t.z * C.inv_a + 0.25);
        h[6] = C.vacancy ? 0.0 : -1.0;
    }
    t.Fx = 0.0; t.Fy = 0.0; t.Fz = 0.0;
    t.rho = 0.0; t.w = 1.0; t.zstop = 0.0;
    t.vmax2a = 0.0; t.amax2a = 0.0;
    t.cx = kSentinel; t.cy = kSentinel; t.cz = kSentinel;
    t.key = A.key[q];
    t.steps = 0;
    t.lineage = A.id0 + q;
    t.next_k = 0;
}

// Termination events after a step: non-finite state, stop (depth linearly
// interpolated in kinetic energy within the step), backscatter, step cap.
template <int L, int LAT>
__device__ __forceinline__ int track_events(TrackRegs<L, LAT>& t, const KernelArgs& A, const SpeciesConst* sp,
                                            double ke0, double z0)
{
    const KernelArgs C = cold_args();
    const bool finite = isfinite(t.x) && isfinite(t.y) && isfinite(t.z) && isfinite(t.vx) &&
                        isfinite(t.vy) && isfinite(t.vz);
    if (!finite) return REEDMD_NONFINITE;
    const double ke = 0.5 * sp[t.species].M1 * (t.vx * t.vx + t.vy * t.vy + t.vz * t.vz);
    if (ke < C.E_stop) {
        const double zr = range_coord(t, C.range_mode);
        t.zstop = (ke0 > C.E_stop) ? z0 + (zr - z0) * (ke0 - C.E_stop) / (ke0 - ke) : z0;
        return REEDMD_STOPPED;
    }
    if (t.z < C.z_start && t.vz < 0.0) return REEDMD_BACKSCATTERED;
    if (C.max_steps > 0 && t.steps >= C.max_steps) return REEDMD_STEPCAP;
    return REEDMD_ACTIVE;
}

__device__ __forceinline__ void add_f64(double* p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void add_i64(long long* p, long long v)
{
    atomicAdd(reinterpret_cast<unsigned long long*>(p), static_cast<unsigned long long>(v));
}
__device__ __forceinline__ void add_i64(int64_t* p, long long v)
{
    atomicAdd(reinterpret_cast<unsigned long long*>(p), static_cast<unsigned long long>(v));
}

// Re-places one depth table (Sec. 2: depths from the statistics gathered so far; Sec. 3:
// criteria updated between complete tracks).  h: the table's stopped weight per depth bin and
// beyond the last bin (n_bins + 1 entries); total: all weight booked for the table; d: on entry
// the previous depths, on return the new ones.  S(z) = (stopped weight with z_stop >= z) / (all booked
// weight) at the bin edges; depth k is where S falls to probs[k], linear in S inside the bin.
// The targets placed this way are the leading ones; the rest, those S does not reach within the
// histogram or that the statistics are too thin for (probs[k] * booked weight < min_weight: less
// than that much weight is expected beyond it; the targets decrease, so the rest are too), keep
// their depths shifted by the move of the last placed depth (unshifted when none is placed);
// then every depth is raised to at least the previous one plus min_gap.
__device__ inline void refine_table(const double* h, double total, int n_bins, double bin_width, int n_thresh,
                                    const double* probs, double min_gap, double min_weight, double* d)
{
    int resolvable = 0;
    while (resolvable < n_thresh && probs[resolvable] * total >= min_weight) ++resolvable;
    if (total > 0.0 && resolvable > 0) {
        double beyond = h[n_bins];                 // stopped weight at or beyond the lower edge of bin b
        for (int b = n_bins - 1; b >= 0; --b) beyond += h[b];
        double s_lo = beyond / total;
        int k = 0;
        double moved = 0.0;                        // move of the last placed depth
        for (int b = 0; b < n_bins && k < resolvable; ++b) {
            beyond -= h[b];
            const double s_hi = beyond / total;
            while (k < resolvable && probs[k] >= s_hi) {
                const double nd = (probs[k] < s_lo)
                                      ? (static_cast<double>(b) + (s_lo - probs[k]) / (s_lo - s_hi)) * bin_width
                                      : static_cast<double>(b) * bin_width;
                moved = nd - d[k];
                d[k] = nd;
                ++k;
            }
            s_lo = s_hi;
        }
        if (k > 0)
            for (int j = k; j < n_thresh; ++j) d[j] += moved;
    }
    for (int k = 1; k < n_thresh; ++k) d[k] = fmax(d[k], d[k - 1] + min_gap);
}

// First claim position of epoch e (ceil(n e / E)).
__device__ __forceinline__ long long epoch_first(long long n, int E, int e)
{
    return (n * e + E - 1) / E;
}

// Table version e of an in-launch refinement, computed by the L lanes of one segment:
// copies every table's statistics as they stand into the snapshot (the lanes take the entries
// in turn; each finished track is booked into exactly one entry of its table's row, so a
// snapshot taken while tracks finish still holds only whole tracks' weights, and its total, the
// sum of the row, is what the row was made of), then lane sl re-places tables sl, sl + L, ...
// from the snapshot starting from version 0 (the caller's depths; a version depends on no other
// version, so nothing waits while it is computed), and publishes the version.  The snapshot
// rows are zero on entry; their last entry receives the total.  Inlined: as a call, the
// registers the call clobbers changed the allocation of the whole kernel and put spill stores
// into the step loop's pair pass.
__device__ __forceinline__ void compute_version(const double* tstat, double* snap_all, double* thr, const double* probs,
                                             double min_gap, double min_weight, double bin_width, int nb, int nt,
                                             int nk, int e, int sl, int L, int* ready)
{
    const size_t sw = static_cast<size_t>(nb + 2);
    for (int tb = 0; tb < nt; ++tb) {
        const double* live = tstat + static_cast<size_t>(tb) * sw;
        double* snap = snap_all + (static_cast<size_t>(e) * nt + tb) * sw;
        double part = 0.0;
        for (size_t i = static_cast<size_t>(sl); i < sw; i += static_cast<size_t>(L)) {
            const double v = __hip_atomic_load(&live[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (i + 1 < sw) snap[i] = v;
            part += v;
        }
        // weights are sums of powers of two: the total is exact in any order
        if (part != 0.0) unsafeAtomicAdd(&snap[sw - 1], part);
    }
    __threadfence();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    for (int tb = sl; tb < nt; tb += L) {
        double* snap = snap_all + (static_cast<size_t>(e) * nt + tb) * sw;
        const double total = __hip_atomic_load(&snap[sw - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const double* first = thr + static_cast<size_t>(tb) * nk;
        double* d = thr + (static_cast<size_t>(e) * nt + tb) * nk;
        for (int k = 0; k < nk; ++k) d[k] = first[k];
        refine_table(snap, total, nb, bin_width, nk, probs, min_gap, min_weight, d);
    }
    __threadfence();
    if (sl == 0) __hip_atomic_store(&ready[e], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Books a finished track (segment leader only).
__device__ __forceinline__ void book_finished(const KernelArgs& A, int status, double w, double zstop,
                                              long long lineage, int next_k, long long steps, int table,
                                              unsigned long long key)
{
    reedmd_stats* S = A.stats;
    if (A.tstat != nullptr && table >= 0) {
        // per-table survival statistics for adaptive cloning depths, each track's weight in
        // exactly one entry: its depth bin, beyond the last bin, or (not stopped in the crystal)
        // the last entry; the row's sum is all weight booked for the table (the table field of
        // a track also carries its table version: version * n_tables + table)
        double* ts = A.tstat + static_cast<size_t>(table % A.n_tables) * (A.n_bins + 2);
        int entry = A.n_bins + 1;
        if (status == REEDMD_STOPPED && zstop >= 0.0) {
            const double fb = floor(zstop / A.bin_width);
            entry = (fb < static_cast<double>(A.n_bins)) ? static_cast<int>(fb) : A.n_bins;
        }
        add_f64(&ts[entry], w);
    }
    add_i64(&S->finished, 1);
    if (status == REEDMD_STOPPED) {
        add_i64(&S->n_stopped, 1);
        add_f64(&S->w_stopped, w);
        if (zstop < 0.0) {
            add_f64(&S->w_underflow, w);
        } else {
            const double fb = floor(zstop / A.bin_width);
            if (!(fb < static_cast<double>(A.n_bins))) add_f64(&S->w_overflow, w);
            else add_f64(&A.hist[static_cast<int>(fb)], w);
        }
        add_f64(&S->sum_wz, w * zstop);
        add_f64(&S->sum_wz2, w * zstop * zstop);
    } else if (status == REEDMD_BACKSCATTERED) {
        add_i64(&S->n_backscattered, 1);
        add_f64(&S->w_backscattered, w);
    } else if (status == REEDMD_CANCELLED) {
        add_i64(&S->n_cancelled, 1);
        add_f64(&S->w_cancelled, w);
    } else {
        if (status == REEDMD_NONFINITE) add_i64(&S->n_nonfinite, 1);
        else add_i64(&S->n_stepcap, 1);
        add_f64(&S->w_quarantined, w);
    }
    if (A.log != nullptr) {
        const long long i = static_cast<long long>(
            atomicAdd(reinterpret_cast<unsigned long long*>(&A.q->log_next), 1ull));
        if (i < A.log_cap) {
            reedmd_result* r = &A.log[i];
            r->lineage = lineage;
            r->status = status;
            r->next_k = next_k;
            r->z_stop = zstop;
            r->w = w;
            r->steps = steps;
            r->key = key;
        }
    }
}

// ---------------------------------------------------------------------------
// Clone queue operations (segment leader), acquire/release at agent scope.
__device__ __forceinline__ long long queue_reserve_push(const KernelArgs& A)
{
    QueueState* q = A.q;
    unsigned long long pos = __hip_atomic_load(&q->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int tries = 0; tries < 256; ++tries) {
        const unsigned long long seq =
            __hip_atomic_load(&A.qseq[pos % A.qcap], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if (seq == pos) {
            unsigned long long expect = pos;
            if (__hip_atomic_compare_exchange_strong(&q->tail, &expect, pos + 1, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                return static_cast<long long>(pos);
            pos = expect;
        } else if (seq < pos) {
            return -1;  // full
        } else {
            pos = __hip_atomic_load(&q->tail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    return -1;
}

__device__ __forceinline__ long long queue_reserve_pop(const KernelArgs& A)
{
    QueueState* q = A.q;
    unsigned long long pos = __hip_atomic_load(&q->head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int tries = 0; tries < 256; ++tries) {
        const unsigned long long seq =
            __hip_atomic_load(&A.qseq[pos % A.qcap], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        if (seq == pos + 1) {
            unsigned long long expect = pos;
            if (__hip_atomic_compare_exchange_strong(&q->head, &expect, pos + 1, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                return static_cast<long long>(pos);
            pos = expect;
        } else if (seq < pos + 1) {
            return -1;  // empty
        } else {
            pos = __hip_atomic_load(&q->head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    return -1;
}

// ---------------------------------------------------------------------------
// Main track kernel: PLAIN (static grid-stride assignment of primaries, clones
// depth first on a per-segment stack) or PERSISTENT (primaries and clones taken
// from device counters and the clone queue until no track is live).
enum : int { kSegNeed = 0, kSegRun = 1, kSegDone = 2 };

template <int L, int MODE, bool F32 = false, int LAT = kDiamond, int VAR = 0>
__global__ void __launch_bounds__(256, REEDMD_WAVES_PER_SIMD(L, LAT)) track_kernel(const KernelArgs A0)
{
    const KernelArgs& A = A0;
    __shared__ double s_sp[kSpeciesLdsDoubles];
    __shared__ double s_force[ForceLds<L, LAT, (VAR & kVarCut) != 0>::kDoubles];
    const SpeciesConst* sp = stage_species(A, s_sp);
    const int lane = threadIdx.x & 63;
    const int sl = lane % L;
    const int seg_in_wave = lane / L;
    const int leader = lane - sl;
    const long long wave = static_cast<long long>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const long long seg = wave * (64 / L) + seg_in_wave;

    constexpr int RW = Lattice<LAT>::kRecWords;
    TrackRegs<L, LAT> t;
    t.fl = force_slab<L, LAT, (VAR & kVarCut) != 0>(s_force);
    t.cx = t.cy = t.cz = kSentinel;
    t.exist = 0;
    t.n_exist = 0;
    int mode = (seg < A.seg_total) ? kSegNeed : kSegDone;
    long long next_primary = seg;
    int top = 0;
    bool fresh = false;
    // steps and pair terms of the running track not yet booked: two 32-bit counters in the
    // track's LDS header, added to by the segment leader every step (a fire-and-forget LDS add
    // instead of a register that the allocator spills and reloads every step) and booked at
    // every poll, every 256 steps of the track, and when the track ends or moves
    unsigned* const cnt = reinterpret_cast<unsigned*>(t.fl + 3 * TrackRegs<L, LAT>::FS + kCountWord);
    auto book_counts = [&](const KernelArgs& C) {
        const unsigned long long v = *reinterpret_cast<volatile unsigned long long*>(cnt);
        *reinterpret_cast<volatile unsigned long long*>(cnt) = 0ull;
        add_i64(&C.stats->track_steps, static_cast<long long>(v & 0xffffffffull));
        add_i64(&C.stats->pair_evals, static_cast<long long>(v >> 32));
    };
    if (sl == 0) *reinterpret_cast<volatile unsigned long long*>(cnt) = 0ull;
    bool cancelled = false;
    bool handoff_now = false;
    double* my_stack = A.stack + static_cast<size_t>(seg < A.seg_total ? seg : 0) *
                                     static_cast<size_t>(A.stack_cap) * RW;

    for (;;) {
        if (mode == kSegNeed) {
            handoff_now = false;
            const KernelArgs A = cold_args();
            if (A.cancel != nullptr) {
                int cv = 0;
                if (sl == 0) cv = __hip_atomic_load(A.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                cancelled = __shfl(cv, leader, 64) != 0;
            }
            // after the tail handoff this launch takes nothing from the queue: what is there
            // (and whatever its segments still hold) is for the 64-lane tail launch
            int hflag = 0;
            if (MODE == kModePersistent && A.handoff_live > 0 && !A.tail) {
                if (sl == 0) hflag = static_cast<int>(__hip_atomic_load(&A.q->handoff, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                hflag = __shfl(hflag, leader, 64);
            }
            bool got = false;
            if (top > 0) {
                --top;
                load_record<L, LAT>(t, my_stack + static_cast<size_t>(top) * RW, sl, A);
                refresh_threshold(t, A);
                got = true;
                handoff_now = hflag != 0;
            } else if (MODE == kModePersistent && A.qcap > 0 && !hflag) {
                long long slot = -1;
                if (sl == 0) slot = queue_reserve_pop(A);
                slot = __shfl(slot, leader, 64);
                if (slot >= 0) {
                    const double* rec = A.qrec + static_cast<size_t>(slot % A.qcap) * RW;
                    load_record<L, LAT>(t, rec, sl, A);
                    refresh_threshold(t, A);
                    __threadfence();
                    if (sl == 0)
                        __hip_atomic_store(&A.qseq[slot % A.qcap], static_cast<unsigned long long>(slot) + A.qcap,
                                           __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    got = true;
                }
            }
            if (!got) {
                long long qi = -1;
                if (MODE == kModePlain) {
                    if (next_primary < A.n) {
                        qi = next_primary;
                        next_primary += A.seg_total;
                    }
                } else {
                    if (sl == 0 && !A.tail && !hflag) {
                        const long long cur = __hip_atomic_load(&A.q->prim_next, __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_AGENT);
                        if (cur < A.n) qi = atomicAdd(reinterpret_cast<unsigned long long*>(&A.q->prim_next), 1ull);
                    }
                    qi = __shfl(qi, leader, 64);
                    if (qi >= A.n) qi = -1;
                }
                int version = 0;
                if (MODE == kModePersistent && A.refine_E > 1) {
                    // in-launch refinement: the epoch of this claim position; its first claimer
                    // computes the epoch's table version (which waits for nothing), then every
                    // segment of a later epoch waits until its version is published (by this
                    // segment, by another segment of this wave in the step above, or by
                    // another wave)
                    if (qi >= 0) version = static_cast<int>((qi * A.refine_E) / A.n);
                    if (qi >= 0 && version > 0 && qi == epoch_first(A.n, A.refine_E, version))
                        compute_version(A.tstat, A.r_snap, const_cast<double*>(A.thr), A.r_probs, A.r_min_gap,
                                        A.r_min_weight, A.bin_width, A.n_bins, A.n_tables, A.n_thresh, version, sl,
                                        L, A.r_ready);
                    if (qi >= 0 && version > 0) {
                        if (sl == 0)
                            while (__hip_atomic_load(&A.r_ready[version], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0)
                                __builtin_amdgcn_s_sleep(4);
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    }
                }
                if (qi >= 0) {
                    start_primary<L, LAT>(t, A, sp, A.order != nullptr ? A.order[qi] : qi);
                    if (t.status != REEDMD_LOST) t.table += version * A.n_tables;
                    if (t.status != REEDMD_LOST) refresh_threshold(t, A);
                    if (sl == 0) add_i64(&A.stats->primaries, 1);
                    fresh = true;
                    got = true;
                }
            }
            if (got) {
                mode = kSegRun;
                if (t.status == REEDMD_LOST) {
                    // invalid species or table index: weight quarantined, error flagged
                    if (sl == 0) {
                        book_finished(A, REEDMD_LOST, t.w, 0.0, t.lineage, t.next_k, t.steps, -1, t.key);
                        add_i64(&A.stats->error_flags, 1);
                        if (MODE == kModePersistent) add_i64(&A.q->live, -1);
                    }
                    mode = kSegNeed;
                    fresh = false;
                } else if (cancelled) {
                    // drain: the track ends where it is, its weight is booked as cancelled
                    if (sl == 0) {
                        book_finished(A, REEDMD_CANCELLED, t.w, 0.0, t.lineage, t.next_k, t.steps, t.table, t.key);
                        if (MODE == kModePersistent) add_i64(&A.q->live, -1);
                    }
                    mode = kSegNeed;
                    fresh = false;
                }
            } else if (MODE == kModePlain) {
                mode = kSegDone;
            } else {
                // nothing to take: leave when no track is live, or when the tail is handed to the
                // wider kernel (every primary claimed and few tracks live; this segment's stack
                // is empty and what is in the queue stays there for the tail kernel)
                long long live = 0;
                int h = 0;
                if (sl == 0) {
                    live = __hip_atomic_load(&A.q->live, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (A.handoff_live > 0 && !A.tail && live > 0) {
                        h = hflag;
                        if (!h && live <= A.handoff_live &&
                            __hip_atomic_load(&A.q->prim_next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= A.n) {
                            __hip_atomic_store(&A.q->handoff, 1ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            h = 1;
                        }
                    }
                    if (A.tail && live > 0) {
                        // leave if the segments that stay (this one gone) are still at least the
                        // reserve; the count is taken first, so concurrent leavers cannot
                        // undercut it
                        const long long keep = live * 2 > kTailReserve ? live * 2 : kTailReserve;
                        const long long gone =
                            static_cast<long long>(atomicAdd(reinterpret_cast<unsigned long long*>(&A.q->tail_left), 1ull)) + 1;
                        if (A.seg_total - gone >= keep) h = 1;
                        else add_i64(&A.q->tail_left, -1);
                    }
                }
                live = __shfl(live, leader, 64);
                h = __shfl(h, leader, 64);
                if (live <= 0 || h) mode = kSegDone;
            }
        }
        if (__all(mode == kSegDone)) break;
        if (mode != kSegRun) {
            __builtin_amdgcn_s_sleep(8);
            continue;
        }

        // ---- one step of a running track ----
        double ke0, z0;
        track_step<L, F32, LAT, VAR>(t, A, sp, sl, fresh, ke0, z0);
        if (sl == 0) {
            const int ne = (VAR & kVarCut) != 0 ? t.n_eval
                                                 : reinterpret_cast<volatile int*>(track_hdr(t) + kExistWord)[0];
            __hip_atomic_fetch_add(&cnt[1], static_cast<unsigned>(ne), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (!fresh) __hip_atomic_fetch_add(&cnt[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        if (fresh) {
            fresh = false;
            continue;
        }
        int st = track_events<L, LAT>(t, A, sp, ke0, z0);
        // poll (cancel word, tail handoff) and book the counts every 256 steps of the track
        if (st == REEDMD_ACTIVE && (t.steps & 255) == 0) {
            const KernelArgs C = cold_args();
            if (sl == 0) book_counts(C);
            if (C.cancel != nullptr) {
                int cv = 0;
                if (sl == 0) cv = __hip_atomic_load(C.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                if (__shfl(cv, leader, 64) != 0) st = REEDMD_CANCELLED;
            }
            if (MODE == kModePersistent && C.handoff_live > 0 && !C.tail) {
                int h = 0;
                if (sl == 0) h = static_cast<int>(__hip_atomic_load(&C.q->handoff, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                handoff_now = __shfl(h, leader, 64) != 0;
            }
        }
        if (st != REEDMD_ACTIVE) {
            handoff_now = false;
            const KernelArgs A = cold_args();
            if (sl == 0) {
                book_finished(A, st, t.w, t.zstop, t.lineage, t.next_k, t.steps, t.table, t.key);
                book_counts(A);
                if (MODE == kModePersistent) add_i64(&A.q->live, -1);
            }
            mode = kSegNeed;
            continue;
        }
        // cloning at depth thresholds (Sec. 2): weight / n_clones, new keys
        const double zr = range_coord(t, A.range_mode);
        if (zr >= t.thr_next) {
            const KernelArgs A = cold_args();
            while (t.next_k < A.n_thresh && zr >= t.thr_next) {
                const int k = t.next_k;
                const unsigned long long parent = t.key;
                t.w = t.w / static_cast<double>(A.n_clones);
                t.next_k = k + 1;
                for (int i = A.n_clones - 1; i >= 1; --i) {
                    t.key = child_key(parent, A.seed, k, i);
                    long long slot = -1;
                    if (MODE == kModePersistent && A.qcap > 0) {
                        if (sl == 0) slot = queue_reserve_push(A);
                        slot = __shfl(slot, leader, 64);
                    }
                    if (slot >= 0) {
                        if (sl == 0) add_i64(&A.q->live, 1);
                        store_record<L, LAT>(t, A.qrec + static_cast<size_t>(slot % A.qcap) * RW, sl);
                        __threadfence();
                        if (sl == 0) {
                            __hip_atomic_store(&A.qseq[slot % A.qcap], static_cast<unsigned long long>(slot) + 1,
                                               __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                            const long long d = static_cast<long long>(slot) + 1 -
                                                static_cast<long long>(__hip_atomic_load(
                                                    &A.q->head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
                            atomicMax(reinterpret_cast<unsigned long long*>(&A.stats->max_queue),
                                      static_cast<unsigned long long>(d > 0 ? d : 0));
                        }
                    } else if (top < A.stack_cap) {
                        if (MODE == kModePersistent && sl == 0) {
                            add_i64(&A.q->live, 1);
                            if (A.qcap > 0) add_i64(&A.stats->stack_overflow, 1);
                        }
                        store_record<L, LAT>(t, my_stack + static_cast<size_t>(top) * RW, sl);
                        ++top;
                    } else {
                        // no room anywhere: the clone's weight is quarantined (ledger stays exact)
                        if (sl == 0) {
                            add_f64(&A.stats->w_quarantined, t.w);
                            add_i64(&A.stats->error_flags, 1);
                        }
                    }
                    if (sl == 0) add_i64(&A.stats->clones, 1);
                }
                t.key = child_key(parent, A.seed, k, 0);
                refresh_threshold(t, A);
            }
        }
        if (MODE == kModePersistent && handoff_now) {
            // tail handoff, after this step's events and cloning: the track goes to the queue
            // as it stands (the record round trip is exact and the segment sums do not depend
            // on the lanes per track, so the wider kernel continues it bit for bit).  If the
            // queue has no room the track goes on here and tries again at the next poll.
            handoff_now = false;
            const KernelArgs C = cold_args();
            long long slot = -1;
            if (sl == 0) slot = queue_reserve_push(C);
            slot = __shfl(slot, leader, 64);
            if (slot >= 0) {
                store_record<L, LAT>(t, C.qrec + static_cast<size_t>(slot % C.qcap) * RW, sl);
                __threadfence();
                if (sl == 0) {
                    __hip_atomic_store(&C.qseq[slot % C.qcap], static_cast<unsigned long long>(slot) + 1,
                                       __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    add_i64(&C.stats->handed_off, 1);
                    book_counts(C);
                }
                mode = kSegNeed;
            }
        }
    }
}

// Builds the starting record of every batch entry (debug / parity entry point).
template <int L, bool F32 = false, int LAT = kDiamond, int VAR = 0>
__global__ void __launch_bounds__(256) init_kernel(const KernelArgs A)
{
    __shared__ double s_sp[kSpeciesLdsDoubles];
    __shared__ double s_force[ForceLds<L, LAT, (VAR & kVarCut) != 0>::kDoubles];
    const SpeciesConst* sp = stage_species(A, s_sp);
    const int lane = threadIdx.x & 63;
    const int sl = lane % L;
    const long long seg = (static_cast<long long>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6)) * (64 / L) + lane / L;
    if (seg >= A.n) return;
    TrackRegs<L, LAT> t;
    t.fl = force_slab<L, LAT, (VAR & kVarCut) != 0>(s_force);
    t.exist = 0;
    start_primary<L, LAT>(t, A, sp, seg);
    double ke0, z0;
    if (t.status != REEDMD_LOST) track_step<L, F32, LAT, VAR>(t, A, sp, sl, true, ke0, z0);
    store_record<L, LAT>(t, A.records + static_cast<size_t>(seg) * Lattice<LAT>::kRecWords, sl);
}

// Advances caller records by nsteps steps without events (debug / parity).
template <int L, bool F32 = false, int LAT = kDiamond, int VAR = 0>
__global__ void __launch_bounds__(256, 2) step_kernel(const KernelArgs A)
{
    __shared__ double s_sp[kSpeciesLdsDoubles];
    __shared__ double s_force[ForceLds<L, LAT, (VAR & kVarCut) != 0>::kDoubles];
    const SpeciesConst* sp = stage_species(A, s_sp);
    const int lane = threadIdx.x & 63;
    const int sl = lane % L;
    const long long seg = (static_cast<long long>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6)) * (64 / L) + lane / L;
    if (seg >= A.n) return;
    TrackRegs<L, LAT> t;
    t.fl = force_slab<L, LAT, (VAR & kVarCut) != 0>(s_force);
    double* rec = A.records + static_cast<size_t>(seg) * Lattice<LAT>::kRecWords;
    load_record<L, LAT>(t, rec, sl, A);
    if (t.status == REEDMD_LOST) return;   // invalid species index: record left as it was
    for (int s = 0; s < A.nsteps; ++s) {
        double ke0, z0;
        track_step<L, F32, LAT, VAR>(t, A, sp, sl, false, ke0, z0);
    }
    store_record<L, LAT>(t, rec, sl);
}

}  // namespace reedmd
