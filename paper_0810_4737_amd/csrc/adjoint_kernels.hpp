// Reverse-mode (adjoint) derivative of the stopping depth of each track with
// respect to the electronic-stopping scale k and the screening-length scale s.
//
// One wavefront (64 lanes, the same slot layout as the track kernel) per
// track.  Forward: the track runs to termination with the ordinary step, a
// checkpoint of its full state every 64 steps, and a log of each step's size
// (dt and which term of the minimum set it) and of the ion's position and
// velocity before it.  Reverse: from the final state, step by step, the state
// before a step is rebuilt from the state after it: the ion from the log, the
// domain atoms by running their part of the step backwards (they feel only the
// ion, so the inverse is explicit: undo the second kick and the drift, evaluate
// the pair terms at the rebuilt positions, undo the first kick), and the
// adjoint of the step is applied in the same pass over the slots.  Atoms that
// a domain move dropped come back from a log the forward writes at each move;
// atoms it created are constants, so their adjoints end at the move.  The state is re-anchored to the
// exact checkpoint at every segment boundary, so reconstruction errors never
// grow over more than 64 steps.  Adjoint state per domain atom (position,
// velocity, force) and the pair terms of the current state live in VGPRs; the
// ion's adjoints are wavefront-uniform.
//
// Per step, forward (see track_step):
//   dt = min(dt_max, dx vmax^-1, sqrt(2 dx) amax^-1/2); h1 = dt/2M1; h2 = dt/2M2
//   v1 = v e^{-g(rho) h1} + F h1;  x1 = x + v1 dt
//   U_j = V_j + f_j h2;  Y_j = X_j + U_j dt          (kept atoms; created atoms are constants)
//   c_j = -V'(r_j; s)/r_j, d_j = x1 - Y_j: F' = sum c_j d_j, f'_j = -c_j d_j, rho' = sum w(r_j)
//   V'_j = U_j + f'_j h2;  v' = (v1 + F' h1) e^{-g(rho') h1}
// with g(rho) = g_const + g_rho rho (both proportional to k), and
//   dc/dr = zz (3 phi'/(a r^3) - 3 phi/r^4 - phi''/(a^2 r^2)),  dc/ds = zz phi''/(s a^2 r).
// The stopping depth z + (z1 - z)(ke0 - E)/(ke0 - ke1) of the last step seeds
// the adjoint.  The active term of the step-size minimum and the particle that
// attains the maximum carry the derivative of dt.
#pragma once
#include "track_kernels.hpp"

namespace reedmd {

// Adjoint of the ion (wavefront-uniform) and of the domain atoms (by register slot).
struct AdjIon {
    double xb[3], vb[3], Fb[3], rhob;
    double kb;            // d z_stop / d k (wavefront-uniform)
};

template <int L>
struct AdjAtoms {
    static constexpr int SL = TrackRegs<L>::SL;
    double Xb[3][SL], Vb[3][SL], fb[3][SL];
};

// Pair term of one atom at squared distance r2 with its derivatives: the force
// coefficient c = -V'(r)/r, dc/dr and dc/ds, the density weight w (normalised)
// and r, 1/r.  The exponentials are the step's (base-2 rates folded per species).
__device__ __forceinline__ void zbl_pair_adjoint(const SpeciesConst& sc, double inv_s, double r2, double& r,
                                                 double& inv_r, double& c, double& c_r, double& c_s, double& w)
{
    const double inv_a = sc.inv_a, zz = sc.zz;
    inv_r = rsqrt_pos(r2);
    r = r2 * inv_r;
    const double e0 = exp2_neg_pair(r, sc.rate[0]);
    const double e1 = exp2_neg_pair(r, sc.rate[1]);
    const double e2 = exp2_neg_pair(r, sc.rate[2]);
    const double e3 = exp2_neg_pair(r, sc.rate[3]);
    const double phi = kZc0 * e0 + kZc1 * e1 + kZc2 * e2 + kZc3 * e3;
    const double dphi = -(kZc0 * kZd0 * e0 + kZc1 * kZd1 * e1 + kZc2 * kZd2 * e2 + kZc3 * kZd3 * e3);
    const double d2phi = kZc0 * kZd0 * kZd0 * e0 + kZc1 * kZd1 * kZd1 * e1 + kZc2 * kZd2 * kZd2 * e2 +
                         kZc3 * kZd3 * kZd3 * e3;
    const double ir2 = inv_r * inv_r;
    // c = zz (phi/r^3 - phi'/(a r^2)), the same value the step computes as -V'(r)/r
    const double dVdr = zz * inv_r * (dphi * inv_a - phi * inv_r);
    c = -dVdr * inv_r;
    c_r = zz * ir2 * (3.0 * dphi * inv_a * inv_r - 3.0 * phi * ir2 - d2phi * inv_a * inv_a);
    c_s = zz * d2phi * inv_a * inv_a * inv_s * inv_r;
    w = sc.wnorm * exp2_neg_pair(r, sc.lam2);
}

// The stopping depth also depends on the state at the start of the last step
// (z0b: d z_stop / d z there; kmb: d z_stop / d ke0 times M1).
__device__ __forceinline__ void seed_last_step(AdjIon& ai, double z0b, double kmb, double vx, double vy, double vz)
{
    ai.xb[2] += z0b;
    ai.vb[0] += kmb * vx;
    ai.vb[1] += kmb * vy;
    ai.vb[2] += kmb * vz;
}

// Step-log entry of one step: dt, the StepInfo code (bit 4: the step moved the
// domain), and the ion's position, velocity, force and density before it.
constexpr int kLogWords = 12;

// Drop-log entry of one domain move: the old centre (3 words, padded to 8),
// then the dropped atoms' positions and velocities, [6][kSlots] by slot.
constexpr int kDropWords = 8 + 6 * kSlots;

// Pair terms of the state held in the registers, per register slot: the
// coefficient c = -V'(r)/r, its derivatives dc/dr and dc/ds, the density
// weight (with its normalisation) and 1/r.  Zero for empty slots.
template <int L>
struct PairState {
    static constexpr int SL = TrackRegs<L>::SL;
    double c[SL], cr[SL], cs[SL], w[SL], ir[SL];
};

template <int L>
__device__ __forceinline__ void pair_state(const TrackRegs<L>& t, const KernelArgs& A, const SpeciesConst& c,
                                           PairState<L>& P)
{
    const KernelArgs K = cold_args();
#pragma unroll
    for (int i = 0; i < TrackRegs<L>::SL; ++i) {
        P.c[i] = 0.0; P.cr[i] = 0.0; P.cs[i] = 0.0; P.w[i] = 0.0; P.ir[i] = 0.0;
        if (!((t.exist >> i) & 1u)) continue;
        const double dx = t.x - t.ax[i], dy = t.y - t.ay[i], dz = t.z - t.az[i];
        double r;
        zbl_pair_adjoint(c, K.inv_s, dx * dx + dy * dy + dz * dz, r, P.ir[i],
                         P.c[i], P.cr[i], P.cs[i], P.w[i]);
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Adjoint of one step n (S_n -> S_{n+1}), with the state rebuilt in the
// registers.  On entry t holds S_{n+1} and P its pair terms, and the adjoint
// arrays hold the adjoint of S_{n+1}; on exit t holds S_n (rebuilt), P the pair
// terms of S_n, and the adjoints those of S_n.  lgn: the step's log entry (dt,
// StepInfo code, ion position, velocity, force and density of S_n).  MOVED: the
// step moved the domain; de is its drop-log entry.  A slot then holds at S_n the atom it held
// at S_{n+1} if that atom was kept, the dropped atom if one left, or nothing.
template <int L, bool MOVED>
__device__ __forceinline__ void reverse_step_regs(AdjIon& ai, AdjAtoms<L>& aa, PairState<L>& P, TrackRegs<L>& t,
                                                  const KernelArgs& A, const SpeciesConst& c, const double* lgn,
                                                  const double* de, int sl, double& sb_lane)
{
    constexpr int SL = TrackRegs<L>::SL;
    constexpr int FS = TrackRegs<L>::FS;
    // the run's scalar settings re-read from the argument segment at every step (scalar loads)
    // instead of registers held across the reverse sweep that the allocator spills
    const KernelArgs K = cold_args();
    // centres of S_{n+1} and S_n; parking place of S_n's empty slots
    const int c1x = t.cx, c1y = t.cy, c1z = t.cz;
    int cnx = c1x, cny = c1y, cnz = c1z;
    double parkx = 0.0, parky = 0.0, parkz = 0.0;
    if constexpr (MOVED) {
        cnx = static_cast<int>(de[0]);
        cny = static_cast<int>(de[1]);
        cnz = static_cast<int>(de[2]);
        const KernelArgs C = cold_args();
        parkx = C.a * (static_cast<double>(cnx) + 0.5);
        parky = C.a * (static_cast<double>(cny) + 0.5);
        parkz = C.a * (static_cast<double>(cnz) + 0.5) - C.park;
    }
    const double* dropped = de + 8;
    unsigned ex_n = 0;
    const double dt = lgn[0];
    const int code = static_cast<int>(reinterpret_cast<const long long*>(lgn)[1]);
    const double h1 = dt * c.half_inv_M1;
    const double h2 = dt * K.half_inv_M2;
    // ---- ion of S_{n+1}; the ion of S_n is the logged one (the chaotic part of the
    //      state is never run backwards)
    const double x1[3] = {t.x, t.y, t.z};
    const double Fp[3] = {t.Fx, t.Fy, t.Fz};
    const double rhop = t.rho;
    const double g2 = c.g_const + c.g_rho * rhop;
    const double fr2 = exp_neg(g2 * h1);
    const double x[3] = {lgn[2], lgn[3], lgn[4]};
    const double v[3] = {lgn[5], lgn[6], lgn[7]};
    const double F[3] = {lgn[8], lgn[9], lgn[10]};
    const double rho = lgn[11];
    const double vp[3] = {t.vx, t.vy, t.vz};
    double q[3];
    for (int k = 0; k < 3; ++k) q[k] = vp[k] / fr2;
    // ---- adjoint of v' = q fr2
    double qb[3], v1b[3], Fpb[3];
    double fr2b = 0.0, h1b = 0.0;
    for (int k = 0; k < 3; ++k) {
        qb[k] = ai.vb[k] * fr2;
        fr2b += ai.vb[k] * q[k];
        v1b[k] = qb[k];
        Fpb[k] = ai.Fb[k] + qb[k] * h1;
        h1b += qb[k] * Fp[k];
    }
    const double g2b = -fr2b * fr2 * h1;
    h1b += -fr2b * fr2 * g2;
    ai.kb += g2b * (c.dg_const + c.dg_rho * rhop);
    const double rhopb = ai.rhob + g2b * c.g_rho;

    // ---- per slot: reconstruct the atom of S_n and its pair term; adjoint of the
    //      second kick, the pair term of S_{n+1}, the drift and the first kick
    double x1b_l[3] = {0.0, 0.0, 0.0};
    double dtb_l = 0.0, h2b_l = 0.0, vm_l = 0.0, fm_l = 0.0;
    double v2s[SL], f2s[SL];   // the slots' |V|^2 and |f|^2 as maximised (the argmax is found by equality)
#pragma unroll
    for (int i = 0; i < SL; ++i) {
        double nXb[3] = {0.0, 0.0, 0.0}, nVb[3] = {0.0, 0.0, 0.0}, nfb[3] = {0.0, 0.0, 0.0};
        v2s[i] = -1.0;
        f2s[i] = -1.0;
        const int s = sl + L * i;
        double* f = t.fl + s;
        const bool e1 = (t.exist >> i) & 1u;   // an atom at S_{n+1}
        bool en = e1, kept = e1;               // an atom at S_n; the same atom at both
        if constexpr (MOVED) {
            const int cell = (s < kSlots) ? (s >> 3) : -1;
            const int rx = cell / 9, ry = (cell / 3) % 3, rz = cell % 3;
            const int oz = cell_of_residue(rz, cnz);
            en = cell >= 0 && oz >= 0;
            kept = e1 && en && cell_of_residue(rx, cnx) == cell_of_residue(rx, c1x) &&
                   cell_of_residue(ry, cny) == cell_of_residue(ry, c1y) && oz == cell_of_residue(rz, c1z);
        }
        // S_{n+1}'s atom and pair terms in this slot (exact zeros when parked)
        const double Y[3] = {t.ax[i], t.ay[i], t.az[i]};
        const double Vp[3] = {t.avx[i], t.avy[i], t.avz[i]};
        const double fp[3] = {f[0], f[FS], f[2 * FS]};
        const double pc = P.c[i], pcr = P.cr[i], pcs = P.cs[i], pw = P.w[i], pir = P.ir[i];
        // S_n's atom: a kept atom runs its part of the step backwards, a dropped one
        // comes from the drop log
        double U[3], X[3], Vn[3] = {0.0, 0.0, 0.0}, fn[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < 3; ++k) {
            U[k] = Vp[k] - fp[k] * h2;
            X[k] = Y[k] - U[k] * dt;
        }
        if constexpr (MOVED) {
            if (en && !kept)
                for (int k = 0; k < 3; ++k) {
                    X[k] = dropped[k * kSlots + s];
                    Vn[k] = dropped[(3 + k) * kSlots + s];
                }
        }
        double cn = 0.0, crn = 0.0, csn = 0.0, wn = 0.0, irn = 0.0;
        if (en) {
            double dn[3], rn;
            for (int k = 0; k < 3; ++k) dn[k] = x[k] - X[k];
            zbl_pair_adjoint(c, K.inv_s, dn[0] * dn[0] + dn[1] * dn[1] + dn[2] * dn[2],
                             rn, irn, cn, crn, csn, wn);
            for (int k = 0; k < 3; ++k) {
                fn[k] = -cn * dn[k];
                if (kept) Vn[k] = U[k] - fn[k] * h2;
            }
            v2s[i] = Vn[0] * Vn[0] + Vn[1] * Vn[1] + Vn[2] * Vn[2];
            f2s[i] = fn[0] * fn[0] + fn[1] * fn[1] + fn[2] * fn[2];
            vm_l = fmax(vm_l, v2s[i]);
            fm_l = fmax(fm_l, f2s[i]);
        }
        // ---- adjoint of the second kick and the pair term of S_{n+1}, and for a kept
        //      atom of its drift and first kick (a created atom is a constant)
        if (e1) {
            double Ub[3], G[3], d[3], cb = 0.0;
            for (int k = 0; k < 3; ++k) {
                Ub[k] = aa.Vb[k][i];
                h2b_l += aa.Vb[k][i] * fp[k];
                d[k] = x1[k] - Y[k];
                G[k] = Fpb[k] - (aa.fb[k][i] + aa.Vb[k][i] * h2);
                cb += G[k] * d[k];
            }
            const double rb = cb * pcr - rhopb * pw * c.inv_lambda;
            sb_lane += cb * pcs;
            for (int k = 0; k < 3; ++k) {
                const double db = pc * G[k] + rb * d[k] * pir;
                x1b_l[k] += db;
                if (kept) {
                    const double Yb = aa.Xb[k][i] - db;
                    nXb[k] = Yb;
                    Ub[k] += Yb * dt;
                    dtb_l += Yb * U[k];
                    nVb[k] = Ub[k];
                    nfb[k] = Ub[k] * h2;
                    h2b_l += Ub[k] * fn[k];
                }
            }
        }
        // ---- S_n into the slot
        if (en) {
            t.ax[i] = X[0]; t.ay[i] = X[1]; t.az[i] = X[2];
            t.avx[i] = Vn[0]; t.avy[i] = Vn[1]; t.avz[i] = Vn[2];
            f[0] = fn[0]; f[FS] = fn[1]; f[2 * FS] = fn[2];
            P.c[i] = cn; P.cr[i] = crn; P.cs[i] = csn; P.w[i] = wn; P.ir[i] = irn;
            ex_n |= 1u << i;
        } else if constexpr (MOVED) {
            t.ax[i] = parkx; t.ay[i] = parky; t.az[i] = parkz;
            t.avx[i] = 0.0; t.avy[i] = 0.0; t.avz[i] = 0.0;
            f[0] = 0.0; f[FS] = 0.0; f[2 * FS] = 0.0;
            P.c[i] = 0.0; P.cr[i] = 0.0; P.cs[i] = 0.0; P.w[i] = 0.0; P.ir[i] = 0.0;
        }
        for (int k = 0; k < 3; ++k) {
            aa.Xb[k][i] = nXb[k];
            aa.Vb[k][i] = nVb[k];
            aa.fb[k][i] = nfb[k];
        }
        // one slot at a time: interleaving the slots' pair terms costs more registers than it hides
        __builtin_amdgcn_sched_barrier(0);
    }
    double x1b[3];
    for (int k = 0; k < 3; ++k) x1b[k] = ai.xb[k] + SegReduce<L>::sum(x1b_l[k]);
    // the atoms' maxima are reduced only when an atom's speed or acceleration set dt
    const int branch = code & 3;
    const double vm = (branch == 1 && !(code & 4)) ? SegReduce<L>::max(vm_l) : 0.0;
    const double fm = (branch == 2 && !(code & 8)) ? SegReduce<L>::max(fm_l) : 0.0;
    // d/dt through the atoms' drifts and, via h2 = dt / 2M2, their kicks: one reduction
    double dtb = SegReduce<L>::sum(dtb_l + h2b_l * K.half_inv_M2);

    // ---- first friction half and kick of the step
    const double g1 = c.g_const + c.g_rho * rho;
    const double fr1 = exp_neg(g1 * h1);
    double v1[3];
    for (int k = 0; k < 3; ++k) v1[k] = v[k] * fr1 + F[k] * h1;

    // ---- adjoint of x1 = x + v1 dt, v1 = v fr1 + F h1, fr1 = exp(-g1 h1)
    double fr1b = 0.0;
    for (int k = 0; k < 3; ++k) {
        v1b[k] += x1b[k] * dt;
        dtb += x1b[k] * v1[k];
        ai.xb[k] = x1b[k];
        ai.vb[k] = v1b[k] * fr1;
        fr1b += v1b[k] * v[k];
        ai.Fb[k] = v1b[k] * h1;
        h1b += v1b[k] * F[k];
    }
    const double g1b = -fr1b * fr1 * h1;
    h1b += -fr1b * fr1 * g1;
    ai.kb += g1b * (c.dg_const + c.dg_rho * rho);
    ai.rhob = g1b * c.g_rho;
    dtb += h1b * c.half_inv_M1;

    if constexpr (MOVED) {
        t.exist = ex_n;
        t.cx = cnx; t.cy = cny; t.cz = cnz;
        t.n_exist = SegReduce<L>::isum(__popc(ex_n));
    }
    t.x = x[0]; t.y = x[1]; t.z = x[2];
    t.vx = v[0]; t.vy = v[1]; t.vz = v[2];
    t.Fx = F[0]; t.Fy = F[1]; t.Fz = F[2];
    t.rho = rho;   // (the atom maxima of t are not kept up to date in the reverse)

    // ---- the active term of the step-size minimum and its maximising particle
    if (branch == 1) {
        const bool ion = (code & 4) != 0;
        const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        const double vmax2b = -0.5 * dtb * dt / (ion ? v2 : vm);
        if (ion) {
            for (int k = 0; k < 3; ++k) ai.vb[k] += 2.0 * vmax2b * v[k];
        } else {
#pragma unroll
            for (int i = 0; i < SL; ++i) {
                if (v2s[i] == vm) {
                    aa.Vb[0][i] += 2.0 * vmax2b * t.avx[i];
                    aa.Vb[1][i] += 2.0 * vmax2b * t.avy[i];
                    aa.Vb[2][i] += 2.0 * vmax2b * t.avz[i];
                }
            }
        }
    } else if (branch == 2) {
        const bool ion = (code & 8) != 0;
        const double f2 = F[0] * F[0] + F[1] * F[1] + F[2] * F[2];
        const double amax2b = -0.25 * dtb * dt / (ion ? f2 * c.inv_M1sq : fm * K.inv_M2sq);
        if (ion) {
            for (int k = 0; k < 3; ++k) ai.Fb[k] += 2.0 * amax2b * F[k] * c.inv_M1sq;
        } else {
#pragma unroll
            for (int i = 0; i < SL; ++i) {
                if (f2s[i] == fm) {
                    const double* f = t.fl + (sl + L * i);
                    const double fx = f[0], fy = f[FS], fz = f[2 * FS];
                    aa.fb[0][i] += 2.0 * amax2b * fx * K.inv_M2sq;
                    aa.fb[1][i] += 2.0 * amax2b * fy * K.inv_M2sq;
                    aa.fb[2][i] += 2.0 * amax2b * fz * K.inv_M2sq;
                }
            }
        }
    }
}

#ifndef REEDMD_GRAD_WAVES_PER_SIMD
#define REEDMD_GRAD_WAVES_PER_SIMD 1
#endif

// One wavefront per primary (batch entry), launched as one-wavefront
// workgroups: tracks differ in length by orders of magnitude, and a finished
// wavefront frees its SIMD for the next track at once.  Writes gout[q] =
// {z_stop, dz/dk, dz/ds, status, steps}; derivatives are zero unless the track
// stopped.
__global__ void __launch_bounds__(64, REEDMD_GRAD_WAVES_PER_SIMD) grad_kernel(const KernelArgs A)
{
    constexpr int L = 64;
    __shared__ SpeciesConst s_sp[kMaxSpecies];
    __shared__ double s_force[ForceLds<L>::kTrackDoubles];
    constexpr int kWords = sizeof(SpeciesConst) * kMaxSpecies / sizeof(double);
    for (int i = threadIdx.x; i < kWords; i += blockDim.x)
        reinterpret_cast<double*>(s_sp)[i] = reinterpret_cast<const double*>(A.sp)[i];
    __syncthreads();
    const SpeciesConst* sp = s_sp;
    const int sl = threadIdx.x & 63;
    const long long local = static_cast<long long>(blockIdx.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const long long q = A.q0 + local;
    if (q >= A.q_end) return;
    double* ck = A.ckpt + static_cast<size_t>(local) * A.ckpt_cap * kRecWords;
    double* dl = A.droplog + static_cast<size_t>(local) * A.drop_cap * kDropWords;
    double* lg = A.steplog + static_cast<size_t>(local) * A.ckpt_cap * 64 * kLogWords;
    double* out = A.gout + static_cast<size_t>(q) * 5;

    TrackRegs<L> t;
    t.fl = force_slab<L>(s_force);
    t.exist = 0;
    start_primary<L>(t, A, sp, q);
    if (t.status == REEDMD_LOST) {
        if (sl == 0) { out[0] = 0.0; out[1] = 0.0; out[2] = 0.0; out[3] = REEDMD_LOST; out[4] = 0.0; }
        return;
    }
    double ke0, z0;
    track_step<L>(t, A, sp, sl, true, ke0, z0);
    store_record<L>(t, ck, sl);

    // ---- forward with a checkpoint every 64 steps and the log of step sizes
    //      and the ion of the state it starts from (steps < ckpt_cap * 64: the loop
    //      ends at the checkpoint capacity)
    //      and, at each domain move, the old centre and the atoms dropped (at most
    //      drop_cap moves: a track that makes more ends as capped)
    int st = REEDMD_ACTIVE;
    int moves = 0;
    for (;;) {
        const long long n = t.steps;
        const int ocx = t.cx, ocy = t.cy, ocz = t.cz;
        const double ion[10] = {t.x, t.y, t.z, t.vx, t.vy, t.vz, t.Fx, t.Fy, t.Fz, t.rho};
        double* de = dl + static_cast<size_t>(moves) * kDropWords;
        StepInfo si;
        track_step<L>(t, A, sp, sl, false, ke0, z0, &si, de + 8);
        const bool moved = t.cx != ocx || t.cy != ocy || t.cz != ocz;
        if (sl == 0) {
            double* e = lg + kLogWords * n;
            e[0] = si.dt;
            reinterpret_cast<long long*>(e)[1] = si.code | (moved ? 16 : 0);
            for (int k = 0; k < 10; ++k) e[2 + k] = ion[k];
            if (moved) {
                de[0] = static_cast<double>(ocx);
                de[1] = static_cast<double>(ocy);
                de[2] = static_cast<double>(ocz);
            }
        }
        if (moved) ++moves;
        st = track_events<L>(t, A, sp, ke0, z0);
        if (st != REEDMD_ACTIVE) break;
        if (moves >= A.drop_cap) { st = REEDMD_STEPCAP; break; }
        if ((t.steps & 63) == 0) {
            const long long k = t.steps >> 6;
            if (k >= A.ckpt_cap) { st = REEDMD_STEPCAP; break; }
            store_record<L>(t, ck + static_cast<size_t>(k) * kRecWords, sl);
        }
    }
    const long long N = t.steps;
    if (st != REEDMD_STOPPED) {
        if (sl == 0) { out[0] = 0.0; out[1] = 0.0; out[2] = 0.0; out[3] = st; out[4] = static_cast<double>(N); }
        return;
    }
    const SpeciesConst& c = sp[t.species];
    const double M1 = c.M1;
    const double zstop = t.zstop;
    // ---- seed: z_stop = z0 + (z1 - z0) theta, theta = (ke0 - E)/(ke0 - ke1)
    const double ke1 = 0.5 * M1 * (t.vx * t.vx + t.vy * t.vy + t.vz * t.vz);
    double z1b = 0.0, ke1b = 0.0, z0b = 1.0, ke0b = 0.0;
    if (ke0 > A.E_stop) {
        const double den = ke0 - ke1;
        const double theta = (ke0 - A.E_stop) / den;
        const double dz = t.z - z0;
        z1b = theta;
        z0b = 1.0 - theta;
        ke1b = dz * (ke0 - A.E_stop) / (den * den);
        ke0b = dz * (A.E_stop - ke1) / (den * den);
    }
    AdjIon ai;
    for (int k = 0; k < 3; ++k) { ai.xb[k] = 0.0; ai.vb[k] = 0.0; ai.Fb[k] = 0.0; }
    ai.xb[2] = z1b;
    ai.vb[0] = ke1b * M1 * t.vx;
    ai.vb[1] = ke1b * M1 * t.vy;
    ai.vb[2] = ke1b * M1 * t.vz;
    ai.rhob = 0.0;
    ai.kb = 0.0;
    AdjAtoms<L> aa;
#pragma unroll
    for (int i = 0; i < TrackRegs<L>::SL; ++i)
        for (int k = 0; k < 3; ++k) { aa.Xb[k][i] = 0.0; aa.Vb[k][i] = 0.0; aa.fb[k][i] = 0.0; }
    double sb_lane = 0.0;

    // ---- reverse, step by step from the final state (t holds S_N)
    __threadfence();   // the logs written by the forward are read by every lane
    PairState<L> P;
    for (long long seg = (N - 1) >> 6; seg >= 0; --seg) {
        const long long start = seg << 6;
        const long long end = (start + 64 < N) ? start + 64 : N;
        // re-anchor to the exact state at the end of the segment
        if (end != N) load_record<L>(t, ck + static_cast<size_t>(end >> 6) * kRecWords, sl, A);
        pair_state<L>(t, A, c, P);
        for (long long n = end - 1; n >= start; --n) {
            const double* lgn = lg + kLogWords * n;
            if (reinterpret_cast<const long long*>(lgn)[1] & 16) {
                --moves;
                reverse_step_regs<L, true>(ai, aa, P, t, A, c, lgn, dl + static_cast<size_t>(moves) * kDropWords, sl,
                                           sb_lane);
            } else {
                reverse_step_regs<L, false>(ai, aa, P, t, A, c, lgn, dl, sl, sb_lane);
            }
            if (n == N - 1) seed_last_step(ai, z0b, ke0b * M1, t.vx, t.vy, t.vz);
        }
    }
    // ---- the starting forces depend on s (positions and velocities are constants)
    {
        const double* r0 = ck;
        const double* a0 = r0 + kHdr;
        const int cz0 = static_cast<int>(reinterpret_cast<const long long*>(r0)[14]);
#pragma unroll
        for (int i = 0; i < TrackRegs<L>::SL; ++i) {
            const int s = sl + L * i;
            if (s >= kSlots) continue;
            if (cell_of_residue((s >> 3) % 3, cz0) < 0) continue;
            double d[3], G[3], cb = 0.0;
            for (int k = 0; k < 3; ++k) {
                d[k] = r0[k] - a0[k * kSlots + s];
                G[k] = ai.Fb[k] - aa.fb[k][i];
                cb += G[k] * d[k];
            }
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            double r, inv_r, cc, c_r, c_s, w;
            zbl_pair_adjoint(c, A.inv_s, r2, r, inv_r, cc, c_r, c_s, w);
            sb_lane += cb * c_s;
        }
    }
    const double dzds = SegReduce<L>::sum(sb_lane);
    if (sl == 0) {
        out[0] = zstop;
        out[1] = ai.kb;
        out[2] = dzds;
        out[3] = REEDMD_STOPPED;
        out[4] = static_cast<double>(N);
    }
}

// Deterministic mean over stopped tracks: res = {count, sum z, sum dz/dk, sum dz/ds}.
__global__ void __launch_bounds__(256) grad_reduce_kernel(const double* gout, long long n, double* res)
{
    __shared__ double sh[4][256];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (long long i = threadIdx.x; i < n; i += blockDim.x) {
        const double* o = gout + static_cast<size_t>(i) * 5;
        if (o[3] == static_cast<double>(REEDMD_STOPPED)) {
            acc[0] += 1.0;
            acc[1] += o[0];
            acc[2] += o[1];
            acc[3] += o[2];
        }
    }
    for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if (threadIdx.x < w)
            for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 4) res[threadIdx.x] = sh[threadIdx.x][0];
}

}  // namespace reedmd
