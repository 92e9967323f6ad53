// Device-side physics for the REED-MD track kernels (gfx950, FP64 VALU).
//
// Everything here is written for one wavefront lane; the track kernels map
// the 216 domain atoms of a track across the lanes of a wavefront segment.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace reedmd {

constexpr int kSlots = 216;       // 27 cells x 8 diamond basis atoms
constexpr int kHdr = 32;          // record header words
constexpr int kRecWords = kHdr + 9 * kSlots;

// Target structures.  Slots are indexed by the ring cell r of a unit cell
// (r = (c_x mod 3)*9 + (c_y mod 3)*3 + (c_z mod 3)) and its basis atom b.
// Diamond: slot r*8 + b, one target species.  Fluorite (UO2, 27 cells of the
// 12-atom cell): the cations (species 0, b = 0..3) in slots r*4 + b, slots
// 108..127 empty, the anions (species 1, b = 4..11) in slots 128 + r*8 + b - 4,
// so that every lane row of 16, 32 or 64 slots holds one target species.
enum : int { kDiamond = 0, kFluorite = 1 };
template <int LAT>
struct Lattice;
template <>
struct Lattice<kDiamond> {
    static constexpr int kSlots = 216, kCellAtoms = 8, kAnion0 = 1 << 20;
    static constexpr int kRecWords = kHdr + 9 * kSlots;
    __device__ static int slot(int r, int b) { return r * 8 + b; }
    __device__ static int cell_of_slot(int s) { return s >> 3; }
    __device__ static int basis_of_slot(int s) { return s & 7; }
};
template <>
struct Lattice<kFluorite> {
    static constexpr int kSlots = 344, kCellAtoms = 12, kAnion0 = 128;
    static constexpr int kRecWords = kHdr + 9 * kSlots;
    __device__ static int slot(int r, int b) { return b < 4 ? r * 4 + b : kAnion0 + r * 8 + (b - 4); }
    __device__ static int cell_of_slot(int s) { return s < 108 ? (s >> 2) : (s < kAnion0 ? -1 : (s - kAnion0) >> 3); }
    __device__ static int basis_of_slot(int s) { return s < kAnion0 ? (s & 3) : 4 + ((s - kAnion0) & 7); }
};
constexpr int kMaxSpecies = 8;
constexpr int kSentinel = -(1 << 29);  // "no domain yet": every slot is regenerated

// Per-species constants, prepared on the host from the ZBL and Lindhard-
// Scharff expressions (see the library's reedmd_create / prepare_species).
struct SpeciesConst {
    double M1;
    double half_inv_M1;   // 1 / (2 M1)
    double inv_a;         // 1 / screening length
    double zz;            // Z1 Z2 e^2 (eV A), 0 when the nuclear force is off
    double inv_lambda;    // 1 / density decay length
    double wnorm;         // 1 / (8 pi lambda^3)
    double g_const;       // friction: gamma = g_const + g_rho * rho
    double g_rho;
    double dg_const;      // d g_const / d k
    double dg_rho;        // d g_rho / d k
    double inv_M1sq;      // 1 / M1^2
    // The screened-Coulomb sum with its constants folded per species:
    //   rate_i = log2(e) d_i / a (base-2 rate),  amp_i = zz c_i,  damp_i = zz c_i d_i / a
    double rate[4], amp[4], damp[4];
    // The same in FP32 for the FP32 pair term (base-2 rates for the hardware 2^x)
    float rate2f[4], amp_f[4], damp_f[4];
    float lam2f, pad_f;
    double lam2;          // log2(e) / lambda, the base-2 rate of the density weight
};

// Pair-term constants of an ion species against the second target species
// (fluorite anions), folded like those above; wnorm includes the ratio of the
// Lindhard-Scharff constants of the two target species (stopping-weighted
// density, Bragg additivity).
struct PairConst {
    double rate[4], amp[4], damp[4];   // rate: base 2, as in SpeciesConst
    double lam2, wnorm;
    float rate2f[4], amp_f[4], damp_f[4];
    float lam2f, pad_f;
};

// ---------------------------------------------------------------------------
// Counter-based random numbers: Philox4x64 with 10 rounds (Salmon, Moraes,
// Dror, Shaw, SC'11).  A round multiplies counter words 0 and 2 by two fixed
// odd 64-bit constants, and builds the next counter from the high halves
// xor-ed with words 1 and 3 and the round key, and from the low halves; the
// key advances by the Weyl increments (golden ratio and sqrt(3)-1 in 64-bit
// fixed point) between rounds.
struct U64x4 {
    uint64_t w[4];
};

__device__ __forceinline__ U64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1)
{
    constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ULL;
    constexpr uint64_t kMulB = 0xCA5A826395121157ULL;
    constexpr uint64_t kWeylA = 0x9E3779B97F4A7C15ULL;
    constexpr uint64_t kWeylB = 0xBB67AE8584CAA73BULL;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hiA = __umul64hi(kMulA, c0), loA = kMulA * c0;
        const uint64_t hiB = __umul64hi(kMulB, c2), loB = kMulB * c2;
        const uint64_t n0 = hiB ^ c1 ^ k0;
        const uint64_t n2 = hiA ^ c3 ^ k1;
        c0 = n0;
        c1 = loB;
        c2 = n2;
        c3 = loA;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    U64x4 o;
    o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
    return o;
}

// (0,1) from the top 52 bits: ((w >> 12) + 1/2) * 2^-52, always an exact double.
__device__ __forceinline__ double open_unit(uint64_t w)
{
    return (static_cast<double>(w >> 12) + 0.5) * 0x1.0p-52;
}

enum : uint64_t { kTagSample = 1, kTagPrimaryKey = 2, kTagThermal = 3, kTagChildKey = 4 };

__device__ __forceinline__ uint64_t child_key(uint64_t key, uint64_t seed, int k, int i)
{
    return philox4x64_10(kTagChildKey, static_cast<uint64_t>(static_cast<int64_t>(k)),
                         static_cast<uint64_t>(static_cast<int64_t>(i)), 0, key, seed).w[0];
}

__device__ __forceinline__ uint64_t primary_key(uint64_t seed, int64_t id)
{
    return philox4x64_10(kTagPrimaryKey, static_cast<uint64_t>(id), 0, 0, seed, 0).w[0];
}

// Thermal displacement (in units of sigma) of basis atom b of cell c of the
// crystal realisation `key`: Box-Muller on the four uniforms of one block
// (cos and sin of the first pair, cos of the second).
__device__ __forceinline__ void thermal_gauss(uint64_t key, uint64_t seed, int cx, int cy, int cz,
                                              int b, double& gx, double& gy, double& gz)
{
    const U64x4 r = philox4x64_10(kTagThermal | (static_cast<uint64_t>(b) << 8),
                                  static_cast<uint64_t>(static_cast<int64_t>(cx)),
                                  static_cast<uint64_t>(static_cast<int64_t>(cy)),
                                  static_cast<uint64_t>(static_cast<int64_t>(cz)), key, seed);
    const double rad0 = sqrt(-2.0 * log(open_unit(r.w[0])));
    const double rad1 = sqrt(-2.0 * log(open_unit(r.w[2])));
    // the angle is 2 pi u with u in (0, 1): sin and cos of pi (2u), where 2u is
    // exact, need no reduction of a large argument
    double s0, c0, s1, c1;
    sincospi(2.0 * open_unit(r.w[1]), &s0, &c0);
    sincospi(2.0 * open_unit(r.w[3]), &s1, &c1);
    gx = rad0 * c0;
    gy = rad0 * s0;
    gz = rad1 * c1;
}

// Fractional basis sites.  Diamond: fcc sites, then the same plus
// (1/4,1/4,1/4).  Fluorite: the fcc sites (cations), then the eight sites with
// every coordinate 1/4 or 3/4 (anions; bit 2 of b - 4 selects x, bit 1 y, bit 0 z).
__device__ __forceinline__ void basis_site(int b, bool fluorite, double& fx, double& fy, double& fz)
{
    if (fluorite && b >= 4) {
        const int j = b - 4;
        fx = ((j >> 2) & 1) ? 0.75 : 0.25;
        fy = ((j >> 1) & 1) ? 0.75 : 0.25;
        fz = (j & 1) ? 0.75 : 0.25;
        return;
    }
    const int q = b & 3;
    const double sh = (b >= 4) ? 0.25 : 0.0;
    fx = ((q == 2 || q == 3) ? 0.5 : 0.0) + sh;
    fy = ((q == 1 || q == 3) ? 0.5 : 0.0) + sh;
    fz = ((q == 1 || q == 2) ? 0.5 : 0.0) + sh;
}

// Position of a newly created atom: ideal site of basis atom b in cell
// (nx,ny,nz) plus its thermal displacement.  Kept out of line (one copy instead
// of one per register slot), so that the rarely taken domain update does not
// raise the register budget of the step: it removes the scalar-register spills
// of the step loop and the stack arrays of the 16-lane layout.
#ifndef REEDMD_INLINE_CREATE
__device__ __attribute__((noinline)) double3 create_atom(uint64_t key, uint64_t seed, int nx, int ny, int nz, int b,
                                                          double a, double sigma, double sigma_b, int fluorite)
#else
__device__ __forceinline__ double3 create_atom(uint64_t key, uint64_t seed, int nx, int ny, int nz, int b,
                                                double a, double sigma, double sigma_b, int fluorite)
#endif
{
    double fx, fy, fz, gx, gy, gz;
    basis_site(b, fluorite != 0, fx, fy, fz);
    if (fluorite && b >= 4) sigma = sigma_b;
    thermal_gauss(key, seed, nx, ny, nz, b, gx, gy, gz);
    return make_double3(a * (static_cast<double>(nx) + fx) + sigma * gx,
                        a * (static_cast<double>(ny) + fy) + sigma * gy,
                        a * (static_cast<double>(nz) + fz) + sigma * gz);
}

// ---------------------------------------------------------------------------
// exp(-y), written from the mathematics: y = n ln2 - r with n the nearest
// integer to y / ln2 (the rounding is done by adding 1.5 * 2^52, whose sum
// holds n in its low mantissa bits, so no conversion is needed), r reduced with
// ln 2 split into a double and its remainder (both FMA-exact), |r| <= ln2/2;
// e^r from a polynomial that minimises the largest relative error on that
// interval (Remez exchange, constant term held at 1), and the scaling by 2^-n
// done by ldexp, which rounds gradual underflow correctly.  Valid for finite
// 0 <= y < 1e9: the kernels' arguments are distances over positive lengths,
// bounded by the parking distance of empty slots (see the library's argument
// checks).
__device__ __forceinline__ double exp_reduce(double y, double& r)
{
    constexpr double kLog2e = 1.4426950408889634;
    constexpr double kLn2Hi = 0x1.62e42fefa39efp-1;
    constexpr double kLn2Lo = 0x1.abc9e3b39803fp-56;
    constexpr double kRound = 0x1.8p52;
    const double nr = fma(-y, kLog2e, kRound);   // kRound + nearest integer to -y / ln2
    const double n = nr - kRound;
    r = fma(-n, kLn2Hi, -y);
    r = fma(-n, kLn2Lo, r);
    return nr;
}

// A constant put into scalar registers where it is used.  FP64 FMAs take no
// 64-bit literal operand, so a polynomial's coefficients live in registers; left
// to itself the compiler hoists the coefficients of an exponential evaluated once
// per step out of the step loop into vector registers, and under register
// pressure spills them to scratch memory and reloads them one by one.
__device__ __forceinline__ double sconst(double v)
{
    asm volatile("" : "+s"(v));
    return v;
}

// Degree 10 (relative error 3.0e-16): the friction factors and other scalars.
__device__ __forceinline__ double exp_neg(double y)
{
    double r;
    const double nr = exp_reduce(y, r);
    double p = sconst(0x1.2a475a7d4ddb2p-22);
    p = fma(p, r, sconst(0x1.730bd57070546p-19));
    p = fma(p, r, sconst(0x1.a017fb6001714p-16));
    p = fma(p, r, sconst(0x1.a01967c4ef7f8p-13));
    p = fma(p, r, sconst(0x1.6c16c20da969ep-10));
    p = fma(p, r, sconst(0x1.11111133719d9p-7));
    p = fma(p, r, sconst(0x1.555555552f919p-5));
    p = fma(p, r, sconst(0x1.5555555548c99p-3));
    p = fma(p, r, sconst(0x1.000000000004bp-1));
    p = fma(p, r, sconst(0x1.0000000000029p+0));
    p = fma(p, r, 1.0);
    return ldexp(p, static_cast<int>(__double2loint(nr)));
}

// 2^(-r k) for the five exponentials of every ion-atom pair term, with the
// base-2 rate k = log2(e) / length folded into the species constants: n, the
// nearest integer to -r k, from one FMA against 1.5 * 2^52, and f = -r k - n in
// [-1/2, 1/2] from a second FMA (r k never rounds on its own); 2^f from the
// degree-8 polynomial that minimises the largest relative error (the Remez
// polynomial of e^x on |x| <= ln2/2, rescaled to 2^f: 1.08e-12), ldexp for the
// scaling.  With the rounding of k (at most 2^-53 r k), the relative error
// stays below 1.15e-12, 90 x inside the per-step tolerance of 1e-10; the ZBL
// sums and the density weight add positive terms only, so the pair term keeps
// that relative accuracy.  Valid for finite 0 <= r k < 1e9.
__device__ __forceinline__ double exp2_neg_pair(double r, double k)
{
    constexpr double kRound = 0x1.8p52;
    const double nr = fma(-r, k, kRound);   // kRound + nearest integer to -r k
    const double n = nr - kRound;
    const double f = fma(-r, k, -n);
    double p = 0x1.66348837e364bp-20;
    p = fma(p, f, 0x1.00ee071f31fb7p-16);
    p = fma(p, f, 0x1.4306c115f9e23p-13);
    p = fma(p, f, 0x1.5d872975bfdb7p-10);
    p = fma(p, f, 0x1.3b2ab7f3b35e8p-7);
    p = fma(p, f, 0x1.c6b08defc2655p-5);
    p = fma(p, f, 0x1.ebfbdff7c5a77p-3);
    p = fma(p, f, 0x1.62e42fef7a78bp-1);
    p = fma(p, f, 1.0);
    return ldexp(p, static_cast<int>(__double2loint(nr)));
}

// exp(-y) with the pair terms' accuracy (the adjoint's pair terms and tests).
__device__ __forceinline__ double exp_neg_pair(double y)
{
    return exp2_neg_pair(y, 1.4426950408889634);
}

// 1/sqrt(x) for finite x > 0: the hardware estimate refined by one
// third-order Newton step on e = 1 - x y^2 (y <- y (1 + e/2 + 3e^2/8)).
__device__ __forceinline__ double rsqrt_pos(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(0.375, e, 0.5), y);
}

// ---------------------------------------------------------------------------
// ZBL universal screening function phi(x) = sum c_i exp(-d_i x).
constexpr double kZc0 = 0.18175, kZc1 = 0.50986, kZc2 = 0.28022, kZc3 = 0.02817;
constexpr double kZd0 = 3.19980, kZd1 = 0.94229, kZd2 = 0.40290, kZd3 = 0.20162;

// Pair term for an ion at separation (dx,dy,dz) = x_ion - x_atom:
//   coef: force on the ion is coef * (dx,dy,dz) (the atom feels the opposite),
//         coef = -V'(r) / r = zz (phi(r/a) / r + (-phi'(r/a)) / a) / r^2
//         with V = zz phi(r/a) / r;
//   ew:   exp(-r/lambda), the density weight without its normalisation; with
//         FK (Firsov local loss) Firsov's kernel shape 1 / (1 + b r)^5, b in
//         c.lam2, taken as 0 beyond kFirsovRange.
// An empty slot sits at the parking distance, where every exponential is 0 and
// so are coef and ew.
constexpr double kFirsovRange = 1.0e3;   // A; every domain atom is within 30 A, parked slots beyond 1e4 A
__device__ __forceinline__ double firsov_shape(double r, double b)
{
    const double t = fma(b, r, 1.0);
    const double t2 = t * t;
    const double w = 1.0 / (t2 * t2 * t);
    return r < kFirsovRange ? w : 0.0;
}

template <bool FK = false, class PC>
__device__ __forceinline__ void zbl_pair(const PC& c, double dx, double dy, double dz, double& coef, double& ew)
{
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double inv_r = rsqrt_pos(r2);
    const double r = r2 * inv_r;
    const double e0 = exp2_neg_pair(r, c.rate[0]);
    const double e1 = exp2_neg_pair(r, c.rate[1]);
    const double e2 = exp2_neg_pair(r, c.rate[2]);
    const double e3 = exp2_neg_pair(r, c.rate[3]);
    const double phi = c.amp[0] * e0 + c.amp[1] * e1 + c.amp[2] * e2 + c.amp[3] * e3;
    const double dphi = c.damp[0] * e0 + c.damp[1] * e1 + c.damp[2] * e2 + c.damp[3] * e3;
    coef = fma(phi, inv_r, dphi) * (inv_r * inv_r);
    if constexpr (FK) ew = firsov_shape(r, c.lam2);
    else ew = exp2_neg_pair(r, c.lam2);
}

// ln x for finite normal x > 0, written from the mathematics: x = m 2^k with m in
// [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s), s = (m - 1) / (m + 1) (m - 1 exact), |s| <= 0.1716,
// from the odd series 2 s (1 + s^2/3 + s^4/5 + ... + s^22/23) (the first term left out is below
// 1e-19 of the sum); k ln 2 with ln 2 split so that k times its leading part is exact.
__device__ __forceinline__ double log_pos(double x)
{
    constexpr double kLn2Hi = 6.93147180369123816490e-01;   // ln 2 to 32 bits
    constexpr double kLn2Lo = 1.90821492927058770002e-10;   // ln 2 - kLn2Hi
    double m = __builtin_amdgcn_frexp_mant(x);               // [1/2, 1)
    int k = __builtin_amdgcn_frexp_exp(x);
    if (m < 0.70710678118654752440) {
        m += m;
        --k;
    }
    const double s = (m - 1.0) / (m + 1.0);
    const double z = s * s;
    double q = 1.0 / 23.0;
    q = fma(q, z, 1.0 / 21.0);
    q = fma(q, z, 1.0 / 19.0);
    q = fma(q, z, 1.0 / 17.0);
    q = fma(q, z, 1.0 / 15.0);
    q = fma(q, z, 1.0 / 13.0);
    q = fma(q, z, 1.0 / 11.0);
    q = fma(q, z, 1.0 / 9.0);
    q = fma(q, z, 1.0 / 7.0);
    q = fma(q, z, 1.0 / 5.0);
    q = fma(q, z, 1.0 / 3.0);
    q = fma(q, z, 1.0);
    const double kd = static_cast<double>(k);
    return fma(kd, kLn2Hi, fma(kd, kLn2Lo, 2.0 * s * q));
}

// ln(1 + x) for finite x >= 0 with its relative accuracy kept for small x: with u = 1 + x
// rounded, ln u scaled by x / (u - 1), the ratio of the exact to the rounded argument.
__device__ __forceinline__ double log1p_pos(double x)
{
    const double u = 1.0 + x;
    return (u == 1.0) ? x : log_pos(u) * (x / (u - 1.0));
}

// Brandt-Kitagawa friction of the ion at speed squared v2 (sqrt(eV/amu))^2:
// pref zeta^2 with pref = k Z1^2 gamma_p (the slow-proton friction of the
// electron gas), zeta the effective-charge fraction in atomic units,
//   zeta = q + (1 - q) / (2 vF^2) ln(1 + (2 Lambda vF)^2),
//   Lambda = 0.48 (1-q)^(2/3) / (Z1^(1/3) (1 - (1-q)/7)),
//   q = 1 - exp(0.803 y^0.3 - 1.3167 y^0.6 - 0.38157 y - 0.008983 y^2) in [0, 1],
//   y = v_r / Z1^(2/3), v_r = v (1 + vF^2 / (5 v^2)) (v >= vF),
//   (3 vF / 4)(1 + 2 v^2 / (3 vF^2) - v^4 / (15 vF^4)) (v < vF)
// (Brandt and Kitagawa 1982; q from the Ziegler-Biersack-Littmark fit).
__device__ __noinline__ double bk_friction(double v2, double pref, double z13, double vF, double inv_vunit)
{
    const double u = sqrt(v2) * inv_vunit;
    const double vF2 = vF * vF;
    double vr;
    if (u >= vF) {
        vr = u * (1.0 + vF2 / (5.0 * u * u));
    } else {
        const double s = u * u / vF2;
        vr = 0.75 * vF * (1.0 + (2.0 / 3.0) * s - s * s / 15.0);
    }
    const double y = vr / (z13 * z13);
    // the powers as exponentials of logarithms (exp_neg takes arguments of either sign here:
    // its reduction holds for |argument| below 700)
    const double y3 = exp_neg(-0.3 * log_pos(y));                                 // y^0.3
    double q = 1.0 - exp_neg(-(0.803 * y3 - 1.3167 * y3 * y3 - 0.38157 * y - 0.008983 * y * y));
    q = fmin(fmax(q, 0.0), 1.0);
    const double nb = 1.0 - q;
    const double nb23 = nb > 0.0 ? exp_neg(-(2.0 / 3.0) * log_pos(nb)) : 0.0;      // nb^(2/3)
    const double lam = 0.48 * nb23 / (z13 * (1.0 - nb / 7.0));
    const double a = 2.0 * lam * vF;
    const double zeta = q + nb / (2.0 * vF2) * log1p_pos(a * a);
    return pref * zeta * zeta;
}

// FP32 variant of the pair term (force precision option; tolerance 1e-5
// relative per step instead of 1e-10): the separation comes in FP64 and is
// rounded once; the distance (hardware 1/sqrt), the four screening terms and
// the density weight (hardware 2^x of an FP32 argument: relative error about
// |argument| x 6e-8, below 2e-6 for every term that is not negligible) and the
// coefficient are FP32.  The caller keeps FP64 for the force components, the
// sums, kicks, drifts and the step size.
template <class PC>
__device__ __forceinline__ void zbl_pair_f32(const PC& c, double dx, double dy, double dz, double& coef, double& ew)
{
    const float x = static_cast<float>(dx), y = static_cast<float>(dy), z = static_cast<float>(dz);
    const float r2 = fmaf(x, x, fmaf(y, y, z * z));
    const float inv_r = __builtin_amdgcn_rsqf(r2);
    const float r = r2 * inv_r;
    const float e0 = __builtin_amdgcn_exp2f(-r * c.rate2f[0]);
    const float e1 = __builtin_amdgcn_exp2f(-r * c.rate2f[1]);
    const float e2 = __builtin_amdgcn_exp2f(-r * c.rate2f[2]);
    const float e3 = __builtin_amdgcn_exp2f(-r * c.rate2f[3]);
    const float phi = c.amp_f[0] * e0 + c.amp_f[1] * e1 + c.amp_f[2] * e2 + c.amp_f[3] * e3;
    const float dphi = c.damp_f[0] * e0 + c.damp_f[1] * e1 + c.damp_f[2] * e2 + c.damp_f[3] * e3;
    coef = static_cast<double>(fmaf(phi, inv_r, dphi) * (inv_r * inv_r));
    ew = static_cast<double>(__builtin_amdgcn_exp2f(-r * c.lam2f));
}

// The unique cell coordinate in {c-1, c, c+1} whose residue mod 3 is `res`.
__device__ __forceinline__ int cell_of_residue(int res, int c)
{
    int off = (res - c) % 3;
    if (off < 0) off += 3;
    return c + (off == 2 ? -1 : off);
}

// True when floor(x / a) == c for certain, decided from x * (1/a) away from the
// cell faces; near a face the caller evaluates floor(x / a) exactly.
__device__ __forceinline__ bool inside_cell(double x, int c, double a, double inv_a)
{
    const double q = x * inv_a - static_cast<double>(c);
    return q > 1e-9 && q < 1.0 - 1e-9;
}

__device__ __forceinline__ int floor_cell(double x, double a)
{
    // clamped so that a runaway (later quarantined) state cannot overflow the cast
    return static_cast<int>(fmin(fmax(floor(x / a), -1.0e8), 1.0e8));
}

}  // namespace reedmd
