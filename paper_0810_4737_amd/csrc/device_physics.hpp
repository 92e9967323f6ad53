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
    constexpr double kTwoPi = 6.283185307179586476925286766559;
    const double rad0 = sqrt(-2.0 * log(open_unit(r.w[0])));
    const double rad1 = sqrt(-2.0 * log(open_unit(r.w[2])));
    double s0, c0, s1, c1;
    sincos(kTwoPi * open_unit(r.w[1]), &s0, &c0);
    sincos(kTwoPi * open_unit(r.w[3]), &s1, &c1);
    gx = rad0 * c0;
    gy = rad0 * s0;
    gz = rad1 * c1;
}

// Fractional diamond-cubic basis: fcc sites, then the same plus (1/4,1/4,1/4).
__device__ __forceinline__ void basis_site(int b, double& fx, double& fy, double& fz)
{
    const int q = b & 3;
    const double sh = (b >= 4) ? 0.25 : 0.0;
    fx = ((q == 2 || q == 3) ? 0.5 : 0.0) + sh;
    fy = ((q == 1 || q == 3) ? 0.5 : 0.0) + sh;
    fz = ((q == 1 || q == 2) ? 0.5 : 0.0) + sh;
}

// Position of a newly created atom: ideal site of basis atom b in cell
// (nx,ny,nz) plus its thermal displacement.  Kept out of line so that the
// rarely taken domain update does not raise the register budget of the step.
#ifdef REEDMD_NOINLINE_CREATE
__device__ __attribute__((noinline)) double3 create_atom(uint64_t key, uint64_t seed, int nx, int ny, int nz, int b,
                                                          double a, double sigma)
#else
__device__ __forceinline__ double3 create_atom(uint64_t key, uint64_t seed, int nx, int ny, int nz, int b,
                                                double a, double sigma)
#endif
{
    double fx, fy, fz, gx, gy, gz;
    basis_site(b, fx, fy, fz);
    thermal_gauss(key, seed, nx, ny, nz, b, gx, gy, gz);
    return make_double3(a * (static_cast<double>(nx) + fx) + sigma * gx,
                        a * (static_cast<double>(ny) + fy) + sigma * gy,
                        a * (static_cast<double>(nz) + fz) + sigma * gz);
}

// ---------------------------------------------------------------------------
// exp(-y) for the force kernels, written from the mathematics: Cody-Waite
// range reduction y = n ln2 + r with ln 2 split into a double and its
// remainder (both FMA-exact), |r| <= ln2/2, the Taylor series of e^r to r^12
// (truncation < 2e-16 relative), and scaling by 2^n (ldexp handles the
// gradual underflow of very small results).  No overflow or NaN handling is
// needed: arguments are distances over positive lengths (y >= 0, bounded).
__device__ __forceinline__ double exp_neg(double y)
{
    constexpr double kLog2e = 1.4426950408889634;
    constexpr double kLn2Hi = 0x1.62e42fefa39efp-1;
    constexpr double kLn2Lo = 0x1.abc9e3b39803fp-56;
    const double t = -fmin(y, 1500.0);
    const double n = rint(t * kLog2e);
    double r = fma(-n, kLn2Hi, t);
    r = fma(-n, kLn2Lo, r);
    double p = 2.08767569878681e-09;            // 1/12!
    p = fma(p, r, 2.505210838544172e-08);       // 1/11!
    p = fma(p, r, 2.755731922398589e-07);       // 1/10!
    p = fma(p, r, 2.7557319223985893e-06);      // 1/9!
    p = fma(p, r, 2.48015873015873e-05);        // 1/8!
    p = fma(p, r, 0.0001984126984126984);       // 1/7!
    p = fma(p, r, 0.001388888888888889);        // 1/6!
    p = fma(p, r, 0.008333333333333333);        // 1/5!
    p = fma(p, r, 0.041666666666666664);        // 1/4!
    p = fma(p, r, 0.16666666666666666);         // 1/3!
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, static_cast<int>(n));
}

// ---------------------------------------------------------------------------
// ZBL universal screening function phi(x) = sum c_i exp(-d_i x).
constexpr double kZc0 = 0.18175, kZc1 = 0.50986, kZc2 = 0.28022, kZc3 = 0.02817;
constexpr double kZd0 = 3.19980, kZd1 = 0.94229, kZd2 = 0.40290, kZd3 = 0.20162;

// Pair term for an ion at separation (dx,dy,dz) = x_ion - x_atom:
//   coef: force on the ion is coef * (dx,dy,dz) (the atom feels the opposite),
//         coef = -V'(r) / r with V = zz phi(r/a) / r;
//   wr:   density weight wnorm * exp(-r/lambda).
__device__ __forceinline__ void zbl_pair(double inv_a, double zz, double inv_lambda, double wnorm, double dx,
                                         double dy, double dz, double& coef, double& wr)
{
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double inv_r = rsqrt(r2);
    const double r = r2 * inv_r;
    const double xs = r * inv_a;
    const double e0 = exp_neg(kZd0 * xs);
    const double e1 = exp_neg(kZd1 * xs);
    const double e2 = exp_neg(kZd2 * xs);
    const double e3 = exp_neg(kZd3 * xs);
    const double phi = kZc0 * e0 + kZc1 * e1 + kZc2 * e2 + kZc3 * e3;
    const double dphi = -(kZc0 * kZd0 * e0 + kZc1 * kZd1 * e1 + kZc2 * kZd2 * e2 + kZc3 * kZd3 * e3);
    // V'(r) = zz (phi'(x) / (a r) - phi(x) / r^2)
    const double dVdr = zz * inv_r * (dphi * inv_a - phi * inv_r);
    coef = -dVdr * inv_r;
    wr = wnorm * exp_neg(r * inv_lambda);
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
