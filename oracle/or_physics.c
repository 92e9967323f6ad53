/*
 * Interaction models for the oracle.  TEST INFRASTRUCTURE ONLY.
 *
 * Sec. 2 ("First", "Second") names the ZBL universal screened nuclear
 * potential as the only ion-atom interaction; its functional form is given
 * by Ziegler, Biersack and Littmark (1985), which the paper cites for it:
 *   V(r) = Z1 Z2 e^2 / r * phi(r / a),   phi(x) = sum_i c_i exp(-d_i x),
 *   a_U = 0.8854 a0 / (Z1^0.23 + Z2^0.23).
 * The screening-length scale s multiplies a_U (a = s a_U); s = 1 is ZBL.
 *
 * Sec. 2 ("Third") models electronic stopping as a local loss that depends
 * on the electron density near the ion.  The configured reading is a local
 * Lindhard-Scharff friction:
 *   S_e(E) = k_L sqrt(E),  k_L = 1.212 Z1^(7/6) Z2 / ((Z1^(2/3)+Z2^(2/3))^(3/2) sqrt(M1))
 *   (eV A^2 with E in eV and M1 in amu),
 * applied as a friction force -gamma(x) v with gamma(x) = k gamma0 rho(x)/N,
 * gamma0 = N k_L sqrt(M1/2), where rho(x) = sum_j w(|x - x_j|) is a local
 * density built from an exponential weight w(r) = exp(-r/lambda)/(8 pi lambda^3)
 * (unit integral, so rho averages to the atomic density N), with
 * lambda = a_U / 0.3 (the Oen-Robinson decay length).
 *
 * Two target species (fluorite): every pair uses the constants of its own
 * target atomic number.  The stopping adds over species (Bragg's rule): each
 * atom's density weight enters rho with the factor k_L(t)/k_L(0), so that
 * gamma = k k_L(0) sqrt(M1/2) rho, and rho averages to sum_t N_t k_L(t)/k_L(0);
 * with one species this is the form above.
 *
 * The paper's own stopping model (Sec. 2, "Third"; its parameters are not
 * printed) has two parts, read here from the works it cites:
 *  - a local inelastic loss after Firsov (1959) in Kishinevskii's local
 *    form: Firsov's energy loss in a collision at distance of closest approach
 *    R is 0.05973 (Z1+Z2)^(5/3) sqrt(E/M1) / (1 + b R)^5 eV with
 *    b = 0.31 (Z1+Z2)^(1/3) per A (E in eV, M1 in amu); its impact-parameter
 *    integral gives Firsov's stopping cross-section
 *    S_F = 0.05973 (Z1+Z2)^(5/3) 2 pi / (12 b^2) sqrt(E/M1) = 0.3254 (Z1+Z2) sqrt(E/M1) eV A^2.
 *    The reading used makes the loss a friction summed over the domain atoms,
 *    gamma_F = sum_j C 3 b^3 / (pi (1 + b r_j)^5), whose radial kernel has unit
 *    volume integral, so an ion crossing a uniform target loses N S_F per unit
 *    length: C = S_F / v = 0.3254 (Z1+Z2) / sqrt(2) (v in sqrt(eV/amu)).  Each
 *    atom uses its own target atomic number.
 *  - a non-local loss after Brandt and Kitagawa (1982): the ion of fractional
 *    ionisation q carries the effective charge zeta Z1 with
 *      zeta = q + (1 - q) / (2 vF^2) ln(1 + (2 Lambda vF)^2)   (atomic units),
 *      Lambda = 0.48 (1-q)^(2/3) / (Z1^(1/3) (1 - (1-q)/7)),
 *    q from the Ziegler-Biersack-Littmark fit
 *      q = 1 - exp(0.803 y^0.3 - 1.3167 y^0.6 - 0.38157 y - 0.008983 y^2),
 *      y = v_r / Z1^(2/3), clamped to [0, 1],
 *    with the relative velocity of ion and electrons v_r = v (1 + vF^2 / (5 v^2))
 *    for v >= vF and (3 vF / 4)(1 + 2 v^2 / (3 vF^2) - v^4 / (15 vF^4)) below; and
 *    the loss is (zeta Z1)^2 times that of a slow proton in an electron gas of
 *    density n_e (Ritchie 1959): friction
 *      gamma_p = 2 / (3 pi) [ln(1 + pi / (alpha rs)) - 1 / (1 + alpha rs / pi)],
 *      alpha = (4 / (9 pi))^(1/3), rs = (3 / (4 pi n_e))^(1/3), vF = (9 pi / 4)^(1/3) / rs.
 *    n_e is the interstitial (muffin-tin residual) electron density, a target
 *    parameter (the paper computes it from a muffin-tin model; the value is not
 *    printed).  Both frictions are scaled by k:
 *      gamma = k (gamma_F(x) + (zeta Z1)^2 gamma_p)   (force -gamma v).
 */
#include <math.h>
#include "or_internal.h"

static const double zbl_c[4] = {0.18175, 0.50986, 0.28022, 0.02817};
static const double zbl_d[4] = {3.19980, 0.94229, 0.40290, 0.20162};

static double target_Z(const or_params* p, int type)
{
    return (double)(type ? p->Z2b : p->Z2);
}

double or_unscaled_screening_length(const or_params* p, int species, int type)
{
    return 0.8854 * OR_BOHR / (pow((double)p->Z1[species], 0.23) + pow(target_Z(p, type), 0.23));
}

double or_screening_length(const or_params* p, int species, int type)
{
    return p->s * or_unscaled_screening_length(p, species, type);
}

/* Constants of one ion species against target species `type` (computed once
 * per force evaluation; the values are the same as computing them per pair). */
void or_pair_constants(const or_params* p, int species, int type, or_pair_consts* c)
{
    c->on = p->pot_mode != OR_POT_NONE;
    c->a = or_screening_length(p, species, type);
    c->zz = (double)p->Z1[species] * target_Z(p, type) * OR_COULOMB;
    c->lambda = or_unscaled_screening_length(p, species, type) / 0.3;
    c->wscale = or_lss_kL(p, species, type) / or_lss_kL(p, species, 0);
    c->firsov = p->stop_mode == OR_STOP_FKBK;
    c->fk_b = or_firsov_b(p, species, type);
    c->fk_norm = or_firsov_norm(p, species, type);
}

/* ZBL pair potential and its radial derivative. */
void or_zbl_c(const or_pair_consts* c, double r, double* V, double* dVdr)
{
    if (!c->on) {
        *V = 0.0;
        *dVdr = 0.0;
        return;
    }
    double x = r / c->a;
    double phi = 0.0, dphi = 0.0;
    for (int i = 0; i < 4; ++i) {
        double e = exp(-zbl_d[i] * x);
        phi += zbl_c[i] * e;
        dphi -= zbl_c[i] * zbl_d[i] * e;
    }
    *V = c->zz * phi / r;
    /* d/dr [zz phi(r/a) / r] = zz (phi'(x)/(a r) - phi(x)/r^2) */
    *dVdr = c->zz * (dphi / (c->a * r) - phi / (r * r));
}

void or_zbl(const or_params* p, int species, int type, double r, double* V, double* dVdr)
{
    or_pair_consts c;
    or_pair_constants(p, species, type, &c);
    or_zbl_c(&c, r, V, dVdr);
}

double or_pair_potential(const or_params* p, int species, int type, double r)
{
    double V, dV;
    or_zbl(p, species, type, r, &V, &dV);
    return V;
}

double or_lss_kL(const or_params* p, int species, int type)
{
    double Z1 = (double)p->Z1[species], Z2 = target_Z(p, type), M1 = p->M1[species];
    double z23 = pow(Z1, 2.0 / 3.0) + pow(Z2, 2.0 / 3.0);
    return 1.212 * pow(Z1, 7.0 / 6.0) * Z2 / (pow(z23, 1.5) * sqrt(M1));
}

/* Atoms of target species `type` per unit volume. */
double or_number_density(const or_params* p, int type)
{
    double per_cell = (p->structure == OR_FLUORITE) ? (type ? 8.0 : 4.0) : (type ? 0.0 : (double)OR_NBASIS);
    return per_cell / (p->a * p->a * p->a);
}

/* Stopping-weighted density of the uniform crystal: sum_t N_t k_L(t)/k_L(0). */
static double uniform_density(const or_params* p, int species)
{
    double n = or_number_density(p, 0);
    if (p->structure == OR_FLUORITE)
        n += or_number_density(p, 1) * or_lss_kL(p, species, 1) / or_lss_kL(p, species, 0);
    return n;
}

double or_density_weight_c(const or_pair_consts* c, double r)
{
    return c->wscale * exp(-r / c->lambda) / (8.0 * OR_PI * c->lambda * c->lambda * c->lambda);
}

double or_density_weight(const or_params* p, int species, int type, double r)
{
    or_pair_consts c;
    or_pair_constants(p, species, type, &c);
    return or_density_weight_c(&c, r);
}

/* Firsov's screening constant b (1/A) and the friction normalisation C 3 b^3 / pi. */
double or_firsov_b(const or_params* p, int species, int type)
{
    return 0.31 * cbrt((double)p->Z1[species] + target_Z(p, type));
}

double or_firsov_norm(const or_params* p, int species, int type)
{
    double zs = (double)p->Z1[species] + target_Z(p, type);
    double C = 0.3254 * zs / sqrt(2.0);
    double b = or_firsov_b(p, species, type);
    return C * 3.0 * b * b * b / OR_PI;
}

double or_firsov_weight_c(const or_pair_consts* c, double r)
{
    return c->fk_norm / pow(1.0 + c->fk_b * r, 5.0);
}

double or_firsov_weight(const or_params* p, int species, int type, double r)
{
    or_pair_consts c;
    or_pair_constants(p, species, type, &c);
    return or_firsov_weight_c(&c, r);
}

/* Atomic units: Hartree (eV), velocity (m/s); the velocity unit sqrt(eV/amu) in m/s. */
#define OR_HARTREE 27.211386245988
#define OR_AU_VELOCITY 2.18769126364e6
static double velocity_unit(void) { return sqrt(1.602176634e-19 / 1.66053906660e-27); }

static double wigner_seitz_radius(const or_params* p)
{
    double n_au = p->n_e * OR_BOHR * OR_BOHR * OR_BOHR;   /* electrons per bohr^3 */
    return cbrt(3.0 / (4.0 * OR_PI * n_au));
}

/* Brandt-Kitagawa effective-charge fraction zeta at ion speed v (sqrt(eV/amu)). */
double or_bk_zeta(const or_params* p, int species, double v)
{
    double Z1 = (double)p->Z1[species];
    double rs = wigner_seitz_radius(p);
    double vF = cbrt(9.0 * OR_PI / 4.0) / rs;
    double u = v * velocity_unit() / OR_AU_VELOCITY;
    double vr;
    if (u >= vF)
        vr = u * (1.0 + vF * vF / (5.0 * u * u));
    else
        vr = 0.75 * vF * (1.0 + 2.0 * u * u / (3.0 * vF * vF) - pow(u, 4.0) / (15.0 * pow(vF, 4.0)));
    double y = vr / pow(Z1, 2.0 / 3.0);
    double q = 1.0 - exp(0.803 * pow(y, 0.3) - 1.3167 * pow(y, 0.6) - 0.38157 * y - 0.008983 * y * y);
    if (q < 0.0) q = 0.0;
    if (q > 1.0) q = 1.0;
    double lam = 0.48 * pow(1.0 - q, 2.0 / 3.0) / (cbrt(Z1) * (1.0 - (1.0 - q) / 7.0));
    return q + (1.0 - q) / (2.0 * vF * vF) * log(1.0 + (2.0 * lam * vF) * (2.0 * lam * vF));
}

/* Slow-proton friction in the electron gas, converted from atomic units
 * (Hartree / bohr per atomic velocity unit) to eV / A per sqrt(eV/amu). */
double or_bk_proton_friction(const or_params* p)
{
    double rs = wigner_seitz_radius(p);
    double alpha = cbrt(4.0 / (9.0 * OR_PI));
    double g_au = 2.0 / (3.0 * OR_PI) * (log(1.0 + OR_PI / (alpha * rs)) - 1.0 / (1.0 + alpha * rs / OR_PI));
    double force_unit = OR_HARTREE / OR_BOHR;
    double speed_unit = OR_AU_VELOCITY / velocity_unit();
    return g_au * force_unit / speed_unit;
}

/* Brandt-Kitagawa friction (zeta Z1)^2 gamma_p at speed v; 0 without electrons. */
double or_bk_gamma(const or_params* p, int species, double v)
{
    if (!(p->n_e > 0.0)) return 0.0;
    double zq = or_bk_zeta(p, species, v) * (double)p->Z1[species];
    return zq * zq * or_bk_proton_friction(p);
}

/* Friction coefficient (force = -gamma v) with the ion's speed squared v2: the
 * Brandt-Kitagawa part depends on the speed, the others do not. */
double or_stopping_gamma(const or_params* p, int species, double rho, double v2)
{
    double g = or_gamma(p, species, rho);
    if (p->stop_mode == OR_STOP_FKBK) g += p->k * or_bk_gamma(p, species, sqrt(v2));
    return g;
}

/* Friction coefficient gamma (force = -gamma v) at local density rho, without
 * the speed-dependent Brandt-Kitagawa part (rho is the Firsov sum in OR_STOP_FKBK). */
double or_gamma(const or_params* p, int species, double rho)
{
    if (p->stop_mode == OR_STOP_OFF) return 0.0;
    if (p->stop_mode == OR_STOP_FKBK) return p->k * rho;
    double N = uniform_density(p, species);
    double gamma0 = N * or_lss_kL(p, species, 0) * sqrt(p->M1[species] / 2.0);
    if (p->stop_mode == OR_STOP_UNIFORM) return p->k * gamma0;
    return p->k * gamma0 * rho / N;
}
