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

/* Friction coefficient gamma (force = -gamma v) at local density rho. */
double or_gamma(const or_params* p, int species, double rho)
{
    if (p->stop_mode == OR_STOP_OFF) return 0.0;
    double N = uniform_density(p, species);
    double gamma0 = N * or_lss_kL(p, species, 0) * sqrt(p->M1[species] / 2.0);
    if (p->stop_mode == OR_STOP_UNIFORM) return p->k * gamma0;
    return p->k * gamma0 * rho / N;
}
