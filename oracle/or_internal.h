/* Internal declarations shared by the oracle's own source files only.
 * TEST INFRASTRUCTURE ONLY (see oracle.h). */
#ifndef REEDMD_OR_INTERNAL_H
#define REEDMD_OR_INTERNAL_H
#include "oracle.h"

/* CODATA 2018: e^2/(4 pi eps0) in eV*A, and the Bohr radius in A. */
#define OR_COULOMB 14.3996454784
#define OR_BOHR 0.529177210903
#define OR_PI 3.14159265358979323846

/* RNG stream tags (first counter word) */
enum { OR_TAG_SAMPLE = 1, OR_TAG_PRIMARY_KEY = 2, OR_TAG_THERMAL = 3, OR_TAG_CHILD_KEY = 4 };

void or_gauss3(uint64_t key, uint64_t seed, int64_t cx, int64_t cy, int64_t cz, int b, double g[3]);
uint64_t or_child_key(uint64_t key, uint64_t seed, int32_t k, int32_t i);
uint64_t or_primary_key(uint64_t seed, int64_t id);

typedef struct {
    int on;
    double a, zz, lambda, wscale;
    int firsov;           /* OR_STOP_FKBK: the stopping weight is Firsov's kernel */
    double fk_b, fk_norm;
} or_pair_consts;
void or_pair_constants(const or_params* p, int species, int type, or_pair_consts* c);
void or_zbl_c(const or_pair_consts* c, double r, double* V, double* dVdr);
double or_density_weight_c(const or_pair_consts* c, double r);
double or_firsov_weight_c(const or_pair_consts* c, double r);

double or_number_density(const or_params* p, int type);
double or_pair_potential(const or_params* p, int species, int type, double r);

void or_compute_forces(const or_params* p, or_track* t);
int or_nbasis(const or_params* p);
double or_type_mass(const or_params* p, int type);

#endif
