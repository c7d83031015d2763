/*
 * fspic_oracle.h -- plain, sequential FP64 reference of the 1D3V electrostatic
 * particle-in-cell cycle with null-collision Monte-Carlo collisions.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, includes or
 * calls this code; only the test suite, the smoke check and the CPU baseline of the
 * benchmark load it.  It shares no source with the HIP path.
 *
 * What it computes follows the paper's cycle (Sec. 2, Fig. "pic_cycle"): linear
 * charge assignment, tridiagonal Poisson solve (Thomas algorithm, Sec. 3.5),
 * leap-frog push with linear field gather (Sec. 3.6), removal of particles that
 * left the box, modified null-collision MCC (Sec. 3.8, eq. null_collision), and the
 * particle array kept sorted by cell (Sec. 3.7), in the normalised units of Sec. 3.3.
 */
#ifndef FSPIC_ORACLE_H
#define FSPIC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_XS_NONE = 0, ORC_XS_CONST_E_ELASTIC = 1, ORC_XS_AR_LIKE = 2 };
enum { ORC_LOAD_RANDOM = 0, ORC_LOAD_QUIET_LANGMUIR = 1 };
enum { ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_CAPACITY = -2, ORC_ERR_ID_OVERFLOW = -5 };

typedef struct orc_params {
    int32_t periodic;        /* 1: periodic box, 0: two absorbing electrodes */
    int32_t n_cells;         /* number of grid cells N */
    int64_t n_e0, n_i0;      /* initial macro-particles per species */
    double length_m, dt_s, n0_m3, te_ev, ti_ev, mass_i_amu;
    double v0_volt, freq_hz, gas_pa, gas_k;
    int32_t xsec;            /* ORC_XS_* */
    double sigma_const_m2, eps_cap_ev;
    uint32_t seed, discharge;
    int32_t load;            /* ORC_LOAD_* */
    double langmuir_amp_cells;
    int32_t langmuir_mode;
    int32_t fp32_offset;     /* 1: positions as cell + FP32 offset, FP32 velocities */
    int32_t eedf_bins;
    double eedf_max_ev;
    int32_t diag_every;
    int64_t avg_start;
    /* Array order after a step: ORC_SORT_CELL keeps the survivors stably sorted by cell
       (Sec. 3.7); ORC_SORT_NONE keeps them in input order (the unsorted variant of
       Sec. 3.2); ORC_SORT_LAG sorts them stably by the cell they occupied at the start of
       the step, so the array is sorted with a lag of one step.  Births follow the
       survivors in every mode. */
    int32_t sort_mode;
    /* ORC_RANK_PARENT_INDEX: births take ids in the array order of their parents;
       ORC_RANK_PARENT_ID: in increasing parent id (for a layout whose order within a
       sorting cell is not fixed). */
    int32_t birth_rank;
    /* Binary Coulomb collisions between particles of one grid cell (Sec. 3.2 names them
       as what fine sorting makes simple): bit 0 e-e, bit 1 i-i, bit 2 e-i; Coulomb
       logarithm. */
    int32_t coulomb;
    double coulomb_log;
    /* Electrode processes (Sec. 2: electrons inserted at the boundaries): each absorbed
       ion emits a secondary electron with probability see_gamma, from a half-Maxwellian
       at see_te_ev; an electron reaching an electrode is reflected with probability
       refl_e. */
    double see_gamma, see_te_ev, refl_e;
    /* External circuit (Sec. 3.5 defers boundary conditions to the literature): a
       capacitor of circuit_cap_f_m2 farad per electrode area in series between the source
       and the driven electrode; 0 keeps the ideal voltage source. */
    double circuit_cap_f_m2;
} orc_params;

enum { ORC_SORT_CELL = 0, ORC_SORT_NONE = 1, ORC_SORT_LAG = 2 };
enum { ORC_RANK_PARENT_INDEX = 0, ORC_RANK_PARENT_ID = 1 };
enum { ORC_COUL_EE = 1, ORC_COUL_II = 2, ORC_COUL_EI = 4 };

typedef struct orc_consts {
    double dx, weight_per_area, kappa[2], phi_scale, vunit, energy_c[2];
    double vth[2], vth_gas, n_gas, nu0[2], p0[2], vhat_amp, drive_phase_per_step;
    double mass[2];
    uint32_t t0[2];
} orc_consts;

typedef struct orc_tallies {
    int64_t step;
    uint32_t next_id[2];
    int64_t absorbed[2][2];           /* [species][wall 0 left, 1 right] */
    double absorbed_energy_ev[2][2];
    int64_t births[2];
    int64_t collisions[2][3];         /* e: elastic, excitation, ionization; i: isotropic, cx */
    int64_t acc_count, eedf_samples;
    int64_t emitted[2];               /* secondary electrons per wall */
    int64_t reflected[2];             /* reflected electrons per wall */
    /* Of the last step, normalised units (energy Q^2 dx / (eps0 A), momentum
       Q^2 dt / (eps0 A), charge Q / A): kinetic energy per species, the mean of the
       values before and after the push (velocities before the collisions); field energy
       1/2 sum over cells of (Phi_j - Phi_j+1)^2; x-momentum sum v_x / |kappa_s| after the
       push; sum of the net node charge; the driven electrode's potential; the charge of
       the driven electrode's conductor (electrode surface + capacitor plate). */
    double kinetic[2], field_energy, momentum, sum_rho, phi0, q_circuit;
} orc_tallies;

typedef struct orc_sim orc_sim;

orc_sim* orc_create(const orc_params* p, int64_t cap_e, int64_t cap_i);
void orc_destroy(orc_sim* s);
int orc_get_consts(const orc_sim* s, orc_consts* out);
int orc_load(orc_sim* s);
int orc_step(orc_sim* s);
int64_t orc_count(const orc_sim* s, int species);
int orc_get_particles(const orc_sim* s, int species, double* x, double* vx, double* vy,
                      double* vz, uint32_t* id);
int orc_set_particles(orc_sim* s, int species, int64_t n, const double* x, const double* vx,
                      const double* vy, const double* vz, const uint32_t* id);
/* what: 0 w_e, 1 w_i, 2 phi, 3 E, 4 acc w_e, 5 acc w_i, 6 acc phi, 7 eedf (bins+1) */
int orc_get_grid(const orc_sim* s, int what, double* out);
int orc_set_grid(orc_sim* s, int what, const double* in);
int orc_get_tallies(const orc_sim* s, orc_tallies* out);
int orc_set_counters(orc_sim* s, int64_t step, uint32_t next_id_e, uint32_t next_id_i);

/* Unit-level entry points used by the pins; the cycle above calls the same routines. */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_u53(uint32_t a, uint32_t b);
void orc_xsec(int model, int species, double eps_ev, double sigma_const, double out[3]);
int orc_solve(int periodic, int n_cells, const double* rho, double phi_left, double* phi,
              double* efield);
void orc_deposit(int periodic, int n_cells, int64_t n, const double* x, double* w);
void orc_stable_sort_by_cell(int64_t n, const int32_t* cell, int n_cells, int64_t* perm);
/* Push n particles once in the field E (node values); flags[i] = 0 kept, 1 left wall, 2 right. */
void orc_push(int periodic, int n_cells, int fp32_offset, double kappa, const double* efield,
              int64_t n, double* x, double* vx, int32_t* flags);
/* One electron-neutral or ion-neutral collision test on a single particle (tag 0 draws).
   Returns the channel taken (0 none, 1.. per species); v is updated in place; for an
   ionisation the secondary electron's and the new ion's velocities are written. */
int orc_collide(const orc_sim* s, int species, uint32_t id, int64_t step, double v[3],
                double v_sec[3], double v_ion[3]);
/* One binary Coulomb collision of a pair (species sa, sb; particle a's id and step key
   the draw); velocities updated in place; n_l_m3 the density that sets the rate.
   Returns 0, or 1 if the pair did not collide (zero relative velocity). */
int orc_coulomb_pair(const orc_sim* s, int sa, int sb, uint32_t id_a, int64_t step,
                     double n_l_m3, double va[3], double vb[3]);
void orc_coulomb_pairs(const orc_sim* s, int sa, int sb, int64_t n, const uint32_t* id_a,
                       int64_t step, double n_l_m3, double* va, double* vb);
/* Secondary electron of an ion absorbed at `wall` (0 at x = 0, 1 at x = N): returns 1 and
   its position and velocity if one is emitted. */
int orc_emit(const orc_sim* s, uint32_t ion_id, int64_t step, int wall, double* x,
             double v[3]);
/* Driven-electrode potential of the series-capacitor circuit for a node charge rho
   (normalised), source value vs and conductor charge q; phi and E are the solution. */
double orc_circuit_solve(const orc_sim* s, const double* rho, double vs, double q, double* phi,
                         double* efield);

#ifdef __cplusplus
}
#endif
#endif
