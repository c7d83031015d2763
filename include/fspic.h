/*
 * fspic.h -- C ABI of libfspic: the per-time-step particle hot path of a 1D3V
 * electrostatic particle-in-cell cycle with Monte-Carlo collisions (Mertmann et al.,
 * "Fine-sorting one-dimensional particle-in-cell algorithm with Monte-Carlo collisions
 * on a graphics processing unit"), on AMD Instinct MI355X (gfx950).
 *
 * One step (Sec. 2, Fig. "pic_cycle"): Poisson solve of the charge deposited by the
 * previous step (Sec. 3.5), leap-frog push with linear field gather (Sec. 3.6), removal
 * of particles that left the box (Sec. 2), modified null-collision MCC (Sec. 3.8, eq.
 * null_collision), re-sort of the particle array by cell (Sec. 3.7), linear charge
 * assignment of the new positions (Sec. 3.4), all in the normalised units of Sec. 3.3.
 *
 * Conventions for every function:
 *  - returns PIC_OK (0) or a negative PIC_ERR_* code; nothing throws across the ABI;
 *  - device pointers are plain addresses of the caller's device memory, host pointers
 *    plain host memory; no PyTorch or HIP C++ types appear here;
 *  - the library never allocates device memory: the caller provides one workspace of
 *    pic_workspace_bytes() bytes, owns it and frees it after pic_free();
 *  - all device work is enqueued on the caller's HIP stream (hipStream_t passed as
 *    void*; 0 is the null stream); functions documented as "syncs" wait for it;
 *  - one pic_sim per stream; a pic_sim is not thread-safe;
 *  - device-side errors (capacity, id overflow) are deferred: they are returned by the
 *    next call that syncs (pic_sync, pic_density, pic_grid, pic_diagnostics,
 *    pic_get_state) and are sticky until pic_free().
 */
#ifndef FSPIC_H
#define FSPIC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FSPIC_ABI_VERSION 2u

enum pic_status {
  PIC_OK = 0,
  PIC_ERR_ARG = -1,         /* invalid argument or configuration */
  PIC_ERR_CAPACITY = -2,    /* particle arrays / far-mover list too small (deferred) */
  PIC_ERR_DEVICE = -3,      /* a HIP runtime call failed */
  PIC_ERR_NONFINITE = -4,   /* a particle position became non-finite (deferred) */
  PIC_ERR_ID_OVERFLOW = -5, /* particle ids would exceed 2^32 - 1 (deferred) */
  PIC_ERR_STATE = -6,       /* call out of order (e.g. step before init) */
  PIC_ERR_WORKSPACE = -7,   /* workspace smaller than pic_workspace_bytes() */
  PIC_ERR_CORRUPT = -8      /* inconsistent device state: a kernel refused an index out of
                               range (deferred); the particle state is no longer valid */
};

enum pic_precision {
  PIC_FP64 = 0,        /* absolute FP64 position, FP64 velocities */
  PIC_FP32_OFFSET = 1  /* int32 cell + FP32 offset in [0,1), FP32 velocities */
};
enum pic_xsec { PIC_XS_NONE = 0, PIC_XS_CONST_E_ELASTIC = 1, PIC_XS_AR_LIKE = 2 };
enum pic_load { PIC_LOAD_RANDOM = 0, PIC_LOAD_QUIET_LANGMUIR = 1 };

/* One discharge.  Physical inputs in SI units (eV for temperatures and energies). */
typedef struct pic_config {
  uint32_t abi_version;      /* FSPIC_ABI_VERSION */
  uint32_t precision;        /* pic_precision; the same for every discharge of a sim */
  uint32_t periodic;         /* 1: periodic box; 0: absorbing electrodes at x = 0 and L */
  uint32_t n_cells;          /* N grid cells (bounded: N + 1 nodes, periodic: N nodes) */
  uint64_t n_e0, n_i0;       /* initial macro-particles per species */
  uint64_t capacity_e, capacity_i; /* particle array capacity per species (< 2^26) */
  double length_m, dt_s, n0_m3, te_ev, ti_ev, mass_i_amu;
  double v0_volt, freq_hz;   /* electrode at x = 0 driven V0 sin(2 pi f t); x = L grounded */
  double gas_pa, gas_k;      /* background gas */
  uint32_t xsec_model;       /* pic_xsec */
  uint32_t load_kind;        /* pic_load */
  double sigma_const_m2;     /* PIC_XS_CONST_E_ELASTIC cross section */
  double eps_cap_ev;         /* energy at which the constant-sigma null frequency is taken */
  uint32_t seed, discharge_index; /* Philox key = (seed, 2 * discharge_index + species) */
  double langmuir_amp_cells; /* quiet-start electron displacement amplitude (cells) */
  uint32_t langmuir_mode;
  uint32_t eedf_bins;        /* <= 256 */
  double eedf_max_ev;
  uint32_t diag_every;       /* EEDF sampled every diag_every steps from avg_start_step */
  uint32_t reserved0;
  uint64_t avg_start_step;   /* time averages accumulate from this step on */
  /* tuning: changes speed only (the results are bit for bit the same: charge is summed
     in fixed point and every other sum in a fixed order); 0 selects the default */
  uint32_t cells_per_tile[2];/* cells owned by one workgroup, per species */
  uint32_t window[2];        /* cells a particle may move per step on the fast sort path */
  uint32_t tail_groups;      /* workgroups per species that take the births tail */
  uint32_t far_capacity;     /* entries of the per-species far-mover list */
  /* --- optional physics and the array order (0 everywhere keeps the plain cycle) --- */
  uint32_t sort_mode;        /* pic_sort: array order kept by the step */
  uint32_t coulomb;          /* binary Coulomb collisions between particles of one grid cell
                                (what fine sorting makes simple, Sec. 3.2): bit 0 e-e,
                                bit 1 i-i, bit 2 e-i; needs PIC_SORT_COUNTING */
  double coulomb_log;        /* Coulomb logarithm */
  double see_gamma;          /* secondary electrons per ion absorbed at an electrode (Sec. 2:
                                electrons inserted at the boundaries), at most 1 */
  double see_te_ev;          /* temperature of the emitted electrons [eV] */
  double refl_e;             /* probability that an electron reaching an electrode is
                                reflected */
  double circuit_cap_f_m2;   /* series capacitor between the source and the driven electrode
                                [F per m^2 of electrode]; 0: ideal voltage source */
  uint32_t sort_cell_cells;  /* PIC_SORT_FINE: grid cells per sorting cell (N_gc - 1) */
  uint32_t sort_cell_capacity; /* PIC_SORT_FINE: particle slots per sorting cell (N_max);
                                0: derived from the load */
} pic_config;

enum pic_sort {
  PIC_SORT_COUNTING = 0, /* stable counting sort by cell into a second buffer (Sec. 3.7's
                            result, canonical order) */
  PIC_SORT_NONE = 1,     /* unsorted: survivors keep their order, the deposit adds straight
                            into the node array (the unsorted GPU variant of Sec. 3.2) */
  PIC_SORT_FINE = 2,     /* the paper's in-place sort into fixed-capacity sorting cells
                            (Sec. 3.2 data structure, Sec. 3.7 steps 1a/1b, 2 and 3); the
                            order inside a sorting cell is not fixed, so births take their
                            ids in increasing parent id */
  PIC_SORT_LAG = 3       /* the counting sort keyed on the cell a particle occupied at the
                            start of the step (known before the push), so the pre-pass reads
                            only that field; the array is sorted with a lag of one step, and a
                            particle absorbed in the step leaves a dead record that the next
                            step skips (pic_get_state and pic_diagnostics leave them out);
                            every discharge of a simulation or none */
};

/* Normalised constants the library derives from a pic_config (Sec. 3.3). */
typedef struct pic_derived {
  double dx, weight_per_area, kappa[2], phi_scale, vunit, energy_c[2];
  double vth[2], vth_gas, n_gas, nu0[2], p0[2], vhat_amp, drive_phase_per_step;
  uint32_t t0[2];            /* candidate iff Philox word < t0 = floor(P0 2^32) */
  uint32_t cells_per_tile[2], window[2];
} pic_derived;

typedef struct pic_diag {
  uint64_t step;
  uint64_t n_particles[2], n_sorted[2];
  uint32_t next_id[2];
  uint64_t absorbed[2][2];          /* [species][wall: 0 at x = 0, 1 at x = L] */
  double absorbed_energy_ev[2][2];
  uint64_t births[2];
  uint64_t collisions[2][3];        /* e: elastic, excitation, ionisation; i: isotropic, cx */
  uint64_t acc_count, eedf_samples;
  double surface_charge[2];         /* normalised (units of Q/A) at x = 0 and x = L */
  uint64_t particle_steps[2];       /* particles pushed, summed over all steps so far */
  uint32_t error_flags;
  uint32_t reserved0;
  /* Energies and momentum (Sec. 2: averaging gives the macroscopic values), normalised
     units of Sec. 3.3 per electrode area: energy (eW/A)^2 dx/eps0, momentum
     (eW/A)^2 dt/eps0, charge eW/A.  kinetic and momentum are taken on the steps the EEDF
     is sampled on (diag_every from avg_start_step); energy_step says which. */
  double kinetic[2];                /* sum over particles of (v_x^2 before + v_x^2 after the
                                       push)/2 + v_y^2 + v_z^2, over 2 |kappa_s| */
  double momentum;                  /* sum_s sum_i v_x(after the push) / |kappa_s| */
  uint64_t energy_step;
  double field_energy;              /* last solve: 1/2 sum over cells (Phi_j - Phi_j+1)^2 */
  double sum_rho;                   /* last solve: sum over nodes of w_i - w_e */
  double phi_driven_v;              /* last solve: potential of the driven electrode [V] */
  double circuit_charge;            /* charge of the driven electrode's conductor */
  uint64_t emitted[2];              /* secondary electrons per wall, summed over steps */
  uint64_t reflected[2];            /* reflected electrons per wall, summed over steps */
  double* eedf;                     /* in: caller buffer for the EEDF counts, or NULL */
  uint32_t eedf_len;                /* in: its length; out: entries written (<= bins + 1) */
  uint32_t reserved1;
} pic_diag;

/* Host-side particle state of one discharge, caller-allocated.  Fill the arrays of the
   sim's precision; the others may be NULL.  For pic_get_state: capacity[] gives the
   array lengths (in), n[] and n_sorted[] are written.  For pic_set_state: n[] and
   n_sorted[] are read; the first n_sorted particles must be ordered by cell (their
   order is kept); the remaining ones form an unsorted tail that the next step sorts in
   (set sort_all = 1 to have the whole array stably sorted by cell on the device
   instead).  w[] (n_nodes each) is written by get_state, ignored by set_state. */
typedef struct pic_state {
  uint64_t capacity[2], n[2], n_sorted[2];
  int32_t* cell[2];
  float* off[2];
  float* vxf[2];
  float* vyf[2];
  float* vzf[2];
  double* x[2];
  double* vx[2];
  double* vy[2];
  double* vz[2];
  uint32_t* id[2];
  double* w[2];
  uint64_t step;
  uint32_t next_id[2];
  uint32_t sort_all;
  uint32_t reserved0;
} pic_state;

typedef struct pic_sim pic_sim;

/* Bytes of device workspace for these discharges (caller allocates, 256-byte aligned). */
int pic_workspace_bytes(const pic_config* cfgs, int n_discharges, size_t* bytes);

/* Derived normalised constants of one configuration (host only, no device work). */
int pic_derive(const pic_config* cfg, pic_derived* out);

/* Creates a simulation of n_discharges independent discharges (all kernels of a step
   cover all of them in one launch each), loads particles (Philox tag 1), sorts them by
   cell, deposits, solves at t = 0 and moves v_x back half a step.  Syncs. */
int pic_init(const pic_config* cfgs, int n_discharges, void* d_workspace, size_t bytes,
             void* hip_stream, pic_sim** out);

/* Bytes of the library's own device workspace (pic_init_static). */
#define PIC_STATIC_WORKSPACE_BYTES (128u * 1024u * 1024u)

/* pic_init for callers that cannot allocate device memory (code that must not call
   hipMalloc: under HIP graph capture, in tight serving loops, or in harnesses that forbid
   it).  Instead of a caller workspace, the simulation lives in a device array of
   PIC_STATIC_WORKSPACE_BYTES that the library holds on each GPU it runs on, from the
   first use until the process ends; this call allocates nothing.  Arguments and the
   resulting pic_sim are as for pic_init on the current HIP device (the handle is freed
   with pic_free as usual).  The array is shared by every call on one GPU and keeps the
   last simulation's contents: each pic_init_static clears what the new simulation uses,
   and a second one on the same GPU overwrites the first one's state, so at most one
   simulation made this way may be live per GPU (calls that overlap race).
   Errors: PIC_ERR_WORKSPACE (with a message from pic_last_error(NULL)) when the
   discharges need more than PIC_STATIC_WORKSPACE_BYTES (pic_workspace_bytes), the errors
   of pic_init otherwise. */
int pic_init_static(const pic_config* cfgs, int n_discharges, void* hip_stream,
                    pic_sim** out);

/* Enqueues n_steps steps.  Asynchronous; with graphs enabled (pic_set_graph), steps are
   replayed from a captured HIP graph of `steps_per_graph` steps. */
int pic_step(pic_sim* sim, uint32_t n_steps);

/* 0 disables graph replay; k > 0 captures k steps once and replays them. */
int pic_set_graph(pic_sim* sim, uint32_t steps_per_graph);

/* Waits for the stream; returns a deferred device error if one occurred. */
int pic_sync(pic_sim* sim);

/* Node profile of one discharge, physical units.  quantity 0 n_e, 1 n_i [m^-3]
   (boundary nodes of a bounded discharge doubled), 2 phi [V] of the last solve;
   kind 0 current, 1 time average from avg_start_step.  Syncs. */
int pic_density(pic_sim* sim, int discharge, int quantity, int kind, double* host_out,
                size_t n_out);

/* Normalised node arrays: 0 w_e, 1 w_i (current particles), 2 phi, 3 E (last solve),
   4 sum of w_e, 5 sum of w_i, 6 sum of phi (time-average accumulators), 7 EEDF counts
   (eedf_bins + 1, last bin = overflow).  Syncs. */
int pic_grid(pic_sim* sim, int discharge, int what, double* host_out, size_t n_out);

int pic_diagnostics(pic_sim* sim, int discharge, pic_diag* out); /* syncs */

int pic_get_state(pic_sim* sim, int discharge, pic_state* st);        /* syncs */
int pic_set_state(pic_sim* sim, int discharge, const pic_state* st);  /* syncs */

/* Per-phase kernel timing.  While enabled, steps launch eagerly (no graph) and every
   kernel is launched with a start and a stop HIP event on the sim's stream, recorded by
   the launch itself around the kernel's execution.  The events of up to 32 steps are in
   flight before they are read, so profiling does not idle the GPU between steps.
   pic_profile(sim, 1|0) turns it on or off and resets the totals; pic_profile_read
   waits for the recorded steps and returns, per phase, the summed milliseconds and the
   number of steps.  Phases: 0 combine, 1 solve, 2 hist, 3 scan (two kernels: from the
   start of the first to the end of the second), 4 main, 5 collide, 6 finalize (two
   kernels), 7 coulomb (zero when no discharge has Coulomb collisions), 8 fine_sort (the
   three steps of PIC_SORT_FINE; zero without it).
   Errors: PIC_ERR_STATE (null sim), PIC_ERR_ARG (null outputs), PIC_ERR_DEVICE. */
int pic_profile(pic_sim* sim, int enable);
int pic_profile_read(pic_sim* sim, double* ms_total, uint64_t* launches, int n_phases);

/* Frees the host handle (not the workspace). */
void pic_free(pic_sim* sim);

/* Message of the last error on this handle (or of the last failed pic_init when sim is
   NULL); owned by the library, valid until the next call. */
const char* pic_last_error(const pic_sim* sim);

#ifdef __cplusplus
}
#endif
#endif
