/*
 * fspic_oracle.c -- plain sequential FP64 reference of the 1D3V electrostatic PIC cycle
 * with null-collision MCC.  TEST INFRASTRUCTURE ONLY (see fspic_oracle.h): only the test
 * suite, the smoke check and the benchmark's CPU baseline load it.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fused multiply-add, so every
 * expression below is evaluated as written, one IEEE operation at a time).
 *
 * Each routine names the passage of the paper it follows.  Where the paper is silent,
 * the reading taken is stated at the routine.
 */
#include "fspic_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* CODATA 2018 constants. */
#define QE 1.602176634e-19
#define ME 9.1093837015e-31
#define EPS0 8.8541878128e-12
#define KB 1.380649e-23
#define AMU 1.66053906660e-27
#define TWO_PI 6.283185307179586476925286766559

/* Ar-like synthetic cross-section model thresholds (eV). */
#define EXC_THRESHOLD 11.5
#define ION_THRESHOLD 15.8

struct orc_sim {
    orc_params p;
    orc_consts k;
    int n_nodes;
    int64_t n[2], cap[2];
    double *x[2], *vx[2], *vy[2], *vz[2];
    uint32_t* id[2];
    /* scratch for the sort and the births */
    double *tx, *tvx, *tvy, *tvz;
    uint32_t* tid;
    int32_t *flags, *cell;
    int32_t* start_cell[2];   /* cell of each particle at the start of the step */
    int64_t* perm;
    double *bx[2], *bvx[2], *bvy[2], *bvz[2];
    /* grid */
    double *w[2], *rho, *phi, *ef;
    double *acc_w[2], *acc_phi, *eedf;
    uint32_t* bparent;        /* parent id of each birth (ionisations, then emissions) */
    int64_t* bkey_perm;
    orc_tallies t;
    /* electrode processes and circuit */
    uint32_t t_see, t_refl;   /* emission / reflection iff a Philox word is below these */
    double vth_see;           /* spread of the emitted electrons' velocity components */
    double cap_norm;          /* series capacitance in units of eps0 A / dx (0: none) */
    double q_tot;             /* charge of the driven electrode's conductor (Q / A units) */
};

/* ------------------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel Random   */
/* Numbers: As Easy as 1, 2, 3", SC'11): a 4-word counter is mixed by ten rounds, each   */
/* two 32x32->64 multiplications whose high halves are xored with the other two words    */
/* and the round key; the 2-word key is advanced by a Weyl sequence between rounds.      */
/* It replaces the paper's per-thread xorshift (Sec. 3.8) so that a draw depends only on */
/* (particle id, step, block, tag) and not on which thread handles the particle.         */
/* ------------------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(pb >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)pb;
        uint32_t n2 = (uint32_t)(pa >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)pa;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53-bit uniform in [0, 1) from two words: all 32 bits of a, top 21 bits of b. */
double orc_u53(uint32_t a, uint32_t b) {
    uint64_t m = ((uint64_t)a << 21) | (uint64_t)(b >> 11);
    return (double)m * (1.0 / 9007199254740992.0);
}

static void draw(const orc_sim* s, int species, uint32_t id, uint32_t step, uint32_t block,
                 uint32_t tag, uint32_t out[4]) {
    uint32_t ctr[4] = {id, step, block, tag};
    uint32_t key[2] = {s->p.seed, 2u * s->p.discharge + (uint32_t)species};
    orc_philox4x32_10(ctr, key, out);
}

/* Two standard normals from one block (Box-Muller on U53 pairs). */
static void normals(const uint32_t b[4], double* z0, double* z1) {
    double ua = orc_u53(b[0], b[1]);
    double ub = orc_u53(b[2], b[3]);
    double r = sqrt(-2.0 * log(1.0 - ua));
    double th = TWO_PI * ub;
    *z0 = r * cos(th);
    *z1 = r * sin(th);
}

/* Isotropic unit vector from one block: cos(theta) = 1 - 2 Ua, phi = 2 pi Ub, the
   first component along the discharge axis. */
static void direction(const uint32_t b[4], double n[3]) {
    double ua = orc_u53(b[0], b[1]);
    double ub = orc_u53(b[2], b[3]);
    double ct = 1.0 - 2.0 * ua;
    double st = sqrt(1.0 - ct * ct);
    double ph = TWO_PI * ub;
    n[0] = ct;
    n[1] = st * cos(ph);
    n[2] = st * sin(ph);
}

/* ------------------------------------------------------------------------------------ */
/* Cross sections (Sec. 3.8 evaluates analytic fits instead of tables; the fits are not */
/* printed, so a synthetic Ar-like model with the same channels and thresholds is used: */
/* electron elastic / 11.5 eV excitation / 15.8 eV ionisation; ion isotropic / charge   */
/* exchange).  sigma in m^2, eps in eV.                                                  */
/* ------------------------------------------------------------------------------------ */
void orc_xsec(int model, int species, double eps, double sigma_const, double out[3]) {
    out[0] = out[1] = out[2] = 0.0;
    if (model == ORC_XS_CONST_E_ELASTIC) {
        if (species == 0) out[0] = sigma_const;
        return;
    }
    if (model != ORC_XS_AR_LIKE) return;
    if (species == 0) {
        double xe = eps / 12.0;
        out[0] = 3e-19 * (xe + 0.05) / (1.0 + xe * xe);
        if (eps > EXC_THRESHOLD) {
            double u = (eps - EXC_THRESHOLD) / 20.0;
            out[1] = 2e-20 * (2.0 * u) / (1.0 + u * u);
        }
        if (eps > ION_THRESHOLD) {
            double u = (eps - ION_THRESHOLD) / 60.0;
            out[2] = 3e-20 * (2.0 * u) / (1.0 + u * u);
        }
    } else {
        out[0] = 2e-19 * (1.0 + 2.0 / (1.0 + eps)) / (1.0 + eps / 100.0);
        out[1] = 3e-19 * (1.0 + 1.0 / (1.0 + eps)) / (1.0 + eps / 1000.0);
    }
}

/* Null-collision frequency "computed once" (Sec. 3.8): a bound of n_g sum_k sigma_k v
   over 0..5000 eV in 0.01 eV steps, raised by 1e-9 relative; for a constant sigma the
   frequency grows without bound and is capped at eps_cap. */
static double null_frequency(const orc_params* p, int species, double n_gas, double mass) {
    if (n_gas <= 0.0) return 0.0;
    if (p->xsec == ORC_XS_NONE) return 0.0;
    if (p->xsec == ORC_XS_CONST_E_ELASTIC) {
        if (species != 0) return 0.0;
        return n_gas * p->sigma_const_m2 * sqrt(2.0 * QE * p->eps_cap_ev / mass);
    }
    double best = 0.0;
    for (int k = 0; k <= 500000; ++k) {
        double eps = (double)k * 0.01;
        double sg[3];
        orc_xsec(p->xsec, species, eps, p->sigma_const_m2, sg);
        double nu = n_gas * (sg[0] + sg[1] + sg[2]) * sqrt(2.0 * QE * eps / mass);
        if (nu > best) best = nu;
    }
    return best * (1.0 + 1e-9);
}

/* Normalised constants (Sec. 3.3): t in dt, x in dx, rho in Q/(A dx), phi in Q dx/(eps0 A),
   E in Q/(eps0 A), v in dx/dt, with Q = e W the charge of one macro-particle; the push
   factor of eq. push_velocity then carries the sign of the species' charge. */
static void derive(const orc_params* p, orc_consts* k) {
    memset(k, 0, sizeof(*k));
    k->dx = p->length_m / (double)p->n_cells;
    k->weight_per_area = p->n0_m3 * p->length_m / (double)p->n_e0;
    k->mass[0] = ME;
    k->mass[1] = p->mass_i_amu * AMU;
    for (int s = 0; s < 2; ++s) {
        double q = (s == 0) ? -1.0 : 1.0;
        k->kappa[s] = q * QE * QE * k->weight_per_area * p->dt_s * p->dt_s /
                      (EPS0 * k->mass[s] * k->dx);
    }
    k->phi_scale = QE * k->weight_per_area * k->dx / EPS0;
    k->vunit = k->dx / p->dt_s;
    for (int s = 0; s < 2; ++s) {
        k->energy_c[s] = 0.5 * k->mass[s] * k->vunit * k->vunit / QE;
        double t_ev = (s == 0) ? p->te_ev : p->ti_ev;
        k->vth[s] = sqrt(t_ev * QE / k->mass[s]) / k->vunit;
    }
    k->vth_gas = sqrt(KB * p->gas_k / k->mass[1]) / k->vunit;
    k->n_gas = (p->gas_pa > 0.0) ? p->gas_pa / (KB * p->gas_k) : 0.0;
    for (int s = 0; s < 2; ++s) {
        k->nu0[s] = null_frequency(p, s, k->n_gas, k->mass[s]);
        /* eq. null_collision: P0 = 1 - exp(-dt nu0); the draw p < P0 is taken on the
           32-bit word, so the threshold is floor(P0 2^32). */
        k->p0[s] = 1.0 - exp(-p->dt_s * k->nu0[s]);
        double t = floor(k->p0[s] * 4294967296.0);
        k->t0[s] = (t >= 4294967295.0) ? 4294967295u : (uint32_t)t;
    }
    k->vhat_amp = p->v0_volt / k->phi_scale;
    k->drive_phase_per_step = TWO_PI * p->freq_hz * p->dt_s;
}

/* ------------------------------------------------------------------------------------ */
/* Field solve (Sec. 3.5): the finite-difference Poisson equation of eq.                */
/* poisson_normalized is tridiagonal and is solved with the Thomas algorithm.            */
/* Bounded: Phi_0 = phi_left (driven electrode), Phi_N = 0 (grounded), unknowns 1..N-1.  */
/* Periodic: mean charge removed, Phi_0 = 0 pinned, same Dirichlet system on 1..N-1.     */
/* E on nodes: centred difference inside; at an electrode, Gauss's law over the half     */
/* cell next to it (E_0 = Phi_0 - Phi_1 - rho_0, E_N = Phi_{N-1} - Phi_N + rho_N).        */
/* ------------------------------------------------------------------------------------ */
static void thomas(int m, const double* d, double* xo) {
    /* Sub- and super-diagonal 1, diagonal -2. */
    if (m <= 0) return;
    double* cp = (double*)malloc(sizeof(double) * (size_t)m);
    double* dp = (double*)malloc(sizeof(double) * (size_t)m);
    cp[0] = 1.0 / -2.0;
    dp[0] = d[0] / -2.0;
    for (int j = 1; j < m; ++j) {
        double den = -2.0 - 1.0 * cp[j - 1];
        cp[j] = 1.0 / den;
        dp[j] = (d[j] - 1.0 * dp[j - 1]) / den;
    }
    xo[m - 1] = dp[m - 1];
    for (int j = m - 2; j >= 0; --j) xo[j] = dp[j] - cp[j] * xo[j + 1];
    free(cp);
    free(dp);
}

int orc_solve(int periodic, int n_cells, const double* rho, double phi_left, double* phi,
              double* ef) {
    int N = n_cells;
    if (N < 1) return ORC_ERR_ARG;
    if (!periodic) {
        int m = N - 1;
        double* d = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
        for (int j = 1; j <= m; ++j) d[j - 1] = -rho[j];
        if (m > 0) {
            d[0] -= phi_left;
            d[m - 1] -= 0.0;
        }
        phi[0] = phi_left;
        phi[N] = 0.0;
        thomas(m, d, phi + 1);
        free(d);
        for (int j = 1; j < N; ++j) ef[j] = (phi[j - 1] - phi[j + 1]) / 2.0;
        ef[0] = phi[0] - phi[1] - rho[0];
        ef[N] = phi[N - 1] - phi[N] + rho[N];
    } else {
        if (N < 3) return ORC_ERR_ARG;
        double mean = 0.0;
        for (int j = 0; j < N; ++j) mean += rho[j];
        mean /= (double)N;
        int m = N - 1;
        double* d = (double*)malloc(sizeof(double) * (size_t)m);
        for (int j = 1; j <= m; ++j) d[j - 1] = -(rho[j] - mean);
        phi[0] = 0.0;
        thomas(m, d, phi + 1);
        free(d);
        for (int j = 0; j < N; ++j) {
            int jm = (j == 0) ? N - 1 : j - 1;
            int jp = (j == N - 1) ? 0 : j + 1;
            ef[j] = (phi[jm] - phi[jp]) / 2.0;
        }
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------------------ */
/* Linear (first-order) charge assignment (Sec. 2, Sec. 3.4): a particle at x in cell   */
/* c = floor(x), f = x - c, adds 1 - f to node c and f to node c + 1.                    */
/* ------------------------------------------------------------------------------------ */
void orc_deposit(int periodic, int n_cells, int64_t n, const double* x, double* w) {
    for (int64_t i = 0; i < n; ++i) {
        double c = floor(x[i]);
        double f = x[i] - c;
        int ci = (int)c;
        int cn = ci + 1;
        if (periodic && cn == n_cells) cn = 0;
        w[ci] += 1.0 - f;
        w[cn] += f;
    }
}

/* ------------------------------------------------------------------------------------ */
/* Leap-frog push (Sec. 3.6): v(t+1/2) = v(t-1/2) + kappa E(x(t)), x(t+1) = x(t) + v(t+1/2)*/
/* with the field gathered linearly from the two nodes of the particle's cell.           */
/* Bounded: inside iff 0 <= x < N, otherwise removed at the wall it crossed.  Periodic:  */
/* x wrapped into [0, N).  In the FP32 cell + offset layout the same update is made in   */
/* single precision on the in-cell offset: f += v; k = floor(f); cell += k; f -= k;       */
/* a rounding to f == 1 moves the particle to offset 0 of the next cell.                 */
/* ------------------------------------------------------------------------------------ */
static inline int wrap_cell(int c, int N) {
    int r = c % N;
    return r < 0 ? r + N : r;
}

void orc_push(int periodic, int n_cells, int fp32, double kappa, const double* ef, int64_t n,
              double* x, double* vx, int32_t* flags) {
    const int N = n_cells;
    for (int64_t i = 0; i < n; ++i) {
        int c = (int)floor(x[i]);
        int cn = c + 1;
        if (periodic && cn == N) cn = 0;
        if (!fp32) {
            double f = x[i] - (double)c;
            double ep = (1.0 - f) * ef[c] + f * ef[cn];
            double v = vx[i] + kappa * ep;
            double xn = x[i] + v;
            int fl = 0;
            if (periodic) {
                while (xn < 0.0) xn += (double)N;
                while (xn >= (double)N) xn -= (double)N;
            } else if (xn < 0.0) {
                fl = 1;
            } else if (xn >= (double)N) {
                fl = 2;
            }
            vx[i] = v;
            x[i] = xn;
            flags[i] = fl;
        } else {
            float f = (float)(x[i] - (double)c);
            float e0 = (float)ef[c];
            float e1 = (float)ef[cn];
            float t = 1.0f - f;
            float a = t * e0;
            float b = f * e1;
            float ep = a + b;
            float kf = (float)kappa;
            float dv = kf * ep;
            float v = (float)vx[i] + dv;
            float fn = f + v;
            float kfl = floorf(fn);
            int cell = c + (int)kfl;
            fn = fn - kfl;
            if (fn >= 1.0f) {
                fn = 0.0f;
                cell += 1;
            }
            int fl = 0;
            if (periodic) {
                cell = wrap_cell(cell, N);
            } else if (cell < 0) {
                fl = 1;
            } else if (cell >= N) {
                fl = 2;
            }
            vx[i] = (double)v;
            x[i] = (double)cell + (double)fn;
            flags[i] = fl;
        }
    }
}

/* ------------------------------------------------------------------------------------ */
/* Stable counting sort by cell (Sec. 3.7: after the sort every particle sits in its    */
/* correct sorting cell; the sorting cell is one grid cell).  Ties keep input order.     */
/* ------------------------------------------------------------------------------------ */
void orc_stable_sort_by_cell(int64_t n, const int32_t* cell, int n_cells, int64_t* perm) {
    int64_t* cnt = (int64_t*)calloc((size_t)n_cells + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) cnt[cell[i] + 1]++;
    for (int c = 0; c < n_cells; ++c) cnt[c + 1] += cnt[c];
    for (int64_t i = 0; i < n; ++i) perm[cnt[cell[i]]++] = i;
    free(cnt);
}

/* ------------------------------------------------------------------------------------ */
/* Modified null-collision MCC (Sec. 3.8, eq. null_collision): every particle draws one  */
/* number p; only p < P0 enters the standard null-collision channel selection, where    */
/* R = U nu0 is compared with the cumulative channel frequencies nu_k = n_g sigma_k v.    */
/* Electrons hit a gas atom at rest; the scattered direction is isotropic; elastic       */
/* recoil loss 2 (m/M)(1 - cos chi); excitation loses 11.5 eV; ionisation loses 15.8 eV */
/* and shares the rest uniformly with a secondary electron, and a new ion is born from  */
/* the gas Maxwellian at the parent's position.  Ions: a gas atom's velocity is drawn,   */
/* g = v - v_gas, eps = m_i g^2 / 2e; isotropic scattering in the centre-of-mass frame   */
/* or charge exchange (the ion takes the atom's velocity).                               */
/* Draw map (counter = id, step, block, tag 0): block 0 -> (w0 test, w1 w2 channel);     */
/* electrons: 1 scattered direction, 2 energy share, 3 secondary direction, 4-5 new ion  */
/* velocity; ions: 1-2 gas velocity, 3 scattering direction.                              */
/* ------------------------------------------------------------------------------------ */
int orc_collide(const orc_sim* s, int species, uint32_t id, int64_t step, double v[3],
                double v_sec[3], double v_ion[3]) {
    const orc_consts* k = &s->k;
    uint32_t st = (uint32_t)step;
    uint32_t b0[4];
    draw(s, species, id, st, 0, 0, b0);
    if (!(b0[0] < k->t0[species])) return 0;
    double r = orc_u53(b0[1], b0[2]) * k->nu0[species];
    if (species == 0) {
        double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
        double eps = k->energy_c[0] * v2;
        double speed = sqrt(v2) * k->vunit;
        double sg[3];
        orc_xsec(s->p.xsec, 0, eps, s->p.sigma_const_m2, sg);
        double nu_el = k->n_gas * sg[0] * speed;
        double nu_ex = k->n_gas * sg[1] * speed;
        double nu_iz = k->n_gas * sg[2] * speed;
        int ch = 0;
        if (r < nu_el) ch = 1;
        else if (r < nu_el + nu_ex) ch = 2;
        else if (r < nu_el + nu_ex + nu_iz) ch = 3;
        if (ch == 0) return 0;
        uint32_t b1[4];
        double n[3];
        draw(s, 0, id, st, 1, 0, b1);
        direction(b1, n);
        if (ch == 1) {
            double vm = sqrt(v2);
            double cchi = (v[0] * n[0] + v[1] * n[1] + v[2] * n[2]) / vm;
            double ep = eps * (1.0 - 2.0 * (k->mass[0] / k->mass[1]) * (1.0 - cchi));
            double vn = sqrt(ep / k->energy_c[0]);
            v[0] = vn * n[0]; v[1] = vn * n[1]; v[2] = vn * n[2];
        } else if (ch == 2) {
            double ep = eps - EXC_THRESHOLD;
            double vn = sqrt(ep / k->energy_c[0]);
            v[0] = vn * n[0]; v[1] = vn * n[1]; v[2] = vn * n[2];
        } else {
            uint32_t b2[4], b3[4], b4[4], b5[4];
            draw(s, 0, id, st, 2, 0, b2);
            draw(s, 0, id, st, 3, 0, b3);
            draw(s, 0, id, st, 4, 0, b4);
            draw(s, 0, id, st, 5, 0, b5);
            double er = eps - ION_THRESHOLD;
            double es = orc_u53(b2[0], b2[1]) * er;
            double epr = er - es;
            double vp = sqrt(epr / k->energy_c[0]);
            v[0] = vp * n[0]; v[1] = vp * n[1]; v[2] = vp * n[2];
            double n2[3];
            direction(b3, n2);
            double vs = sqrt(es / k->energy_c[0]);
            v_sec[0] = vs * n2[0]; v_sec[1] = vs * n2[1]; v_sec[2] = vs * n2[2];
            double z0, z1, z2, z3;
            normals(b4, &z0, &z1);
            normals(b5, &z2, &z3);
            v_ion[0] = k->vth_gas * z0;
            v_ion[1] = k->vth_gas * z1;
            v_ion[2] = k->vth_gas * z2;
        }
        return ch;
    } else {
        uint32_t b1[4], b2[4];
        draw(s, 1, id, st, 1, 0, b1);
        draw(s, 1, id, st, 2, 0, b2);
        double z0, z1, z2, z3;
        normals(b1, &z0, &z1);
        normals(b2, &z2, &z3);
        double vg[3] = {k->vth_gas * z0, k->vth_gas * z1, k->vth_gas * z2};
        double g[3] = {v[0] - vg[0], v[1] - vg[1], v[2] - vg[2]};
        double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
        double eps = k->energy_c[1] * g2;
        double speed = sqrt(g2) * k->vunit;
        double sg[3];
        orc_xsec(s->p.xsec, 1, eps, s->p.sigma_const_m2, sg);
        double nu_is = k->n_gas * sg[0] * speed;
        double nu_cx = k->n_gas * sg[1] * speed;
        int ch = 0;
        if (r < nu_is) ch = 1;
        else if (r < nu_is + nu_cx) ch = 2;
        if (ch == 0) return 0;
        if (ch == 1) {
            uint32_t b3[4];
            double n[3];
            draw(s, 1, id, st, 3, 0, b3);
            direction(b3, n);
            double gm = sqrt(g2);
            for (int a = 0; a < 3; ++a) v[a] = 0.5 * (v[a] + vg[a]) + 0.5 * gm * n[a];
        } else {
            for (int a = 0; a < 3; ++a) v[a] = vg[a];
        }
        return ch;
    }
}

/* A probability as the threshold of a 32-bit Philox word: the event happens iff the word
   is below floor(p 2^32) (p >= 1: always, except the word 2^32 - 1). */
static uint32_t word_threshold(double p) {
    if (!(p > 0.0)) return 0u;
    double t = floor(p * 4294967296.0);
    return (t >= 4294967295.0) ? 4294967295u : (uint32_t)t;
}

/* ------------------------------------------------------------------------------------ */
/* Simulation object                                                                     */
/* ------------------------------------------------------------------------------------ */
static void* xcalloc(size_t n, size_t sz) { return calloc(n ? n : 1, sz); }

orc_sim* orc_create(const orc_params* p, int64_t cap_e, int64_t cap_i) {
    if (!p || p->n_cells < 1 || cap_e < 0 || cap_i < 0) return NULL;
    if (p->periodic && p->n_cells < 3) return NULL;
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    s->p = *p;
    derive(p, &s->k);
    s->n_nodes = p->periodic ? p->n_cells : p->n_cells + 1;
    s->cap[0] = cap_e;
    s->cap[1] = cap_i;
    int64_t cmax = cap_e > cap_i ? cap_e : cap_i;
    for (int sp = 0; sp < 2; ++sp) {
        size_t c = (size_t)s->cap[sp];
        s->x[sp] = (double*)xcalloc(c, sizeof(double));
        s->vx[sp] = (double*)xcalloc(c, sizeof(double));
        s->vy[sp] = (double*)xcalloc(c, sizeof(double));
        s->vz[sp] = (double*)xcalloc(c, sizeof(double));
        s->id[sp] = (uint32_t*)xcalloc(c, sizeof(uint32_t));
        s->bx[sp] = (double*)xcalloc(c, sizeof(double));
        s->bvx[sp] = (double*)xcalloc(c, sizeof(double));
        s->bvy[sp] = (double*)xcalloc(c, sizeof(double));
        s->bvz[sp] = (double*)xcalloc(c, sizeof(double));
        s->w[sp] = (double*)xcalloc((size_t)s->n_nodes, sizeof(double));
        s->start_cell[sp] = (int32_t*)xcalloc(c, sizeof(int32_t));
        s->acc_w[sp] = (double*)xcalloc((size_t)s->n_nodes, sizeof(double));
    }
    s->tx = (double*)xcalloc((size_t)cmax, sizeof(double));
    s->tvx = (double*)xcalloc((size_t)cmax, sizeof(double));
    s->tvy = (double*)xcalloc((size_t)cmax, sizeof(double));
    s->tvz = (double*)xcalloc((size_t)cmax, sizeof(double));
    s->tid = (uint32_t*)xcalloc((size_t)cmax, sizeof(uint32_t));
    s->flags = (int32_t*)xcalloc((size_t)cmax, sizeof(int32_t));
    s->cell = (int32_t*)xcalloc((size_t)cmax, sizeof(int32_t));
    s->perm = (int64_t*)xcalloc((size_t)cmax, sizeof(int64_t));
    s->rho = (double*)xcalloc((size_t)s->n_nodes, sizeof(double));
    s->phi = (double*)xcalloc((size_t)s->n_nodes, sizeof(double));
    s->ef = (double*)xcalloc((size_t)s->n_nodes, sizeof(double));
    s->acc_phi = (double*)xcalloc((size_t)s->n_nodes, sizeof(double));
    s->eedf = (double*)xcalloc((size_t)(p->eedf_bins > 0 ? p->eedf_bins + 1 : 1), sizeof(double));
    s->bparent = (uint32_t*)xcalloc((size_t)cmax, sizeof(uint32_t));
    s->bkey_perm = (int64_t*)xcalloc((size_t)cmax, sizeof(int64_t));
    s->t_see = word_threshold(p->see_gamma);
    s->t_refl = word_threshold(p->refl_e);
    s->vth_see = sqrt(p->see_te_ev * QE / ME) / s->k.vunit;
    s->cap_norm = (p->circuit_cap_f_m2 > 0.0 && !p->periodic)
                      ? p->circuit_cap_f_m2 * s->k.dx / EPS0 : 0.0;
    return s;
}

void orc_destroy(orc_sim* s) {
    if (!s) return;
    for (int sp = 0; sp < 2; ++sp) {
        free(s->x[sp]); free(s->vx[sp]); free(s->vy[sp]); free(s->vz[sp]); free(s->id[sp]);
        free(s->bx[sp]); free(s->bvx[sp]); free(s->bvy[sp]); free(s->bvz[sp]);
        free(s->w[sp]); free(s->acc_w[sp]);
    }
    free(s->tx); free(s->tvx); free(s->tvy); free(s->tvz); free(s->tid);
    free(s->flags); free(s->cell); free(s->start_cell[0]); free(s->start_cell[1]); free(s->perm);
    free(s->rho); free(s->phi); free(s->ef); free(s->acc_phi); free(s->eedf);
    free(s->bparent); free(s->bkey_perm);
    free(s);
}

int orc_get_consts(const orc_sim* s, orc_consts* out) {
    *out = s->k;
    return ORC_OK;
}

int64_t orc_count(const orc_sim* s, int sp) { return s->n[sp]; }

/* Re-order species sp by a stable sort on `key` (input order breaks ties); with key NULL
   the key is the cell the particle is in, floor(x). */
static void sort_species_by(orc_sim* s, int sp, const int32_t* key) {
    int64_t n = s->n[sp];
    if (!key) {
        for (int64_t i = 0; i < n; ++i) s->cell[i] = (int32_t)floor(s->x[sp][i]);
        key = s->cell;
    }
    orc_stable_sort_by_cell(n, key, s->p.n_cells, s->perm);
    for (int64_t j = 0; j < n; ++j) {
        int64_t i = s->perm[j];
        s->tx[j] = s->x[sp][i]; s->tvx[j] = s->vx[sp][i]; s->tvy[j] = s->vy[sp][i];
        s->tvz[j] = s->vz[sp][i]; s->tid[j] = s->id[sp][i];
    }
    memcpy(s->x[sp], s->tx, sizeof(double) * (size_t)n);
    memcpy(s->vx[sp], s->tvx, sizeof(double) * (size_t)n);
    memcpy(s->vy[sp], s->tvy, sizeof(double) * (size_t)n);
    memcpy(s->vz[sp], s->tvz, sizeof(double) * (size_t)n);
    memcpy(s->id[sp], s->tid, sizeof(uint32_t) * (size_t)n);
}

static void sort_species(orc_sim* s, int sp) { sort_species_by(s, sp, NULL); }

static void deposit_all(orc_sim* s) {
    for (int sp = 0; sp < 2; ++sp) {
        memset(s->w[sp], 0, sizeof(double) * (size_t)s->n_nodes);
        orc_deposit(s->p.periodic, s->p.n_cells, s->n[sp], s->x[sp], s->w[sp]);
    }
}

/* ------------------------------------------------------------------------------------ */
/* Series capacitor between the source and the driven electrode (an external circuit;   */
/* Sec. 3.5 leaves boundary conditions to the literature).  The electrode and the plate */
/* joined to it form one conductor whose charge q changes only by the particles it      */
/* absorbs or emits.  Its plasma-side surface charge is sigma_0 = E_0, which for the     */
/* tridiagonal system grows with the electrode potential as sigma_0 = sigma_z + Phi_0/N  */
/* (sigma_z: the value for Phi_0 = 0); the plate holds q - sigma_0, so                    */
/* Phi_0 = V_s + (q - sigma_0)/C, solved for Phi_0 in closed form each step.              */
/* ------------------------------------------------------------------------------------ */
double orc_circuit_solve(const orc_sim* s, const double* rho, double vs, double q, double* phi,
                         double* ef) {
    const int N = s->p.n_cells;
    const double C = s->cap_norm;
    orc_solve(0, N, rho, 0.0, phi, ef);
    double sigma_z = ef[0];
    double phi0 = (vs + (q - sigma_z) / C) / (1.0 + 1.0 / ((double)N * C));
    orc_solve(0, N, rho, phi0, phi, ef);
    return phi0;
}

/* Field of step `step` from the current node weights; with `init` the circuit's charge is
   set so that the capacitor starts uncharged.  Records the net charge and field energy. */
static void solve_at(orc_sim* s, int64_t step, int init) {
    double sr = 0.0;
    for (int j = 0; j < s->n_nodes; ++j) {
        s->rho[j] = s->w[1][j] - s->w[0][j];
        sr += s->rho[j];
    }
    double vl = 0.0;
    if (!s->p.periodic)
        vl = s->k.vhat_amp * sin(s->k.drive_phase_per_step * (double)step);
    if (s->cap_norm > 0.0) {
        if (init) {
            orc_solve(0, s->p.n_cells, s->rho, 0.0, s->phi, s->ef);
            /* uncharged capacitor: Phi_0 = V_s, so q = sigma_0 = sigma_z + V_s / N */
            s->q_tot = s->ef[0] + vl / (double)s->p.n_cells;
        }
        vl = orc_circuit_solve(s, s->rho, vl, s->q_tot, s->phi, s->ef);
    } else {
        orc_solve(s->p.periodic, s->p.n_cells, s->rho, vl, s->phi, s->ef);
    }
    const int N = s->p.n_cells;
    double fe = 0.0;
    for (int j = 0; j < N; ++j) {
        double a = s->phi[j];
        double b = (s->p.periodic && j == N - 1) ? s->phi[0] : s->phi[j + 1];
        fe += (a - b) * (a - b);
    }
    s->t.field_energy = 0.5 * fe;
    s->t.sum_rho = sr;
    s->t.phi0 = s->p.periodic ? 0.0 : s->phi[0];
    s->t.q_circuit = s->q_tot;
}

/* Conversion of an FP64 position to the cell + FP32 offset layout: the offset is x - cell
   rounded toward zero, so it stays below 1. */
static double to_fp32_offset(double x) {
    double c = floor(x);
    double d = x - c;
    float f = (float)d;
    if ((double)f > d) f = nextafterf(f, 0.0f);
    return c + (double)f;
}

/* Initial load (tag 1, step word 0), initial sort, field and half-step back-push.
   Random: x = U53 N (block 0); Maxwellian velocities, thermal speed sqrt(kT/m), from
   blocks 1 and 2.  Quiet Langmuir start: x_k = (k + 1/2) N / N_s, electrons displaced by
   A sin(2 pi m x / N), cold.  Leap-frog start (Sec. 3.6): v_x(-1/2) = v_x(0) - kappa E / 2. */
int orc_load(orc_sim* s) {
    const orc_params* p = &s->p;
    const int N = p->n_cells;
    int64_t n0[2] = {p->n_e0, p->n_i0};
    for (int sp = 0; sp < 2; ++sp) {
        if (n0[sp] > s->cap[sp]) return ORC_ERR_CAPACITY;
        if (n0[sp] > 4294967295LL) return ORC_ERR_ID_OVERFLOW;
        s->n[sp] = n0[sp];
        for (int64_t i = 0; i < n0[sp]; ++i) {
            uint32_t id = (uint32_t)i;
            double x, v[3] = {0.0, 0.0, 0.0};
            if (p->load == ORC_LOAD_RANDOM) {
                uint32_t b0[4], b1[4], b2[4];
                draw(s, sp, id, 0, 0, 1, b0);
                draw(s, sp, id, 0, 1, 1, b1);
                draw(s, sp, id, 0, 2, 1, b2);
                x = orc_u53(b0[0], b0[1]) * (double)N;
                double z0, z1, z2, z3;
                normals(b1, &z0, &z1);
                normals(b2, &z2, &z3);
                v[0] = s->k.vth[sp] * z0;
                v[1] = s->k.vth[sp] * z1;
                v[2] = s->k.vth[sp] * z2;
            } else {
                x = ((double)i + 0.5) * (double)N / (double)n0[sp];
                if (sp == 0) {
                    x = x + p->langmuir_amp_cells *
                                sin(TWO_PI * (double)p->langmuir_mode * x / (double)N);
                    while (x < 0.0) x += (double)N;
                    while (x >= (double)N) x -= (double)N;
                }
            }
            if (p->fp32_offset) {
                x = to_fp32_offset(x);
                for (int a = 0; a < 3; ++a) v[a] = (double)(float)v[a];
            }
            s->x[sp][i] = x;
            s->vx[sp][i] = v[0];
            s->vy[sp][i] = v[1];
            s->vz[sp][i] = v[2];
            s->id[sp][i] = id;
        }
        s->t.next_id[sp] = (uint32_t)n0[sp];
        sort_species(s, sp);
    }
    deposit_all(s);
    solve_at(s, 0, 1);
    for (int sp = 0; sp < 2; ++sp) {
        double kap = s->k.kappa[sp];
        for (int64_t i = 0; i < s->n[sp]; ++i) {
            double x = s->x[sp][i];
            int c = (int)floor(x);
            int cn = c + 1;
            if (p->periodic && cn == N) cn = 0;
            if (!p->fp32_offset) {
                double f = x - (double)c;
                double ep = (1.0 - f) * s->ef[c] + f * s->ef[cn];
                s->vx[sp][i] = s->vx[sp][i] - 0.5 * kap * ep;
            } else {
                float f = (float)(x - (double)c);
                float t = 1.0f - f;
                float a = t * (float)s->ef[c];
                float b = f * (float)s->ef[cn];
                float ep = a + b;
                float hk = 0.5f * (float)kap;
                float dv = hk * ep;
                s->vx[sp][i] = (double)((float)s->vx[sp][i] - dv);
            }
        }
    }
    s->t.step = 0;
    return ORC_OK;
}

static int is_eedf_step(const orc_sim* s, int64_t step) {
    if (s->p.eedf_bins <= 0 || s->p.diag_every <= 0) return 0;
    if (step < s->p.avg_start) return 0;
    return ((step - s->p.avg_start) % s->p.diag_every) == 0;
}

/* ------------------------------------------------------------------------------------ */
/* Electrode processes (Sec. 2: if secondary electrons or reflection are featured,       */
/* electrons are inserted at the boundaries).  Draws: counter (id, step, block, tag 0)   */
/* under the key of the particle's own species, blocks 6-8 (the collision draws use 0-5).*/
/* Reflection: block 6 word 0 below floor(r 2^32); the electron is mirrored in the wall   */
/* it crossed (x -> -x or 2N - x, v_x -> -v_x).  Secondary emission: an absorbed ion's    */
/* block 6 word 0 below floor(gamma 2^32) emits one electron: |v_x| Rayleigh-distributed  */
/* (the flux of a Maxwellian at see_te_ev through the wall; block 7 words 0-1), v_y, v_z */
/* normal (block 8), pointing into the box, at the distance a random fraction of one     */
/* step's flight from the wall (block 7 words 2-3).                                      */
/* ------------------------------------------------------------------------------------ */
int orc_emit(const orc_sim* s, uint32_t ion_id, int64_t step, int wall, double* x, double v[3]) {
    uint32_t b6[4], b7[4], b8[4];
    draw(s, 1, ion_id, (uint32_t)step, 6, 0, b6);
    if (!(b6[0] < s->t_see)) return 0;
    draw(s, 1, ion_id, (uint32_t)step, 7, 0, b7);
    draw(s, 1, ion_id, (uint32_t)step, 8, 0, b8);
    double ua = orc_u53(b7[0], b7[1]);
    double uf = orc_u53(b7[2], b7[3]);
    double vn = s->vth_see * sqrt(-2.0 * log(1.0 - ua));
    double z0, z1;
    normals(b8, &z0, &z1);
    const double N = (double)s->p.n_cells;
    if (wall == 0) {
        v[0] = vn;
        *x = uf * vn;
    } else {
        v[0] = -vn;
        *x = N - uf * vn;
    }
    v[1] = s->vth_see * z0;
    v[2] = s->vth_see * z1;
    if (!(*x >= 0.0 && *x < N)) return 0;
    return 1;
}

/* Mirror an electron that crossed a wall; returns 1 if it is back inside the box. */
static int reflect(const orc_sim* s, double* x, double* vx, int wall) {
    const int N = s->p.n_cells;
    if (!s->p.fp32_offset) {
        *x = (wall == 0) ? -*x : 2.0 * (double)N - *x;
    } else {
        /* the same mirror on the cell + FP32 offset layout: cell c, offset f -> cell
           -c - 1 (or 2N - c - 1), offset 1 - f */
        int c = (int)floor(*x);
        float f = (float)(*x - (double)c);
        int cn = (wall == 0) ? -c - 1 : 2 * N - c - 1;
        float fn = 1.0f - f;
        if (fn >= 1.0f) {
            fn = 0.0f;
            cn += 1;
        }
        *x = (double)cn + (double)fn;
    }
    *vx = -*vx;
    return (*x >= 0.0 && *x < (double)N);
}

/* ------------------------------------------------------------------------------------ */
/* Binary Coulomb collision of two particles of one cell (the collisions fine sorting   */
/* makes straightforward, Sec. 3.2), after Takizuka and Abe (J. Comput. Phys. 25, 205,  */
/* 1977): the relative velocity u = v_a - v_b is turned by an angle Theta with          */
/* tan(Theta/2) = delta, delta normal with variance                                      */
/*   q_a^2 q_b^2 n_L lnLambda dt / (8 pi eps0^2 m_ab^2 |u|^3)   (m_ab reduced mass),     */
/* about a uniformly drawn azimuth Phi; both particles share the change so that the     */
/* pair's momentum and kinetic energy are unchanged.  Draws: counter (id_a, step, block, */
/* tag 2) under particle a's species key; like pairs blocks 0 (delta) and 1 (Phi),      */
/* electron-ion pairs blocks 2 and 3.                                                    */
/* ------------------------------------------------------------------------------------ */
int orc_coulomb_pair(const orc_sim* s, int sa, int sb, uint32_t id_a, int64_t step,
                     double n_l, double va[3], double vb[3]) {
    const orc_consts* k = &s->k;
    double u[3] = {va[0] - vb[0], va[1] - vb[1], va[2] - vb[2]};
    double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    if (!(u2 > 0.0)) return 1;
    double um = sqrt(u2);
    double ma = k->mass[sa], mb = k->mass[sb];
    double mab = ma * mb / (ma + mb);
    double usi = um * k->vunit;
    double var = (QE * QE) * (QE * QE) * n_l * s->p.coulomb_log * s->p.dt_s /
                 (8.0 * (TWO_PI / 2.0) * EPS0 * EPS0 * mab * mab * usi * usi * usi);
    uint32_t blk = (sa == sb) ? 0u : 2u;
    uint32_t b0[4], b1[4];
    draw(s, sa, id_a, (uint32_t)step, blk, 2, b0);
    draw(s, sa, id_a, (uint32_t)step, blk + 1u, 2, b1);
    double z0, z1;
    normals(b0, &z0, &z1);
    double delta = sqrt(var) * z0;
    double ph = TWO_PI * orc_u53(b1[0], b1[1]);
    double sth = 2.0 * delta / (1.0 + delta * delta);
    double omc = 2.0 * delta * delta / (1.0 + delta * delta);
    double cph = cos(ph), sph = sin(ph);
    double up = sqrt(u[0] * u[0] + u[1] * u[1]);
    double du[3];
    if (up > 0.0) {
        du[0] = (u[0] / up) * u[2] * sth * cph - (u[1] / up) * um * sth * sph - u[0] * omc;
        du[1] = (u[1] / up) * u[2] * sth * cph + (u[0] / up) * um * sth * sph - u[1] * omc;
        du[2] = -up * sth * cph - u[2] * omc;
    } else {
        du[0] = u[2] * sth * cph;
        du[1] = u[2] * sth * sph;
        du[2] = -u[2] * omc;
    }
    double fa = mb / (ma + mb), fb = ma / (ma + mb);
    for (int a = 0; a < 3; ++a) {
        va[a] = va[a] + fa * du[a];
        vb[a] = vb[a] - fb * du[a];
    }
    return 0;
}

/* The pair collision applied to n pairs (a_k, b_k) with ids id_a[k] in turn (velocities as
   n x 3 arrays); a helper of the pins, the cycle pairs particles in coulomb_step. */
void orc_coulomb_pairs(const orc_sim* s, int sa, int sb, int64_t n, const uint32_t* id_a,
                       int64_t step, double n_l, double* va, double* vb) {
    for (int64_t q = 0; q < n; ++q)
        orc_coulomb_pair(s, sa, sb, id_a[q], step, n_l, va + 3 * q, vb + 3 * q);
}

/* Coulomb collisions of the cell-sorted survivors [0, nsurv[s]) of both species: in every
   cell the like particles pair up in array order (first with second, third with fourth,
   ...; an odd one out does not collide), then the k-th electron of the cell pairs with
   its k-th ion.  n_L: the cell density of the species (like pairs) or the lower of the
   two (electron-ion). */
static void coulomb_step(orc_sim* s, const int64_t nsurv[2], int64_t step) {
    const int N = s->p.n_cells;
    const double dens = s->k.weight_per_area / s->k.dx;
    int64_t* start[2];
    for (int sp = 0; sp < 2; ++sp) {
        start[sp] = (int64_t*)calloc((size_t)N + 1, sizeof(int64_t));
        for (int64_t i = 0; i < nsurv[sp]; ++i) start[sp][(int)floor(s->x[sp][i]) + 1]++;
        for (int c = 0; c < N; ++c) start[sp][c + 1] += start[sp][c];
    }
    for (int sp = 0; sp < 2; ++sp) {
        if (!(s->p.coulomb & (sp == 0 ? ORC_COUL_EE : ORC_COUL_II))) continue;
        for (int c = 0; c < N; ++c) {
            int64_t a = start[sp][c], n = start[sp][c + 1] - a;
            for (int64_t q = 0; q + 1 < n; q += 2) {
                int64_t i = a + q, j = a + q + 1;
                double va[3] = {s->vx[sp][i], s->vy[sp][i], s->vz[sp][i]};
                double vb[3] = {s->vx[sp][j], s->vy[sp][j], s->vz[sp][j]};
                orc_coulomb_pair(s, sp, sp, s->id[sp][i], step, (double)n * dens, va, vb);
                s->vx[sp][i] = va[0]; s->vy[sp][i] = va[1]; s->vz[sp][i] = va[2];
                s->vx[sp][j] = vb[0]; s->vy[sp][j] = vb[1]; s->vz[sp][j] = vb[2];
            }
        }
    }
    if (s->p.coulomb & ORC_COUL_EI) {
        for (int c = 0; c < N; ++c) {
            int64_t ae = start[0][c], ne = start[0][c + 1] - ae;
            int64_t ai = start[1][c], ni = start[1][c + 1] - ai;
            int64_t np = ne < ni ? ne : ni;
            for (int64_t q = 0; q < np; ++q) {
                int64_t i = ae + q, j = ai + q;
                double va[3] = {s->vx[0][i], s->vy[0][i], s->vz[0][i]};
                double vb[3] = {s->vx[1][j], s->vy[1][j], s->vz[1][j]};
                orc_coulomb_pair(s, 0, 1, s->id[0][i], step, (double)np * dens, va, vb);
                s->vx[0][i] = va[0]; s->vy[0][i] = va[1]; s->vz[0][i] = va[2];
                s->vx[1][j] = vb[0]; s->vy[1][j] = vb[1]; s->vz[1][j] = vb[2];
            }
        }
    }
    if (s->p.fp32_offset)
        for (int sp = 0; sp < 2; ++sp)
            for (int64_t i = 0; i < nsurv[sp]; ++i) {
                s->vx[sp][i] = (double)(float)s->vx[sp][i];
                s->vy[sp][i] = (double)(float)s->vy[sp][i];
                s->vz[sp][i] = (double)(float)s->vz[sp][i];
            }
    free(start[0]);
    free(start[1]);
}

/* Births ordered by parent id within [lo, hi) (a stable sort of their indices). */
struct birth_key {
    uint32_t key;
    int64_t idx;
};
static int cmp_birth_key(const void* a, const void* b) {
    const struct birth_key* x = (const struct birth_key*)a;
    const struct birth_key* y = (const struct birth_key*)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}
static void order_births_by_parent(orc_sim* s, int64_t lo, int64_t hi, int64_t* perm) {
    int64_t n = hi - lo;
    struct birth_key* k = (struct birth_key*)xcalloc((size_t)n, sizeof(struct birth_key));
    for (int64_t i = 0; i < n; ++i) {
        k[i].key = s->bparent[lo + i];
        k[i].idx = lo + i;
    }
    qsort(k, (size_t)n, sizeof(struct birth_key), cmp_birth_key);
    for (int64_t i = 0; i < n; ++i) perm[lo + i] = k[i].idx;
    free(k);
}

/* One PIC cycle (Sec. 2, Fig. pic_cycle): field from rho_n, push, removal at the walls
   (with electrode reflection and emission when featured), MCC on the survivors, re-sort
   by cell, charge assignment of the new positions. */
int orc_step(orc_sim* s) {
    const orc_params* p = &s->p;
    const orc_consts* k = &s->k;
    const int64_t step = s->t.step;
    solve_at(s, step, 0);
    if (step >= p->avg_start) {
        for (int j = 0; j < s->n_nodes; ++j) {
            s->acc_w[0][j] += s->w[0][j];
            s->acc_w[1][j] += s->w[1][j];
            s->acc_phi[j] += s->phi[j];
        }
        s->t.acc_count++;
    }
    int64_t nb[2] = {0, 0}; /* births this step per species */
    int64_t nb_iz = 0;      /* ionisations (the first nb_iz births of both species) */
    int64_t nsurv[2];
    int64_t cond0 = 0;      /* charge conducted into the driven electrode (units of Q) */
    double mom = 0.0;
    /* electrons first: their ionisations create the births of both species */
    for (int sp = 0; sp < 2; ++sp) {
        int64_t n = s->n[sp];
        double ak = fabs(k->kappa[sp]);
        memcpy(s->tvx, s->vx[sp], sizeof(double) * (size_t)n); /* v_x before the push */
        if (p->sort_mode == ORC_SORT_LAG)
            for (int64_t i = 0; i < n; ++i) s->start_cell[sp][i] = (int32_t)floor(s->x[sp][i]);
        orc_push(p->periodic, p->n_cells, p->fp32_offset, k->kappa[sp], s->ef, n, s->x[sp],
                 s->vx[sp], s->flags);
        double ke = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double v0 = s->tvx[i], v1 = s->vx[sp][i];
            double vyz = s->vy[sp][i] * s->vy[sp][i] + s->vz[sp][i] * s->vz[sp][i];
            ke += (0.5 * (v0 * v0 + v1 * v1) + vyz) / (2.0 * ak);
            mom += v1 / ak;
        }
        s->t.kinetic[sp] = ke;
        if (sp == 0 && is_eedf_step(s, step)) {
            double inv_w = (double)p->eedf_bins / p->eedf_max_ev;
            for (int64_t i = 0; i < n; ++i) {
                double v2 = s->vx[0][i] * s->vx[0][i] + s->vy[0][i] * s->vy[0][i] +
                            s->vz[0][i] * s->vz[0][i];
                double eps = k->energy_c[0] * v2;
                double b = floor(eps * inv_w);
                int bin = (b >= (double)p->eedf_bins) ? p->eedf_bins : (int)b;
                s->eedf[bin] += 1.0;
            }
            s->t.eedf_samples++;
        }
        int64_t m = 0;
        for (int64_t i = 0; i < n; ++i) {
            double v[3] = {s->vx[sp][i], s->vy[sp][i], s->vz[sp][i]};
            if (s->flags[i] != 0) {
                int wall = s->flags[i] - 1;
                if (sp == 0 && s->t_refl > 0u) {
                    uint32_t b6[4];
                    draw(s, 0, s->id[0][i], (uint32_t)step, 6, 0, b6);
                    if (b6[0] < s->t_refl && reflect(s, &s->x[0][i], &v[0], wall)) {
                        s->t.reflected[wall]++;
                        s->flags[i] = 0;
                    }
                }
            }
            if (s->flags[i] != 0) {
                int wall = s->flags[i] - 1;
                s->t.absorbed[sp][wall]++;
                s->t.absorbed_energy_ev[sp][wall] +=
                    k->energy_c[sp] * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                if (wall == 0) cond0 += (sp == 0) ? -1 : 1;
                if (sp == 1 && s->t_see > 0u) {
                    double xe, ve[3];
                    if (orc_emit(s, s->id[1][i], step, wall, &xe, ve)) {
                        if (nb[0] >= s->cap[0]) return ORC_ERR_CAPACITY;
                        if (p->fp32_offset) {
                            xe = to_fp32_offset(xe);
                            for (int a = 0; a < 3; ++a) ve[a] = (double)(float)ve[a];
                        }
                        s->bx[0][nb[0]] = xe;
                        s->bvx[0][nb[0]] = ve[0]; s->bvy[0][nb[0]] = ve[1];
                        s->bvz[0][nb[0]] = ve[2];
                        s->bparent[nb[0]] = s->id[1][i];
                        nb[0]++;
                        s->t.emitted[wall]++;
                        if (wall == 0) cond0 += 1;
                    }
                }
                continue;
            }
            double vs[3], vi[3];
            int ch = orc_collide(s, sp, s->id[sp][i], step, v, vs, vi);
            if (ch > 0) s->t.collisions[sp][ch - 1]++;
            if (p->fp32_offset)
                for (int a = 0; a < 3; ++a) v[a] = (double)(float)v[a];
            if (sp == 0 && ch == 3) {
                if (nb[0] >= s->cap[0] || nb[1] >= s->cap[1]) return ORC_ERR_CAPACITY;
                if (p->fp32_offset)
                    for (int a = 0; a < 3; ++a) {
                        vs[a] = (double)(float)vs[a];
                        vi[a] = (double)(float)vi[a];
                    }
                s->bx[0][nb[0]] = s->x[0][i];
                s->bvx[0][nb[0]] = vs[0]; s->bvy[0][nb[0]] = vs[1]; s->bvz[0][nb[0]] = vs[2];
                s->bparent[nb[0]] = s->id[0][i];
                s->bx[1][nb[1]] = s->x[0][i];
                s->bvx[1][nb[1]] = vi[0]; s->bvy[1][nb[1]] = vi[1]; s->bvz[1][nb[1]] = vi[2];
                nb[0]++;
                nb[1]++;
                nb_iz++;
            }
            /* survivors are compacted in input order */
            s->start_cell[sp][m] = s->start_cell[sp][i];
            s->x[sp][m] = s->x[sp][i];
            s->vx[sp][m] = v[0]; s->vy[sp][m] = v[1]; s->vz[sp][m] = v[2];
            s->id[sp][m] = s->id[sp][i];
            m++;
        }
        nsurv[sp] = m;
    }
    s->t.momentum = mom;
    s->q_tot += (double)cond0;
    for (int sp = 0; sp < 2; ++sp) {
        if (nsurv[sp] + nb[sp] > s->cap[sp]) return ORC_ERR_CAPACITY;
        if ((uint64_t)s->t.next_id[sp] + (uint64_t)nb[sp] > 4294967295ULL)
            return ORC_ERR_ID_OVERFLOW;
    }
    /* birth order: ionisations in parent order, then emissions in parent-ion order;
       with ORC_RANK_PARENT_ID each group by increasing parent id */
    int64_t* bperm = s->bkey_perm;
    for (int64_t b = 0; b < nb[0]; ++b) bperm[b] = b;
    if (p->birth_rank == ORC_RANK_PARENT_ID) {
        order_births_by_parent(s, 0, nb_iz, bperm);
        order_births_by_parent(s, nb_iz, nb[0], bperm);
    }
    for (int sp = 0; sp < 2; ++sp) {
        s->n[sp] = nsurv[sp];
        if (p->sort_mode == ORC_SORT_CELL) sort_species(s, sp);
        else if (p->sort_mode == ORC_SORT_LAG) sort_species_by(s, sp, s->start_cell[sp]);
    }
    if (p->coulomb && p->sort_mode == ORC_SORT_CELL) coulomb_step(s, nsurv, step);
    for (int sp = 0; sp < 2; ++sp) {
        for (int64_t b = 0; b < nb[sp]; ++b) {
            int64_t j = nsurv[sp] + b;
            int64_t src = bperm[b]; /* the ion births follow the ionisations' order */
            s->x[sp][j] = s->bx[sp][src];
            s->vx[sp][j] = s->bvx[sp][src];
            s->vy[sp][j] = s->bvy[sp][src];
            s->vz[sp][j] = s->bvz[sp][src];
            s->id[sp][j] = s->t.next_id[sp] + (uint32_t)b;
        }
        s->n[sp] = nsurv[sp] + nb[sp];
        s->t.next_id[sp] += (uint32_t)nb[sp];
        s->t.births[sp] += nb[sp];
    }
    deposit_all(s);
    s->t.step = step + 1;
    return ORC_OK;
}

int orc_get_particles(const orc_sim* s, int sp, double* x, double* vx, double* vy, double* vz,
                      uint32_t* id) {
    size_t n = (size_t)s->n[sp];
    if (x) memcpy(x, s->x[sp], n * sizeof(double));
    if (vx) memcpy(vx, s->vx[sp], n * sizeof(double));
    if (vy) memcpy(vy, s->vy[sp], n * sizeof(double));
    if (vz) memcpy(vz, s->vz[sp], n * sizeof(double));
    if (id) memcpy(id, s->id[sp], n * sizeof(uint32_t));
    return ORC_OK;
}

int orc_set_particles(orc_sim* s, int sp, int64_t n, const double* x, const double* vx,
                      const double* vy, const double* vz, const uint32_t* id) {
    if (n < 0 || n > s->cap[sp]) return ORC_ERR_CAPACITY;
    for (int64_t i = 0; i < n; ++i)
        if (!(x[i] >= 0.0 && x[i] < (double)s->p.n_cells)) return ORC_ERR_ARG;
    s->n[sp] = n;
    memcpy(s->x[sp], x, (size_t)n * sizeof(double));
    memcpy(s->vx[sp], vx, (size_t)n * sizeof(double));
    memcpy(s->vy[sp], vy, (size_t)n * sizeof(double));
    memcpy(s->vz[sp], vz, (size_t)n * sizeof(double));
    memcpy(s->id[sp], id, (size_t)n * sizeof(uint32_t));
    /* the node weights always describe the particles held */
    memset(s->w[sp], 0, sizeof(double) * (size_t)s->n_nodes);
    orc_deposit(s->p.periodic, s->p.n_cells, n, s->x[sp], s->w[sp]);
    return ORC_OK;
}

int orc_get_grid(const orc_sim* s, int what, double* out) {
    size_t nn = (size_t)s->n_nodes;
    switch (what) {
    case 0: memcpy(out, s->w[0], nn * sizeof(double)); break;
    case 1: memcpy(out, s->w[1], nn * sizeof(double)); break;
    case 2: memcpy(out, s->phi, nn * sizeof(double)); break;
    case 3: memcpy(out, s->ef, nn * sizeof(double)); break;
    case 4: memcpy(out, s->acc_w[0], nn * sizeof(double)); break;
    case 5: memcpy(out, s->acc_w[1], nn * sizeof(double)); break;
    case 6: memcpy(out, s->acc_phi, nn * sizeof(double)); break;
    case 7: memcpy(out, s->eedf, (size_t)(s->p.eedf_bins + 1) * sizeof(double)); break;
    default: return ORC_ERR_ARG;
    }
    return ORC_OK;
}

int orc_set_grid(orc_sim* s, int what, const double* in) {
    size_t nn = (size_t)s->n_nodes;
    if (what == 0) memcpy(s->w[0], in, nn * sizeof(double));
    else if (what == 1) memcpy(s->w[1], in, nn * sizeof(double));
    else return ORC_ERR_ARG;
    return ORC_OK;
}

int orc_get_tallies(const orc_sim* s, orc_tallies* out) {
    *out = s->t;
    return ORC_OK;
}

int orc_set_counters(orc_sim* s, int64_t step, uint32_t ne, uint32_t ni) {
    s->t.step = step;
    s->t.next_id[0] = ne;
    s->t.next_id[1] = ni;
    return ORC_OK;
}
