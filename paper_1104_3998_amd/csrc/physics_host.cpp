// physics_host.cpp -- host-side derivation of the normalised constants of one discharge
// (Sec. 3.3) and of the tile geometry of the step kernels.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "host_common.h"

namespace fspic {

namespace {
constexpr double kQe = 1.602176634e-19;    // CODATA 2018
constexpr double kMe = 9.1093837015e-31;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kKb = 1.380649e-23;
constexpr double kAmu = 1.66053906660e-27;
constexpr double kTwoPiH = 6.283185307179586476925286766559;

// Synthetic Ar-like cross sections (m^2) in place of the paper's unprinted argon fits.
void cross_sections(int model, int species, double eps, double sc, double s[3]) {
  s[0] = s[1] = s[2] = 0.0;
  if (model == PIC_XS_CONST_E_ELASTIC) {
    if (species == 0) s[0] = sc;
    return;
  }
  if (model != PIC_XS_AR_LIKE) return;
  if (species == 0) {
    const double xe = eps / 12.0;
    s[0] = 3e-19 * (xe + 0.05) / (1.0 + xe * xe);
    if (eps > 11.5) {
      const double u = (eps - 11.5) / 20.0;
      s[1] = 2e-20 * (2.0 * u) / (1.0 + u * u);
    }
    if (eps > 15.8) {
      const double u = (eps - 15.8) / 60.0;
      s[2] = 3e-20 * (2.0 * u) / (1.0 + u * u);
    }
  } else {
    s[0] = 2e-19 * (1.0 + 2.0 / (1.0 + eps)) / (1.0 + eps / 100.0);
    s[1] = 3e-19 * (1.0 + 1.0 / (1.0 + eps)) / (1.0 + eps / 1000.0);
  }
}

// Null-collision frequency, computed once per species (Sec. 3.8): the largest total
// frequency n_g sum sigma v over 0..5000 eV (0.01 eV grid) raised by 1e-9; for a
// constant sigma, the frequency at eps_cap.
double null_frequency(const pic_config& c, int species, double n_gas, double mass) {
  if (n_gas <= 0.0 || c.xsec_model == PIC_XS_NONE) return 0.0;
  if (c.xsec_model == PIC_XS_CONST_E_ELASTIC) {
    if (species != 0) return 0.0;
    return n_gas * c.sigma_const_m2 * std::sqrt(2.0 * kQe * c.eps_cap_ev / mass);
  }
  double best = 0.0;
  for (int k = 0; k <= 500000; ++k) {
    const double eps = static_cast<double>(k) * 0.01;
    double s[3];
    cross_sections(static_cast<int>(c.xsec_model), species, eps, c.sigma_const_m2, s);
    const double nu = n_gas * (s[0] + s[1] + s[2]) * std::sqrt(2.0 * kQe * eps / mass);
    best = nu > best ? nu : best;
  }
  return best * (1.0 + 1e-9);
}

int largest_divisor_at_most(int n, int c) {
  for (int d = std::min(c, n); d >= 1; --d)
    if (n % d == 0) return d;
  return 1;
}
}  // namespace

double electron_mass() { return kMe; }
double ion_mass(const pic_config& c) { return c.mass_i_amu * kAmu; }

// Coulomb pair coefficients e^4 lnLambda dt / (8 pi eps0^2 m_ab^2) [SI] of e-e, i-i and e-i
// pairs (m_ab the reduced mass of the pair).
void coulomb_coefficients(const pic_config& c, double coef[3]) {
  const double me = kMe, mi = ion_mass(c);
  const double mab[3] = {0.5 * me, 0.5 * mi, me * mi / (me + mi)};
  for (int k = 0; k < 3; ++k)
    coef[k] = (kQe * kQe) * (kQe * kQe) * c.coulomb_log * c.dt_s /
              (8.0 * (kTwoPiH / 2.0) * kEps0 * kEps0 * mab[k] * mab[k]);
}

// A probability as the threshold of a 32-bit Philox word: the event happens iff the word
// is below floor(p 2^32) (p >= 1: always, except for the word 2^32 - 1).
uint32_t word_threshold(double p) {
  if (!(p > 0.0)) return 0u;
  const double t = std::floor(p * 4294967296.0);
  return t >= 4294967295.0 ? 4294967295u : static_cast<uint32_t>(t);
}

// Spread sqrt(e T / m_e) of each velocity component of the secondary electrons, in cells
// per step.
double see_spread(const pic_config& c, const pic_derived& k) {
  return std::sqrt(c.see_te_ev * kQe / kMe) / k.vunit;
}

// Series capacitance in the units of the normalised field equations (eps0 A / dx per
// electrode area A), 0 for the ideal source or a periodic box.
double circuit_cap_norm(const pic_config& c, const pic_derived& k) {
  if (!(c.circuit_cap_f_m2 > 0.0) || c.periodic) return 0.0;
  return c.circuit_cap_f_m2 * k.dx / kEps0;
}

int validate_config(const pic_config& c, std::string* why) {
  auto bad = [&](const char* m) {
    *why = m;
    return PIC_ERR_ARG;
  };
  if (c.abi_version != FSPIC_ABI_VERSION) return bad("abi_version mismatch");
  if (c.precision != PIC_FP64 && c.precision != PIC_FP32_OFFSET) return bad("precision");
  if (c.n_cells < 1 || c.n_cells > kMaxCells) return bad("n_cells out of [1, 16384]");
  if (c.periodic && c.n_cells < 3) return bad("periodic box needs >= 3 cells");
  if (c.n_e0 < 1) return bad("n_e0 must be >= 1 (it sets the macro-particle weight)");
  if (c.capacity_e < c.n_e0 || c.capacity_i < c.n_i0) return bad("capacity below n0");
  // the kernels address an array element by a 32-bit byte offset: both buffers of an
  // 8-byte field, or the candidate records (48 bytes in FP64), must stay below 4 GiB
  if (c.capacity_e >= (1ull << 26) || c.capacity_i >= (1ull << 26))
    return bad("capacity must be < 2^26 per species");
  if (!(c.length_m > 0) || !(c.dt_s > 0) || !(c.n0_m3 > 0) || !(c.mass_i_amu > 0))
    return bad("length, dt, n0 and ion mass must be positive");
  if (!(c.te_ev >= 0) || !(c.ti_ev >= 0) || !(c.gas_pa >= 0) || !(c.gas_k > 0))
    return bad("temperatures / gas pressure");
  if (c.xsec_model > PIC_XS_AR_LIKE) return bad("xsec_model");
  if (c.load_kind > PIC_LOAD_QUIET_LANGMUIR) return bad("load_kind");
  if (c.eedf_bins > 256) return bad("eedf_bins > 256");
  if (c.eedf_bins > 0 && !(c.eedf_max_ev > 0)) return bad("eedf_max_ev");
  if (c.xsec_model == PIC_XS_CONST_E_ELASTIC && !(c.eps_cap_ev > 0)) return bad("eps_cap_ev");
  if (c.sort_mode > PIC_SORT_LAG) return bad("sort_mode");
  if (c.sort_mode == PIC_SORT_FINE) {
    if (c.see_gamma > 0.0) return bad("secondary emission is not built for PIC_SORT_FINE");
    if (c.sort_cell_capacity > static_cast<uint32_t>(kMaxFineSlots))
      return bad("sort_cell_capacity > 65536");
    for (int sp = 0; sp < 2; ++sp) {
      const uint32_t g = c.cells_per_tile[sp] > 0 ? c.cells_per_tile[sp]
                                                  : (c.sort_cell_cells > 0 ? c.sort_cell_cells : 2);
      if (c.periodic && c.n_cells % g != 0)
        return bad("periodic fine sort: the sorting cell size must divide n_cells");
    }
  }
  if (c.coulomb > 7) return bad("coulomb: bits 0-2 only");
  if (c.coulomb != 0 && c.sort_mode != PIC_SORT_COUNTING)
    return bad("coulomb collisions pair the particles of a cell: need PIC_SORT_COUNTING");
  if (c.coulomb != 0 && !(c.coulomb_log > 0.0)) return bad("coulomb_log must be > 0");
  if (!(c.see_gamma >= 0.0 && c.see_gamma <= 1.0)) return bad("see_gamma must be in [0, 1]");
  if (!(c.refl_e >= 0.0 && c.refl_e <= 1.0)) return bad("refl_e must be in [0, 1]");
  if (c.see_gamma > 0.0 && !(c.see_te_ev > 0.0)) return bad("see_te_ev must be > 0");
  if ((c.see_gamma > 0.0 || c.refl_e > 0.0) && c.periodic)
    return bad("electrode processes need a bounded discharge");
  if (!(c.circuit_cap_f_m2 >= 0.0)) return bad("circuit_cap_f_m2 must be >= 0");
  return PIC_OK;
}

int derive(const pic_config& c, pic_derived* k) {
  std::memset(k, 0, sizeof(*k));
  k->dx = c.length_m / static_cast<double>(c.n_cells);
  k->weight_per_area = c.n0_m3 * c.length_m / static_cast<double>(c.n_e0);
  const double mass[2] = {kMe, c.mass_i_amu * kAmu};
  for (int s = 0; s < 2; ++s) {
    const double q = s == 0 ? -1.0 : 1.0;
    // eq. push_velocity with Q = e W, M = m W
    k->kappa[s] = q * kQe * kQe * k->weight_per_area * c.dt_s * c.dt_s /
                  (kEps0 * mass[s] * k->dx);
  }
  k->phi_scale = kQe * k->weight_per_area * k->dx / kEps0;
  k->vunit = k->dx / c.dt_s;
  for (int s = 0; s < 2; ++s) {
    k->energy_c[s] = 0.5 * mass[s] * k->vunit * k->vunit / kQe;
    const double t_ev = s == 0 ? c.te_ev : c.ti_ev;
    k->vth[s] = std::sqrt(t_ev * kQe / mass[s]) / k->vunit;
  }
  k->vth_gas = std::sqrt(kKb * c.gas_k / mass[1]) / k->vunit;
  k->n_gas = c.gas_pa > 0.0 ? c.gas_pa / (kKb * c.gas_k) : 0.0;
  for (int s = 0; s < 2; ++s) {
    k->nu0[s] = null_frequency(c, s, k->n_gas, mass[s]);
    k->p0[s] = 1.0 - std::exp(-c.dt_s * k->nu0[s]);  // eq. null_collision
    const double t = std::floor(k->p0[s] * 4294967296.0);
    k->t0[s] = t >= 4294967295.0 ? 4294967295u : static_cast<uint32_t>(t);
  }
  k->vhat_amp = c.v0_volt / k->phi_scale;
  k->drive_phase_per_step = kTwoPiH * c.freq_hz * c.dt_s;
  TileChoice tc[2];
  choose_tiles(c, *k, tc);
  for (int s = 0; s < 2; ++s) {
    k->cells_per_tile[s] = static_cast<uint32_t>(tc[s].C);
    k->window[s] = static_cast<uint32_t>(tc[s].D);
  }
  return PIC_OK;
}

// Tile geometry.  A workgroup owns C consecutive cells (the paper's "one thread block
// per sorting cell", Sec. 3.2, with C cells per block instead of one) and sorts the
// particles that stay within D cells of them; the rest take the far-mover path.
// Default sizes (measured on the large discharge and the batched scan): an electron tile
// holds about 2e3 null-collision candidates (P0 of its particles), between 2.5e3 and 2e4
// particles, so that the MCC pass amortises its per-tile work over enough candidates
// without making a few very long workgroups; an ion tile holds about 2.5e3 particles (ions
// have few candidates), and their many short workgroups fill the gaps around the long
// electron ones in the particle pass.
void choose_tiles(const pic_config& c, const pic_derived& k, TileChoice tc[2]) {
  const int N = static_cast<int>(c.n_cells);
  const uint64_t n0[2] = {c.n_e0, c.n_i0};
  const int d_default[2] = {32, 4};
  for (int s = 0; s < 2; ++s) {
    tc[s].nmax = 0;
    if (c.sort_mode == PIC_SORT_FINE) {
      // the paper's sorting cells: G grid cells each (N_gc = G + 1 grid points), nmax
      // slots each (default: 2.5 times the load's mean count of the species per sorting
      // cell, plus 64, in whole wavefronts)
      // (cells_per_tile, a tuning field, may set it per species)
      const int g0 = c.cells_per_tile[s] > 0 ? static_cast<int>(c.cells_per_tile[s])
                                             : (c.sort_cell_cells > 0 ? static_cast<int>(c.sort_cell_cells) : 2);
      const int G = std::max(1, std::min(g0, std::min(kMaxCellsPerTile, N)));
      const uint64_t n0s = s == 0 ? c.n_e0 : c.n_i0;
      int nmax = static_cast<int>(c.sort_cell_capacity);
      if (nmax <= 0) {
        const double mean = static_cast<double>(n0s) * G / N;
        nmax = static_cast<int>(std::ceil((2.5 * mean + 64.0) / 64.0)) * 64;
      }
      tc[s].C = G;
      tc[s].D = std::max(0, std::min(c.window[s] > 0 ? static_cast<int>(c.window[s]) : d_default[s],
                                     (kMaxWindow - G) / 2));
      if (c.periodic) tc[s].D = std::max(0, std::min(tc[s].D, (N - 2 * G - 1) / 2));
      tc[s].W = G + 2 * tc[s].D;
      tc[s].n_tiles = (N + G - 1) / G;
      tc[s].n_tail = 0;
      tc[s].nmax = nmax;
      continue;
    }
    if (c.sort_mode == PIC_SORT_NONE) {
      // unsorted: the array is cut into equal index ranges (tail-like tiles), about 2048
      // particles of the capacity each; no cell windows
      const uint64_t cap = s == 0 ? c.capacity_e : c.capacity_i;
      tc[s].C = 1;
      tc[s].D = 0;
      tc[s].W = 1;
      tc[s].n_tiles = static_cast<int>(std::max<uint64_t>(1, std::min<uint64_t>(65536, (cap + 2047) / 2048)));
      tc[s].n_tail = 0;
      continue;
    }
    int C;
    if (c.cells_per_tile[s] > 0) {
      C = static_cast<int>(c.cells_per_tile[s]);
    } else {
      const double target =
          s == 0 ? std::min(2.0e4, std::max(2.5e3, 2.0e3 / std::max(k.p0[0], 1e-9))) : 2.5e3;
      const double ppc = std::max(1.0, static_cast<double>(n0[s]) / N);
      C = static_cast<int>(std::lround(target / ppc));
    }
    C = std::max(1, std::min(C, std::min(64, N)));
    int D = c.window[s] > 0 ? static_cast<int>(c.window[s]) : d_default[s];
    if (c.periodic) {
      // C divides N, and the tile with its window (C + 2D cells) leaves at least C + 1
      // other cells, so no window wraps onto its own tile
      for (;;) {
        C = largest_divisor_at_most(N, C);
        const int room = N - 2 * C - 1;
        if (room >= 0 || C == 1) {
          D = std::max(0, std::min(D, room / 2));
          break;
        }
        C = C - 1;
      }
    }
    D = std::max(0, std::min(D, (kMaxWindow - C) / 2));
    tc[s].C = C;
    tc[s].D = D;
    tc[s].W = C + 2 * D;
    tc[s].n_tiles = (N + C - 1) / C;
    // tail tiles: about one per 128 cell tiles (births are well under 1% of a step's
    // particles), each with a global rank row per wave over all cells
    tc[s].n_tail = c.tail_groups > 0 ? static_cast<int>(c.tail_groups)
                                     : std::max(1, std::min(16, tc[s].n_tiles / 128));
  }
}

}  // namespace fspic
