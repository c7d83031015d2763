// api.cpp -- the C ABI of libfspic (include/fspic.h): configuration checks, the carve-up
// of the caller's workspace, the launch sequence of a step (eager or replayed from a
// captured HIP graph), state upload/download and diagnostics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "host_common.h"

using namespace fspic;

namespace {

thread_local std::string g_init_error;

constexpr int kPhases = 9;
constexpr int kRing = 32;  // steps whose phase events are in flight before they are read

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bump allocator over the workspace; with base == nullptr it only measures.
struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = align_up(off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * (count ? count : 1);
    return p;
  }
};

struct Plan {
  std::vector<pic_config> cfg;
  std::vector<pic_derived> der;
  std::vector<TileChoice> tiles;  // 2 per discharge
  std::vector<SpeciesDev> sp;
  std::vector<DischargeDev> ds;
  std::vector<int2> tile_table;
  std::vector<int2> node_table, cell_table;  // blocks of nodes / cells per species
  std::vector<int4> collide_table;           // MCC workgroups
  SimDev sim{};
  SimDev* d_sim = nullptr;
  SpeciesDev* d_sp = nullptr;
  DischargeDev* d_ds = nullptr;
  int2* d_tt = nullptr;
  int2* d_nt = nullptr;
  int2* d_ct = nullptr;
  int4* d_cw = nullptr;
  LaunchInfo li{};
  size_t bytes = 0;
};

// Workgroup -> tile table of the particle kernels: the (small) tail tiles first, so that
// they start early, then the cell tiles in order.  (Giving each XCD one contiguous run of
// tiles was measured slower for k_main: the particle density, and with it the work per
// tile, varies along the discharge, and contiguous runs load the XCDs unevenly.)
std::vector<int2> tile_order(const std::vector<int2>& tail, const std::vector<int2>& cells) {
  std::vector<int2> list(tail);
  list.insert(list.end(), cells.begin(), cells.end());
  return list;
}

int build_plan(const pic_config* cfgs, int n, char* ws, Plan* pl, std::string* why) {
  if (!cfgs || n < 1) {
    *why = "need at least one configuration";
    return PIC_ERR_ARG;
  }
  pl->cfg.assign(cfgs, cfgs + n);
  pl->der.resize(n);
  pl->tiles.resize(2 * n);
  for (int d = 0; d < n; ++d) {
    std::string w;
    const int rc = validate_config(cfgs[d], &w);
    if (rc != PIC_OK) {
      *why = "discharge " + std::to_string(d) + ": " + w;
      return rc;
    }
    if (cfgs[d].precision != cfgs[0].precision) {
      *why = "all discharges of a simulation must use the same precision";
      return PIC_ERR_ARG;
    }
    if ((cfgs[d].sort_mode == PIC_SORT_LAG) != (cfgs[0].sort_mode == PIC_SORT_LAG)) {
      *why = "the lagged sort is chosen for all discharges of a simulation or none";
      return PIC_ERR_ARG;
    }
    derive(cfgs[d], &pl->der[d]);
    choose_tiles(cfgs[d], pl->der[d], &pl->tiles[2 * d]);
  }
  const bool fp32 = cfgs[0].precision == PIC_FP32_OFFSET;
  pl->li.lag = cfgs[0].sort_mode == PIC_SORT_LAG;
  Carver cv{ws};
  pl->sp.assign(2 * n, SpeciesDev{});
  pl->ds.assign(n, DischargeDev{});
  pl->tile_table.clear();
  std::vector<int2> cell_tiles, tail_tiles;
  int max_nodes = 0, max_cap = 0, max_cells = 0;
  for (int d = 0; d < n; ++d) {
    const pic_config& c = cfgs[d];
    const pic_derived& k = pl->der[d];
    const int N = static_cast<int>(c.n_cells);
    const int nn = c.periodic ? N : N + 1;
    max_nodes = std::max(max_nodes, nn);
    max_cells = std::max(max_cells, N);
    DischargeDev& D = pl->ds[d];
    D.n_cells = N;
    D.periodic = static_cast<int>(c.periodic);
    D.n_nodes = nn;
    D.spec0 = 2 * d;
    for (int s = 0; s < 2; ++s) {
      D.w[s] = cv.take<double>(nn);
      D.acc_w[s] = cv.take<double>(nn);
    }
    D.phi = cv.take<double>(nn);
    D.E64 = cv.take<double>(nn);
    D.E32 = cv.take<float>(nn);
    D.acc_phi = cv.take<double>(nn);
    D.dstat = cv.take<double>(DS_N);
    D.energy_step = cv.take<unsigned long long>(1);
    D.cap_norm = circuit_cap_norm(c, k);
    D.coulomb = static_cast<int32_t>(c.coulomb);
    coulomb_coefficients(c, D.coul_coef);
    D.coul_dens = k.weight_per_area / k.dx;
    D.vunit = k.vunit;
    D.mfrac_e = ion_mass(c) / (electron_mass() + ion_mass(c));
    D.mfrac_i = electron_mass() / (electron_mass() + ion_mass(c));
    if (c.coulomb) pl->li.coulomb = true;
    D.acc_count = cv.take<unsigned long long>(1);
    D.eedf_samples = cv.take<unsigned long long>(1);
    D.eedf_bins = static_cast<int>(c.eedf_bins);
    D.eedf = cv.take<unsigned long long>(c.eedf_bins + 1);
    D.diag_every = static_cast<int>(c.diag_every);
    D.eedf_inv_width = c.eedf_bins > 0 ? static_cast<double>(c.eedf_bins) / c.eedf_max_ev : 0.0;
    D.vhat_amp = k.vhat_amp;
    D.phase_per_step = k.drive_phase_per_step;
    D.avg_start = static_cast<int64_t>(c.avg_start_step);
    for (int s = 0; s < 2; ++s) {
      SpeciesDev& S = pl->sp[2 * d + s];
      const TileChoice& tc = pl->tiles[2 * d + s];
      uint32_t cap = static_cast<uint32_t>(s == 0 ? c.capacity_e : c.capacity_i);
      if (c.sort_mode == PIC_SORT_FINE) {
        // every sorting cell's slots, and the contiguous arrays of the load / set_state
        const uint64_t slots = static_cast<uint64_t>(tc.n_tiles) * static_cast<uint64_t>(tc.nmax);
        if (tc.nmax > kMaxFineSlots || slots >= (1ull << 26)) {
          *why = "discharge " + std::to_string(d) + ": fine sort needs " + std::to_string(slots) +
                 " slots (sorting cells x sort_cell_capacity): must be < 2^26, at most 65536 "
                 "per sorting cell";
          return PIC_ERR_ARG;
        }
        cap = std::max<uint32_t>(cap, static_cast<uint32_t>(slots));
        pl->li.fine = true;
      }
      max_cap = std::max(max_cap, static_cast<int>(cap));
      S.ds = d;
      S.sp = s;
      S.mode = static_cast<int32_t>(c.sort_mode);
      S.n_cells = N;
      S.periodic = static_cast<int>(c.periodic);
      S.C = tc.C;
      S.D = tc.D;
      S.W = tc.W;
      S.n_tiles = tc.n_tiles;
      S.n_tail = tc.n_tail;
      S.n_nodes = nn;
      S.cap = cap;
      S.far_cap = c.far_capacity > 0 ? c.far_capacity : std::max<uint32_t>(65536u, cap / 8u);
      // particle and candidate arrays hold one element past the capacity: a sink that
      // lanes without a record to store write to, so that stores are not branched over
      const size_t cap1 = static_cast<size_t>(cap) + 1;
      // the two buffers of a field are one allocation, buffer 1 a fixed distance above
      // buffer 0, so the kernels reach both from one base pointer
      // velocity records: FP32 16 bytes (vx, vy, vz, id), FP64 24 bytes (vx, vy, vz);
      // the buffer distance a multiple of 256 and of the record size
      const size_t rv = fp32 ? 16 : 24;
      const size_t st4 = align_up(4 * cap1, 256), st8 = align_up(8 * cap1, 256);
      const size_t stv = align_up(rv * cap1, fp32 ? 256 : 768);
      S.bstride4 = static_cast<uint32_t>(st4);
      S.bstride8 = static_cast<uint32_t>(st8);
      S.bstridev = static_cast<uint32_t>(stv);
      const int last_rec = fp32 ? F_ID : F_VZ;  // the last field in the velocity record
      for (int f = 0; f < 6; ++f) {
        if (!fp32 && f == 1) {
          S.fld[0][f] = S.fld[1][f] = nullptr;
          continue;
        }
        if (f >= F_VX && f <= last_rec) continue;  // the velocity records, below
        const size_t st = (fp32 || f == F_ID) ? st4 : st8;
        char* pair = cv.take<char>(2 * st);
        S.fld[0][f] = pair;
        S.fld[1][f] = pair ? pair + st : nullptr;
      }
      {
        char* pair = cv.take<char>(2 * stv);
        for (int b = 0; b < 2; ++b)
          for (int f = F_VX; f <= last_rec; ++f)
            S.fld[b][f] = pair ? pair + b * stv + (rv / 4) * (f - F_VX) : nullptr;
      }
      // velocity records of n elements: the vx, vy, vz (FP32 also id) pointers into one array
      auto vel_records = [&](void** fl, size_t n) {
        char* v = cv.take<char>(rv * n);
        for (int f = F_VX; f <= last_rec; ++f) fl[f] = v ? v + (rv / 4) * (f - F_VX) : nullptr;
      };
      if (s == 0) {
        for (int b = 0; b < 2; ++b) {
          if (fp32) {
            S.stage[b][F32_CELL] = cv.take<int>(cap);
            S.stage[b][F32_OFF] = cv.take<float>(cap);
            vel_records(S.stage[b], cap);
          } else {
            S.stage[b][F64_X] = cv.take<double>(cap);
            S.stage[b][1] = nullptr;
            vel_records(S.stage[b], cap);
          }
          S.stage[b][F_ID] = nullptr;
        }
      }
      for (int f = 0; f < 6; ++f) S.fine[f] = nullptr;
      S.nmax = static_cast<uint32_t>(tc.nmax);
      S.fcnt = S.flv = S.fpid = S.fpid_list = nullptr;
      if (c.sort_mode == PIC_SORT_FINE) {
        for (int f = 0; f < 6; ++f) {
          if (!fp32 && f == 1) continue;
          if (f >= F_VX && f <= last_rec) continue;
          S.fine[f] = cv.take<char>(((fp32 || f == F_ID) ? 4 : 8) * cap1);
        }
        vel_records(S.fine, cap1);
        S.fcnt = cv.take<uint32_t>(static_cast<size_t>(tc.n_tiles));
        S.flv = cv.take<uint32_t>(static_cast<size_t>(tc.n_tiles));
        if (s == 0) {
          S.fpid = cv.take<uint32_t>(cap);
          S.fpid_list = cv.take<uint32_t>(cap);
        }
      }
      S.n_total = cv.take<uint32_t>(2);
      S.n_sorted = cv.take<uint32_t>(2);
      S.n_holes = cv.take<uint32_t>(2);
      S.next_id = cv.take<uint32_t>(1);
      S.cell_start = cv.take<uint32_t>(2 * (N + 1));
      S.hist = cv.take<uint32_t>(static_cast<size_t>(tc.n_tiles) * kWaves * tc.W);
      S.tilerel = cv.take<uint32_t>(static_cast<size_t>(tc.n_tiles) * kWaves * tc.W);
      S.thist = cv.take<uint32_t>(static_cast<size_t>(tc.n_tail) * kWaves * N);
      S.trel = cv.take<uint32_t>(static_cast<size_t>(tc.n_tail) * kWaves * N);
      S.partial = cv.take<unsigned long long>(static_cast<size_t>(tc.n_tiles) * (tc.W + 1));
      S.far_w = cv.take<unsigned long long>(nn);
      S.far_count = cv.take<uint32_t>(1);
      S.far_list = cv.take<uint4>(S.far_cap);
      S.far_grouped = cv.take<uint4>(S.far_cap);
      S.far_cell_cnt = cv.take<uint32_t>(N);
      S.far_fill = cv.take<uint32_t>(N);
      S.far_base = cv.take<uint32_t>(N);
      S.base = cv.take<uint32_t>(N);
      S.far_dest = cv.take<uint32_t>(cap);
      const int ntt = tc.n_tiles + tc.n_tail;
      S.cand = cv.take<char>((fp32 ? 32 : 48) * cap1);
      S.cand_cnt = cv.take<uint32_t>(static_cast<size_t>(ntt) * kWaves);
      S.birth_cnt = cv.take<uint32_t>(ntt);
      S.stage_first = cv.take<uint32_t>(ntt);
      // births of both species are ranked over the electron tiles
      const int ntt_e = pl->tiles[2 * d].n_tiles + pl->tiles[2 * d].n_tail;
      S.birth_base = cv.take<uint32_t>(std::max(ntt, ntt_e) + 1);
      S.fin = cv.take<uint32_t>(2);
      S.absorbed = cv.take<unsigned long long>(2);
      S.absorbed_energy = cv.take<double>(2);
      S.births = cv.take<unsigned long long>(1);
      S.collisions = cv.take<unsigned long long>(3);
      S.emitted = cv.take<unsigned long long>(2);
      S.reflected = cv.take<unsigned long long>(2);
      S.psteps = cv.take<unsigned long long>(1);
      S.tstats = cv.take<TileStats>(static_cast<size_t>(ntt));
      S.ev_bits = cv.take<uint32_t>((static_cast<size_t>(ntt) + 31) / 32);
      S.tcount = cv.take<uint2>(static_cast<size_t>(ntt));
      S.tke = cv.take<double>(2 * static_cast<size_t>(ntt));
      S.t_refl = s == 0 ? word_threshold(c.refl_e) : 0u;
      S.t_see = s == 1 ? word_threshold(c.see_gamma) : 0u;
      S.vth_see = see_spread(c, k);
      for (int f = 0; f < 6; ++f) S.em_stage[f] = nullptr;
      S.ab_list = nullptr;
      S.ab_cnt = S.em_cnt = S.em_lo = S.em_base = nullptr;
      if (S.t_see) {
        pl->li.emission = true;
        S.ab_list = cv.take<uint2>(cap);
        // emitted electrons wait at their parent ion's index: electron records, cap_i long
        if (fp32) {
          S.em_stage[F32_CELL] = cv.take<int>(cap);
          S.em_stage[F32_OFF] = cv.take<float>(cap);
          vel_records(S.em_stage, cap);
          S.em_stage[F_ID] = nullptr;
        } else {
          S.em_stage[F64_X] = cv.take<double>(cap);
          vel_records(S.em_stage, cap);
        }
        S.ab_cnt = cv.take<uint32_t>(static_cast<size_t>(ntt) * kWaves);
        S.em_cnt = cv.take<uint32_t>(static_cast<size_t>(ntt) * kWaves);
        S.em_lo = cv.take<uint32_t>(static_cast<size_t>(ntt) * kWaves);
        S.em_base = cv.take<uint32_t>(static_cast<size_t>(ntt) * kWaves + 1);
      }
      {
        // fixed-point deposit: a node's weight never exceeds the species' capacity, so
        // 2^shift (cap + 1) < 2^63 keeps every sum in 64 bits; at most 52 bits of fraction
        int bits = 0;
        while ((uint64_t{1} << bits) <= static_cast<uint64_t>(cap) + 1) ++bits;
        const int shift = std::min(52, 63 - bits);
        S.dep_one = uint64_t{1} << shift;
        S.dep_scale = std::ldexp(1.0, shift);
        S.dep_inv = std::ldexp(1.0, -shift);
      }
      S.kappa = k.kappa[s];
      S.kappa_f = static_cast<float>(k.kappa[s]);
      S.t0 = k.t0[s];
      S.energy_c = k.energy_c[s];
      S.vunit = k.vunit;
      S.n_gas = k.n_gas;
      S.nu0 = k.nu0[s];
      S.vth_gas = k.vth_gas;
      S.mass_ratio = electron_mass() / ion_mass(c);
      S.key0 = c.seed;
      S.key1 = 2u * c.discharge_index + static_cast<uint32_t>(s);
      S.xsec = static_cast<int>(c.xsec_model);
      S.sigma_const = c.sigma_const_m2;
      S.n_init = static_cast<uint32_t>(s == 0 ? c.n_e0 : c.n_i0);
      S.load_kind = static_cast<int>(c.load_kind);
      S.lang_mode = static_cast<int>(c.langmuir_mode);
      S.vth = k.vth[s];
      S.lang_amp = c.langmuir_amp_cells;
      for (int t = 0; t < tc.n_tiles; ++t) cell_tiles.push_back(make_int2(2 * d + s, t));
      for (int j = 0; j < tc.n_tail; ++j) tail_tiles.push_back(make_int2(2 * d + s, tc.n_tiles + j));
    }
  }
  pl->tile_table = tile_order(tail_tiles, cell_tiles);
  const int n_gtiles = 256;
  for (int i = 0; i < 2 * n; ++i)
    pl->sp[i].gsort_hist = cv.take<uint32_t>(static_cast<size_t>(n_gtiles) * pl->sp[i].n_cells);
  pl->sim.step = cv.take<unsigned long long>(1);
  pl->sim.error = cv.take<uint32_t>(1);
  pl->sim.fin_count = cv.take<uint32_t>(1);
  pl->sim.n_ds = n;
  pl->sim.n_spec = 2 * n;
  pl->sim.total_tiles = static_cast<int>(pl->tile_table.size());
  pl->sim.max_nodes = max_nodes;
  int max_window = 1;
  for (const SpeciesDev& S : pl->sp) max_window = std::max(max_window, static_cast<int>(S.W));
  pl->sim.max_window = max_window;
  pl->d_ds = cv.take<DischargeDev>(n);
  pl->d_sp = cv.take<SpeciesDev>(2 * n);
  pl->d_tt = cv.take<int2>(pl->tile_table.size());
  // the per-node and per-cell kernels take only the blocks that exist (a batch of
  // discharges of different sizes would otherwise launch its largest size for every one);
  // k_combine takes kCombineNodes nodes per workgroup, k_scan_cells kScanCells cells
  pl->node_table.clear();
  pl->cell_table.clear();
  for (int i = 0; i < 2 * n; ++i) {
    for (int j = 0; j < pl->sp[i].n_nodes; j += kCombineNodes)
      pl->node_table.push_back(make_int2(i, j));
    // no per-cell offsets when unsorted or sorted in place
    if (pl->sp[i].mode == kModeNone || pl->sp[i].mode == kModeFine) continue;
    for (int c = 0; c < pl->sp[i].n_cells; c += kScanCells)
      pl->cell_table.push_back(make_int2(i, c));
  }
  // MCC work: each electron tile alone (up to a few thousand candidates); the ion tiles'
  // lists several tiles at a time, as many as make about one workgroup pass of candidates
  // at the load (P0 of the ion tile's particles), at most kIonGroup: every workgroup pays
  // the collision path's long dependent chain once per pass however few lanes it has, and
  // few ion workgroups leave the CU slots to the long electron ones (large discharge: 64
  // tiles of a handful of candidates each; high-pressure discharges: one or two tiles of
  // a few hundred).  Electron work first, the long workgroups starting early.  With few
  // electron tiles (under four per CU) a workgroup has eight waves instead of four: each
  // lane's collision is a long dependent chain, and two four-wave workgroups per CU leave
  // the SIMDs idle (large discharge: 68 -> 61 us); with many, four-wave workgroups
  // schedule better (batched scan: 1.30 against 1.47 ms).
  int e_tiles = 0;
  for (int i = 0; i < 2 * n; i += 2) e_tiles += pl->sp[i].n_tiles + pl->sp[i].n_tail;
  const int cwg = e_tiles < kCollideWideBelow ? kCollideWide : kWG;
  pl->collide_table.clear();
  for (int pass = 0; pass < 2; ++pass)
    for (int i = pass; i < 2 * n; i += 2) {
      const SpeciesDev& S = pl->sp[i];
      const int nt = S.n_tiles + S.n_tail;
      int g = 1;
      if (pass == 1) {
        const int d = i / 2;
        const double per_tile = static_cast<double>(pl->cfg[d].n_i0) /
                                static_cast<double>(std::max(1, S.n_tiles)) * pl->der[d].p0[1];
        g = static_cast<int>(std::min<double>(kIonGroup,
                                              std::max(1.0, cwg / std::max(per_tile, 1e-9))));
      }
      for (int t = 0; t < nt; t += g)
        pl->collide_table.push_back(make_int4(i, t, std::min(g, nt - t), 0));
    }
  pl->d_nt = cv.take<int2>(pl->node_table.size());
  pl->d_ct = cv.take<int2>(pl->cell_table.size());
  pl->d_cw = cv.take<int4>(pl->collide_table.size());
  pl->d_sim = cv.take<SimDev>(1);
  pl->sim.ds = pl->d_ds;
  pl->sim.sp = pl->d_sp;
  pl->sim.tile_table = pl->d_tt;
  pl->sim.node_table = pl->d_nt;
  pl->sim.cell_table = pl->d_ct;
  pl->sim.collide_table = pl->d_cw;
  pl->bytes = align_up(cv.off, 256);
  LaunchInfo& li = pl->li;
  li.n_ds = n;
  li.n_spec = 2 * n;
  li.total_tiles = pl->sim.total_tiles;
  li.max_nodes = max_nodes;
  li.max_cap = max_cap;
  li.n_gtiles = n_gtiles;
  li.max_cells = max_cells;
  li.max_window = max_window;
  li.n_node_wgs = static_cast<int>(pl->node_table.size());
  li.n_cell_wgs = static_cast<int>(pl->cell_table.size());
  li.n_collide_wgs = static_cast<int>(pl->collide_table.size());
  li.collide_wg = cwg;
  li.fp32 = fp32;
  return PIC_OK;
}

}  // namespace

namespace fspic {
void set_init_error(const std::string& msg) { g_init_error = msg; }
}  // namespace fspic

struct pic_sim {
  Plan pl;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  std::string err;
  uint32_t sticky = 0;
  // graph replay
  uint32_t graph_k = 0;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap_stream = nullptr;
  // profiling
  bool prof = false;
  hipEvent_t ev[kRing][2 * kPhases] = {};
  int ring_used = 0;  // steps recorded in the ring and not yet read
  double ms[kPhases] = {};
  uint64_t cnt[kPhases] = {};
};

#define HIPCHECK(sim, expr)                                                   \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess) {                                                   \
      (sim)->err = std::string(#expr) + ": " + hipGetErrorString(e_);         \
      return PIC_ERR_DEVICE;                                                  \
    }                                                                         \
  } while (0)

static int launch_check(pic_sim* sim, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    sim->err = std::string(what) + ": " + hipGetErrorString(e);
    return PIC_ERR_DEVICE;
  }
  return PIC_OK;
}

static int map_error_bits(uint32_t bits) {
  if (bits & kErrIdOverflow) return PIC_ERR_ID_OVERFLOW;
  if (bits & (kErrCapacity | kErrFarOverflow | kErrFarGroup)) return PIC_ERR_CAPACITY;
  if (bits & kErrNonfinite) return PIC_ERR_NONFINITE;
  if (bits & kErrState) return PIC_ERR_CORRUPT;
  return PIC_OK;
}

static const char* error_text(uint32_t bits) {
  if (bits & kErrIdOverflow) return "particle ids exhausted (2^32 - 1)";
  if (bits & kErrCapacity) return "births did not fit the particle capacity";
  if (bits & kErrFarOverflow) return "far-mover list overflow (raise far_capacity / window)";
  if (bits & kErrFarGroup) return "too many far movers into one cell (raise window)";
  if (bits & kErrNonfinite) return "a particle position was not finite or not in a cell";
  if (bits & kErrState) return "inconsistent device state: an index out of range was refused";
  return "";
}

// deferred device errors that still leave the host copies readable
static bool readable(int rc) {
  return rc == PIC_OK || rc == PIC_ERR_CAPACITY || rc == PIC_ERR_ID_OVERFLOW ||
         rc == PIC_ERR_NONFINITE || rc == PIC_ERR_CORRUPT;
}

extern "C" int pic_workspace_bytes(const pic_config* cfgs, int n, size_t* bytes) {
  if (!bytes) return PIC_ERR_ARG;
  Plan pl;
  std::string why;
  const int rc = build_plan(cfgs, n, nullptr, &pl, &why);
  if (rc != PIC_OK) {
    g_init_error = why;
    return rc;
  }
  *bytes = pl.bytes;
  return PIC_OK;
}

extern "C" int pic_derive(const pic_config* cfg, pic_derived* out) {
  if (!cfg || !out) return PIC_ERR_ARG;
  std::string why;
  const int rc = validate_config(*cfg, &why);
  if (rc != PIC_OK) {
    g_init_error = why;
    return rc;
  }
  return derive(*cfg, out);
}

// Reads the phase events of the steps recorded so far (waits for the last of them) and
// adds their durations to the per-phase totals.  Events are read in batches so that a
// profiled run keeps the GPU as busy as an unprofiled one.
static int drain_profile(pic_sim* sim) {
  if (sim->ring_used == 0) return PIC_OK;
  // the finalize phase's end event (12, 13) is the last one a step records
  HIPCHECK(sim, hipEventSynchronize(sim->ev[sim->ring_used - 1][13]));
  for (int k = 0; k < sim->ring_used; ++k)
    for (int p = 0; p < kPhases; ++p) {
      float ms = 0.0f;
      HIPCHECK(sim, hipEventElapsedTime(&ms, sim->ev[k][2 * p], sim->ev[k][2 * p + 1]));
      sim->ms[p] += ms;
      sim->cnt[p] += 1;
    }
  sim->ring_used = 0;
  return PIC_OK;
}

static int step_once(pic_sim* sim, hipStream_t st) {
  const LaunchInfo& li = sim->pl.li;
  const SimDev* d = sim->pl.d_sim;
  if (!sim->prof) {
    launch_combine(li, d, st);
    launch_solve(li, d, 0, st);
    launch_hist(li, d, st);
    launch_scan(li, d, st);
    launch_main(li, d, st);
    launch_collide(li, d, st);
    if (li.coulomb) launch_coulomb(li, d, st);
    if (li.fine) launch_fine_sort(li, d, st);
    launch_finalize(li, d, st);
    if (li.fine) launch_fine_births(li, d, st);
    return launch_check(sim, "step launch");
  }
  if (sim->ring_used == kRing) {
    const int rc = drain_profile(sim);
    if (rc != PIC_OK) return rc;
  }
  hipEvent_t* ev = sim->ev[sim->ring_used];
  launch_combine(li, d, st, ev[0], ev[1]);
  launch_solve(li, d, 0, st, ev[2], ev[3]);
  launch_hist(li, d, st, ev[4], ev[5]);
  launch_scan(li, d, st, ev[6], ev[7]);
  launch_main(li, d, st, ev[8], ev[9]);
  launch_collide(li, d, st, ev[10], ev[11]);
  if (li.coulomb) {
    launch_coulomb(li, d, st, ev[14], ev[15]);
  } else {
    HIPCHECK(sim, hipEventRecord(ev[14], st));
    HIPCHECK(sim, hipEventRecord(ev[15], st));
  }
  if (li.fine) {
    launch_fine_sort(li, d, st, ev[16], ev[17]);
  } else {
    HIPCHECK(sim, hipEventRecord(ev[16], st));
    HIPCHECK(sim, hipEventRecord(ev[17], st));
  }
  launch_finalize(li, d, st, ev[12], ev[13]);
  if (li.fine) launch_fine_births(li, d, st);
  sim->ring_used += 1;
  return launch_check(sim, "step launch");
}

extern "C" int pic_init(const pic_config* cfgs, int n, void* d_workspace, size_t bytes,
                        void* hip_stream, pic_sim** out) {
  if (!out) return PIC_ERR_ARG;
  *out = nullptr;
  pic_sim* sim = new pic_sim();
  std::string why;
  int rc = build_plan(cfgs, n, static_cast<char*>(d_workspace), &sim->pl, &why);
  if (rc == PIC_OK && !d_workspace) {
    why = "workspace pointer is null";
    rc = PIC_ERR_ARG;
  }
  if (rc == PIC_OK && bytes < sim->pl.bytes) {
    why = "workspace of " + std::to_string(bytes) + " bytes, need " +
          std::to_string(sim->pl.bytes);
    rc = PIC_ERR_WORKSPACE;
  }
  if (rc == PIC_OK && (reinterpret_cast<uintptr_t>(d_workspace) & 255u)) {
    why = "workspace must be 256-byte aligned";
    rc = PIC_ERR_ARG;
  }
  if (rc != PIC_OK) {
    g_init_error = why;
    delete sim;
    return rc;
  }
  sim->ws = static_cast<char*>(d_workspace);
  sim->stream = static_cast<hipStream_t>(hip_stream);
  Plan& pl = sim->pl;
  hipStream_t st = sim->stream;
  auto fail = [&](int code) {
    g_init_error = sim->err;
    delete sim;
    return code;
  };
#define INITCHECK(expr)                                                     \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess) {                                                 \
      sim->err = std::string(#expr) + ": " + hipGetErrorString(e_);         \
      return fail(PIC_ERR_DEVICE);                                          \
    }                                                                       \
  } while (0)
  launch_zero(sim->ws, pl.bytes, st);  // pl.bytes is a multiple of 256
  INITCHECK(hipMemcpyAsync(pl.d_ds, pl.ds.data(), sizeof(DischargeDev) * pl.ds.size(),
                           hipMemcpyHostToDevice, st));
  INITCHECK(hipMemcpyAsync(pl.d_sp, pl.sp.data(), sizeof(SpeciesDev) * pl.sp.size(),
                           hipMemcpyHostToDevice, st));
  INITCHECK(hipMemcpyAsync(pl.d_tt, pl.tile_table.data(), sizeof(int2) * pl.tile_table.size(),
                           hipMemcpyHostToDevice, st));
  INITCHECK(hipMemcpyAsync(pl.d_nt, pl.node_table.data(), sizeof(int2) * pl.node_table.size(),
                           hipMemcpyHostToDevice, st));
  INITCHECK(hipMemcpyAsync(pl.d_ct, pl.cell_table.data(), sizeof(int2) * pl.cell_table.size(),
                           hipMemcpyHostToDevice, st));
  INITCHECK(hipMemcpyAsync(pl.d_cw, pl.collide_table.data(),
                           sizeof(int4) * pl.collide_table.size(), hipMemcpyHostToDevice, st));
  INITCHECK(hipMemcpyAsync(pl.d_sim, &pl.sim, sizeof(SimDev), hipMemcpyHostToDevice, st));
  for (const SpeciesDev& S : pl.sp)
    INITCHECK(hipMemcpyAsync(S.next_id, &S.n_init, sizeof(uint32_t), hipMemcpyHostToDevice, st));
  // load into buffer 1 (n_total[1] = n_init), sort into buffer 0
  for (const SpeciesDev& S : pl.sp)
    INITCHECK(hipMemcpyAsync(S.n_total + 1, &S.n_init, sizeof(uint32_t), hipMemcpyHostToDevice, st));
  launch_load(pl.li, pl.d_sim, 1, st);
  launch_general_sort(pl.li, pl.d_sim, 1, 0, st);
  if (pl.li.fine) launch_fine_scatter(pl.li, pl.d_sim, 0, st);
  launch_deposit_tiles(pl.li, pl.d_sim, -1, st);
  launch_combine(pl.li, pl.d_sim, st);
  launch_solve(pl.li, pl.d_sim, 1, st);
  launch_halfstep(pl.li, pl.d_sim, st);
  if (launch_check(sim, "init launch") != PIC_OK) return fail(PIC_ERR_DEVICE);
  INITCHECK(hipStreamSynchronize(st));
  uint32_t bits = 0;
  INITCHECK(hipMemcpy(&bits, pl.sim.error, sizeof(bits), hipMemcpyDeviceToHost));
  if (bits) {
    sim->err = error_text(bits);
    return fail(map_error_bits(bits));
  }
#undef INITCHECK
  *out = sim;
  return PIC_OK;
}

static int ensure_graph(pic_sim* sim) {
  if (sim->exec || sim->graph_k == 0) return PIC_OK;
  if (!sim->cap_stream) HIPCHECK(sim, hipStreamCreateWithFlags(&sim->cap_stream, hipStreamNonBlocking));
  HIPCHECK(sim, hipStreamBeginCapture(sim->cap_stream, hipStreamCaptureModeThreadLocal));
  const bool prof = sim->prof;
  sim->prof = false;
  for (uint32_t k = 0; k < sim->graph_k; ++k) step_once(sim, sim->cap_stream);
  sim->prof = prof;
  hipGraph_t g = nullptr;
  HIPCHECK(sim, hipStreamEndCapture(sim->cap_stream, &g));
  hipError_t e = hipGraphInstantiate(&sim->exec, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) {
    sim->exec = nullptr;
    sim->err = std::string("hipGraphInstantiate: ") + hipGetErrorString(e);
    return PIC_ERR_DEVICE;
  }
  return PIC_OK;
}

extern "C" int pic_step(pic_sim* sim, uint32_t n_steps) {
  if (!sim) return PIC_ERR_STATE;
  uint32_t done = 0;
  if (sim->graph_k > 0 && !sim->prof && n_steps >= sim->graph_k) {
    const int rc = ensure_graph(sim);
    if (rc != PIC_OK) return rc;
    while (n_steps - done >= sim->graph_k) {
      HIPCHECK(sim, hipGraphLaunch(sim->exec, sim->stream));
      done += sim->graph_k;
    }
  }
  for (; done < n_steps; ++done) {
    const int rc = step_once(sim, sim->stream);
    if (rc != PIC_OK) return rc;
  }
  return PIC_OK;
}

extern "C" int pic_set_graph(pic_sim* sim, uint32_t k) {
  if (!sim) return PIC_ERR_STATE;
  if (sim->exec) {
    hipGraphExecDestroy(sim->exec);
    sim->exec = nullptr;
  }
  sim->graph_k = k;
  return PIC_OK;
}

extern "C" int pic_sync(pic_sim* sim) {
  if (!sim) return PIC_ERR_STATE;
  HIPCHECK(sim, hipStreamSynchronize(sim->stream));
  uint32_t bits = 0;
  HIPCHECK(sim, hipMemcpy(&bits, sim->pl.sim.error, sizeof(bits), hipMemcpyDeviceToHost));
  sim->sticky |= bits;
  if (sim->sticky) {
    sim->err = error_text(sim->sticky);
    return map_error_bits(sim->sticky);
  }
  return PIC_OK;
}

template <class T>
static int d2h(pic_sim* sim, T* host, const T* dev, size_t count) {
  if (count == 0) return PIC_OK;
  HIPCHECK(sim, hipMemcpy(host, dev, sizeof(T) * count, hipMemcpyDeviceToHost));
  return PIC_OK;
}

template <class T>
static int h2d(pic_sim* sim, T* dev, const T* host, size_t count) {
  if (count == 0) return PIC_OK;
  HIPCHECK(sim, hipMemcpyAsync(dev, host, sizeof(T) * count, hipMemcpyHostToDevice, sim->stream));
  HIPCHECK(sim, hipStreamSynchronize(sim->stream));
  return PIC_OK;
}

// FP32 velocity records (vx, vy, vz, id words) and the host's per-field arrays (any of
// them may be null: not wanted).
struct VelRec {
  float vx, vy, vz;
  uint32_t id;
};
static_assert(sizeof(VelRec) == 16, "16-byte velocity records");

static void split_vel(const VelRec& r, size_t o, float* vx, float* vy, float* vz, uint32_t* id) {
  if (vx) vx[o] = r.vx;
  if (vy) vy[o] = r.vy;
  if (vz) vz[o] = r.vz;
  if (id) id[o] = r.id;
}

// FP64 velocity records (vx, vy, vz)
struct VelRec64 {
  double vx, vy, vz;
};
static_assert(sizeof(VelRec64) == 24, "24-byte velocity records");

static void split_vel64(const VelRec64& r, size_t o, double* vx, double* vy, double* vz) {
  if (vx) vx[o] = r.vx;
  if (vy) vy[o] = r.vy;
  if (vz) vz[o] = r.vz;
}

static uint64_t device_step(pic_sim* sim, int* rc) {
  unsigned long long st = 0;
  *rc = d2h(sim, &st, sim->pl.sim.step, 1);
  return st;
}

// Recomputes the node weights of the current particles (the combine of the next step).
static int refresh_weights(pic_sim* sim) {
  launch_combine(sim->pl.li, sim->pl.d_sim, sim->stream);
  int rc = launch_check(sim, "combine");
  if (rc != PIC_OK) return rc;
  HIPCHECK(sim, hipStreamSynchronize(sim->stream));
  return PIC_OK;
}

extern "C" int pic_grid(pic_sim* sim, int d, int what, double* out, size_t n_out) {
  if (!sim) return PIC_ERR_STATE;
  if (d < 0 || d >= sim->pl.li.n_ds || !out || what < 0 || what > 7) return PIC_ERR_ARG;
  const DischargeDev& D = sim->pl.ds[d];
  const size_t need = what == 7 ? static_cast<size_t>(D.eedf_bins) + 1 : D.n_nodes;
  if (n_out < need) return PIC_ERR_ARG;
  int rc = pic_sync(sim);
  if (!readable(rc)) return rc;
  const int sticky = rc;
  if (what <= 1) {
    rc = refresh_weights(sim);
    if (rc != PIC_OK) return rc;
  }
  switch (what) {
    case 0: rc = d2h(sim, out, D.w[0], need); break;
    case 1: rc = d2h(sim, out, D.w[1], need); break;
    case 2: rc = d2h(sim, out, D.phi, need); break;
    case 3: rc = d2h(sim, out, D.E64, need); break;
    case 4: rc = d2h(sim, out, D.acc_w[0], need); break;
    case 5: rc = d2h(sim, out, D.acc_w[1], need); break;
    case 6: rc = d2h(sim, out, D.acc_phi, need); break;
    default: {
      std::vector<unsigned long long> tmp(need);
      rc = d2h(sim, tmp.data(), D.eedf, need);
      for (size_t i = 0; i < need; ++i) out[i] = static_cast<double>(tmp[i]);
    }
  }
  return rc != PIC_OK ? rc : sticky;
}

extern "C" int pic_density(pic_sim* sim, int d, int quantity, int kind, double* out,
                           size_t n_out) {
  if (!sim) return PIC_ERR_STATE;
  if (d < 0 || d >= sim->pl.li.n_ds || !out || quantity < 0 || quantity > 2 || kind < 0 ||
      kind > 1)
    return PIC_ERR_ARG;
  const DischargeDev& D = sim->pl.ds[d];
  const pic_derived& k = sim->pl.der[d];
  const size_t nn = D.n_nodes;
  if (n_out < nn) return PIC_ERR_ARG;
  const int what = kind == 0 ? quantity : 4 + quantity;
  int rc = pic_grid(sim, d, what, out, n_out);
  if (!readable(rc)) return rc;
  double norm = 1.0;
  if (kind == 1) {
    unsigned long long c = 0;
    const int r2 = d2h(sim, &c, D.acc_count, 1);
    if (r2 != PIC_OK) return r2;
    norm = c > 0 ? 1.0 / static_cast<double>(c) : 0.0;
  }
  if (quantity <= 1) {
    const double f = norm * k.weight_per_area / k.dx;
    for (size_t j = 0; j < nn; ++j) out[j] *= f;
    if (!D.periodic) {
      out[0] *= 2.0;
      out[nn - 1] *= 2.0;
    }
  } else {
    const double f = norm * k.phi_scale;
    for (size_t j = 0; j < nn; ++j) out[j] *= f;
  }
  return rc;
}

extern "C" int pic_diagnostics(pic_sim* sim, int d, pic_diag* out) {
  if (!sim) return PIC_ERR_STATE;
  if (d < 0 || d >= sim->pl.li.n_ds || !out) return PIC_ERR_ARG;
  const int sticky = pic_sync(sim);
  if (sticky == PIC_ERR_DEVICE) return sticky;
  double* const eedf_out = out->eedf;
  const uint32_t eedf_cap = out->eedf_len;
  std::memset(out, 0, sizeof(*out));
  int rc;
  const uint64_t step = device_step(sim, &rc);
  if (rc != PIC_OK) return rc;
  const int p = static_cast<int>(step & 1);
  out->step = step;
  const DischargeDev& D = sim->pl.ds[d];
  for (int s = 0; s < 2; ++s) {
    const SpeciesDev& S = sim->pl.sp[2 * d + s];
    uint32_t nt = 0, ns = 0, nid = 0;
    unsigned long long ab[2] = {0, 0}, bi = 0, co[3] = {0, 0, 0};
    double ae[2] = {0, 0};
    uint32_t holes = 0;
    if ((rc = d2h(sim, &nt, S.n_total + p, 1)) != PIC_OK) return rc;
    if ((rc = d2h(sim, &ns, S.n_sorted + p, 1)) != PIC_OK) return rc;
    if ((rc = d2h(sim, &holes, S.n_holes + p, 1)) != PIC_OK) return rc;
    nt -= std::min(holes, nt);  // the lagged sort's dead records are not particles
    ns -= std::min(holes, ns);
    if ((rc = d2h(sim, &nid, S.next_id, 1)) != PIC_OK) return rc;
    if ((rc = d2h(sim, ab, S.absorbed, 2)) != PIC_OK) return rc;
    if ((rc = d2h(sim, ae, S.absorbed_energy, 2)) != PIC_OK) return rc;
    if ((rc = d2h(sim, &bi, S.births, 1)) != PIC_OK) return rc;
    if ((rc = d2h(sim, co, S.collisions, 3)) != PIC_OK) return rc;
    unsigned long long ps = 0;
    if ((rc = d2h(sim, &ps, S.psteps, 1)) != PIC_OK) return rc;
    out->particle_steps[s] = ps;
    out->n_particles[s] = nt;
    out->n_sorted[s] = ns;
    out->next_id[s] = nid;
    for (int w = 0; w < 2; ++w) {
      out->absorbed[s][w] = ab[w];
      out->absorbed_energy_ev[s][w] = ae[w];
    }
    out->births[s] = bi;
    for (int c = 0; c < 3; ++c) out->collisions[s][c] = co[c];
    unsigned long long em[2] = {0, 0}, rf[2] = {0, 0};
    if ((rc = d2h(sim, em, S.emitted, 2)) != PIC_OK) return rc;
    if ((rc = d2h(sim, rf, S.reflected, 2)) != PIC_OK) return rc;
    for (int w = 0; w < 2; ++w) {
      out->emitted[w] += em[w];
      out->reflected[w] += rf[w];
    }
  }
  double ds[DS_N] = {};
  unsigned long long est = 0;
  if ((rc = d2h(sim, ds, D.dstat, DS_N)) != PIC_OK) return rc;
  if ((rc = d2h(sim, &est, D.energy_step, 1)) != PIC_OK) return rc;
  out->kinetic[0] = ds[DS_KIN_E];
  out->kinetic[1] = ds[DS_KIN_I];
  out->momentum = ds[DS_MOM];
  out->energy_step = est;
  out->field_energy = ds[DS_FIELD];
  out->sum_rho = ds[DS_SUM_RHO];
  out->phi_driven_v = ds[DS_PHI0] * sim->pl.der[d].phi_scale;
  out->circuit_charge = ds[DS_Q];
  out->eedf = eedf_out;
  if (eedf_out && eedf_cap > 0) {
    const size_t n = std::min<size_t>(eedf_cap, static_cast<size_t>(D.eedf_bins) + 1);
    std::vector<unsigned long long> tmp(n);
    if ((rc = d2h(sim, tmp.data(), D.eedf, n)) != PIC_OK) return rc;
    for (size_t i = 0; i < n; ++i) eedf_out[i] = static_cast<double>(tmp[i]);
    out->eedf_len = static_cast<uint32_t>(n);
  }
  unsigned long long ac = 0, es = 0;
  if ((rc = d2h(sim, &ac, D.acc_count, 1)) != PIC_OK) return rc;
  if ((rc = d2h(sim, &es, D.eedf_samples, 1)) != PIC_OK) return rc;
  out->acc_count = ac;
  out->eedf_samples = es;
  double e0 = 0, en = 0;
  if ((rc = d2h(sim, &e0, D.E64, 1)) != PIC_OK) return rc;
  if ((rc = d2h(sim, &en, D.E64 + (D.n_nodes - 1), 1)) != PIC_OK) return rc;
  out->surface_charge[0] = D.periodic ? 0.0 : e0;
  out->surface_charge[1] = D.periodic ? 0.0 : -en;
  out->error_flags = sim->sticky;
  return sticky;
}

// Host copy of a fine-sorted species: the slots of every sorting cell, compacted in
// sorting-cell order.
template <class T>
static int fine_gather(pic_sim* sim, const SpeciesDev& S, const void* dev, T* host,
                       const std::vector<uint32_t>& cnt) {
  if (!host) return PIC_OK;
  std::vector<T> all(static_cast<size_t>(S.n_tiles) * S.nmax);
  int rc = d2h(sim, all.data(), static_cast<const T*>(dev), all.size());
  if (rc != PIC_OK) return rc;
  size_t o = 0;
  for (int k = 0; k < S.n_tiles; ++k) {
    const T* src = all.data() + static_cast<size_t>(k) * S.nmax;
    std::copy(src, src + std::min(cnt[k], S.nmax), host + o);
    o += std::min(cnt[k], S.nmax);
  }
  return PIC_OK;
}

static int fine_state_to_host(pic_sim* sim, const SpeciesDev& S, bool fp32, pic_state* st,
                              int s) {
  std::vector<uint32_t> cnt(S.n_tiles);
  int rc = d2h(sim, cnt.data(), S.fcnt, cnt.size());
  if (rc != PIC_OK) return rc;
  uint64_t n = 0;
  for (uint32_t c : cnt) n += std::min(c, S.nmax);
  if (n != st->n[s]) {
    sim->err = "pic_get_state: sorting-cell counts disagree with the particle count";
    return PIC_ERR_CORRUPT;
  }
  void* const* f = S.fine;
  if (fp32) {
    if ((rc = fine_gather(sim, S, f[F32_CELL], st->cell[s], cnt))) return rc;
    if ((rc = fine_gather(sim, S, f[F32_OFF], st->off[s], cnt))) return rc;
    std::vector<VelRec> rec(static_cast<size_t>(n));
    if ((rc = fine_gather(sim, S, f[F_VX], rec.data(), cnt))) return rc;
    for (size_t i = 0; i < rec.size(); ++i)
      split_vel(rec[i], i, st->vxf[s], st->vyf[s], st->vzf[s], st->id[s]);
    return PIC_OK;
  } else {
    if ((rc = fine_gather(sim, S, f[F64_X], st->x[s], cnt))) return rc;
    std::vector<VelRec64> rec(static_cast<size_t>(n));
    if ((rc = fine_gather(sim, S, f[F_VX], rec.data(), cnt))) return rc;
    for (size_t i = 0; i < rec.size(); ++i) split_vel64(rec[i], i, st->vx[s], st->vy[s], st->vz[s]);
  }
  return fine_gather(sim, S, f[F_ID], st->id[s], cnt);
}

// Host copy of a species under the lagged sort: the nt records of buffer p without the
// dead ones (cell -1, or x < 0).
template <class T>
static int lag_gather(pic_sim* sim, const void* dev, T* host, const std::vector<char>& live) {
  if (!host) return PIC_OK;
  std::vector<T> all(live.size());
  int rc = d2h(sim, all.data(), static_cast<const T*>(dev), all.size());
  if (rc != PIC_OK) return rc;
  size_t o = 0;
  for (size_t i = 0; i < live.size(); ++i)
    if (live[i]) host[o++] = all[i];
  return PIC_OK;
}

static int lag_state_to_host(pic_sim* sim, const SpeciesDev& S, bool fp32, int p, uint32_t nt,
                             pic_state* st, int s) {
  std::vector<char> live(nt);
  int rc;
  void* const* f = S.fld[p];
  if (fp32) {
    std::vector<int32_t> cell(nt);
    if ((rc = d2h(sim, cell.data(), static_cast<const int32_t*>(f[F32_CELL]), nt))) return rc;
    for (uint32_t i = 0; i < nt; ++i) live[i] = cell[i] >= 0;
    if ((rc = lag_gather(sim, f[F32_CELL], st->cell[s], live))) return rc;
    if ((rc = lag_gather(sim, f[F32_OFF], st->off[s], live))) return rc;
    size_t n_live = 0;
    for (char l : live) n_live += l ? 1 : 0;
    std::vector<VelRec> rec(n_live);
    if ((rc = lag_gather(sim, f[F_VX], rec.data(), live))) return rc;
    for (size_t i = 0; i < rec.size(); ++i)
      split_vel(rec[i], i, st->vxf[s], st->vyf[s], st->vzf[s], st->id[s]);
    return PIC_OK;
  } else {
    std::vector<double> x(nt);
    if ((rc = d2h(sim, x.data(), static_cast<const double*>(f[F64_X]), nt))) return rc;
    for (uint32_t i = 0; i < nt; ++i) live[i] = x[i] >= 0.0;
    if ((rc = lag_gather(sim, f[F64_X], st->x[s], live))) return rc;
    size_t n_live = 0;
    for (char l : live) n_live += l ? 1 : 0;
    std::vector<VelRec64> rec(n_live);
    if ((rc = lag_gather(sim, f[F_VX], rec.data(), live))) return rc;
    for (size_t i = 0; i < rec.size(); ++i) split_vel64(rec[i], i, st->vx[s], st->vy[s], st->vz[s]);
  }
  return lag_gather(sim, f[F_ID], st->id[s], live);
}

extern "C" int pic_get_state(pic_sim* sim, int d, pic_state* st) {
  if (!sim) return PIC_ERR_STATE;
  if (d < 0 || d >= sim->pl.li.n_ds || !st) return PIC_ERR_ARG;
  const int sticky = pic_sync(sim);
  if (sticky == PIC_ERR_DEVICE) return sticky;
  int rc;
  const uint64_t step = device_step(sim, &rc);
  if (rc != PIC_OK) return rc;
  const int p = static_cast<int>(step & 1);
  const bool fp32 = sim->pl.li.fp32;
  if ((rc = refresh_weights(sim)) != PIC_OK) return rc;
  const DischargeDev& D = sim->pl.ds[d];
  for (int s = 0; s < 2; ++s) {
    const SpeciesDev& S = sim->pl.sp[2 * d + s];
    uint32_t nt = 0, ns = 0, nid = 0;
    if ((rc = d2h(sim, &nt, S.n_total + p, 1)) != PIC_OK) return rc;
    if ((rc = d2h(sim, &ns, S.n_sorted + p, 1)) != PIC_OK) return rc;
    if ((rc = d2h(sim, &nid, S.next_id, 1)) != PIC_OK) return rc;
    st->n[s] = nt;
    st->n_sorted[s] = ns;
    st->next_id[s] = nid;
    uint32_t holes = 0;
    if ((rc = d2h(sim, &holes, S.n_holes + p, 1)) != PIC_OK) return rc;
    if (nt - std::min(holes, nt) > st->capacity[s]) {
      sim->err = "pic_get_state: host arrays smaller than the particle count";
      return PIC_ERR_CAPACITY;
    }
    if (S.mode == kModeLag && holes > 0) {
      // the dead records of the last step are left out (they lie in the sorted prefix)
      if ((rc = lag_state_to_host(sim, S, fp32, p, nt, st, s)) != PIC_OK) return rc;
      st->n[s] = nt - holes;
      st->n_sorted[s] = ns - std::min(holes, ns);
      if (st->w[s] && (rc = d2h(sim, st->w[s], D.w[s], D.n_nodes))) return rc;
      continue;
    }
    if (S.mode == kModeFine) {
      // sorting cells one after the other, each its fcnt particles
      st->n_sorted[s] = nt;
      if ((rc = fine_state_to_host(sim, S, fp32, st, s)) != PIC_OK) return rc;
      if (st->w[s] && (rc = d2h(sim, st->w[s], D.w[s], D.n_nodes))) return rc;
      continue;
    }
    void* const* f = S.fld[p];
    if (fp32) {
      if (st->cell[s] && (rc = d2h(sim, st->cell[s], static_cast<const int32_t*>(f[F32_CELL]), nt))) return rc;
      if (st->off[s] && (rc = d2h(sim, st->off[s], static_cast<const float*>(f[F32_OFF]), nt))) return rc;
      if (st->vxf[s] || st->vyf[s] || st->vzf[s] || st->id[s]) {
        std::vector<VelRec> rec(nt);
        if ((rc = d2h(sim, rec.data(), static_cast<const VelRec*>(f[F_VX]), nt))) return rc;
        for (uint32_t i = 0; i < nt; ++i)
          split_vel(rec[i], i, st->vxf[s], st->vyf[s], st->vzf[s], st->id[s]);
      }
    } else {
      if (st->x[s] && (rc = d2h(sim, st->x[s], static_cast<const double*>(f[F64_X]), nt))) return rc;
      if (st->vx[s] || st->vy[s] || st->vz[s]) {
        std::vector<VelRec64> rec(nt);
        if ((rc = d2h(sim, rec.data(), static_cast<const VelRec64*>(f[F_VX]), nt))) return rc;
        for (uint32_t i = 0; i < nt; ++i) split_vel64(rec[i], i, st->vx[s], st->vy[s], st->vz[s]);
      }
      if (st->id[s] && (rc = d2h(sim, st->id[s], static_cast<const uint32_t*>(f[F_ID]), nt))) return rc;
    }
    if (st->w[s] && (rc = d2h(sim, st->w[s], D.w[s], D.n_nodes))) return rc;
  }
  st->step = step;
  return sticky;
}

extern "C" int pic_set_state(pic_sim* sim, int d, const pic_state* st) {
  if (!sim) return PIC_ERR_STATE;
  if (d < 0 || d >= sim->pl.li.n_ds || !st) return PIC_ERR_ARG;
  int rc = pic_sync(sim);
  if (rc == PIC_ERR_DEVICE) return rc;
  const uint64_t cur = device_step(sim, &rc);
  if (rc != PIC_OK) return rc;
  if (sim->pl.li.n_ds > 1 && st->step != cur) {
    sim->err = "pic_set_state: in a batched simulation the step must stay the same";
    return PIC_ERR_ARG;
  }
  const bool fp32 = sim->pl.li.fp32;
  const DischargeDev& D = sim->pl.ds[d];
  const int N = D.n_cells;
  // a fine-sorted discharge is rebuilt from a cell sort of the whole state
  const bool fine = sim->pl.sp[2 * d].mode == kModeFine || sim->pl.sp[2 * d + 1].mode == kModeFine;
  const bool sort_all = st->sort_all || fine;
  // validate on the host before anything is uploaded
  for (int s = 0; s < 2; ++s) {
    const SpeciesDev& S = sim->pl.sp[2 * d + s];
    // an unsorted species keeps any order: no sorted prefix to check
    const uint64_t n = st->n[s],
                   ns = (sort_all || S.mode == kModeNone) ? 0 : st->n_sorted[s];
    if (n > S.cap || ns > n) {
      sim->err = "pic_set_state: counts exceed capacity";
      return PIC_ERR_ARG;
    }
    if (n && !st->id[s]) return PIC_ERR_ARG;
    long prev = -1;
    for (uint64_t i = 0; i < n; ++i) {
      long c;
      if (fp32) {
        if (!st->cell[s] || !st->off[s] || !st->vxf[s] || !st->vyf[s] || !st->vzf[s]) return PIC_ERR_ARG;
        const float o = st->off[s][i];
        c = st->cell[s][i];
        if (c < 0 || c >= N || !(o >= 0.0f && o < 1.0f)) {
          sim->err = "pic_set_state: position outside the box";
          return PIC_ERR_ARG;
        }
      } else {
        if (!st->x[s] || !st->vx[s] || !st->vy[s] || !st->vz[s]) return PIC_ERR_ARG;
        const double x = st->x[s][i];
        if (!(x >= 0.0 && x < static_cast<double>(N))) {
          sim->err = "pic_set_state: position outside the box";
          return PIC_ERR_ARG;
        }
        c = static_cast<long>(std::floor(x));
      }
      if (i < ns) {
        if (c < prev) {
          sim->err = "pic_set_state: the first n_sorted particles are not ordered by cell";
          return PIC_ERR_ARG;
        }
        prev = c;
      }
    }
  }
  // the step counter decides which buffer holds the state
  unsigned long long stp = st->step;
  if ((rc = h2d(sim, sim->pl.sim.step, &stp, 1)) != PIC_OK) return rc;
  const int p = static_cast<int>(stp & 1);
  const int up = sort_all ? p ^ 1 : p;
  for (int s = 0; s < 2; ++s) {
    const SpeciesDev& S = sim->pl.sp[2 * d + s];
    const uint32_t n = static_cast<uint32_t>(st->n[s]);
    const uint32_t ns = (sort_all || S.mode == kModeNone)
                            ? n : static_cast<uint32_t>(st->n_sorted[s]);
    void* const* f = S.fld[up];
    if (fp32) {
      if ((rc = h2d(sim, static_cast<int32_t*>(f[F32_CELL]), st->cell[s], n))) return rc;
      if ((rc = h2d(sim, static_cast<float*>(f[F32_OFF]), st->off[s], n))) return rc;
      std::vector<VelRec> rec(n);
      for (uint32_t i = 0; i < n; ++i)
        rec[i] = VelRec{st->vxf[s][i], st->vyf[s][i], st->vzf[s][i], st->id[s][i]};
      if ((rc = h2d(sim, static_cast<VelRec*>(f[F_VX]), rec.data(), n))) return rc;
    } else {
      if ((rc = h2d(sim, static_cast<double*>(f[F64_X]), st->x[s], n))) return rc;
      std::vector<VelRec64> rec(n);
      for (uint32_t i = 0; i < n; ++i) rec[i] = VelRec64{st->vx[s][i], st->vy[s][i], st->vz[s][i]};
      if ((rc = h2d(sim, static_cast<VelRec64*>(f[F_VX]), rec.data(), n))) return rc;
      if ((rc = h2d(sim, static_cast<uint32_t*>(f[F_ID]), st->id[s], n))) return rc;
    }
    const uint32_t cnt[2] = {n, ns};
    const uint32_t no_holes[2] = {0u, 0u};
    if ((rc = h2d(sim, S.n_total + up, &cnt[0], 1))) return rc;
    if ((rc = h2d(sim, S.n_sorted + up, &cnt[1], 1))) return rc;
    if ((rc = h2d(sim, S.n_holes, no_holes, 2))) return rc;
    const uint32_t nid = st->next_id[s];
    if ((rc = h2d(sim, S.next_id, &nid, 1))) return rc;
    launch_zero(S.far_w, sizeof(unsigned long long) * S.n_nodes, sim->stream);
  }
  if (sort_all) {
    // the general sort covers every species; keep the other discharges' buffers intact by
    // sorting only when this is the only discharge
    if (sim->pl.li.n_ds != 1) {
      sim->err = "pic_set_state: sort_all (and a fine-sorted state) is only available for a "
                 "single discharge";
      return PIC_ERR_ARG;
    }
    launch_general_sort(sim->pl.li, sim->pl.d_sim, up, p, sim->stream);
    if (fine) launch_fine_scatter(sim->pl.li, sim->pl.d_sim, p, sim->stream);
  } else {
    for (int s = 0; s < 2; ++s) launch_cell_start(sim->pl.li, sim->pl.d_sim, 2 * d + s, p, sim->stream);
  }
  launch_deposit_tiles(sim->pl.li, sim->pl.d_sim, d, sim->stream);
  if ((rc = launch_check(sim, "set_state")) != PIC_OK) return rc;
  HIPCHECK(sim, hipStreamSynchronize(sim->stream));
  return PIC_OK;
}

extern "C" int pic_profile(pic_sim* sim, int enable) {
  if (!sim) return PIC_ERR_STATE;
  if (enable && !sim->ev[0][0])
    for (int k = 0; k < kRing; ++k)
      for (int i = 0; i < 2 * kPhases; ++i) HIPCHECK(sim, hipEventCreate(&sim->ev[k][i]));
  if (sim->prof) {
    const int rc = drain_profile(sim);
    if (rc != PIC_OK) return rc;
  }
  sim->prof = enable != 0;
  for (int i = 0; i < kPhases; ++i) {
    sim->ms[i] = 0.0;
    sim->cnt[i] = 0;
  }
  return PIC_OK;
}

extern "C" int pic_profile_read(pic_sim* sim, double* ms, uint64_t* launches, int n) {
  if (!sim || !ms || !launches) return PIC_ERR_ARG;
  const int rc = drain_profile(sim);
  if (rc != PIC_OK) return rc;
  for (int i = 0; i < n && i < kPhases; ++i) {
    ms[i] = sim->ms[i];
    launches[i] = sim->cnt[i];
  }
  return PIC_OK;
}

extern "C" void pic_free(pic_sim* sim) {
  if (!sim) return;
  if (sim->stream) hipStreamSynchronize(sim->stream);
  if (sim->exec) hipGraphExecDestroy(sim->exec);
  if (sim->cap_stream) hipStreamDestroy(sim->cap_stream);
  for (int k = 0; k < kRing; ++k)
    for (int i = 0; i < 2 * kPhases; ++i)
      if (sim->ev[k][i]) hipEventDestroy(sim->ev[k][i]);
  delete sim;
}

extern "C" const char* pic_last_error(const pic_sim* sim) {
  return sim ? sim->err.c_str() : g_init_error.c_str();
}
