// sim_layout.h -- descriptors shared by the host side of libfspic and its kernels.
//
// One SpeciesDev per (discharge, species) and one DischargeDev per discharge live in
// the caller's workspace; every kernel of a step reads them, so a step's launches have
// identical arguments from one step to the next (which is what lets a captured HIP
// graph replay any number of steps).  Buffers that change role every step (the two
// particle arrays, cell offsets and counts) are indexed by the parity of the device
// step counter.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace fspic {

// Device code sees the descriptors' array pointers as global-memory pointers, so loads and
// stores through them compile to global_* instructions.  Through a generic pointer they
// would be flat_* instructions, which also count against the LDS wait counter and make
// every LDS access in a loop wait for the loads in flight.  Host code sees plain pointers
// of the same size and layout.
// The descriptors themselves are read through constant-address-space pointers: they do not
// change during a launch, and the compiler then reads them with scalar loads.
#if defined(__HIP_DEVICE_COMPILE__)
#define FSPIC_GLOBAL __attribute__((address_space(1)))
#define FSPIC_CONST __attribute__((address_space(4)))
#else
#define FSPIC_GLOBAL
#define FSPIC_CONST
#endif
#define GM FSPIC_GLOBAL
#define CM FSPIC_CONST

constexpr int kWG = 256;             // threads per workgroup of the particle kernels
constexpr int kWaves = kWG / 64;     // wave64
constexpr int kMaxWindow = 256;      // histogram window W = C + 2D (8-bit slot keys)
constexpr int kSolveWG = 1024;       // threads of the per-discharge solve / scan kernels
constexpr int kCombineLanes = 8;     // lanes per node in k_combine
constexpr int kCombineNodes = 32;    // nodes of a k_combine workgroup (256 threads)
constexpr int kCollideWide = 512;    // threads of an MCC workgroup when electron tiles are few
constexpr int kCollideWideBelow = 1024;  // ... fewer than this (four per CU of the MI355X)
constexpr int kIonGroup = 64;        // ion tiles whose candidate lists one MCC workgroup takes
constexpr int kScanLanes = 16;       // lanes per cell in k_scan_cells
constexpr int kScanCells = 16;       // cells of a k_scan_cells workgroup (256 threads)
constexpr int kMaxCells = 16384;     // LDS histogram of the general (initial) sort
constexpr int kMaxEedfBins = 256;
constexpr int kMaxCellsPerTile = 64;
constexpr int kMaxFineSlots = 65536; // slots of one fine-sort sorting cell (LDS bit masks)

enum ErrorBits : uint32_t {
  kErrCapacity = 1u,     // births did not fit the particle arrays
  kErrFarOverflow = 2u,  // far-mover list overflowed (raise far_capacity or window)
  kErrIdOverflow = 4u,   // particle ids would pass 2^32 - 1
  kErrFarGroup = 8u,     // too many far movers into one cell in one step
  kErrState = 16u,       // inconsistent device state (an index out of range was refused)
  kErrNonfinite = 32u,   // a particle's position was not finite or not in a cell
};

// Wall events of one tile in one step (written only by the tiles that have any, which
// mark themselves in the species' event bitmap), combined in tile order by k_birth_scan
// (so the totals do not depend on the order tiles finish in).
struct TileStats {
  double abs_e[2];    // energy of the particles absorbed at each wall [eV]
  uint32_t abs_n[2];  // particles absorbed at each wall
  uint32_t emit[2];   // secondary electrons emitted at each wall (ion species)
  uint32_t refl[2];   // electrons reflected at each wall (electron species)
};


// Per-discharge results of the last step, normalised units (energy Q^2 dx / (eps0 A),
// charge Q / A, potential Q dx / (eps0 A)).
enum : int {
  DS_KIN_E = 0,     // kinetic energy of the electrons (energy steps)
  DS_KIN_I = 1,     // kinetic energy of the ions (energy steps)
  DS_MOM = 2,       // x-momentum sum_s sum v_x / |kappa_s| (energy steps)
  DS_FIELD = 3,     // field energy 1/2 sum over cells of (Phi_j - Phi_j+1)^2
  DS_SUM_RHO = 4,   // net node charge sum_j (w_i - w_e)
  DS_PHI0 = 5,      // potential of the driven electrode
  DS_Q = 6,         // charge of the driven electrode's conductor (series capacitor)
  DS_Q_INIT = 7,    // that charge at the load
  DS_N = 8
};

// Per-particle record fields of the two layouts.  The velocity is kept as one record per
// particle, so that the MCC pass writes a collided particle's velocity with one store
// into one cache line (two at most):
// * FP32: cell and offset in arrays of their own (4 bytes each); vx, vy, vz, id together
//   in an array of 16-byte records, the field pointers of vx, vy, vz and id pointing 0,
//   4, 8 and 12 bytes into it (element stride 16 bytes);
// * FP64: x and id in arrays of their own (8 and 4 bytes); vx, vy, vz in an array of
//   24-byte records, their field pointers 0, 8 and 16 bytes into it (stride 24 bytes).
enum : int { F32_CELL = 0, F32_OFF = 1, F_VX = 2, F_VY = 3, F_VZ = 4, F_ID = 5 };
enum : int { F64_X = 0 };

// Array order a species keeps (pic_sort).
enum : int32_t { kModeCounting = 0, kModeNone = 1, kModeFine = 2, kModeLag = 3 };

struct SpeciesDev {
  int32_t ds, sp, n_cells, periodic;
  int32_t mode;                // kMode*: counting sort, unsorted (range tiles), fine sort
  int32_t C, D, W, n_tiles;        // cell tiles: tile t owns cells [tC, tC + C)
  int32_t n_tail;                  // tail tiles: the unsorted births at the end of the array
  int32_t n_nodes;
  uint32_t cap, far_cap;
  // particle arrays: [buffer][field]; FP32 cell+offset: cell, off, vx, vy, vz, id;
  // FP64: x, (unused), vx, vy, vz, id
  void GM* fld[2][6];
  uint32_t bstride4, bstride8;  // fld[1][f] - fld[0][f] in bytes for 4- and 8-byte fields
  uint32_t bstridev;            // ... for the velocity records (a multiple of the record size)
  // birth staging (electron species only): [0] secondary electrons, [1] new ions;
  // fields as in fld
  void GM* stage[2][6];
  uint32_t GM* n_total;        // [2] particles in buffer b
  uint32_t GM* n_sorted;       // [2] length of the cell-sorted prefix of buffer b
  uint32_t GM* n_holes;        // [2] lagged sort: dead records (absorbed) in buffer b
  uint32_t GM* next_id;        // [1]
  uint32_t GM* cell_start;     // [2][n_cells + 1] first index of each cell in the sorted prefix
  // A tile's index range is split into kWaves contiguous sub-ranges, one per wave, in
  // order; each (tile, wave) keeps its own histogram row so the waves never synchronise.
  uint32_t GM* hist;           // [n_tiles * kWaves * W] post-push cell histogram per (tile, wave)
  uint32_t GM* tilerel;        // [n_tiles * kWaves * W] offset of (tile, wave) in cell c from base[c]
  uint32_t GM* thist;          // [n_tail * kWaves * n_cells] post-push cell counts per tail row
  uint32_t GM* trel;           // [n_tail * kWaves * n_cells] running offset of a tail row in cell c
  // Charge deposits are integers: a weight w in [0, 1] is added as round(w 2^dep_shift),
  // so sums are exact and do not depend on the order of the additions.
  unsigned long long GM* partial;  // [n_tiles * (W + 1)] tile deposit windows
  unsigned long long GM* far_w;    // [n_nodes] deposits of far movers, tail tiles and births
  uint32_t GM* far_count;      // [1]
  uint4 GM* far_list;          // [far_cap] far movers of the cell tiles: (cell, index, tile, 0)
  uint4 GM* far_grouped;       // [far_cap] far list grouped by cell
  uint32_t GM* far_cell_cnt;   // [n_cells]
  uint32_t GM* far_fill;       // [n_cells]
  uint32_t GM* far_base;       // [n_cells]
  uint32_t GM* base;           // [n_cells] first output index of each cell
  uint32_t GM* far_dest;       // [cap] output index of each far mover, by input index
  void GM* cand;               // [cap + 1] MCC candidate records (output slot, id, cell and the
                               // post-push position and velocity; 32 B in FP32, 48 B in FP64),
                               // stored in the input-index range of the wave that found them
  uint32_t GM* cand_cnt;       // [(n_tiles + n_tail) * kWaves] candidates per (tile, wave)
  uint32_t GM* birth_cnt;      // [n_tiles + n_tail] births of each electron tile
  uint32_t GM* stage_first;    // [n_tiles + n_tail] first staging index of a tile's births
  uint32_t GM* birth_base;     // [n_tiles + n_tail + 1] exclusive scan of the electron births
                               // (electron species only)
  uint32_t GM* fin;            // [2] births that fit this step, id of the first
  unsigned long long GM* absorbed;   // [2] per wall (0 left, 1 right)
  double GM* absorbed_energy;        // [2] eV
  unsigned long long GM* births;     // [1]
  unsigned long long GM* collisions; // [3]
  unsigned long long GM* emitted;    // [2] secondary electrons emitted per wall (ions)
  unsigned long long GM* reflected;  // [2] electrons reflected per wall (electrons)
  unsigned long long GM* psteps;     // [1] particles stepped, summed over steps
  TileStats GM* tstats;              // [n_tiles + n_tail] this step's wall events per tile
  uint32_t GM* ev_bits;              // [(n_tiles + n_tail + 31) / 32] tiles with wall events
  uint2 GM* tcount;                  // [n_tiles + n_tail] particles pushed, alive per tile
  double GM* tke;                    // [2 (n_tiles + n_tail)] kinetic energy, momentum sums
                                     // per tile (energy steps)
  // fixed-point deposit: one = 2^dep_shift, inv = 2^-dep_shift
  unsigned long long dep_one;
  double dep_scale, dep_inv;
  // physics (normalised units)
  double kappa;
  float kappa_f;
  uint32_t t0;
  double energy_c, vunit, n_gas, nu0, vth_gas, mass_ratio;
  uint32_t key0, key1;
  int32_t xsec;
  double sigma_const;
  // electrode processes: reflection threshold (electrons) and emission threshold (ions) of
  // a Philox word, and the spread of the emitted electrons' velocity components
  uint32_t t_refl, t_see;
  double vth_see;
  // secondary emission (ion species): k_main lists the absorbed ions (id, wall status) in
  // their (tile, wave) unit's index range, in input order; k_emit stores the emitted
  // electrons (electron records in the fields of `fld`) compacted at the front of the same
  // range.  Per (tile, wave): absorbed count, first list index, emitted count and (after
  // k_birth_scan) the exclusive scan of the emitted counts
  uint2 GM* ab_list;           // [cap]
  void GM* em_stage[6];        // [cap] each
  uint32_t GM* ab_cnt;         // [(n_tiles + n_tail) * kWaves]
  uint32_t GM* em_lo;          // [(n_tiles + n_tail) * kWaves]
  uint32_t GM* em_cnt;         // [(n_tiles + n_tail) * kWaves]
  uint32_t GM* em_base;        // [(n_tiles + n_tail) * kWaves + 1]
  // fine sort (the paper's fixed-capacity sorting cells, kModeFine): sorting cell k (the
  // tile k, C grid cells) holds its particles in slots [k nmax, k nmax + fcnt[k]) of the
  // `fine` arrays (fields as in fld), sorted in place every step; its free slots at the end
  // park the particles that leave it (flv of them) until they are moved
  void GM* fine[6];
  uint32_t nmax;
  uint32_t GM* fcnt;           // [n_tiles]
  uint32_t GM* flv;            // [n_tiles]
  uint32_t GM* fpid;           // [cap] parent id of each staged birth (electron species)
  uint32_t GM* fpid_list;      // [cap] the step's birth parent ids in birth order
  uint32_t GM* gsort_hist;     // [n_gtiles * n_cells] general sort scratch (initial sort)
  // initial load
  uint32_t n_init;
  int32_t load_kind, lang_mode;
  double vth, lang_amp;
};

struct DischargeDev {
  int32_t n_cells, periodic, n_nodes, spec0;
  double GM* w[2];             // current node weights of electrons and ions
  double GM* phi;
  double GM* E64;
  float GM* E32;
  double GM* acc_w[2];
  double GM* acc_phi;
  double GM* dstat;            // [DS_N] results of the last step
  unsigned long long GM* energy_step;  // step of the last kinetic-energy sums
  unsigned long long GM* acc_count;
  unsigned long long GM* eedf;          // [eedf_bins + 1]
  unsigned long long GM* eedf_samples;
  int32_t eedf_bins, diag_every;
  double eedf_inv_width;
  double vhat_amp, phase_per_step;
  double cap_norm;             // series capacitance in units of eps0 A / dx; 0: ideal source
  int64_t avg_start;
  // binary Coulomb collisions in a cell: bit 0 e-e, bit 1 i-i, bit 2 e-i
  int32_t coulomb;
  double coul_coef[3];         // e^4 lnLambda dt / (8 pi eps0^2 m_ab^2) of e-e, i-i, e-i [SI]
  double coul_dens;            // density of one macro-particle per cell [m^-3]
  double vunit;                // dx / dt [m/s]
  double mfrac_e, mfrac_i;     // an e-i pair's shares of the change: m_i / M, m_e / M
};

struct SimDev {
  unsigned long long GM* step;
  uint32_t GM* error;
  uint32_t GM* fin_count;       // workgroups of the finalize kernel done this step
  int32_t n_ds, n_spec, total_tiles, max_nodes;
  int32_t max_window;        // largest histogram window W of all species
  const DischargeDev CM* ds;
  const SpeciesDev CM* sp;
  const int2 CM* tile_table;  // workgroup -> (species index, local tile)
  const int2 CM* node_table;  // k_combine workgroup -> (species index, first of kCombineNodes nodes)
  const int2 CM* cell_table;  // k_scan_cells workgroup -> (species index, first of kScanCells cells)
  // k_collide workgroup -> (species index, first tile, tiles, 0): one electron tile, or up
  // to kIonGroup consecutive ion tiles
  const int4 CM* collide_table;
};

}  // namespace fspic
