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

constexpr int kWG = 256;             // threads per workgroup of the particle kernels
constexpr int kWaves = kWG / 64;     // wave64
constexpr int kMaxWindow = 256;      // histogram window W = C + 2D (8-bit slot keys)
constexpr int kSolveWG = 1024;       // threads of the per-discharge solve / scan kernels
constexpr int kMaxCells = 16384;     // LDS histogram of the general (initial) sort
constexpr int kMaxEedfBins = 256;
constexpr int kMaxCellsPerTile = 64;

enum ErrorBits : uint32_t {
  kErrCapacity = 1u,     // births did not fit the particle arrays
  kErrFarOverflow = 2u,  // far-mover list overflowed (raise far_capacity or window)
  kErrIdOverflow = 4u,   // particle ids would pass 2^32 - 1
  kErrFarGroup = 8u,     // too many far movers into one cell in one step
  kErrState = 16u,       // inconsistent device state (an index out of range was refused)
};

// Per-particle record fields of the two layouts.
enum : int { F32_CELL = 0, F32_OFF = 1, F_VX = 2, F_VY = 3, F_VZ = 4, F_ID = 5 };
enum : int { F64_X = 0 };

struct SpeciesDev {
  int32_t ds, sp, n_cells, periodic;
  int32_t C, D, W, n_tiles;        // cell tiles: tile t owns cells [tC, tC + C)
  int32_t tile_base;               // first global workgroup index of the cell tiles
  int32_t n_tail, tail_base;       // workgroups that take the unsorted tail (births)
  int32_t n_nodes;
  uint32_t cap, far_cap;
  // particle arrays: [buffer][field]; FP32 cell+offset: cell, off, vx, vy, vz, id;
  // FP64: x, (unused), vx, vy, vz, id
  void* fld[2][6];
  // birth staging (electron species only): [0] secondary electrons, [1] new ions;
  // fields as in fld
  void* stage[2][6];
  uint32_t* n_total;        // [2] particles in buffer b
  uint32_t* n_sorted;       // [2] length of the cell-sorted prefix of buffer b
  uint32_t* next_id;        // [1]
  uint32_t* cell_start;     // [2][n_cells + 1] first index of each cell in the sorted prefix
  uint32_t* hist;           // [n_tiles * W] post-push cell histogram of each tile
  uint32_t* tilerel;        // [n_tiles * W] offset of tile t inside cell c, relative to base[c]
  void* partial;            // [n_tiles * (W + 1)] tile deposit windows (float or double)
  double* far_w;            // [n_nodes] deposits of far movers and births
  uint32_t* far_count;      // [1]
  uint4* far_list;          // [far_cap] (cell, index, source tile, 0)
  uint4* far_grouped;       // [far_cap] far list grouped by cell
  uint32_t* far_cell_cnt;   // [n_cells]
  uint32_t* far_fill;       // [n_cells]
  uint32_t* far_base;       // [n_cells]
  uint32_t* base;           // [n_cells] first output index of each cell
  uint32_t* far_dest;       // [cap] output index of each far mover, by input index
  uint4* cand;              // [cap] MCC candidates (output slot, id, channel words), stored
                            // in each tile's input-index range
  uint32_t* cand_cnt;       // [n_tiles + n_tail]
  uint32_t* birth_cnt;      // [n_tiles + n_tail] births of each electron tile
  uint32_t* tile_first;     // [n_tiles + n_tail] first input index of each tile
  uint32_t* birth_base;     // [n_tiles + n_tail + 1] exclusive scan of the electron births
  unsigned long long* absorbed;   // [2] per wall (0 left, 1 right)
  double* absorbed_energy;        // [2] eV
  unsigned long long* births;     // [1]
  unsigned long long* collisions; // [3]
  double* ke_sum;                 // [4] sum vx^2, vy^2, vz^2, vx (diagnostic steps)
  unsigned long long* psteps;     // [1] particles stepped, summed over steps
  // physics (normalised units)
  double kappa;
  float kappa_f;
  uint32_t t0;
  double energy_c, vunit, n_gas, nu0, vth_gas, mass_ratio;
  uint32_t key0, key1;
  int32_t xsec;
  double sigma_const;
  uint32_t* gsort_hist;     // [n_gtiles * n_cells] general sort scratch (initial sort)
  // initial load
  uint32_t n_init;
  int32_t load_kind, lang_mode;
  double vth, lang_amp;
};

struct DischargeDev {
  int32_t n_cells, periodic, n_nodes, spec0;
  double* w[2];             // current node weights of electrons and ions
  double* phi;
  double* E64;
  float* E32;
  double* acc_w[2];
  double* acc_phi;
  double* scratch;          // [n_nodes] solver scratch
  unsigned long long* acc_count;
  unsigned long long* eedf;          // [eedf_bins + 1]
  unsigned long long* eedf_samples;
  int32_t eedf_bins, diag_every;
  double eedf_inv_width;
  double vhat_amp, phase_per_step;
  int64_t avg_start;
};

struct SimDev {
  unsigned long long* step;
  uint32_t* error;
  uint32_t* fin_count;       // workgroups of the finalize kernel done this step
  int32_t n_ds, n_spec, total_tiles, max_nodes;
  DischargeDev* ds;
  SpeciesDev* sp;
  int2* tile_table;          // workgroup -> (species index, local tile)
};

}  // namespace fspic
