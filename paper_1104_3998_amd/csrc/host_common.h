// host_common.h -- declarations shared by the host-side files of libfspic.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/fspic.h"
#include "sim_layout.h"

namespace fspic {

struct TileChoice {
  int C, D, W, n_tiles, n_tail;
  int nmax;  // fine sort: slots per sorting cell
};

int validate_config(const pic_config& c, std::string* why);
// message returned by pic_last_error(NULL) (errors before a pic_sim exists)
void set_init_error(const std::string& msg);
int derive(const pic_config& c, pic_derived* k);
void choose_tiles(const pic_config& c, const pic_derived& k, TileChoice tc[2]);
double electron_mass();
double ion_mass(const pic_config& c);
double circuit_cap_norm(const pic_config& c, const pic_derived& k);
void coulomb_coefficients(const pic_config& c, double coef[3]);
uint32_t word_threshold(double p);
double see_spread(const pic_config& c, const pic_derived& k);

// Launch geometry the host needs beside the device descriptors.
struct LaunchInfo {
  int n_ds, n_spec, total_tiles, max_nodes, max_cap, n_gtiles, max_cells, max_window;
  int n_node_wgs, n_cell_wgs;  // entries of the node and cell block tables
  int n_collide_wgs;           // entries of the MCC work table
  int collide_wg;              // threads of an MCC workgroup (kWG or kCollideWide)
  bool fp32;
  bool coulomb;                // some discharge has Coulomb collisions
  bool emission;               // some discharge has secondary emission
  bool fine;                   // some species is fine-sorted
  bool lag;                    // every species uses the lagged counting sort
};

// Step kernels (kernels_step.hip).  `sim` points at the SimDev copy in device memory.
// With events e0 / e1, they are recorded at the start / end of the phase's kernels.
void launch_combine(const LaunchInfo& li, const SimDev* sim, hipStream_t st,
                    hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_solve(const LaunchInfo& li, const SimDev* sim, int init_mode, hipStream_t st,
                  hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_hist(const LaunchInfo& li, const SimDev* sim, hipStream_t st,
                 hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_scan(const LaunchInfo& li, const SimDev* sim, hipStream_t st,
                 hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_main(const LaunchInfo& li, const SimDev* sim, hipStream_t st,
                 hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_collide(const LaunchInfo& li, const SimDev* sim, hipStream_t st,
                    hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_finalize(const LaunchInfo& li, const SimDev* sim, hipStream_t st,
                     hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Fine sort (kernels_fine.hip): steps 1-3 after the MCC; births into their sorting cells
// after k_birth_scan; the set-up scatter of a cell-sorted contiguous buffer
void launch_fine_sort(const LaunchInfo& li, const SimDev* sim, hipStream_t st,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
void launch_fine_births(const LaunchInfo& li, const SimDev* sim, hipStream_t st);
void launch_fine_scatter(const LaunchInfo& li, const SimDev* sim, int src, hipStream_t st);
// Coulomb collisions (kernels_coulomb.hip)
void launch_coulomb(const LaunchInfo& li, const SimDev* sim, hipStream_t st,
                    hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);

// Set-up kernels (kernels_setup.hip).
void launch_load(const LaunchInfo& li, const SimDev* sim, int dst_buf, hipStream_t st);
void launch_general_sort(const LaunchInfo& li, const SimDev* sim, int src_buf, int dst_buf,
                         hipStream_t st);
void launch_cell_start(const LaunchInfo& li, const SimDev* sim, int spec, int buf,
                       hipStream_t st);
void launch_deposit_tiles(const LaunchInfo& li, const SimDev* sim, int ds_filter,
                          hipStream_t st);
void launch_halfstep(const LaunchInfo& li, const SimDev* sim, hipStream_t st);
// zero fill of `bytes` (a multiple of 8) at the 8-byte aligned device address p
void launch_zero(void* p, size_t bytes, hipStream_t st);

}  // namespace fspic
