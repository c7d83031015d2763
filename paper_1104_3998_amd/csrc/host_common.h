// host_common.h -- declarations shared by the host-side files of libfspic.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/fspic.h"
#include "sim_layout.h"

namespace fspic {

struct TileChoice {
  int C, D, W, n_tiles, n_tail;
};

int validate_config(const pic_config& c, std::string* why);
int derive(const pic_config& c, pic_derived* k);
void choose_tiles(const pic_config& c, const pic_derived& k, TileChoice tc[2]);
double electron_mass();
double ion_mass(const pic_config& c);

// Launch geometry the host needs beside the device descriptors.
struct LaunchInfo {
  int n_ds, n_spec, total_tiles, max_nodes, max_cap, n_gtiles, max_cells, max_window;
  int n_node_wgs, n_cell_wgs;  // entries of the node and cell block tables
  int n_collide_wgs;           // entries of the MCC work table
  bool fp32;
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

// Set-up kernels (kernels_setup.hip).
void launch_load(const LaunchInfo& li, const SimDev* sim, int dst_buf, hipStream_t st);
void launch_general_sort(const LaunchInfo& li, const SimDev* sim, int src_buf, int dst_buf,
                         hipStream_t st);
void launch_cell_start(const LaunchInfo& li, const SimDev* sim, int spec, int buf,
                       hipStream_t st);
void launch_deposit_tiles(const LaunchInfo& li, const SimDev* sim, int ds_filter,
                          hipStream_t st);
void launch_halfstep(const LaunchInfo& li, const SimDev* sim, hipStream_t st);

}  // namespace fspic
