// kernels_fine.hip -- the paper's fine sort (Sec. 3.2 data structure, Sec. 3.7 algorithm)
// on gfx950, the alternative to the stable counting sort.
//
// Each sorting cell k (C grid cells, the paper's N_gc = C + 1 grid points) owns nmax slots
// of the particle arrays; its particles fill the first fcnt[k].  The push (k_main) updates
// every particle in its slot.  Then, as in the paper:
//   step 1 (k_fine_sort1, one workgroup per sorting cell; the paper's steps 1a and 1b):
//     particles that left the sorting cell are copied to its free slots at the end, and
//     the gaps they and the absorbed particles leave are filled with the last particles
//     that stayed;
//   step 2 (k_fine_sort2): each sorting cell takes from its two neighbours' parked
//     particles the ones that moved into it;
//   step 3 (k_fine_sort3): the rare particles that moved farther than one sorting cell
//     are appended to their sorting cell with a global atomic counter (the algorithm's
//     one global atomic).
// The paper ranks with shared-memory atomic counters; here every rank inside a workgroup
// comes from ordered scans of LDS bit masks, so steps 1 and 2 place the particles the same
// way every run.  Step 3 and the births (k_fine_births) take their slots from global
// atomics, so the order inside a sorting cell is not fixed (the set of particles of each
// sorting cell is); births therefore take their ids in increasing parent id.
#include <hip/hip_ext.h>

#include <type_traits>

#include "device_common.h"
#include "host_common.h"

namespace fspic {

namespace {

struct F32 {};
struct F64 {};

template <class P>
struct FReal;
template <>
struct FReal<F32> {
  using type = float;
};
template <>
struct FReal<F64> {
  using type = double;
};

constexpr int kFineWG = 256;
constexpr uint32_t kMaxFineBirths = 65536;  // births per step and discharge (fine sort)
constexpr int kMaxFineWords = kMaxFineSlots / 32;

// cell of the particle in slot i of the fine arrays, -1 for a dead slot
template <class P>
__device__ __forceinline__ int fine_cell(const SpeciesDev& s, uint32_t i) {
  if constexpr (std::is_same<P, F32>::value) {
    return ldg<int>(s.fine[F32_CELL], i);
  } else {
    const double x = ldg<double>(s.fine[F64_X], i);
    return x >= 0.0 ? static_cast<int>(floor(x)) : -1;
  }
}

// whole record from slot a to slot b of the fine arrays
template <class P>
__device__ __forceinline__ void fine_copy(const SpeciesDev& s, uint32_t a, uint32_t b) {
  using real = typename FReal<P>::type;
  if constexpr (std::is_same<P, F32>::value) {
    stg<int>(s.fine[F32_CELL], b, ldg<int>(s.fine[F32_CELL], a));
    stg<float>(s.fine[F32_OFF], b, ldg<float>(s.fine[F32_OFF], a));
    stg<uint4>(s.fine[F_VX], b, ldg<uint4>(s.fine[F_VX], a));  // velocity and id record
  } else {
    stg<double>(s.fine[F64_X], b, ldg<double>(s.fine[F64_X], a));
    stg<Vel3d>(s.fine[F_VX], b, ldg<Vel3d>(s.fine[F_VX], a));
    stg<uint32_t>(s.fine[F_ID], b, ldg<uint32_t>(s.fine[F_ID], a));
  }
}

// sorting cell of a particle in cell c
__device__ __forceinline__ int sort_cell_of(const SpeciesDev& s, int c) { return c / s.C; }

// Position of the set bit of rank t (0-based) among the bits of `m`.
__device__ __forceinline__ int select_bit(uint32_t m, int t) {
  for (int k = 0; k < t; ++k) m &= m - 1u;
  return __ffs(static_cast<int>(m)) - 1;
}

// Exclusive scan of n words' popcounts held in `words` into `pre` (LDS), by one workgroup;
// returns the total.
__device__ uint32_t popcount_scan(const uint32_t* words, uint32_t* pre, int n, uint32_t* lds) {
  for (int w = threadIdx.x; w < n; w += blockDim.x) pre[w] = __popc(words[w]);
  return array_exclusive_scan(pre, n, lds);
}

// ------------------------------------------------------------------------------------
// Step 1: sorting cell k after the push.  Slot j < n is a stayer (still in k), a leaver
// (alive, now in another sorting cell) or dead (absorbed).  Leavers are copied to the
// free slots at the end, leaver r to slot nmax - 1 - r; then the g-th gap below S (the
// number of stayers) takes the g-th stayer at or above S.  Afterwards the stayers fill
// [0, S) and the L leavers [nmax - L, nmax).
// ------------------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(kFineWG) void k_fine_sort1(const SimDev* __restrict__ simp) {
  const SimDev& sim = *simp;
  const int2 tt = sim.tile_table[blockIdx.x];
  const SpeciesDev s = sim.sp[tt.x];
  if (s.mode != kModeFine) return;
  const int k = tt.y;
  const uint32_t base = static_cast<uint32_t>(k) * s.nmax;
  const uint32_t n = min(s.fcnt[k], s.nmax);
  __shared__ uint32_t stay[kMaxFineWords], leave[kMaxFineWords];
  __shared__ uint32_t stay_pre[kMaxFineWords], leave_pre[kMaxFineWords];
  __shared__ uint32_t lds[kFineWG / 64 + 1];
  const int nw = static_cast<int>((n + 31u) / 32u);
  for (int w = threadIdx.x; w < nw; w += blockDim.x) stay[w] = leave[w] = 0u;
  __syncthreads();
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
    const int c = fine_cell<P>(s, base + j);
    const uint32_t bit = 1u << (j & 31u);
    if (c >= 0) {
      if (sort_cell_of(s, c) == k) atomicOr(&stay[j >> 5], bit);
      else atomicOr(&leave[j >> 5], bit);
    }
  }
  __syncthreads();
  const uint32_t S = popcount_scan(stay, stay_pre, nw, lds);
  const uint32_t L = popcount_scan(leave, leave_pre, nw, lds);
  if (n + L > s.nmax) {
    // the parked leavers would overwrite particles not yet moved: the sorting cell is full
    // (the state is no longer valid; nothing is parked for steps 2 and 3)
    if (threadIdx.x == 0) {
      atomicOr(sim.error, kErrCapacity);
      s.flv[k] = 0u;
    }
    return;
  }
  // 1a: leavers to the end, in slot order from the last slot down
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
    const uint32_t m = leave[j >> 5];
    if (!((m >> (j & 31u)) & 1u)) continue;
    const uint32_t r = leave_pre[j >> 5] + __popc(m & ((1u << (j & 31u)) - 1u));
    fine_copy<P>(s, base + j, base + s.nmax - 1u - r);
  }
  __syncthreads();  // the leavers' slots are read before they are refilled
  // 1b: gaps below S take the stayers above S, in order
  const uint32_t stays_below_S = [&] {
    const uint32_t w = S >> 5;
    if (w >= static_cast<uint32_t>(nw)) return S;
    return stay_pre[w] + __popc(stay[w] & ((1u << (S & 31u)) - 1u));
  }();
  for (uint32_t j = threadIdx.x; j < S; j += blockDim.x) {
    const uint32_t m = stay[j >> 5];
    if ((m >> (j & 31u)) & 1u) continue;
    // gap rank among the gaps below S, and the stayer of that rank above S
    const uint32_t g = j - (stay_pre[j >> 5] + __popc(m & ((1u << (j & 31u)) - 1u)));
    const uint32_t want = stays_below_S + g;  // rank among all stayers, < S
    if (want >= S) continue;                  // cannot happen: as many donors as gaps
    int lo = 0, hi = nw - 1;                  // last word whose prefix <= want
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (stay_pre[mid] <= want) lo = mid;
      else hi = mid - 1;
    }
    const uint32_t src = static_cast<uint32_t>(lo) * 32u +
                         static_cast<uint32_t>(select_bit(stay[lo], static_cast<int>(want - stay_pre[lo])));
    fine_copy<P>(s, base + src, base + j);
  }
  if (threadIdx.x == 0) {
    s.fcnt[k] = S;
    s.flv[k] = L;
  }
}

// ------------------------------------------------------------------------------------
// Step 2: sorting cell k takes, from the parked leavers of its left and then its right
// neighbour (in their parked order), those now in k, appended after its stayers.
// ------------------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(kFineWG) void k_fine_sort2(const SimDev* __restrict__ simp) {
  const SimDev& sim = *simp;
  const int2 tt = sim.tile_table[blockIdx.x];
  const SpeciesDev s = sim.sp[tt.x];
  if (s.mode != kModeFine) return;
  const int k = tt.y, nt = s.n_tiles;
  const uint32_t base = static_cast<uint32_t>(k) * s.nmax;
  __shared__ uint32_t lds[kFineWG / 64 + 1];
  uint32_t fill = s.fcnt[k];
  const uint32_t my_parked = s.flv[k];
  for (int side = 0; side < 2; ++side) {
    int nb = side == 0 ? k - 1 : k + 1;
    if (s.periodic) nb = (nb + nt) % nt;
    if (nb < 0 || nb >= nt || nb == k) continue;
    if (side == 1 && s.periodic && nt == 2) continue;  // the same neighbour on both sides
    const uint32_t nl = s.flv[nb];
    const uint32_t nbase = static_cast<uint32_t>(nb) * s.nmax + s.nmax - nl;
    for (uint32_t b = 0; b < nl; b += blockDim.x) {
      const uint32_t j = b + threadIdx.x;
      bool mine = false;
      if (j < nl) mine = sort_cell_of(s, fine_cell<P>(s, nbase + j)) == k;
      uint32_t total;
      const uint32_t r = block_exclusive_scan<uint32_t>(mine ? 1u : 0u, lds, total);
      if (mine) {
        const uint32_t dst = fill + r;
        if (dst + my_parked < s.nmax) fine_copy<P>(s, nbase + j, base + dst);
        else atomicOr(sim.error, kErrCapacity);
      }
      fill += total;
    }
  }
  if (threadIdx.x == 0) s.fcnt[k] = min(fill, s.nmax - my_parked);
}

// ------------------------------------------------------------------------------------
// Step 3: sorting cell k sends its parked leavers that moved farther than one sorting cell
// to their sorting cells, taking the slot from that cell's counter (global atomic).
// ------------------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(kFineWG) void k_fine_sort3(const SimDev* __restrict__ simp) {
  const SimDev& sim = *simp;
  const int2 tt = sim.tile_table[blockIdx.x];
  const SpeciesDev s = sim.sp[tt.x];
  if (s.mode != kModeFine) return;
  const int k = tt.y, nt = s.n_tiles;
  const uint32_t nl = s.flv[k];
  const uint32_t pbase = static_cast<uint32_t>(k) * s.nmax + s.nmax - nl;
  for (uint32_t j = threadIdx.x; j < nl; j += blockDim.x) {
    const int c = fine_cell<P>(s, pbase + j);
    const int dk = sort_cell_of(s, c);
    int left = k - 1, right = k + 1;
    if (s.periodic) {
      left = (left + nt) % nt;
      right = right % nt;
    }
    if (dk == left || dk == right || dk < 0 || dk >= nt) continue;
    // the destination's own parked leavers stay untouched until its step 3 has read them
    const uint32_t slot = atomicAdd(&s.fcnt[dk], 1u);
    if (slot + s.flv[dk] < s.nmax) fine_copy<P>(s, pbase + j, static_cast<uint32_t>(dk) * s.nmax + slot);
    else atomicOr(sim.error, kErrCapacity);
  }
}

// ------------------------------------------------------------------------------------
// Births of the step (electron ionisations, staged by k_collide at the parent's slot
// range with the parent's id): birth b takes rank = the number of births whose parent id
// is smaller (parent ids are distinct), id next_id + rank, and a slot at the end of the
// sorting cell of its position (atomic counter), for both species.  One workgroup per
// discharge; births that did not fit the capacity (k_birth_scan) are dropped.
// ------------------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(kSolveWG) void k_fine_births(const SimDev* __restrict__ simp) {
  using real = typename FReal<P>::type;
  const SimDev& sim = *simp;
  const DischargeDev dd = sim.ds[blockIdx.x];
  const SpeciesDev se = sim.sp[dd.spec0];
  if (se.mode != kModeFine) return;
  const int nt = se.n_tiles + se.n_tail;
  const uint32_t B = se.birth_base[nt];
  if (B == 0u) return;
  if (B > kMaxFineBirths) {  // the rank below is quadratic in B
    if (threadIdx.x == 0) atomicOr(sim.error, kErrCapacity);
    return;
  }
  // parent ids in birth order (electron tiles in order, each in its staging order)
  for (uint32_t g = threadIdx.x; g < B; g += blockDim.x) {
    int lo = 0, hi = nt - 1;  // tile u with birth_base[u] <= g < birth_base[u + 1]
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (se.birth_base[mid] <= g) lo = mid;
      else hi = mid - 1;
    }
    const uint32_t si = se.stage_first[lo] + (g - se.birth_base[lo]);
    se.fpid_list[g] = si < se.cap ? se.fpid[si] : 0xFFFFFFFFu;
    se.far_dest[g] = si;  // staging index of birth g (far_dest is free in this mode)
  }
  __syncthreads();
  for (uint32_t g = threadIdx.x; g < B; g += blockDim.x) {
    const uint32_t pid = se.fpid_list[g];
    uint32_t rank = 0u;
    for (uint32_t h = 0; h < B; ++h) rank += se.fpid_list[h] < pid ? 1u : 0u;
    const uint32_t si = se.far_dest[g];
    if (si >= se.cap) continue;
    for (int sp = 0; sp < 2; ++sp) {
      const SpeciesDev s = sim.sp[dd.spec0 + sp];
      const uint32_t fit = s.fin[0], nid = s.fin[1];
      if (rank >= fit) continue;
      void GM* const* src = se.stage[sp];
      int cell;
      real pos;
      if constexpr (std::is_same<P, F32>::value) {
        cell = ldg<int>(src[F32_CELL], si);
        pos = ldg<float>(src[F32_OFF], si);
      } else {
        pos = ldg<double>(src[F64_X], si);
        cell = static_cast<int>(floor(pos));
      }
      const int dk = cell / s.C;
      const uint32_t slot = atomicAdd(&s.fcnt[dk], 1u);
      if (slot >= s.nmax) {
        atomicOr(sim.error, kErrCapacity);
        continue;
      }
      const uint32_t b = static_cast<uint32_t>(dk) * s.nmax + slot;
      if constexpr (std::is_same<P, F32>::value) {
        stg<int>(s.fine[F32_CELL], b, cell);
        stg<float>(s.fine[F32_OFF], b, pos);
        uint4 v = ldg<uint4>(src[F_VX], si);  // the staged birth's velocity record
        v.w = nid + rank;
        stg<uint4>(s.fine[F_VX], b, v);
      } else {
        stg<double>(s.fine[F64_X], b, pos);
        stg<Vel3d>(s.fine[F_VX], b, ldg<Vel3d>(src[F_VX], si));
        stg<uint32_t>(s.fine[F_ID], b, nid + rank);
      }
      // deposit (fixed point, order-free)
      const double fr = std::is_same<P, F32>::value ? static_cast<double>(pos)
                                                     : static_cast<double>(pos) - floor(static_cast<double>(pos));
      const unsigned long long F = fix_weight(fr, s.dep_scale);
      int cn = cell + 1;
      if (s.periodic && cn == s.n_cells) cn = 0;
      atomicAdd(&s.far_w[cell], s.dep_one - F);
      atomicAdd(&s.far_w[cn], F);
    }
  }
}

// ------------------------------------------------------------------------------------
// Set-up: the cell-sorted contiguous buffer `src` into the sorting cells, in order (the
// particles of sorting cell k are the contiguous run of its cells).
// ------------------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(kFineWG) void k_fine_scatter(const SimDev* __restrict__ simp,
                                                          int src) {
  using real = typename FReal<P>::type;
  const SimDev& sim = *simp;
  const int2 tt = sim.tile_table[blockIdx.x];
  const SpeciesDev s = sim.sp[tt.x];
  if (s.mode != kModeFine) return;
  const int k = tt.y, N = s.n_cells;
  const uint32_t GM* cs = s.cell_start + src * (N + 1);
  const uint32_t a = cs[k * s.C], b = cs[min(k * s.C + s.C, N)];
  const uint32_t n = b > a ? b - a : 0u;
  if (n > s.nmax) {
    if (threadIdx.x == 0) atomicOr(sim.error, kErrCapacity);
    return;
  }
  void GM* const* f = s.fld[src];
  const uint32_t base = static_cast<uint32_t>(k) * s.nmax;
  for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) {
    const uint32_t i = a + j, o = base + j;
    if constexpr (std::is_same<P, F32>::value) {
      stg<int>(s.fine[F32_CELL], o, ldg<int>(f[F32_CELL], i));
      stg<float>(s.fine[F32_OFF], o, ldg<float>(f[F32_OFF], i));
      stg<uint4>(s.fine[F_VX], o, ldg<uint4>(f[F_VX], i));  // velocity and id record
    } else {
      stg<double>(s.fine[F64_X], o, ldg<double>(f[F64_X], i));
      stg<Vel3d>(s.fine[F_VX], o, ldg<Vel3d>(f[F_VX], i));
      stg<uint32_t>(s.fine[F_ID], o, ldg<uint32_t>(f[F_ID], i));
    }
  }
  if (threadIdx.x == 0) s.fcnt[k] = n;
}

template <typename K, typename... Args>
void launch_ev(K kernel, dim3 grid, dim3 block, hipStream_t st, hipEvent_t e0, hipEvent_t e1,
               Args... args) {
  if (e0 || e1) hipExtLaunchKernelGGL(kernel, grid, block, 0, st, e0, e1, 0, args...);
  else kernel<<<grid, block, 0, st>>>(args...);
}

}  // namespace

void launch_fine_sort(const LaunchInfo& li, const SimDev* sim, hipStream_t st, hipEvent_t e0,
                      hipEvent_t e1) {
  const dim3 grid(li.total_tiles), block(kFineWG);
  const hipEvent_t none = nullptr;
  if (li.fp32) {
    launch_ev(k_fine_sort1<F32>, grid, block, st, e0, none, sim);
    launch_ev(k_fine_sort2<F32>, grid, block, st, none, none, sim);
    launch_ev(k_fine_sort3<F32>, grid, block, st, none, e1, sim);
  } else {
    launch_ev(k_fine_sort1<F64>, grid, block, st, e0, none, sim);
    launch_ev(k_fine_sort2<F64>, grid, block, st, none, none, sim);
    launch_ev(k_fine_sort3<F64>, grid, block, st, none, e1, sim);
  }
}

void launch_fine_births(const LaunchInfo& li, const SimDev* sim, hipStream_t st) {
  if (li.fp32) k_fine_births<F32><<<li.n_ds, kSolveWG, 0, st>>>(sim);
  else k_fine_births<F64><<<li.n_ds, kSolveWG, 0, st>>>(sim);
}

void launch_fine_scatter(const LaunchInfo& li, const SimDev* sim, int src, hipStream_t st) {
  if (li.fp32) k_fine_scatter<F32><<<li.total_tiles, kFineWG, 0, st>>>(sim, src);
  else k_fine_scatter<F64><<<li.total_tiles, kFineWG, 0, st>>>(sim, src);
}

}  // namespace fspic
