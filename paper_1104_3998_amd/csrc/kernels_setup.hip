// kernels_setup.hip -- kernels that build a state rather than advance it: the initial
// load, the general stable counting sort by cell (used once at load time and for states
// handed in unsorted), the charge deposit of a sorted state and the half-step back-push
// that starts the leap-frog (Sec. 3.6).
#include <algorithm>
#include <type_traits>

#include "device_common.h"
#include "host_common.h"

namespace fspic {

struct S32 {};
struct S64 {};

template <class P>
struct Rec;
template <>
struct Rec<S32> {
  using real = float;
  static constexpr int n_fields = 6;
};
template <>
struct Rec<S64> {
  using real = double;
};

__device__ __forceinline__ int cell_of32(void GM* const* f, uint32_t i) {
  return static_cast<const int GM*>(f[F32_CELL])[i];
}
__device__ __forceinline__ int cell_of64(void GM* const* f, uint32_t i) {
  return static_cast<int>(floor(static_cast<const double GM*>(f[F64_X])[i]));
}

template <class P>
__device__ __forceinline__ int cell_of(void GM* const* f, uint32_t i) {
  if constexpr (std::is_same<P, S32>::value) return cell_of32(f, i);
  else return cell_of64(f, i);
}

template <class P>
__device__ __forceinline__ void copy_record(void GM* const* src, uint32_t i, void GM* const* dst,
                                            uint32_t j) {
  if constexpr (std::is_same<P, S32>::value) {
    static_cast<int GM*>(dst[F32_CELL])[j] = static_cast<const int GM*>(src[F32_CELL])[i];
    static_cast<float GM*>(dst[F32_OFF])[j] = static_cast<const float GM*>(src[F32_OFF])[i];
    // velocity and id: one 16-byte record
    static_cast<uint4 GM*>(dst[F_VX])[j] = static_cast<const uint4 GM*>(src[F_VX])[i];
  } else {
    static_cast<double GM*>(dst[F64_X])[j] = static_cast<const double GM*>(src[F64_X])[i];
    static_cast<Vel3d GM*>(dst[F_VX])[j] = static_cast<const Vel3d GM*>(src[F_VX])[i];
    static_cast<uint32_t GM*>(dst[F_ID])[j] = static_cast<const uint32_t GM*>(src[F_ID])[i];
  }
}

// ------------------------------------------------------------------------------------
// Initial load (tag 1, step word 0), particle i gets id i.  Random: x = U53 N from block
// 0, Maxwellian velocities (thermal speed sqrt(kT/m)) from blocks 1-2 by Box-Muller.
// Quiet start: x_k = (k + 1/2) N / N_s, electrons displaced by A sin(2 pi m x / N), cold.
// The FP32 layout keeps cell = floor(x) and the offset x - cell rounded toward zero.
// ------------------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(256) void k_load(const SimDev* __restrict__ simp, int dst) {
  const SimDev& sim = *simp;
  const SpeciesDev s = sim.sp[blockIdx.y];
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s.n_init) return;
  const int N = s.n_cells;
  const double dn = static_cast<double>(N);
  double x, v[3] = {0.0, 0.0, 0.0};
  if (s.load_kind == 0) {
    const uint4 b0 = philox(i, 0u, 0u, 1u, s.key0, s.key1);
    const uint4 b1 = philox(i, 0u, 1u, 1u, s.key0, s.key1);
    const uint4 b2 = philox(i, 0u, 2u, 1u, s.key0, s.key1);
    x = u53(b0.x, b0.y) * dn;
    double z0, z1, z2, z3;
    normals64(b1, z0, z1);
    normals64(b2, z2, z3);
    v[0] = s.vth * z0;
    v[1] = s.vth * z1;
    v[2] = s.vth * z2;
  } else {
    x = (static_cast<double>(i) + 0.5) * dn / static_cast<double>(s.n_init);
    if (s.sp == 0) {
      x = x + s.lang_amp * sin(kTwoPi * static_cast<double>(s.lang_mode) * x / dn);
      for (int it = 0; it < 4 && x < 0.0; ++it) x += dn;
      for (int it = 0; it < 4 && x >= dn; ++it) x -= dn;
    }
  }
  void GM* const* f = s.fld[dst];
  if constexpr (std::is_same<P, S32>::value) {
    const double c = floor(x);
    static_cast<int GM*>(f[F32_CELL])[i] = static_cast<int>(c);
    static_cast<float GM*>(f[F32_OFF])[i] = __double2float_rz(x - c);
    static_cast<uint4 GM*>(f[F_VX])[i] =
        make_uint4(__float_as_uint(static_cast<float>(v[0])), __float_as_uint(static_cast<float>(v[1])),
                   __float_as_uint(static_cast<float>(v[2])), i);
  } else {
    static_cast<double GM*>(f[F64_X])[i] = x;
    static_cast<Vel3d GM*>(f[F_VX])[i] = Vel3d{v[0], v[1], v[2]};
    static_cast<uint32_t GM*>(f[F_ID])[i] = i;
  }
}

// ------------------------------------------------------------------------------------
// General stable counting sort by cell of buffer `src` into `dst` (n = n_total[src]).
// Tiles of consecutive particles are taken by single-wave workgroups: (1) LDS histogram
// of the whole cell range per tile, (2) per cell an exclusive scan over tiles plus an
// exclusive scan over cells, (3) each wave scatters its tile 64 particles at a time,
// ranking equal cells by lane order, so the order inside a cell is the input order.
// ------------------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(64) void k_gsort_hist(const SimDev* __restrict__ simp, int src,
                                                   int n_gtiles) {
  extern __shared__ uint32_t hist[];
  const SimDev& sim = *simp;
  const SpeciesDev s = sim.sp[blockIdx.y];
  const int N = s.n_cells;
  const uint32_t n = s.n_total[src];
  const uint32_t per = (n + n_gtiles - 1) / n_gtiles;
  const uint32_t lo = min(n, blockIdx.x * per), hi = min(n, lo + per);
  for (int c = threadIdx.x; c < N; c += blockDim.x) hist[c] = 0u;
  __syncthreads();
  void GM* const* f = s.fld[src];
  for (uint32_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    int c = cell_of<P>(f, i);
    c = c < 0 ? 0 : (c >= N ? N - 1 : c);
    atomicAdd(&hist[c], 1u);
  }
  __syncthreads();
  uint32_t* gh = s.gsort_hist + static_cast<size_t>(blockIdx.x) * N;
  for (int c = threadIdx.x; c < N; c += blockDim.x) gh[c] = hist[c];
}

__global__ __launch_bounds__(kSolveWG) void k_gsort_scan(const SimDev* __restrict__ simp,
                                                         int src, int dst, int n_gtiles) {
  const SimDev& sim = *simp;
  const SpeciesDev s = sim.sp[blockIdx.x];
  __shared__ uint32_t lds[kSolveWG / 64 + 1];
  const int N = s.n_cells;
  const uint32_t n = s.n_total[src];
  for (int c = threadIdx.x; c < N; c += blockDim.x) {
    uint32_t run = 0;
    for (int g = 0; g < n_gtiles; ++g) {
      uint32_t* e = s.gsort_hist + static_cast<size_t>(g) * N + c;
      const uint32_t v = *e;
      *e = run;
      run += v;
    }
    s.base[c] = run;
  }
  array_exclusive_scan(s.base, N, lds);
  uint32_t* cs = s.cell_start + dst * (N + 1);
  for (int c = threadIdx.x; c < N; c += blockDim.x) cs[c] = s.base[c];
  if (threadIdx.x == 0) {
    cs[N] = n;
    s.n_total[dst] = n;
    s.n_sorted[dst] = n;
  }
}

template <class P>
__global__ __launch_bounds__(64) void k_gsort_scatter(const SimDev* __restrict__ simp, int src,
                                                      int dst, int n_gtiles) {
  extern __shared__ uint32_t run[];
  const SimDev& sim = *simp;
  const SpeciesDev s = sim.sp[blockIdx.y];
  const int N = s.n_cells;
  const uint32_t n = s.n_total[src];
  const uint32_t per = (n + n_gtiles - 1) / n_gtiles;
  const uint32_t lo = min(n, blockIdx.x * per), hi = min(n, lo + per);
  const uint32_t* gh = s.gsort_hist + static_cast<size_t>(blockIdx.x) * N;
  for (int c = threadIdx.x; c < N; c += blockDim.x) run[c] = s.base[c] + gh[c];
  __syncthreads();
  const int lane = threadIdx.x;
  const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  void GM* const* fs = s.fld[src];
  void GM* const* fd = s.fld[dst];
  for (uint32_t b = lo; b < hi; b += 64) {
    const uint32_t i = b + lane;
    bool active = i < hi;
    int key = 0;
    if (active) {
      key = cell_of<P>(fs, i);
      key = key < 0 ? 0 : (key >= N ? N - 1 : key);
    }
    uint32_t pos = 0;
    unsigned long long act = __ballot(active);
    while (act) {
      const int leader = __ffsll(static_cast<long long>(act)) - 1;
      const int lk = __shfl(key, leader, 64);
      const bool mine = active && key == lk;
      const unsigned long long mm = __ballot(mine);
      if (mine) {
        pos = run[lk] + static_cast<uint32_t>(__popcll(mm & lt));
        active = false;
      }
      __builtin_amdgcn_wave_barrier();
      if (lane == leader) run[lk] += static_cast<uint32_t>(__popcll(mm));
      __builtin_amdgcn_wave_barrier();
      act = __ballot(active);
    }
    if (i < hi && pos < s.cap) copy_record<P>(fs, i, fd, pos);
  }
}

// cell_start of buffer `buf` from its sorted prefix (state handed in by the caller)
template <class P>
__global__ __launch_bounds__(256) void k_cell_start(const SimDev* __restrict__ simp, int spec,
                                                    int buf) {
  const SimDev& sim = *simp;
  const SpeciesDev s = sim.sp[spec];
  const int N = s.n_cells;
  const uint32_t ns = s.n_sorted[buf];
  uint32_t* cs = s.cell_start + buf * (N + 1);
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  void GM* const* f = s.fld[buf];
  if (ns == 0) {
    for (int c = i; c <= N; c += gridDim.x * blockDim.x) cs[c] = 0u;
    return;
  }
  if (i >= ns) return;
  const int ci = cell_of<P>(f, i);
  const int cp = i > 0 ? cell_of<P>(f, i - 1) : -1;
  for (int c = cp + 1; c <= ci; ++c) cs[c] = i;
  if (i == ns - 1)
    for (int c = ci + 1; c <= N; ++c) cs[c] = ns;
}

// ------------------------------------------------------------------------------------
// Charge deposit of an unmoved sorted state into the tile windows (plus the tail into
// the far array), in the layout k_combine reads.  ds_filter >= 0 limits it to one
// discharge.
// ------------------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(256) void k_deposit_tiles(const SimDev* __restrict__ simp,
                                                       int ds_filter) {
  const SimDev& sim = *simp;
  const int2 tt = sim.tile_table[blockIdx.x];
  const SpeciesDev s = sim.sp[tt.x];
  if (ds_filter >= 0 && s.ds != ds_filter) return;
  const int p = static_cast<int>(*sim.step & 1ull);
  const int t = tt.y;
  const int N = s.n_cells, W = s.W;
  // fixed-point node weights of the window (integer atomics: exact in any order)
  __shared__ unsigned long long dep[kMaxWindow + 1];
  uint32_t lo, hi;
  const bool tail = (t >= s.n_tiles || s.mode == kModeNone) && s.mode != kModeFine;
  void GM* const* f = s.mode == kModeFine ? s.fine : s.fld[p];
  if (s.mode == kModeFine) {
    lo = static_cast<uint32_t>(t) * s.nmax;
    hi = lo + min(s.fcnt[t], s.nmax);
  } else if (s.mode == kModeNone) {
    const uint32_t nt = s.n_total[p];
    const uint32_t per = (nt + s.n_tiles - 1) / s.n_tiles;
    lo = min(nt, static_cast<uint32_t>(t) * per);
    hi = min(nt, lo + per);
  } else if (!tail) {
    const uint32_t* cs = s.cell_start + p * (N + 1);
    lo = cs[t * s.C];
    hi = cs[min(t * s.C + s.C, N)];
  } else {
    const uint32_t ns = s.n_sorted[p], nt = s.n_total[p];
    const uint32_t ntail = nt > ns ? nt - ns : 0u;
    const uint32_t per = (ntail + s.n_tail - 1) / s.n_tail;
    lo = min(nt, ns + static_cast<uint32_t>(t - s.n_tiles) * per);
    hi = min(nt, lo + per);
  }
  for (int k = threadIdx.x; k <= W; k += blockDim.x) dep[k] = 0ull;
  __syncthreads();
  for (uint32_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    int c;
    double fr;
    if constexpr (std::is_same<P, S32>::value) {
      c = static_cast<const int GM*>(f[F32_CELL])[i];
      fr = static_cast<double>(static_cast<const float GM*>(f[F32_OFF])[i]);
    } else {
      const double x = static_cast<const double GM*>(f[F64_X])[i];
      const double cc = floor(x);
      c = static_cast<int>(cc);
      fr = x - cc;
    }
    if (c < 0 || c >= N) continue;
    const unsigned long long F = fix_weight(fr, s.dep_scale);
    const int k = tail ? -1 : window_slot(s, t, c);
    if (k >= 0) {
      atomicAdd(&dep[k], s.dep_one - F);
      atomicAdd(&dep[k + 1], F);
    } else {
      int cn = c + 1;
      if (s.periodic && cn == N) cn = 0;
      atomicAdd(&s.far_w[c], s.dep_one - F);
      atomicAdd(&s.far_w[cn], F);
    }
  }
  __syncthreads();
  if (!tail) {
    unsigned long long GM* part = s.partial + static_cast<size_t>(t) * (W + 1);
    for (int k = threadIdx.x; k <= W; k += blockDim.x) part[k] = dep[k];
  }
}

// Leap-frog start (Sec. 3.6): v_x(-1/2) = v_x(0) - kappa E(x_0) / 2.
template <class P>
__global__ __launch_bounds__(256) void k_halfstep(const SimDev* __restrict__ simp) {
  const SimDev& sim = *simp;
  const SpeciesDev s = sim.sp[blockIdx.y];
  const DischargeDev dd = sim.ds[s.ds];
  const int p = static_cast<int>(*sim.step & 1ull);
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  void GM* const* f = s.fld[p];
  if (s.mode == kModeFine) {  // slot i of sorting cell i / nmax
    if (i >= s.cap || (i % s.nmax) >= s.fcnt[i / s.nmax]) return;
    f = s.fine;
  } else if (i >= s.n_total[p]) {
    return;
  }
  const int N = s.n_cells;
  if constexpr (std::is_same<P, S32>::value) {
    const int c = static_cast<const int GM*>(f[F32_CELL])[i];
    if (c < 0 || c >= N) return;
    const int cn = (s.periodic && c + 1 == N) ? 0 : c + 1;
    const float fr = static_cast<const float GM*>(f[F32_OFF])[i];
    const float t = 1.0f - fr;
    const float a = t * dd.E32[c];
    const float b = fr * dd.E32[cn];
    const float ep = a + b;
    const float hk = 0.5f * s.kappa_f;
    const float dv = hk * ep;
    float* vx = static_cast<float GM*>(f[F_VX]);  // velocity records: 4 floats each
    vx[4 * static_cast<size_t>(i)] = vx[4 * static_cast<size_t>(i)] - dv;
  } else {
    const double x = static_cast<const double GM*>(f[F64_X])[i];
    if (!(x >= 0.0 && x < static_cast<double>(N))) return;
    const double cc = floor(x);
    const int c = static_cast<int>(cc);
    const int cn = (s.periodic && c + 1 == N) ? 0 : c + 1;
    const double fr = x - cc;
    const double ep = (1.0 - fr) * dd.E64[c] + fr * dd.E64[cn];
    double* vx = static_cast<double GM*>(f[F_VX]);  // velocity records: 3 doubles each
    vx[3 * static_cast<size_t>(i)] = vx[3 * static_cast<size_t>(i)] - 0.5 * s.kappa * ep;
  }
}

// Zero fill of n 8-byte words (a kernel rather than a memset node, so that the same code
// stays correct if a caller records it into a HIP graph).
__global__ __launch_bounds__(256) void k_zero(unsigned long long* p, size_t n) {
  for (size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<size_t>(gridDim.x) * blockDim.x)
    p[i] = 0ull;
}

// ------------------------------------------------------------------------------------
// host launchers
// ------------------------------------------------------------------------------------
void launch_zero(void* p, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 8;
  if (n == 0) return;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 4096);
  k_zero<<<static_cast<unsigned>(blocks), 256, 0, st>>>(static_cast<unsigned long long*>(p), n);
}

void launch_load(const LaunchInfo& li, const SimDev* sim, int dst_buf, hipStream_t st) {
  dim3 grid((li.max_cap + 255) / 256, li.n_spec);
  if (li.fp32) k_load<S32><<<grid, 256, 0, st>>>(sim, dst_buf);
  else k_load<S64><<<grid, 256, 0, st>>>(sim, dst_buf);
}

void launch_general_sort(const LaunchInfo& li, const SimDev* sim, int src_buf, int dst_buf,
                         hipStream_t st) {
  dim3 grid(li.n_gtiles, li.n_spec);
  const size_t lds = static_cast<size_t>(li.max_cells) * sizeof(uint32_t);
  if (li.fp32) k_gsort_hist<S32><<<grid, 64, lds, st>>>(sim, src_buf, li.n_gtiles);
  else k_gsort_hist<S64><<<grid, 64, lds, st>>>(sim, src_buf, li.n_gtiles);
  k_gsort_scan<<<li.n_spec, kSolveWG, 0, st>>>(sim, src_buf, dst_buf, li.n_gtiles);
  if (li.fp32) k_gsort_scatter<S32><<<grid, 64, lds, st>>>(sim, src_buf, dst_buf, li.n_gtiles);
  else k_gsort_scatter<S64><<<grid, 64, lds, st>>>(sim, src_buf, dst_buf, li.n_gtiles);
}

void launch_cell_start(const LaunchInfo& li, const SimDev* sim, int spec, int buf,
                       hipStream_t st) {
  const int blocks = (li.max_cap + 255) / 256 + 1;
  if (li.fp32) k_cell_start<S32><<<blocks, 256, 0, st>>>(sim, spec, buf);
  else k_cell_start<S64><<<blocks, 256, 0, st>>>(sim, spec, buf);
}

void launch_deposit_tiles(const LaunchInfo& li, const SimDev* sim, int ds_filter,
                          hipStream_t st) {
  if (li.fp32) k_deposit_tiles<S32><<<li.total_tiles, 256, 0, st>>>(sim, ds_filter);
  else k_deposit_tiles<S64><<<li.total_tiles, 256, 0, st>>>(sim, ds_filter);
}

void launch_halfstep(const LaunchInfo& li, const SimDev* sim, hipStream_t st) {
  dim3 grid((li.max_cap + 255) / 256, li.n_spec);
  if (li.fp32) k_halfstep<S32><<<grid, 256, 0, st>>>(sim);
  else k_halfstep<S64><<<grid, 256, 0, st>>>(sim);
}

}  // namespace fspic
