// device_common.h -- device-side building blocks of the PIC-MCC step kernels:
// counter-based draws, the Ar-like cross sections, the leap-frog push of both particle
// layouts, the collision kinematics, tile-window geometry and workgroup scans.
//
// Everything here is evaluated one IEEE operation at a time (the library is built with
// -ffp-contract=off), so the push and the collision decisions come out identical in
// every kernel that calls them.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "sim_layout.h"

namespace fspic {

// ------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64
// multiplications on the 4-word counter, the key advanced by a Weyl sequence between
// rounds.  Stateless, keyed by (seed, 2 * discharge + species), counter (id, step, block,
// tag): any thread can produce any particle's draw, unlike the per-thread xorshift
// state of the paper's Sec. 3.8.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                        uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // one 32x32->64 product per multiplier (a single v_mad_u64_u32)
    const uint64_t pa = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t pb = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    const uint32_t n0 = static_cast<uint32_t>(pb >> 32) ^ c1 ^ k0;
    const uint32_t n2 = static_cast<uint32_t>(pa >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = static_cast<uint32_t>(pb);
    c2 = n2;
    c3 = static_cast<uint32_t>(pa);
  }
  return make_uint4(c0, c1, c2, c3);
}

// uniform in [0, 1) from 53 bits: all of a, the top 21 bits of b
__device__ __forceinline__ double u53(uint32_t a, uint32_t b) {
  const uint64_t m = (static_cast<uint64_t>(a) << 21) | static_cast<uint64_t>(b >> 11);
  return static_cast<double>(m) * (1.0 / 9007199254740992.0);
}

constexpr double kTwoPi = 6.283185307179586476925286766559;

__device__ __forceinline__ void normals64(uint4 b, double& z0, double& z1) {
  const double ua = u53(b.x, b.y);
  const double ub = u53(b.z, b.w);
  const double r = sqrt(-2.0 * log(1.0 - ua));
  const double th = kTwoPi * ub;
  double sn, cs;
  sincos(th, &sn, &cs);  // one argument reduction for both
  z0 = r * cs;
  z1 = r * sn;
}

// isotropic unit vector, first component along the discharge axis
__device__ __forceinline__ void direction64(uint4 b, double& n0, double& n1, double& n2) {
  const double ua = u53(b.x, b.y);
  const double ub = u53(b.z, b.w);
  const double ct = 1.0 - 2.0 * ua;
  const double st = sqrt(1.0 - ct * ct);
  const double ph = kTwoPi * ub;
  double sn, cs;
  sincos(ph, &sn, &cs);
  n0 = ct;
  n1 = st * cs;
  n2 = st * sn;
}

__device__ __forceinline__ void direction32(uint4 b, float& n0, float& n1, float& n2) {
  const double ua = u53(b.x, b.y);
  const double ub = u53(b.z, b.w);
  const float ct = static_cast<float>(1.0 - 2.0 * ua);
  const float st = sqrtf(fmaxf(0.0f, 1.0f - ct * ct));
  const float ph = static_cast<float>(kTwoPi * ub);
  float sn, cs;
  sincosf(ph, &sn, &cs);
  n0 = ct;
  n1 = st * cs;
  n2 = st * sn;
}

// ------------------------------------------------------------------------------------
// Cross sections: synthetic Ar-like model standing in for the paper's analytic argon fits
// (Sec. 3.8): electrons elastic / excitation (11.5 eV) / ionisation (15.8 eV), ions
// isotropic / charge exchange; constant-sigma electron-elastic model; sigma in m^2.
// ------------------------------------------------------------------------------------
enum { XS_NONE = 0, XS_CONST_E_ELASTIC = 1, XS_AR_LIKE = 2 };
constexpr double kExcEv = 11.5;
constexpr double kIonEv = 15.8;

// Each of the model's fractions is evaluated over one common denominator: the same
// functions with one division instead of two or three, which round differently from the
// nested form by a few units in the last place.
//   elastic     3e-19 (x + 0.05) / (1 + x^2), x = eps / 12  =  3.6e-18 (eps + 0.6) / (144 + eps^2)
//   excitation  2e-20 2u / (1 + u^2), u = (eps - 11.5) / 20  =  8e-19 a / (400 + a^2)
//   ionisation  3e-20 2u / (1 + u^2), u = (eps - 15.8) / 60  =  3.6e-18 a / (3600 + a^2)
__device__ __forceinline__ void xsec_electron(int model, double eps, double sc, double& el,
                                              double& ex, double& iz) {
  el = ex = iz = 0.0;
  if (model == XS_CONST_E_ELASTIC) {
    el = sc;
    return;
  }
  if (model != XS_AR_LIKE) return;
  el = 3.6e-18 * (eps + 0.6) / (144.0 + eps * eps);
  if (eps > kExcEv) {
    const double a = eps - kExcEv;
    ex = 8e-19 * a / (400.0 + a * a);
  }
  if (eps > kIonEv) {
    const double a = eps - kIonEv;
    iz = 3.6e-18 * a / (3600.0 + a * a);
  }
}

//   isotropic       2e-19 (1 + 2 / (1 + eps)) / (1 + eps / 100)
//                   =  2e-17 (3 + eps) / ((1 + eps) (100 + eps))
//   charge exchange 3e-19 (1 + 1 / (1 + eps)) / (1 + eps / 1000)
//                   =  3e-16 (2 + eps) / ((1 + eps) (1000 + eps))
__device__ __forceinline__ void xsec_ion(int model, double eps, double& is, double& cx) {
  is = cx = 0.0;
  if (model != XS_AR_LIKE) return;
  const double e1 = 1.0 + eps;
  is = 2e-17 * (3.0 + eps) / (e1 * (100.0 + eps));
  cx = 3e-16 * (2.0 + eps) / (e1 * (1000.0 + eps));
}

// ------------------------------------------------------------------------------------
// Leap-frog push with linear gather (Sec. 3.6) and the wall test (Sec. 2):
// status 0 kept, 1 left the box at x < 0, 2 at x >= N, 3 not a finite position.
// ------------------------------------------------------------------------------------
// FP32 cell + offset: the update is made on the offset so its resolution does not
// depend on the cell index.
__device__ __forceinline__ int push32(int c, float f, float vx, float e0, float e1, float kf,
                                      int N, int periodic, int& d, float& fo, float& vo) {
  const float t = 1.0f - f;
  const float a = t * e0;
  const float b = f * e1;
  const float ep = a + b;
  const float dv = kf * ep;
  const float v = vx + dv;
  float fn = f + v;
  const float kfl = floorf(fn);
  vo = v;
  if (!(fabsf(kfl) < 1.0e9f)) {
    d = 0;
    fo = 0.0f;
    return 3;
  }
  int dd = c + static_cast<int>(kfl);
  fn = fn - kfl;
  if (fn >= 1.0f) {
    fn = 0.0f;
    dd += 1;
  }
  fo = fn;
  if (periodic) {
    dd %= N;
    if (dd < 0) dd += N;
    d = dd;
    return 0;
  }
  d = dd;
  if (dd < 0) return 1;
  if (dd >= N) return 2;
  return 0;
}

// FP64 absolute position.
__device__ __forceinline__ int push64(double x, double vx, double e0, double e1, double kappa,
                                      int N, int periodic, double& xo, double& vo, int& d) {
  const double c = floor(x);
  const double f = x - c;
  const double ep = (1.0 - f) * e0 + f * e1;
  const double v = vx + kappa * ep;
  double xn = x + v;
  vo = v;
  const double dn = static_cast<double>(N);
  if (!(fabs(xn) < 1.0e15)) {
    xo = 0.0;
    d = 0;
    return 3;
  }
  if (periodic) {
    if (xn < 0.0 || xn >= dn) {
      const double k = floor(xn / dn);
      xn = xn - k * dn;
      for (int it = 0; it < 4 && xn < 0.0; ++it) xn += dn;
      for (int it = 0; it < 4 && xn >= dn; ++it) xn -= dn;
    }
    xo = xn;
    int dd = static_cast<int>(floor(xn));
    if (dd >= N) dd = N - 1;
    if (dd < 0) dd = 0;
    d = dd;
    return 0;
  }
  xo = xn;
  if (xn < 0.0) {
    d = -1;
    return 1;
  }
  if (xn >= dn) {
    d = N;
    return 2;
  }
  d = static_cast<int>(floor(xn));
  return 0;
}

// ------------------------------------------------------------------------------------
// Electrode processes (Sec. 2: electrons inserted at the boundaries when secondary
// emission or reflection is featured).  A reflected electron is mirrored in the wall it
// crossed (x -> -x or 2N - x, v_x -> -v_x); st is its wall status (1: x < 0, 2: x >= N).
// Returns whether the mirrored position is inside the box.
// ------------------------------------------------------------------------------------
// FP32 cell + offset: cell c, offset f -> cell -c - 1 (or 2N - c - 1), offset 1 - f.
__device__ __forceinline__ bool mirror32(int N, int st, int& d, float& f) {
  int cn = st == 1 ? -d - 1 : 2 * N - d - 1;
  float fn = 1.0f - f;
  if (fn >= 1.0f) {
    fn = 0.0f;
    cn += 1;
  }
  d = cn;
  f = fn;
  return cn >= 0 && cn < N;
}

__device__ __forceinline__ bool mirror64(int N, int st, double& x, int& d) {
  const double dn = static_cast<double>(N);
  x = st == 1 ? -x : 2.0 * dn - x;
  if (!(x >= 0.0 && x < dn)) return false;
  d = static_cast<int>(floor(x));
  return true;
}

// Secondary electron of an ion absorbed at wall st (1: x = 0, 2: x = N), from the ion's
// Philox blocks 7 and 8 (block 6 word 0 decided the emission): normal speed Rayleigh-
// distributed with scale vth (the flux of a Maxwellian through the wall), tangential
// components normal, starting a uniform fraction of its first step's flight from the wall.
// Returns whether the start position is inside the box.
__device__ __forceinline__ bool emitted_electron(int N, int st, double vth, uint4 b7, uint4 b8,
                                                 double& x, double v[3]) {
  const double ua = u53(b7.x, b7.y);
  const double uf = u53(b7.z, b7.w);
  const double vn = vth * sqrt(-2.0 * log(1.0 - ua));
  double z0, z1;
  normals64(b8, z0, z1);
  const double dn = static_cast<double>(N);
  if (st == 1) {
    v[0] = vn;
    x = uf * vn;
  } else {
    v[0] = -vn;
    x = dn - uf * vn;
  }
  v[1] = vth * z0;
  v[2] = vth * z1;
  return x >= 0.0 && x < dn;
}

// ------------------------------------------------------------------------------------
// Tile-window geometry.  Cell tile t of a species owns cells [tC, tC + C); its window
// starts at cell tC - D.  A histogram window spans W = C + 2D cells, a deposit window
// W + 1 nodes.  for_covering visits, in increasing tile index, every tile whose window
// (of `span` slots) contains cell / node j, with j's slot in that window.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ int floordiv(int a, int b) {
  return a >= 0 ? a / b : -((-a + b - 1) / b);
}

template <class F>
__device__ __forceinline__ void for_covering(const SpeciesDev& s, int j, int span, F&& f) {
  const int C = s.C, D = s.D, n = s.n_tiles, N = s.n_cells;
  const int thi = floordiv(j + D, C);
  const int tlo = floordiv(j + D - span, C) + 1;
  if (!s.periodic) {
    const int a = tlo < 0 ? 0 : tlo;
    const int b = thi > n - 1 ? n - 1 : thi;
    for (int t = a; t <= b; ++t) f(t, j - t * C + D);
    return;
  }
  auto slot = [&](int t) {
    int k = (j - t * C + D) % N;
    return k < 0 ? k + N : k;
  };
  if (tlo < 0) {
    for (int t = 0; t <= thi; ++t) f(t, slot(t));
    for (int t = tlo + n; t <= n - 1; ++t) f(t, slot(t));
  } else if (thi > n - 1) {
    for (int t = 0; t <= thi - n; ++t) f(t, slot(t));
    for (int t = tlo; t <= n - 1; ++t) f(t, slot(t));
  } else {
    for (int t = tlo; t <= thi; ++t) f(t, slot(t));
  }
}

// The tiles of for_covering as (at most) two index ranges [a0, b0], [a1, b1], visited in
// that order (an empty range has b < a), and the slot of cell / node j in tile t's window.
__device__ __forceinline__ void covering_ranges(const SpeciesDev& s, int j, int span, int a[2],
                                                int b[2]) {
  const int C = s.C, D = s.D, n = s.n_tiles;
  const int thi = floordiv(j + D, C);
  const int tlo = floordiv(j + D - span, C) + 1;
  a[1] = 0;
  b[1] = -1;
  if (!s.periodic) {
    a[0] = tlo < 0 ? 0 : tlo;
    b[0] = thi > n - 1 ? n - 1 : thi;
  } else if (tlo < 0) {
    a[0] = 0;
    b[0] = thi;
    a[1] = tlo + n;
    b[1] = n - 1;
  } else if (thi > n - 1) {
    a[0] = 0;
    b[0] = thi - n;
    a[1] = tlo;
    b[1] = n - 1;
  } else {
    a[0] = tlo;
    b[0] = thi;
  }
}

__device__ __forceinline__ int covering_slot(const SpeciesDev& s, int j, int t) {
  int k = j - t * s.C + s.D;
  if (s.periodic) {
    k %= s.n_cells;
    if (k < 0) k += s.n_cells;
  }
  return k;
}

// slot of cell d in the window of tile t, or -1 if outside [0, W)
__device__ __forceinline__ int window_slot(const SpeciesDev& s, int t, int d) {
  int k = d - (t * s.C - s.D);
  if (s.periodic) {
    k %= s.n_cells;
    if (k < 0) k += s.n_cells;
  }
  return (k >= 0 && k < s.W) ? k : -1;
}

// ------------------------------------------------------------------------------------
// Wave-level helpers.
// ------------------------------------------------------------------------------------
// Element i of a global array, addressed by a 32-bit byte offset from the array's base.
// Every array of the library is smaller than 4 GiB (the capacities are checked on the
// host), and in this form the base stays in scalar registers and the memory instruction
// takes the 32-bit offset (no 64-bit address arithmetic per access).
template <class T>
__device__ __forceinline__ T ldg(const void GM* base, uint32_t i) {
  return *reinterpret_cast<const T GM*>(reinterpret_cast<const char GM*>(base) +
                                        i * static_cast<uint32_t>(sizeof(T)));
}

template <class T>
__device__ __forceinline__ void stg(void GM* base, uint32_t i, T v) {
  *reinterpret_cast<T GM*>(reinterpret_cast<char GM*>(base) + i * static_cast<uint32_t>(sizeof(T))) = v;
}

// A velocity written or copied as one record (FP32: the first 12 bytes of the 16-byte
// record; FP64: the whole 24-byte record).
struct alignas(4) Vel3 {
  float x, y, z;
};
struct alignas(8) Vel3d {
  double x, y, z;
};

// Index of this thread's wave in the workgroup, as a wave-uniform (scalar) value.
__device__ __forceinline__ int wave_id() {
  return __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) >> 6);
}

__device__ __forceinline__ unsigned long long lanes_below() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ unsigned long long lanes_above() {
  const int lane = threadIdx.x & 63;
  return lane == 63 ? 0ull : (~0ull << (lane + 1));
}

// Mask of the active lanes whose key equals this lane's key (keys < 2^nbits); valid for
// active lanes.  One ballot per key bit, so the cost does not depend on how many lanes
// share a key.
__device__ __forceinline__ unsigned long long match_key(int key, bool act, int nbits) {
  unsigned long long m = __ballot(act);
  for (int b = 0; b < nbits; ++b) {
    const bool bit = act && ((key >> b) & 1);
    const unsigned long long mb = __ballot(bit);
    m &= bit ? mb : ~mb;
  }
  return m;
}

// The same mask, one pass per distinct key among the active lanes: cheaper when a wave's
// keys take few values (a chunk of 64 cell-sorted particles lands in a few window slots).
__device__ __forceinline__ unsigned long long match_key_few(int key, bool act) {
  unsigned long long todo = __ballot(act);
  unsigned long long mine = 0ull;
  while (todo) {  // wave-uniform
    const int first = __ffsll(static_cast<long long>(todo)) - 1;
    const int k0 = __builtin_amdgcn_readlane(key, first);
    // lanes holding k0 (one compare into a scalar mask), restricted to the active ones
    const unsigned long long m =
        __builtin_amdgcn_uicmp(static_cast<unsigned>(key), static_cast<unsigned>(k0), 32) &
        todo;
    if (act && key == k0) mine = m;
    todo &= ~m;
  }
  return mine;
}

template <class T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = x + __shfl_xor(x, o, 64);
  return x;
}

// ------------------------------------------------------------------------------------
// Fixed-point charge weights.  A particle at in-cell offset f adds 1 - f to the node on
// its left and f to the node on its right (Sec. 3.4).  The library adds them as the
// integers one - F and F with F = round(f 2^shift): integer sums are exact whatever the
// order of the additions, so the node weights come out bit for bit the same however the
// work is scheduled.  shift leaves room for the species' whole capacity in 64 bits.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long fix_weight(double f, double scale) {
  // f * scale < 2^53: the product is exact and rint gives the nearest integer
  return static_cast<unsigned long long>(rint(f * scale));
}

// ------------------------------------------------------------------------------------
// Workgroup scans (fixed summation order, so results do not depend on scheduling).
// ------------------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const T y = __shfl_up(x, o, 64);
    if (lane >= o) x = x + y;
  }
  return x;
}

// Exclusive scan of one value per thread over the workgroup; `lds` holds blockDim/64+1
// entries.  Returns the exclusive prefix, writes the total.
template <class T>
__device__ __forceinline__ T block_exclusive_scan(T v, T* lds, T& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const T inc = wave_inclusive_scan(v);
  if (lane == 63) lds[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T r = T(0);
    for (int i = 0; i < nw; ++i) {
      const T t = lds[i];
      lds[i] = r;
      r = r + t;
    }
    lds[nw] = r;
  }
  __syncthreads();
  const T ex = lds[w] + (inc - v);
  total = lds[nw];
  __syncthreads();
  return ex;
}

// Sum of one value per thread over the workgroup in a fixed order (a butterfly inside
// each wave, then the waves in order); `lds` holds blockDim/64 entries.  Every thread
// gets the total.
template <class T>
__device__ __forceinline__ T block_sum_fixed(T v, T* lds) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  if (lane == 0) lds[w] = v;
  __syncthreads();
  T r = T(0);
  for (int i = 0; i < nw; ++i) r = r + lds[i];
  __syncthreads();
  return r;
}

// Exclusive scan of src[0..n) into dst[0..n) by one workgroup (dst may be src: in place);
// returns the total.  Thread t takes the contiguous part [t per, (t + 1) per); parts of
// up to kScanPer elements are read into registers at once, so that their loads are in
// flight together.  The caller orders any earlier writes of src with a barrier; the
// barrier at the end makes the workgroup's own stores visible to it (its waves share one
// CU; no device-scope fence, which on this GPU writes back the whole L2).
constexpr int kScanPer = 16;
template <class T, class Ptr>
__device__ T array_exclusive_scan_to(Ptr src, Ptr dst, int n, T* lds) {
  const int per = (n + blockDim.x - 1) / blockDim.x;
  const int lo = threadIdx.x * per;
  const int hi = lo + per < n ? lo + per : n;
  T sum = T(0);
  T total;
  if (per <= kScanPer) {
    T v[kScanPer];
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      v[k] = T(0);
      if (lo + k < hi) v[k] = src[lo + k];
    }
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) sum = sum + v[k];
    T run = block_exclusive_scan(sum, lds, total);
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      if (lo + k < hi) dst[lo + k] = run;
      run = run + v[k];
    }
  } else {
    for (int i = lo; i < hi; ++i) sum = sum + src[i];
    T run = block_exclusive_scan(sum, lds, total);
    for (int i = lo; i < hi; ++i) {
      const T v = src[i];
      dst[i] = run;
      run = run + v;
    }
  }
  __syncthreads();
  return total;
}

// In-place exclusive scan of a[0..n) by one workgroup; returns the total (a barrier first
// orders the workgroup's earlier writes of a).
template <class T, class Ptr>
__device__ T array_exclusive_scan(Ptr a, int n, T* lds) {
  __syncthreads();
  return array_exclusive_scan_to<T>(a, a, n, lds);
}

}  // namespace fspic
