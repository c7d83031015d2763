// kernels_step.hip -- the kernels of one PIC-MCC step (Sec. 2 cycle), in launch order:
//
//   k_combine   node weights w_s = sum of the tile deposit windows + far/birth deposits
//   k_solve     Poisson + field on the nodes (Sec. 3.5), one workgroup per discharge
//   k_hist      per-tile LDS histogram of the post-push cells (sort pre-pass, Sec. 3.7)
//   k_scan_cells / k_scan_base
//               per-(tile, cell) output offsets; far movers ranked
//   k_main      push + gather (Sec. 3.6), walls (Sec. 2), stable scatter into the sorted
//               output, LDS deposit (Sec. 3.4), null-collision candidate test
//   k_collide   MCC of the candidates (Sec. 3.8), births staged in parent order
//   k_finalize  births appended in parent order, counters, step advance
//
// A tile is the set of particles of C consecutive cells (the paper puts one sorting cell
// per thread block, Sec. 3.2); the output of a tile's particles can only land within D
// cells of its cells except for rare far movers, so the stable counting sort needs
// only a (C + 2D)-slot histogram per tile.  Charge is deposited as fixed-point integers
// (device_common.h, fix_weight): the bulk into per-tile LDS windows, far movers, tail
// particles and births (a small fraction) into a per-node array with integer atomics, so
// every node weight is an exact, order-independent sum.
#include <hip/hip_ext.h>

#include <type_traits>

#include "device_common.h"
#include "host_common.h"

namespace fspic {

struct P32 {};
struct P64 {};

// One particle array (or staging set) as the kernels address it: the field pointers of
// buffer 0 (in scalar registers for the whole particle loop) and the byte distance to the
// array wanted, so that the two buffers of a field share one base pointer and differ only
// in a 32-bit offset (boff4 for 4-byte fields, boff8 for 8-byte ones, boffv for the
// FP32 velocity records).
struct RecPtr {
  void GM* f[6];
  uint32_t boff4, boff8, boffv;
};

// buffer b of the species' particle arrays (a fine-sorted species has one set of arrays,
// sorted in place)
__device__ __forceinline__ RecPtr rec_buf(const SpeciesDev CM* s, int b) {
  RecPtr r;
  if (s->mode == kModeFine) {
#pragma unroll
    for (int k = 0; k < 6; ++k) r.f[k] = s->fine[k];
    r.boff4 = r.boff8 = r.boffv = 0u;
    return r;
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) r.f[k] = s->fld[0][k];
  r.boff4 = b ? s->bstride4 : 0u;
  r.boff8 = b ? s->bstride8 : 0u;
  r.boffv = b ? s->bstridev : 0u;
  return r;
}

// a birth staging set (its own pointers)
__device__ __forceinline__ RecPtr rec_stage(const SpeciesDev CM* s, int k6) {
  RecPtr r;
#pragma unroll
  for (int k = 0; k < 6; ++k) r.f[k] = s->stage[k6][k];
  r.boff4 = r.boff8 = r.boffv = 0u;
  return r;
}

// element at a 32-bit byte offset from a field's base
template <class T>
__device__ __forceinline__ T ldo(const void GM* base, uint32_t off) {
  return *reinterpret_cast<const T GM*>(reinterpret_cast<const char GM*>(base) + off);
}

template <class T>
__device__ __forceinline__ void sto(void GM* base, uint32_t off, T v) {
  *reinterpret_cast<T GM*>(reinterpret_cast<char GM*>(base) + off) = v;
}

// byte offset of velocity record i (from the vx field's pointer): FP32 16-byte records
// (vx, vy, vz, id), FP64 24-byte records (vx, vy, vz)
template <class P>
__device__ __forceinline__ uint32_t vel_off(const RecPtr& f, uint32_t i);

template <class P>
struct Part0;
template <>
struct Part0<P32> {
  using real = float;
};
template <>
struct Part0<P64> {
  using real = double;
};

template <>
__device__ __forceinline__ uint32_t vel_off<P32>(const RecPtr& f, uint32_t i) {
  return f.boffv + i * 16u;
}
template <>
__device__ __forceinline__ uint32_t vel_off<P64>(const RecPtr& f, uint32_t i) {
  return f.boffv + i * 24u;
}

// Velocity of record i (the MCC pass's update of a collided particle): one 12- or 24-byte
// store into the record.
template <class P>
__device__ __forceinline__ void store_velocity(const RecPtr& f, uint32_t i,
                                               const typename Part0<P>::real v[3]) {
  if constexpr (std::is_same<P, P32>::value) {
    sto<Vel3>(f.f[F_VX], vel_off<P>(f, i), Vel3{v[0], v[1], v[2]});
  } else {
    sto<Vel3d>(f.f[F_VX], vel_off<P>(f, i), Vel3d{v[0], v[1], v[2]});
  }
}

// Velocity of record i of a staging set (births, emitted electrons).
template <class P>
__device__ __forceinline__ void load_velocity(const RecPtr& f, uint32_t i,
                                              typename Part0<P>::real v[3]) {
  if constexpr (std::is_same<P, P32>::value) {
    const Vel3 q = ldo<Vel3>(f.f[F_VX], vel_off<P>(f, i));
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
  } else {
    const Vel3d q = ldo<Vel3d>(f.f[F_VX], vel_off<P>(f, i));
    v[0] = q.x;
    v[1] = q.y;
    v[2] = q.z;
  }
}

// byte offset of record i's id (from the id field's pointer)
template <class P>
__device__ __forceinline__ uint32_t id_off(const RecPtr& f, uint32_t i) {
  if constexpr (std::is_same<P, P32>::value) return vel_off<P>(f, i);
  else return f.boff4 + i * 4u;
}

// One MCC candidate record: output slot, id, post-push cell, position word and velocity.
// FP32: two 16-byte halves (slot, id, cell, offset bits) (vx, vy, vz, -); FP64: three
// (slot, id, cell, -) (x, vx) (vy, vz).
template <class P>
__device__ __forceinline__ void cand_store(void GM* base, uint32_t e, uint32_t dst,
                                           uint32_t id, int d, typename Part0<P>::real pos,
                                           typename Part0<P>::real vx,
                                           typename Part0<P>::real vy,
                                           typename Part0<P>::real vz) {
  if constexpr (std::is_same<P, P32>::value) {
    const uint32_t o = e * 32u;
    sto<uint4>(base, o, make_uint4(dst, id, static_cast<uint32_t>(d), __float_as_uint(pos)));
    sto<float4>(base, o + 16u, make_float4(vx, vy, vz, 0.0f));
  } else {
    const uint32_t o = e * 48u;
    sto<uint4>(base, o, make_uint4(dst, id, static_cast<uint32_t>(d), 0u));
    sto<double2>(base, o + 16u, make_double2(pos, vx));
    sto<double2>(base, o + 32u, make_double2(vy, vz));
  }
}

template <class P>
__device__ __forceinline__ uint4 cand_load(const void GM* base, uint32_t e,
                                           typename Part0<P>::real& pos,
                                           typename Part0<P>::real v[3]) {
  if constexpr (std::is_same<P, P32>::value) {
    const uint32_t o = e * 32u;
    const uint4 a = ldo<uint4>(base, o);
    const float4 b = ldo<float4>(base, o + 16u);
    pos = __uint_as_float(a.w);
    v[0] = b.x;
    v[1] = b.y;
    v[2] = b.z;
    return a;
  } else {
    const uint32_t o = e * 48u;
    const uint4 a = ldo<uint4>(base, o);
    const double2 b = ldo<double2>(base, o + 16u);
    const double2 c = ldo<double2>(base, o + 32u);
    pos = b.x;
    v[0] = b.y;
    v[1] = c.x;
    v[2] = c.y;
    return a;
  }
}

template <class P>
struct Part;

template <>
struct Part<P32> {
  using real = float;
  int cell;
  float off, vx, vy, vz;
  uint32_t id;
  __device__ __forceinline__ void load(const RecPtr& f, uint32_t i) {
    const uint32_t o = f.boff4 + i * 4u;
    cell = ldo<int>(f.f[F32_CELL], o);
    off = ldo<float>(f.f[F32_OFF], o);
    const uint4 v = ldo<uint4>(f.f[F_VX], vel_off<P32>(f, i));
    vx = __uint_as_float(v.x);
    vy = __uint_as_float(v.y);
    vz = __uint_as_float(v.z);
    id = v.w;
  }
};

template <>
struct Part<P64> {
  using real = double;
  double x, vx, vy, vz;
  uint32_t id;
  __device__ __forceinline__ void load(const RecPtr& f, uint32_t i) {
    x = ldo<double>(f.f[F64_X], f.boff8 + i * 8u);
    const Vel3d v = ldo<Vel3d>(f.f[F_VX], vel_off<P64>(f, i));
    vx = v.x;
    vy = v.y;
    vz = v.z;
    id = ldo<uint32_t>(f.f[F_ID], f.boff4 + i * 4u);
  }
};

// Stores one record: cell d and offset (FP32) or absolute x (FP64), velocity, and the id
// unless kWithId is false (birth staging keeps no id: k_finalize numbers the births when it
// appends them; the FP64 staging arrays have no id field, the FP32 ones get 0 in the
// record's id word).
template <class P, bool kWithId = true>
__device__ __forceinline__ void store_record(const RecPtr& f, uint32_t i, int d,
                                             typename Part<P>::real pos,
                                             typename Part<P>::real vx,
                                             typename Part<P>::real vy,
                                             typename Part<P>::real vz, uint32_t id) {
  const uint32_t o4 = f.boff4 + i * 4u;
  if constexpr (std::is_same<P, P32>::value) {
    sto<int>(f.f[F32_CELL], o4, d);
    sto<float>(f.f[F32_OFF], o4, pos);
    sto<uint4>(f.f[F_VX], vel_off<P32>(f, i),
               make_uint4(__float_as_uint(vx), __float_as_uint(vy), __float_as_uint(vz),
                          kWithId ? id : 0u));
  } else {
    sto<double>(f.f[F64_X], f.boff8 + i * 8u, pos);
    sto<Vel3d>(f.f[F_VX], vel_off<P64>(f, i), Vel3d{vx, vy, vz});
    if constexpr (kWithId) sto<uint32_t>(f.f[F_ID], o4, id);
  }
}

// In-place update of a fine-sorted particle's position and v_x (the other fields do not
// change in the push); a particle that left the box gets the dead marker (cell -1, or a
// negative x) that k_fine_sort1 removes.
template <class P>
__device__ __forceinline__ void store_in_place(const RecPtr& f, uint32_t i, bool alive, int d,
                                               typename Part<P>::real pos,
                                               typename Part<P>::real vx) {
  const uint32_t o4 = f.boff4 + i * 4u;
  if constexpr (std::is_same<P, P32>::value) {
    sto<int>(f.f[F32_CELL], o4, alive ? d : -1);
    sto<float>(f.f[F32_OFF], o4, pos);
    sto<float>(f.f[F_VX], vel_off<P32>(f, i), vx);
  } else {
    sto<double>(f.f[F64_X], f.boff8 + i * 8u, alive ? pos : -1.0);
    sto<double>(f.f[F_VX], vel_off<P64>(f, i), vx);
  }
}

struct TileRange {
  uint32_t lo, hi;
  int c0;
  bool tail;
  bool fine;  // a sorting cell of a fine-sorted species
};

__device__ __forceinline__ TileRange tile_range(const SpeciesDev& s, int t, int p) {
  TileRange r;
  r.fine = false;
  if (s.mode == kModeFine) {
    // sorting cell t: its slots in the fine arrays
    r.tail = false;
    r.fine = true;
    r.c0 = t * s.C;
    r.lo = static_cast<uint32_t>(t) * s.nmax;
    r.hi = r.lo + min(s.fcnt[t], s.nmax);
    return r;
  }
  if (s.mode == kModeNone) {
    // unsorted: the array [0, n) cut into n_tiles equal ranges, handled like tail tiles
    r.tail = true;
    r.c0 = 0;
    const uint32_t nt = s.n_total[p];
    const uint32_t per = (nt + s.n_tiles - 1) / s.n_tiles;
    r.lo = min(nt, static_cast<uint32_t>(t) * per);
    r.hi = min(nt, r.lo + per);
    return r;
  }
  r.tail = t >= s.n_tiles;
  if (!r.tail) {
    r.c0 = t * s.C;
    const int c1 = min(r.c0 + s.C, s.n_cells);
    const uint32_t GM* cs = s.cell_start + p * (s.n_cells + 1);
    r.lo = cs[r.c0];
    r.hi = cs[c1];
  } else {
    r.c0 = 0;
    const uint32_t ns = s.n_sorted[p], nt = s.n_total[p];
    const uint32_t ntail = nt > ns ? nt - ns : 0u;
    const uint32_t per = (ntail + s.n_tail - 1) / s.n_tail;
    const uint32_t j = static_cast<uint32_t>(t - s.n_tiles);
    r.lo = min(nt, ns + j * per);
    r.hi = min(nt, r.lo + per);
  }
  if (r.hi < r.lo) r.hi = r.lo;
  return r;
}

// A tile's index range [lo, hi) is cut into kWaves contiguous pieces (multiples of 64
// particles except the last); wave w takes piece w, so the waves of a tile need no
// synchronisation and each (tile, wave) is its own unit of the stable order.
struct WaveRange {
  uint32_t lo, hi;
};

// piece w of a tile (any lane may ask for any piece)
__device__ __forceinline__ WaveRange piece_range(const TileRange& r, int w) {
  const uint32_t n = r.hi - r.lo;
  const uint32_t q = (n + kWaves * 64 - 1) / (kWaves * 64) * 64;
  WaveRange wr;
  wr.lo = min(r.hi, r.lo + static_cast<uint32_t>(w) * q);
  wr.hi = min(r.hi, wr.lo + q);
  return wr;
}

// the piece of the calling wave, as wave-uniform values (keeps the particle loop a scalar
// loop): w must be the same in every lane
__device__ __forceinline__ WaveRange wave_range(const TileRange& r, int w) {
  WaveRange wr = piece_range(r, w);
  wr.lo = __builtin_amdgcn_readfirstlane(wr.lo);
  wr.hi = __builtin_amdgcn_readfirstlane(wr.hi);
  return wr;
}

// Streams a wave's range [lo, hi) through `body` in chunks of 64 consecutive particles
// (lane l takes lo + 64 j + l), U chunks per pass, with the loads of the next pass issued
// before the current pass is worked on.  `body(item, index, valid)` runs on all 64 lanes.
// The loads are not conditional (lanes past the end re-read the last element), so a
// pass always issues the same memory instructions; with the bodies' stores also
// unconditional, the compiler can wait for exactly the loads of the pass it needs instead
// of for every outstanding access.
template <class T, int U, class Load, class Body>
__device__ __forceinline__ void stream_range(uint32_t lo, uint32_t hi, Load&& load,
                                             Body&& body) {
  if (lo >= hi) return;
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t last = hi - 1u;
  T nxt[U];
#pragma unroll
  for (int u = 0; u < U; ++u) load(nxt[u], min(lo + static_cast<uint32_t>(u) * 64u + lane, last));
  for (uint32_t b = lo; b < hi; b += U * 64u) {
    T cur[U];
#pragma unroll
    for (int u = 0; u < U; ++u) cur[u] = nxt[u];
#pragma unroll
    for (int u = 0; u < U; ++u)
      load(nxt[u], min(b + static_cast<uint32_t>(U + u) * 64u + lane, last));
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t i = b + static_cast<uint32_t>(u) * 64u + lane;
      body(cur[u], i, i < hi);
    }
  }
}

// The same, from the end of the range backwards: pass by pass and chunk by chunk in
// decreasing index order (lanes inside a chunk still ascend; lanes before the start
// re-read the first element).
template <class T, int U, class Load, class Body>
__device__ __forceinline__ void stream_range_rev(uint32_t lo, uint32_t hi, Load&& load,
                                                 Body&& body) {
  if (lo >= hi) return;
  const int lane = static_cast<int>(threadIdx.x & 63u);
  const int ilo = static_cast<int>(lo), ihi = static_cast<int>(hi);
  T nxt[U];
#pragma unroll
  for (int u = 0; u < U; ++u) load(nxt[u], static_cast<uint32_t>(max(ihi - 64 * (u + 1) + lane, ilo)));
  for (int b = ihi; b > ilo; b -= U * 64) {
    T cur[U];
#pragma unroll
    for (int u = 0; u < U; ++u) cur[u] = nxt[u];
#pragma unroll
    for (int u = 0; u < U; ++u)
      load(nxt[u], static_cast<uint32_t>(max(b - 64 * (U + u + 1) + lane, ilo)));
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = b - 64 * (u + 1) + lane;
      body(cur[u], static_cast<uint32_t>(max(i, ilo)), i >= ilo);
    }
  }
}

// In k_main the even waves of a cell tile walk their piece backwards: each cell's output
// sub-run of a wave is then filled from its end, and the cache lines that two neighbouring
// sub-runs share are written by both neighbours at about the same time (at the start or
// at the end of both passes) instead of once early and once late, when a half-written
// line has long been written back.
__device__ __forceinline__ bool wave_reversed(const TileRange& r, int w) {
  return !r.tail && !r.fine && (w & 1) == 0;
}

// The fields the push reads (the sort pre-pass loads only these).
template <class P>
struct PushIn;

template <>
struct PushIn<P32> {
  int cell;
  float off, vx;
  __device__ __forceinline__ void load(const RecPtr& f, uint32_t i) {
    const uint32_t o = f.boff4 + i * 4u;
    cell = ldo<int>(f.f[F32_CELL], o);
    off = ldo<float>(f.f[F32_OFF], o);
    vx = ldo<float>(f.f[F_VX], vel_off<P32>(f, i));
  }
};

template <>
struct PushIn<P64> {
  double x, vx;
  __device__ __forceinline__ void load(const RecPtr& f, uint32_t i) {
    x = ldo<double>(f.f[F64_X], f.boff8 + i * 8u);
    vx = ldo<double>(f.f[F_VX], vel_off<P64>(f, i));
  }
};

// The stored cell only (the lagged sort's key; the pre-pass then reads 4 of 24 bytes in
// FP32): -1 for a dead record.
template <class P>
struct KeyIn;

template <>
struct KeyIn<P32> {
  int cell;
  __device__ __forceinline__ void load(const RecPtr& f, uint32_t i) {
    cell = ldo<int>(f.f[F32_CELL], f.boff4 + i * 4u);
  }
  __device__ __forceinline__ int key() const { return cell; }
};

template <>
struct KeyIn<P64> {
  double x;
  __device__ __forceinline__ void load(const RecPtr& f, uint32_t i) {
    x = ldo<double>(f.f[F64_X], f.boff8 + i * 8u);
  }
  __device__ __forceinline__ int key() const { return x >= 0.0 ? static_cast<int>(floor(x)) : -1; }
};

// stored cell of a full record (-1: dead)
template <class P>
__device__ __forceinline__ int stored_cell(const Part<P>& q) {
  if constexpr (std::is_same<P, P32>::value) return q.cell;
  else return q.x >= 0.0 ? static_cast<int>(floor(q.x)) : -1;
}

__device__ __forceinline__ int key_bits(int n) {
  int b = 0;
  while ((1 << b) < n) ++b;
  return b;
}
// Loads the field of the tile's nodes [c0, c0 + C] into LDS (node index wrapped when
// periodic).  Tail tiles read the global array instead.
template <class real>
__device__ __forceinline__ void load_field_window(const SpeciesDev& s, const real GM* E,
                                                  const TileRange& r, real* Elds) {
  if (r.tail) return;
  for (int k = threadIdx.x; k <= s.C; k += blockDim.x) {
    int n = r.c0 + k;
    if (s.periodic) n %= s.n_cells;
    if (n > s.n_nodes - 1) n = s.n_nodes - 1;
    Elds[k] = E[n];
  }
}

// Lagged sort: the field at the W + 1 nodes of tile r's window (slot k of the window is
// cell t C - D + k; the nodes past the ends of a bounded grid are never read).
template <class real>
__device__ __forceinline__ void load_field_window_lag(const SpeciesDev& s, const real GM* E,
                                                      const TileRange& r, int tile, real* Elds) {
  if (r.tail) return;
  for (int k = threadIdx.x; k <= s.W; k += blockDim.x) {
    int n = tile * s.C - s.D + k;
    if (s.periodic) {
      n %= s.n_cells;
      if (n < 0) n += s.n_cells;
    }
    n = n < 0 ? 0 : (n > s.n_nodes - 1 ? s.n_nodes - 1 : n);
    Elds[k] = E[n];
  }
}

// Field at a node.  A cell tile's particles sit in its own cells, so their nodes are in
// the tile's LDS window (the clamp only guards a corrupt state); tail particles read the
// global array.  kTail is a compile-time flag so that the two reads stay an LDS read and
// a global read (a run-time choice between the two pointers would make a flat load).
template <class real, bool kTail>
__device__ __forceinline__ real field_at(const SpeciesDev& s, const real GM* E, const real* Elds,
                                         const TileRange& r, int node) {
  if constexpr (!kTail) {
    int k = node - r.c0;
    k = k < 0 ? 0 : (k > s.C ? s.C : k);
    return Elds[k];
  } else {
    if (s.periodic && node >= s.n_cells) node -= s.n_cells;
    return E[node];
  }
}

// Push one particle: returns status (0 kept, 1/2 wall, 3 invalid), the destination cell
// d, the new position word (offset or x) and the new v_x.
template <class P, bool kTail, class Q>
__device__ __forceinline__ int push_particle(const SpeciesDev& s, const DischargeDev& dd,
                                             const typename Part<P>::real* Elds,
                                             const TileRange& r, const Q& q, int& d,
                                             typename Part<P>::real& pos,
                                             typename Part<P>::real& vxn) {
  if constexpr (std::is_same<P, P32>::value) {
    const int c = q.cell;
    if (c < 0 || c >= s.n_cells) {
      d = 0;
      pos = 0.0f;
      vxn = q.vx;
      return 3;
    }
    const float e0 = field_at<float, kTail>(s, dd.E32, Elds, r, c);
    const float e1 = field_at<float, kTail>(s, dd.E32, Elds, r, c + 1);
    return push32(c, q.off, q.vx, e0, e1, s.kappa_f, s.n_cells, s.periodic, d, pos, vxn);
  } else {
    if (!(q.x >= 0.0 && q.x < static_cast<double>(s.n_cells))) {
      d = 0;
      pos = 0.0;
      vxn = q.vx;
      return 3;
    }
    const int c = static_cast<int>(floor(q.x));
    const double e0 = field_at<double, kTail>(s, dd.E64, Elds, r, c);
    const double e1 = field_at<double, kTail>(s, dd.E64, Elds, r, c + 1);
    return push64(q.x, q.vx, e0, e1, s.kappa, s.n_cells, s.periodic, pos, vxn, d);
  }
}

// Lagged sort: push a record whose present cell has window slot ek of its tile (ek >= 0:
// the two nodes are window entries ek and ek + 1) or lies outside the window (ek < 0:
// global field array).
template <class P, class Q>
__device__ __forceinline__ int push_particle_lag(const SpeciesDev& s, const DischargeDev& dd,
                                                 const typename Part<P>::real* Elds, int ek,
                                                 const Q& q, int& d, typename Part<P>::real& pos,
                                                 typename Part<P>::real& vxn) {
  using real = typename Part<P>::real;
  int c;
  if constexpr (std::is_same<P, P32>::value) {
    c = q.cell;
    if (c < 0 || c >= s.n_cells) {
      d = 0;
      pos = 0.0f;
      vxn = q.vx;
      return 3;
    }
  } else {
    if (!(q.x >= 0.0 && q.x < static_cast<double>(s.n_cells))) {
      d = 0;
      pos = 0.0;
      vxn = q.vx;
      return 3;
    }
    c = static_cast<int>(floor(q.x));
  }
  const real GM* E = std::is_same<P, P32>::value ? reinterpret_cast<const real GM*>(dd.E32)
                                                  : reinterpret_cast<const real GM*>(dd.E64);
  real e0, e1;
  if (ek >= 0) {
    e0 = Elds[ek];
    e1 = Elds[ek + 1];
  } else {
    const int c1 = (s.periodic && c + 1 >= s.n_cells) ? c + 1 - s.n_cells : c + 1;
    e0 = E[c];
    e1 = E[c1];
  }
  if constexpr (std::is_same<P, P32>::value)
    return push32(c, q.off, q.vx, e0, e1, s.kappa_f, s.n_cells, s.periodic, d, pos, vxn);
  else
    return push64(q.x, q.vx, e0, e1, s.kappa, s.n_cells, s.periodic, pos, vxn, d);
}

// Electrode reflection of an electron that reached a wall (st 1 or 2; Sec. 2), decided by
// word 0 of its Philox block 6: returns the new status, 0 when mirrored back into the box.
template <class P>
__device__ __forceinline__ int reflect_at_wall(const SpeciesDev& s, uint32_t id, uint32_t step32,
                                               int st, int& d, typename Part<P>::real& pos,
                                               typename Part<P>::real& vxn) {
  if (!(philox(id, step32, 6u, 0u, s.key0, s.key1).x < s.t_refl)) return st;
  bool in;
  if constexpr (std::is_same<P, P32>::value) in = mirror32(s.n_cells, st, d, pos);
  else in = mirror64(s.n_cells, st, pos, d);
  vxn = -vxn;
  return in ? 0 : st;
}

__device__ __forceinline__ bool diag_step(const DischargeDev& dd, unsigned long long step) {
  if (dd.eedf_bins <= 0 || dd.diag_every <= 0) return false;
  const long long st = static_cast<long long>(step);
  if (st < dd.avg_start) return false;
  return ((st - dd.avg_start) % dd.diag_every) == 0;
}

// ====================================================================================
// k_combine: w_s[j] = sum over the tiles whose deposit window holds node j + the far /
// birth deposits.  kCombineLanes lanes per node (a node is covered by about (W + 1) / C
// windows): lane l adds windows l, l + kCombineLanes, ... in order, then the lanes' sums
// meet in a fixed butterfly, so the result is reproducible.  Grid: one workgroup per
// block of kCombineNodes nodes of a species (node_table).
// ====================================================================================
__global__ __launch_bounds__(kCombineNodes * kCombineLanes) void k_combine(
    const SimDev* __restrict__ simp) {
  const SimDev& sim = *simp;
  const int2 nt = sim.node_table[blockIdx.x];
  const SpeciesDev s = sim.sp[nt.x];
  const int l = static_cast<int>(threadIdx.x) % kCombineLanes;
  const int j = nt.y + static_cast<int>(threadIdx.x) / kCombineLanes;
  const bool live = j < s.n_nodes;  // the butterfly below needs every lane of a node
  const unsigned long long GM* part = s.partial;
  const int span = s.W + 1;
  unsigned long long sum = 0ull;
  if (live && s.mode != kModeNone) {  // unsorted: every deposit is in the node array
    int a[2], b[2];
    covering_ranges(s, j, span, a, b);
    const int n0 = b[0] >= a[0] ? b[0] - a[0] + 1 : 0;
    const int n1 = b[1] >= a[1] ? b[1] - a[1] + 1 : 0;
    for (int u = l; u < n0 + n1; u += kCombineLanes) {
      const int t = u < n0 ? a[0] + u : a[1] + (u - n0);
      sum += part[static_cast<size_t>(t) * span + covering_slot(s, j, t)];
    }
  }
#pragma unroll
  for (int o = kCombineLanes / 2; o >= 1; o >>= 1)
    sum += static_cast<unsigned long long>(__shfl_xor(static_cast<long long>(sum), o, 64));
  if (live && l == 0)
    sim.ds[s.ds].w[s.sp][j] = static_cast<double>(sum + s.far_w[j]) * s.dep_inv;
}

// Exclusive scan of kV values per thread over the workgroup in one pass (the order of
// block_exclusive_scan for each); lds holds kV * (blockDim / 64 + 1) doubles.
template <int kV>
__device__ __forceinline__ void block_exclusive_scan_n(double (&v)[kV], double* lds,
                                                       double (&total)[kV]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double inc[kV];
#pragma unroll
  for (int q = 0; q < kV; ++q) {
    inc[q] = wave_inclusive_scan(v[q]);
    if (lane == 63) lds[q * (kSolveWG / 64 + 1) + w] = inc[q];
  }
  __syncthreads();
  if (threadIdx.x < kV) {
    double* l = lds + threadIdx.x * (kSolveWG / 64 + 1);
    double r = 0.0;
    for (int i = 0; i < nw; ++i) {
      const double t = l[i];
      l[i] = r;
      r = r + t;
    }
    l[nw] = r;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kV; ++q) {
    const double* l = lds + q * (kSolveWG / 64 + 1);
    total[q] = l[nw];
    v[q] = l[w] + (inc[q] - v[q]);
  }
  __syncthreads();
}

// ====================================================================================
// k_solve: one workgroup per discharge.  The finite-difference Poisson system of eq.
// poisson_normalized (Sec. 3.5) with Phi_0 = V(t_n), Phi_N = 0 (or periodic, mean charge
// removed, Phi_0 = 0) is solved exactly as the paper's tridiagonal system, but in the
// parallel form of its two recurrences: the slopes s_j = Phi_{j+1} - Phi_j obey
// s_j = s_0 - R_j with R_j = sum_{k=1..j} rho_k, s_0 fixed by the two end potentials;
// Phi is the running sum of s.  E_j = -(s_{j-1} + s_j)/2 inside; at an electrode Gauss's
// law over the half cell: E_0 = -s_0 - rho_0, E_N = -s_{N-1} + rho_N.
// With a series capacitor C between the source V_s and the driven electrode (an external
// circuit; Sec. 3.5 leaves boundary conditions to the literature), the electrode and the
// plate joined to it hold the charge q, which changes only by the particles absorbed or
// emitted there.  E_0 grows with Phi_0 as E_0 = sigma_z + Phi_0 / N (sigma_z: the value
// for Phi_0 = 0), the plate holds q - E_0, and Phi_0 = V_s + (q - E_0) / C gives
// Phi_0 = (V_s + (q - sigma_z) / C) / (1 + 1 / (N C)).
// The step's net charge, field energy and electrode potential are kept for diagnostics.
// Two workgroup-wide scans: one over rho (its prefix gives R; the totals of rho_k and
// k rho_k give sum_j R_j, hence s_0), one over the slopes (Phi and the field energy).
// ====================================================================================
__global__ __launch_bounds__(kSolveWG) void k_solve(const SimDev* __restrict__ simp,
                                                    int init_mode) {
  const SimDev& sim = *simp;
  const DischargeDev dd = sim.ds[blockIdx.x];
  __shared__ double lds_n[3 * (kSolveWG / 64 + 1)];
  __shared__ double sv[kMaxCells + 1];  // rho_j, then the slope s_j
  const unsigned long long step = init_mode ? 0ull : *sim.step;
  const int N = dd.n_cells;
  const int nn = dd.n_nodes;
  const double GM* we = dd.w[0];
  const double GM* wi = dd.w[1];
  const int tid = threadIdx.x;
  // thread tid owns the nodes [lo, hi) and the cells [lo, hc)
  const int per = (nn + static_cast<int>(blockDim.x) - 1) / static_cast<int>(blockDim.x);
  const int lo = tid * per;
  const int hi = min(lo + per, nn);
  const int hc = min(hi, N);
  const double rho_wall0 = wi[0] - we[0];
  const double rho_wallN = dd.periodic ? 0.0 : wi[N] - we[N];
  // One pass over the charge: the net charge of all nodes, and over the cells 1..N-1 the
  // sums of rho_k and of k rho_k, whose prefixes give R_j = sum_{k=1..j} (rho_k - mean)
  // and sum_j R_j = N P - K - mean N (N - 1) / 2 (P, K their totals) without a scan of R.
  double v3[3] = {0.0, 0.0, 0.0}, t3[3];
  constexpr int kB = 8;  // nodes of a thread read at once (their loads in flight together)
  for (int j0 = lo; j0 < hi; j0 += kB) {
    double a[kB], b[kB];
#pragma unroll
    for (int k = 0; k < kB; ++k) {
      a[k] = 0.0;
      b[k] = 0.0;
      if (j0 + k < hi) {
        a[k] = wi[j0 + k];
        b[k] = we[j0 + k];
      }
    }
#pragma unroll
    for (int k = 0; k < kB; ++k) {
      const int j = j0 + k;
      if (j >= hi) break;
      const double r = a[k] - b[k];
      sv[j] = r;
      v3[2] += r;
      if (j >= 1 && j < N) {
        v3[0] += r;
        v3[1] += static_cast<double>(j) * r;
      }
    }
  }
  block_exclusive_scan_n<3>(v3, lds_n, t3);
  const double sum_rho = t3[2];
  // mean charge of the cells (periodic only)
  const double mean = dd.periodic ? (rho_wall0 + t3[0]) / static_cast<double>(N) : 0.0;
  const double Nd = static_cast<double>(N);
  const double sum_r = Nd * t3[0] - t3[1] - mean * Nd * (Nd - 1.0) * 0.5;
  const double vs = dd.periodic ? 0.0 : dd.vhat_amp * sin(dd.phase_per_step * static_cast<double>(step));
  double a = vs;
  double q = 0.0;
  if (dd.cap_norm > 0.0) {
    const double sigma_z = -(sum_r / Nd) - rho_wall0;
    if (init_mode) {
      q = sigma_z + vs / Nd;  // capacitor uncharged at the load
    } else {
      const SpeciesDev se = sim.sp[dd.spec0];
      const SpeciesDev si = sim.sp[dd.spec0 + 1];
      q = dd.dstat[DS_Q_INIT] + static_cast<double>(si.absorbed[0]) -
          static_cast<double>(se.absorbed[0]) + static_cast<double>(si.emitted[0]);
    }
    a = (vs + (q - sigma_z) / dd.cap_norm) / (1.0 + 1.0 / (Nd * dd.cap_norm));
  }
  const double s0 = (0.0 - a + sum_r) / Nd;
  // s_j = s0 - R_j into LDS (read across the thread boundary by E below); their sum
  // (Phi_j = a + sum_{m<j} s_m) and sum of squares (field energy) in one more pass
  double v2[2] = {0.0, 0.0}, t2[2];
  {
    double run = v3[0];  // sum_{k=1..lo-1} rho_k
    for (int j = lo; j < hc; ++j) {
      if (j >= 1) run += sv[j];
      const double sj = s0 - (run - static_cast<double>(j) * mean);
      sv[j] = sj;
      v2[0] += sj;
      v2[1] += sj * sj;
    }
  }
  block_exclusive_scan_n<2>(v2, lds_n, t2);
  double GM* phi = dd.phi;
  {
    double run = v2[0] + a;
    for (int j = lo; j < hc; ++j) {
      phi[j] = run;
      run += sv[j];
    }
  }
  if (!dd.periodic && tid == 0) phi[N] = 0.0;
  const double field = 0.5 * t2[1];
  // E from the slopes
  for (int j = lo; j < hi; ++j) {
    double e;
    if (dd.periodic) {
      const int jm = j == 0 ? N - 1 : j - 1;
      e = -(sv[jm] + sv[j]) / 2.0;
    } else if (j == 0) {
      e = -sv[0] - rho_wall0;
    } else if (j == N) {
      e = -sv[N - 1] + rho_wallN;
    } else {
      e = -(sv[j - 1] + sv[j]) / 2.0;
    }
    dd.E64[j] = e;
    dd.E32[j] = static_cast<float>(e);
  }
  if (tid == 0) {
    dd.dstat[DS_FIELD] = field;
    dd.dstat[DS_SUM_RHO] = sum_rho;
    dd.dstat[DS_PHI0] = dd.periodic ? 0.0 : a;
    dd.dstat[DS_Q] = q;
    if (init_mode) dd.dstat[DS_Q_INIT] = q;
  }
  __syncthreads();  // the phi stores above are read by other threads below
  if (!init_mode && static_cast<long long>(step) >= dd.avg_start) {
    constexpr int kA = 4;  // nodes of a thread updated at once
    const int B = static_cast<int>(blockDim.x);
    for (int j0 = tid; j0 < nn; j0 += kA * B) {
      double x0[kA], x1[kA], x2[kA], y0[kA], y1[kA], y2[kA];
#pragma unroll
      for (int k = 0; k < kA; ++k) {
        const int j = j0 + k * B;
        x0[k] = x1[k] = x2[k] = y0[k] = y1[k] = y2[k] = 0.0;
        if (j < nn) {
          x0[k] = dd.acc_w[0][j];
          x1[k] = dd.acc_w[1][j];
          x2[k] = dd.acc_phi[j];
          y0[k] = we[j];
          y1[k] = wi[j];
          y2[k] = phi[j];
        }
      }
#pragma unroll
      for (int k = 0; k < kA; ++k) {
        const int j = j0 + k * B;
        if (j < nn) {
          dd.acc_w[0][j] = x0[k] + y0[k];
          dd.acc_w[1][j] = x1[k] + y1[k];
          dd.acc_phi[j] = x2[k] + y2[k];
        }
      }
    }
    if (tid == 0) *dd.acc_count += 1ull;
  }
  if (!init_mode && tid == 0 && diag_step(dd, step)) *dd.eedf_samples += 1ull;
  // per-step far-mover state of both species starts empty; a fine-sorted species counts
  // its survivors into n_sorted of the step's output parity.  (Not at the load: the far
  // array then holds part of the load's deposit, which the first step's combine reads.)
  for (int sp = 0; sp < 2 && !init_mode; ++sp) {
    const SpeciesDev s = sim.sp[dd.spec0 + sp];
    for (int j = tid; j < nn; j += blockDim.x) s.far_w[j] = 0ull;
    for (int c = tid; c < N; c += blockDim.x) s.far_cell_cnt[c] = 0u;
    if (tid == 0) *s.far_count = 0u;
    if (tid == 0 && s.mode == kModeFine) s.n_sorted[(step + 1ull) & 1ull] = 0u;
  }
}

// ====================================================================================
// k_hist: post-push cell histogram (sort pre-pass).  Each wave counts its own piece of
// the tile into its own LDS histogram over the tile's window with LDS atomic increments,
// spread over lane-indexed copies (a chunk of 64 particles comes from one cell and lands
// in a few slots; with one copy the increments would queue on those slots).  Particles
// that leave the window go to the far list.  A tail tile (the unsorted births at the end of the array)
// has no window: each of its waves counts into its own global row over all cells.
// ====================================================================================
constexpr int kHistCopies = 8;

template <class P>
struct HistU;
template <>
struct HistU<P32> {
  static constexpr int value = 4;
};
template <>
struct HistU<P64> {
  static constexpr int value = 2;
};

// kLag: the lagged sort (the array ordered by the cell each particle held at the start of
// the step; Sec. 3.7 only needs the order to be close): the key is the cell stored in the
// record at the start of the step, so the pre-pass reads that field only and pushes
// nothing.
template <class P, bool kLag>
__global__ __launch_bounds__(kWG) void k_hist(const SimDev* __restrict__ simp) {
  using real = typename Part<P>::real;
  const SimDev& sim = *simp;
  const int2 tt = sim.tile_table[blockIdx.x];
  const SpeciesDev s = sim.sp[tt.x];
  if (s.mode == kModeFine) return;  // sorted in place after the push: no pre-pass
  const DischargeDev dd = sim.ds[s.ds];
  const unsigned long long step = *sim.step;
  const uint32_t step32 = static_cast<uint32_t>(step);
  const int p = static_cast<int>(step & 1ull);
  const TileRange r = tile_range(s, tt.y, p);
  __shared__ real Elds[kMaxCellsPerTile + 1];
  __shared__ uint32_t hq[kWaves][64][2];
  // per-wave histograms, kHistCopies copies each (lane l counts into copy l mod
  // kHistCopies, so an LDS atomic has few lanes on one slot); W_max slots per copy
  extern __shared__ uint32_t hdyn[];
  const int tid = threadIdx.x, lane = tid & 63, wv = wave_id();
  const unsigned long long lt = lanes_below();
  const real GM* E = std::is_same<P, P32>::value ? reinterpret_cast<const real GM*>(dd.E32)
                                                  : reinterpret_cast<const real GM*>(dd.E64);
  if constexpr (!kLag) load_field_window<real>(s, E, r, Elds);  // lagged: no push here
  const int W = s.W;
  const int Wm = sim.max_window;
  for (int k = tid; k < kWaves * kHistCopies * Wm; k += kWG) hdyn[k] = 0u;
  uint32_t* h = hdyn + wv * kHistCopies * Wm;
  uint32_t* hl = h + (lane & (kHistCopies - 1)) * Wm;
  __syncthreads();
  const WaveRange wr = wave_range(r, wv);
  const RecPtr in = rec_buf(&sim.sp[tt.x], p);
  auto load = [&](PushIn<P>& q, uint32_t i) { q.load(in, i); };
  if (kLag && !r.tail) {
    // lagged: histogram of the stored cells of the live records (dead ones skipped)
    uint32_t qn = 0;  // wave-uniform
    auto flush = [&]() {
      uint32_t e0 = 0u;
      if (lane == 0) e0 = atomicAdd(s.far_count, qn);
      e0 = __shfl(e0, 0, 64);
      const uint32_t j = static_cast<uint32_t>(lane);
      if (j < qn) {
        const uint32_t e = e0 + j;
        const uint32_t d = hq[wv][j][0];
        if (e < s.far_cap) {
          s.far_list[e] = make_uint4(d, hq[wv][j][1], static_cast<uint32_t>(tt.y), 0u);
          atomicAdd(&s.far_cell_cnt[d], 1u);
        }
      }
      qn = 0;
    };
    auto kload = [&](KeyIn<P>& q, uint32_t i) { q.load(in, i); };
    stream_range<KeyIn<P>, 8>(wr.lo, wr.hi, kload, [&](const KeyIn<P>& q, uint32_t i, bool valid) {
      const int key = valid ? q.key() : -1;
      const bool live = key >= 0 && key < s.n_cells;
      const int k = live ? window_slot(s, tt.y, key) : -1;
      if (k >= 0) atomicAdd(&hl[k], 1u);
      const bool far = live && k < 0;
      const unsigned long long fm = __ballot(far);
      if (fm) {
        if (qn + static_cast<uint32_t>(__popcll(fm)) > 64u) flush();
        if (far) {
          const uint32_t j = qn + static_cast<uint32_t>(__popcll(fm & lt));
          hq[wv][j][0] = static_cast<uint32_t>(key);
          hq[wv][j][1] = i;
        }
        qn += static_cast<uint32_t>(__popcll(fm));
      }
    });
    if (qn) flush();
    uint32_t GM* row = s.hist + (static_cast<size_t>(tt.y) * kWaves + wv) * W;
    for (int k = lane; k < W; k += 64) {
      uint32_t n = 0u;
#pragma unroll
      for (int c = 0; c < kHistCopies; ++c) n += h[c * Wm + k];
      row[k] = n;
    }
  } else if (kLag) {
    // lagged tail: each wave counts its live records' stored cells into its global row
    uint32_t GM* row = s.thist +
                       static_cast<size_t>((tt.y - s.n_tiles) * kWaves + wv) * s.n_cells;
    auto kload = [&](KeyIn<P>& q, uint32_t i) { q.load(in, i); };
    stream_range<KeyIn<P>, 8>(wr.lo, wr.hi, kload, [&](const KeyIn<P>& q, uint32_t i, bool valid) {
      const int key = valid ? q.key() : -1;
      if (key >= 0 && key < s.n_cells) atomicAdd(&row[key], 1u);
    });
  } else if (!r.tail) {
    // far movers wait in a per-wave LDS queue and are appended to the far list after the
    // loop (a returning atomic inside the loop would make it wait for the next loads)
    uint32_t qn = 0;  // wave-uniform
    auto flush = [&]() {
      uint32_t e0 = 0u;
      if (lane == 0) e0 = atomicAdd(s.far_count, qn);
      e0 = __shfl(e0, 0, 64);
      const uint32_t j = static_cast<uint32_t>(lane);  // the queue holds at most 64
      if (j < qn) {
        const uint32_t e = e0 + j;
        const uint32_t d = hq[wv][j][0];
        if (e < s.far_cap) {
          s.far_list[e] = make_uint4(d, hq[wv][j][1], static_cast<uint32_t>(tt.y), 0u);
          atomicAdd(&s.far_cell_cnt[d], 1u);
        }
      }
      qn = 0;
    };
    stream_range<PushIn<P>, HistU<P>::value>(
        wr.lo, wr.hi, load, [&](const PushIn<P>& q, uint32_t i, bool valid) {
          int st = 4, d = 0;
          real pos, vxn;
          if (valid) st = push_particle<P, false>(s, dd, Elds, r, q, d, pos, vxn);
          if (s.t_refl && (st == 1 || st == 2))
            st = reflect_at_wall<P>(s, ldo<uint32_t>(in.f[F_ID], id_off<P>(in, i)), step32, st,
                                    d, pos, vxn);
          const int k = st == 0 ? window_slot(s, tt.y, d) : -1;
          const bool near = k >= 0;
          if (near) atomicAdd(&hl[k], 1u);
          const bool far = st == 0 && !near;
          const unsigned long long fm = __ballot(far);
          if (fm) {
            if (qn + static_cast<uint32_t>(__popcll(fm)) > 64u) flush();
            if (far) {
              const uint32_t j = qn + static_cast<uint32_t>(__popcll(fm & lt));
              hq[wv][j][0] = static_cast<uint32_t>(d);
              hq[wv][j][1] = i;
            }
            qn += static_cast<uint32_t>(__popcll(fm));
          }
        });
    if (qn) flush();
    uint32_t GM* row = s.hist + (static_cast<size_t>(tt.y) * kWaves + wv) * W;
    for (int k = lane; k < W; k += 64) {  // the wave's own copies: no barrier needed
      uint32_t n = 0u;
#pragma unroll
      for (int c = 0; c < kHistCopies; ++c) n += h[c * Wm + k];
      row[k] = n;
    }
  } else if (s.mode == kModeNone) {
    // unsorted: survivors of the wave's piece, in input order
    uint32_t cnt = 0u;  // wave-uniform
    stream_range<PushIn<P>, HistU<P>::value>(
        wr.lo, wr.hi, load, [&](const PushIn<P>& q, uint32_t i, bool valid) {
          int st = 4, d = 0;
          real pos, vxn;
          if (valid) st = push_particle<P, true>(s, dd, Elds, r, q, d, pos, vxn);
          if (s.t_refl && (st == 1 || st == 2))
            st = reflect_at_wall<P>(s, ldo<uint32_t>(in.f[F_ID], id_off<P>(in, i)), step32, st,
                                    d, pos, vxn);
          cnt += static_cast<uint32_t>(__popcll(__ballot(st == 0)));
        });
    if (lane == 0) s.hist[tt.y * kWaves + wv] = cnt;
  } else {
    uint32_t GM* row = s.thist +
                    static_cast<size_t>((tt.y - s.n_tiles) * kWaves + wv) * s.n_cells;
    stream_range<PushIn<P>, HistU<P>::value>(
        wr.lo, wr.hi, load, [&](const PushIn<P>& q, uint32_t i, bool valid) {
          int st = 4, d = 0;
          real pos, vxn;
          if (valid) st = push_particle<P, true>(s, dd, Elds, r, q, d, pos, vxn);
          if (s.t_refl && (st == 1 || st == 2))
            st = reflect_at_wall<P>(s, ldo<uint32_t>(in.f[F_ID], id_off<P>(in, i)), step32, st,
                                    d, pos, vxn);
          if (st == 0) atomicAdd(&row[d], 1u);
        });
  }
}

// ====================================================================================
// Output offsets.  Output order = stable sort of the survivors by cell (ties in input
// order).  The units of that order are, in input order: the (tile, wave) pieces of the
// cell tiles, then the (tail tile, wave) pieces of the tail.  For cell c:
//   count(c) = histogram entries of the covering (tile, wave) units + far movers into c
//              + tail-row entries,
//   base(c)  = exclusive scan of count;
//   a cell-tile unit (t, w) starts at base(c) + (far movers into c from tiles < t)
//              + (entries of the covering units before (t, w));
//   a far mover from tile u starts at base(c) + (its rank by index among the far movers
//              into c) + (entries of the covering units of tiles < u);
//   tail row j starts after all of the cell tiles' particles and far movers in c and the
//              tail rows before j.
// k_scan_cells does the per-cell part across the whole chip (and clears the tail rows
// for the next step); k_scan_base (one workgroup per discharge and species) scans over
// cells and places the far movers.
// ====================================================================================
constexpr uint32_t kMaxFarGroup = 8192;

// kScanLanes lanes per cell: lane u takes the covering (tile, wave) units u, u + kScanLanes,
// ... of the cell (in the order of the stable sort), and a scan over the cell's lanes gives
// every unit its offset.  Grid: one workgroup per block of kScanCells cells of a species.
template <class T>
__device__ __forceinline__ T group_inclusive_scan(T x) {  // over aligned groups of kScanLanes
  const int g = static_cast<int>(threadIdx.x) & (kScanLanes - 1);
#pragma unroll
  for (int o = 1; o < kScanLanes; o <<= 1) {
    const T y = __shfl_up(x, o, kScanLanes);
    if (g >= o) x = x + y;
  }
  return x;
}

__global__ __launch_bounds__(kScanCells * kScanLanes) void k_scan_cells(
    const SimDev* __restrict__ simp) {
  const SimDev& sim = *simp;
  const int2 ct = sim.cell_table[blockIdx.x];
  const SpeciesDev s = sim.sp[ct.x];
  const int g = static_cast<int>(threadIdx.x) & (kScanLanes - 1);
  const int c = ct.y + static_cast<int>(threadIdx.x) / kScanLanes;
  const int N = s.n_cells;
  const bool live = c < N;  // the group scans below need every lane of a cell
  const int W = s.W;
  int a[2] = {0, 0}, b[2] = {-1, -1};
  if (live) covering_ranges(s, c, W, a, b);
  const int n0 = b[0] >= a[0] ? b[0] - a[0] + 1 : 0;
  const int n1 = b[1] >= a[1] ? b[1] - a[1] + 1 : 0;
  const int units = (n0 + n1) * kWaves;
  const int rows = live ? s.n_tail * kWaves : 0;
  // Loads of up to kB passes are issued together, then scanned: one memory round trip
  // for the usual cell (at most kB * kScanLanes units and tail rows).
  constexpr int kB = 4;
  uint32_t run = 0;
  const uint32_t nfar = live ? s.far_cell_cnt[c] : 0u;
  for (int u0 = 0; __any(u0 < units); u0 += kScanLanes * kB) {
    uint32_t v[kB];
    size_t o[kB];
#pragma unroll
    for (int q = 0; q < kB; ++q) {
      const int u = u0 + q * kScanLanes + g;
      v[q] = 0u;
      o[q] = 0;
      if (u < units) {
        const int ti = u / kWaves, w = u - ti * kWaves;
        const int t = ti < n0 ? a[0] + ti : a[1] + (ti - n0);
        o[q] = (static_cast<size_t>(t) * kWaves + w) * W + covering_slot(s, c, t);
        v[q] = s.hist[o[q]];
      }
    }
#pragma unroll
    for (int q = 0; q < kB; ++q) {
      const int u = u0 + q * kScanLanes + g;
      const uint32_t inc = group_inclusive_scan(v[q]);
      if (u < units) s.tilerel[o[q]] = run + inc - v[q];
      run += __shfl(inc, kScanLanes - 1, kScanLanes);
    }
  }
  run += nfar;
  for (int j0 = 0; __any(j0 < rows); j0 += kScanLanes * kB) {
    uint32_t v[kB];
#pragma unroll
    for (int q = 0; q < kB; ++q) {
      const int jj = j0 + q * kScanLanes + g;
      v[q] = jj < rows ? s.thist[static_cast<size_t>(jj) * N + c] : 0u;
    }
#pragma unroll
    for (int q = 0; q < kB; ++q) {
      const int jj = j0 + q * kScanLanes + g;
      const uint32_t inc = group_inclusive_scan(v[q]);
      if (jj < rows) {
        const size_t o = static_cast<size_t>(jj) * N + c;
        s.trel[o] = run + inc - v[q];
        s.thist[o] = 0u;
      }
      run += __shfl(inc, kScanLanes - 1, kScanLanes);
    }
  }
  if (live && g == 0) s.base[c] = run;
}

__global__ __launch_bounds__(kSolveWG) void k_scan_base(const SimDev* __restrict__ simp) {
  const SimDev& sim = *simp;
  const SpeciesDev s = sim.sp[blockIdx.x];
  __shared__ uint32_t lds[kSolveWG / 64 + 1];
  const int q = static_cast<int>((*sim.step + 1ull) & 1ull);
  const int N = s.n_cells, W = s.W;
  if (s.mode == kModeFine) return;
  if (s.mode == kModeNone) {
    // unsorted: each (tile, wave) unit's survivors start after those of the units before
    const uint32_t n_surv = array_exclusive_scan_to(s.hist, s.tilerel, s.n_tiles * kWaves, lds);
    if (threadIdx.x == 0) s.n_sorted[q] = n_surv;
    return;
  }
  const uint32_t fc = *s.far_count;
  const uint32_t F = fc < s.far_cap ? fc : s.far_cap;
  if (threadIdx.x == 0 && fc > s.far_cap) atomicOr(sim.error, kErrFarOverflow);
  const uint32_t n_surv = array_exclusive_scan(s.base, N, lds);
  if (F > 0) {
    for (int c = threadIdx.x; c < N; c += blockDim.x) {
      s.far_fill[c] = 0u;
      s.far_base[c] = s.far_cell_cnt[c];
    }
    array_exclusive_scan(s.far_base, N, lds);
    for (uint32_t e = threadIdx.x; e < F; e += blockDim.x) {
      const uint4 v = s.far_list[e];
      if (v.x >= static_cast<uint32_t>(N)) {
        atomicOr(sim.error, kErrState);
        continue;
      }
      const uint32_t pos = s.far_base[v.x] + atomicAdd(&s.far_fill[v.x], 1u);
      if (pos < F) s.far_grouped[pos] = v;
    }
    __syncthreads();  // one workgroup: a barrier makes its global stores visible to it
    // the cell-tile units' offsets in cells that receive far movers from lower tiles
    for (int c = threadIdx.x; c < N; c += blockDim.x) {
      const uint32_t g = s.far_cell_cnt[c];
      if (g == 0u) continue;
      if (g > kMaxFarGroup) {
        atomicOr(sim.error, kErrFarGroup);
        continue;
      }
      const uint32_t gb = s.far_base[c];
      for_covering(s, c, W, [&](int t, int k) {
        uint32_t fb = 0;
        for (uint32_t m = 0; m < g; ++m) fb += s.far_grouped[gb + m].z < static_cast<uint32_t>(t);
        if (fb == 0u) return;
        for (int w = 0; w < kWaves; ++w)
          s.tilerel[(static_cast<size_t>(t) * kWaves + w) * W + k] += fb;
      });
    }
    for (uint32_t e = threadIdx.x; e < F; e += blockDim.x) {
      const uint4 v = s.far_grouped[e];
      if (v.x >= static_cast<uint32_t>(N) || v.y >= s.cap) continue;
      const int c = static_cast<int>(v.x);
      const uint32_t g = s.far_cell_cnt[c];
      const uint32_t gb = s.far_base[c];
      if (g > kMaxFarGroup) continue;
      uint32_t rank = 0;
      for (uint32_t m = 0; m < g; ++m) rank += s.far_grouped[gb + m].y < v.y;
      uint32_t nb = 0;
      for_covering(s, c, W, [&](int t, int k) {
        if (static_cast<uint32_t>(t) < v.z)
          for (int w = 0; w < kWaves; ++w)
            nb += s.hist[(static_cast<size_t>(t) * kWaves + w) * W + k];
      });
      s.far_dest[v.y] = s.base[c] + rank + nb;
    }
  }
  uint32_t GM* cs = s.cell_start + q * (N + 1);
  {
    constexpr int kC = 8;  // cells of a thread copied at once
    const int B = static_cast<int>(blockDim.x);
    for (int c0 = threadIdx.x; c0 < N; c0 += kC * B) {
      uint32_t v[kC];
#pragma unroll
      for (int k = 0; k < kC; ++k) v[k] = c0 + k * B < N ? s.base[c0 + k * B] : 0u;
#pragma unroll
      for (int k = 0; k < kC; ++k)
        if (c0 + k * B < N) cs[c0 + k * B] = v[k];
    }
  }
  if (threadIdx.x == 0) {
    cs[N] = n_surv;
    s.n_sorted[q] = n_surv;
  }
}
// ====================================================================================
// k_main: the fused particle pass of one tile.  Each wave streams its piece of the tile:
// push + gather (Sec. 3.6), walls and EEDF (Sec. 2), the stable scatter of the survivors
// (its own running offset per window slot, so the output order is the one the histograms
// promised), the null-collision test (candidates listed with their post-push state),
// and the linear deposit into its own LDS window (Sec. 3.4).  Tail tiles rank their
// particles per cell against their global tail rows.
// ====================================================================================
constexpr uint32_t kNoDest = 0xFFFFFFFFu;
constexpr int kFarQ = 64;           // per-wave queue of far movers (one chunk always fits)

// Copies of the tile's deposit window: lane l adds into copy l mod kDepCopies, so one
// atomic instruction has few lanes on any one address (the 64 particles of a chunk come
// from one cell and land in a handful of slots).
constexpr int kDepCopies = 8;

template <class P, bool kLag>
struct MainShared {
  using real = typename Part<P>::real;
  // the field at the tile's nodes (lagged sort: at the nodes of its whole window, since a
  // record's present cell may lie up to D cells outside the tile)
  real Elds[(kLag ? kMaxWindow : kMaxCellsPerTile) + 1];
  uint32_t off[kWaves][kMaxWindow];  // next output index of each (wave, window slot)
  // sum of the fixed-point right-node weights F of the near particles of each window slot,
  // in kDepCopies copies shared by the waves; the slot's particle count comes from the
  // tile's histogram rows, so the left node's share (count * one - sum F) needs no atomics
  unsigned long long dep[kDepCopies][kMaxWindow];
  uint32_t cnt[kMaxWindow];          // fine sort: near particles per window slot
  uint32_t eedf[kMaxEedfBins + 1];
  double wst[kWaves][4];             // per-wave sums: kinetic, momentum, absorbed energy x2
  uint32_t wcnt[kWaves][8];          // per-wave counts: absorbed, emitted, reflected x2, pushed, alive
  uint32_t err;                      // error bits found by the tile
  // far movers deferred to the end of each wave's loop: index, cell, position word,
  // vx, vy, vz (FP32 bits), id, candidate entry; FP64 keeps the reals in fqd and only
  // index, cell, id, candidate entry here
  uint32_t fq[kWaves][kFarQ][std::is_same<real, double>::value ? 4 : 8];
  double fqd[kWaves][std::is_same<real, double>::value ? kFarQ : 1][4];
};

// One collision test of a candidate (Sec. 3.8): returns the channel (0 null).
template <class P>
__device__ int collide(const SpeciesDev& s, uint32_t id, uint32_t step, uint32_t w1,
                       uint32_t w2, typename Part<P>::real v[3], typename Part<P>::real vs[3],
                       typename Part<P>::real vi[3]) {
  using real = typename Part<P>::real;
  const double r = u53(w1, w2) * s.nu0;
  if (s.sp == 0) {
    const double vx = v[0], vy = v[1], vz = v[2];
    const double v2 = vx * vx + vy * vy + vz * vz;
    const double eps = s.energy_c * v2;
    const double speed = sqrt(v2) * s.vunit;
    double el, ex, iz;
    xsec_electron(s.xsec, eps, s.sigma_const, el, ex, iz);
    const double nu_el = s.n_gas * el * speed;
    const double nu_ex = s.n_gas * ex * speed;
    const double nu_iz = s.n_gas * iz * speed;
    int ch = 0;
    if (r < nu_el) ch = 1;
    else if (r < nu_el + nu_ex) ch = 2;
    else if (r < nu_el + nu_ex + nu_iz) ch = 3;
    if (ch == 0) return 0;
    const uint4 b1 = philox(id, step, 1u, 0u, s.key0, s.key1);
    if (ch == 1) {
      if constexpr (std::is_same<P, P32>::value) {
        float n0, n1, n2;
        direction32(b1, n0, n1, n2);
        const float vm = sqrtf(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
        const float cchi = (v[0] * n0 + v[1] * n1 + v[2] * n2) / vm;
        const float fac = 1.0f - 2.0f * static_cast<float>(s.mass_ratio) * (1.0f - cchi);
        const float vn = vm * sqrtf(fac);
        v[0] = vn * n0;
        v[1] = vn * n1;
        v[2] = vn * n2;
      } else {
        double n0, n1, n2;
        direction64(b1, n0, n1, n2);
        const double vm = sqrt(v2);
        const double cchi = (vx * n0 + vy * n1 + vz * n2) / vm;
        const double ep = eps * (1.0 - 2.0 * s.mass_ratio * (1.0 - cchi));
        const double vn = sqrt(ep / s.energy_c);
        v[0] = vn * n0;
        v[1] = vn * n1;
        v[2] = vn * n2;
      }
    } else if (ch == 2) {
      double n0, n1, n2;
      direction64(b1, n0, n1, n2);
      const double vn = sqrt((eps - kExcEv) / s.energy_c);
      v[0] = static_cast<real>(vn * n0);
      v[1] = static_cast<real>(vn * n1);
      v[2] = static_cast<real>(vn * n2);
    } else {
      // draws taken one block at a time (blocks 2..5) to keep few values live
      const double er = eps - kIonEv;
      const uint4 b2 = philox(id, step, 2u, 0u, s.key0, s.key1);
      const double es = u53(b2.x, b2.y) * er;
      const double epr = er - es;
      double n0, n1, n2;
      direction64(b1, n0, n1, n2);
      const double vp = sqrt(epr / s.energy_c);
      v[0] = static_cast<real>(vp * n0);
      v[1] = static_cast<real>(vp * n1);
      v[2] = static_cast<real>(vp * n2);
      direction64(philox(id, step, 3u, 0u, s.key0, s.key1), n0, n1, n2);
      const double vsm = sqrt(es / s.energy_c);
      vs[0] = static_cast<real>(vsm * n0);
      vs[1] = static_cast<real>(vsm * n1);
      vs[2] = static_cast<real>(vsm * n2);
      double z0, z1, z2, z3;
      normals64(philox(id, step, 4u, 0u, s.key0, s.key1), z0, z1);
      vi[0] = static_cast<real>(s.vth_gas * z0);
      vi[1] = static_cast<real>(s.vth_gas * z1);
      normals64(philox(id, step, 5u, 0u, s.key0, s.key1), z2, z3);
      vi[2] = static_cast<real>(s.vth_gas * z2);
    }
    return ch;
  }
  // ion: sample the gas atom, test with the relative speed
  const uint4 b1 = philox(id, step, 1u, 0u, s.key0, s.key1);
  const uint4 b2 = philox(id, step, 2u, 0u, s.key0, s.key1);
  double z0, z1, z2, z3;
  normals64(b1, z0, z1);
  normals64(b2, z2, z3);
  const double vg[3] = {s.vth_gas * z0, s.vth_gas * z1, s.vth_gas * z2};
  const double vv[3] = {v[0], v[1], v[2]};
  const double g[3] = {vv[0] - vg[0], vv[1] - vg[1], vv[2] - vg[2]};
  const double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
  const double eps = s.energy_c * g2;
  const double speed = sqrt(g2) * s.vunit;
  double sis, scx;
  xsec_ion(s.xsec, eps, sis, scx);
  const double nu_is = s.n_gas * sis * speed;
  const double nu_cx = s.n_gas * scx * speed;
  int ch = 0;
  if (r < nu_is) ch = 1;
  else if (r < nu_is + nu_cx) ch = 2;
  if (ch == 1) {
    const uint4 b3 = philox(id, step, 3u, 0u, s.key0, s.key1);
    double n0, n1, n2;
    direction64(b3, n0, n1, n2);
    const double gm = sqrt(g2);
    const double nn[3] = {n0, n1, n2};
    for (int a = 0; a < 3; ++a) v[a] = static_cast<real>(0.5 * (vv[a] + vg[a]) + 0.5 * gm * nn[a]);
  } else if (ch == 2) {
    for (int a = 0; a < 3; ++a) v[a] = static_cast<real>(vg[a]);
  }
  return ch;
}

// Fixed-point weight F = round(f 2^shift) of the right-hand node of a particle's cell
// (Sec. 3.4: the left-hand node takes one - F); pos is the FP32 offset or the FP64 x.
template <class P>
__device__ __forceinline__ unsigned long long right_weight(const SpeciesDev& s,
                                                           typename Part<P>::real pos) {
  double f;
  if constexpr (std::is_same<P, P32>::value) {
    f = static_cast<double>(pos);
  } else {
    f = pos - floor(pos);
  }
  return fix_weight(f, s.dep_scale);
}

// Deposit of one particle in cell d straight into the per-node array (integer atomics).
template <class P>
__device__ __forceinline__ void far_deposit(const SpeciesDev& s, int d,
                                            typename Part<P>::real pos) {
  const unsigned long long F = right_weight<P>(s, pos);
  int dn = d + 1;
  if (s.periodic && dn == s.n_cells) dn = 0;
  atomicAdd(&s.far_w[d], s.dep_one - F);
  atomicAdd(&s.far_w[dn], F);
}

// Chunks of 64 particles per pass of a wave's loop.  Besides keeping loads in flight, a
// longer pass writes more of a wave's output sub-run of each cell at once: the sub-run's
// cache lines are then completed by fewer partial writes spread over less time (measured
// against 1-8 on the large discharge).
template <class P>
struct MainU;
template <>
struct MainU<P32> {
  static constexpr int value = 6;
};
template <>
struct MainU<P64> {
  static constexpr int value = 3;
};

// Four waves per SIMD (at most 128 VGPRs): with fewer, too few loads are in flight.
// kLag: the lagged sort -- the scatter key is the cell stored at the start of the step
// (known before the push), the record written holds the post-push state, and a particle
// absorbed in this step leaves a dead record in the slot the pre-pass counted for it
// (the next step skips it).
template <class P, bool kLag>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(4))) void k_main(
    const SimDev* __restrict__ simp) {
  using real = typename Part<P>::real;
  const SimDev& sim = *simp;
  const int2 tt = sim.tile_table[blockIdx.x];
  const SpeciesDev s = sim.sp[tt.x];
  const DischargeDev dd = sim.ds[s.ds];
  const unsigned long long step = *sim.step;
  const uint32_t step32 = static_cast<uint32_t>(step);
  const int p = static_cast<int>(step & 1ull), pq = p ^ 1;
  const TileRange r = tile_range(s, tt.y, p);
  const int tile = tt.y;
  __shared__ MainShared<P, kLag> sh;
  const int tid = threadIdx.x, lane = tid & 63, wv = wave_id();
  const unsigned long long lt = lanes_below(), gt = lanes_above();
  const bool energy_on = diag_step(dd, step);
  const bool eedf_on = s.sp == 0 && energy_on;
  // after a far-list overflow or an overfull far group, far_dest is not valid this step
  const bool far_ok = (*sim.error & (kErrFarOverflow | kErrFarGroup)) == 0u;
  const uint32_t n_out = s.n_sorted[pq];
  const uint32_t sink = s.cap;  // the extra element past the capacity of every array
  const real GM* E = std::is_same<P, P32>::value ? reinterpret_cast<const real GM*>(dd.E32)
                                                  : reinterpret_cast<const real GM*>(dd.E64);
  if constexpr (kLag) load_field_window_lag<real>(s, E, r, tile, sh.Elds);
  else load_field_window<real>(s, E, r, sh.Elds);
  const int W = s.W;
  if (!r.tail && !r.fine) {
    for (int k = tid; k < kWaves * W; k += kWG) {
      const int w = k / W, kk = k - w * W;
      int c = tile * s.C - s.D + kk;
      if (s.periodic) {
        c %= s.n_cells;
        if (c < 0) c += s.n_cells;
      }
      // running output index of (wave, slot): the start of its sub-run, or the end for
      // a wave that walks backwards
      const size_t o = (static_cast<size_t>(tile) * kWaves + w) * W + kk;
      sh.off[w][kk] = (c >= 0 && c < s.n_cells)
                          ? s.base[c] + s.tilerel[o] + (wave_reversed(r, w) ? s.hist[o] : 0u)
                          : 0u;
    }
  }
  for (int k = tid; k < kDepCopies * W; k += kWG) sh.dep[k / W][k % W] = 0ull;
  const bool lds_counts = r.fine || kLag;  // deposit counts kept in LDS (no histogram rows)
  if (lds_counts)
    for (int k = tid; k < W; k += kWG) sh.cnt[k] = 0u;
  if (eedf_on)
    for (int k = tid; k <= dd.eedf_bins; k += kWG) sh.eedf[k] = 0u;
  if (tid == 0) sh.err = 0u;
  if (tid < kWaves * 4) sh.wst[tid / 4][tid % 4] = 0.0;
  __syncthreads();
  // Sums of the tile are built chunk by chunk in a fixed order (a butterfly over the
  // chunk's lanes, added to the wave's own LDS entry), so no per-lane accumulator stays
  // live through the particle loop.
  uint32_t n_abs0 = 0u, n_abs1 = 0u;    // wave-uniform
  uint32_t n_wall[4] = {0u, 0u, 0u, 0u};  // emitted x2 (k_emit), reflected x2 (wave-uniform)
  uint32_t n_pushed = 0u, n_alive = 0u;  // wave-uniform
  uint32_t n_em = 0u;                   // absorbed ions listed by this wave (emission)
  const WaveRange wr = wave_range(r, wv);
  const RecPtr in = rec_buf(&sim.sp[tt.x], p);
  const RecPtr out = rec_buf(&sim.sp[tt.x], pq);
  uint32_t n_cand = 0;  // candidates of this wave so far (wave-uniform)
  auto load = [&](Part<P>& q, uint32_t i) { q.load(in, i); };

  // Push, walls (reflection, absorption, emission), EEDF, energy sums and the
  // null-collision test: common to both kinds of tile.
  // ek: the lagged sort's window slot of the record's present cell (cell tiles only)
  auto push_and_test = [&](auto tail_tag, auto rev_tag, const Part<P>& q, bool valid, int& d,
                           real& pos, real& vxn, bool& cand, int ek) {
    constexpr bool kTail = decltype(tail_tag)::value;
    constexpr bool kRev = decltype(rev_tag)::value;
    int st = 4;
    if (valid) {
      if constexpr (kLag && !kTail) st = push_particle_lag<P>(s, dd, sh.Elds, ek, q, d, pos, vxn);
      else st = push_particle<P, kTail>(s, dd, sh.Elds, r, q, d, pos, vxn);
    }
    if (energy_on) {  // wave-uniform: after the push, before the walls
      double v1 = 0.0, ke = 0.0, v2 = 0.0;
      if (st < 3) {
        const double vyz = static_cast<double>(q.vy) * static_cast<double>(q.vy) +
                           static_cast<double>(q.vz) * static_cast<double>(q.vz);
        v1 = static_cast<double>(vxn);
        v2 = v1 * v1 + vyz;
        // kinetic energy as the mean of v_x^2 before and after the push
        const double v0 = static_cast<double>(q.vx);
        ke = 0.5 * (v0 * v0 + v1 * v1) + vyz;
      }
      const double sk = wave_sum(ke), sm = wave_sum(v1);
      if (lane == 0) {
        sh.wst[wv][0] += sk;
        sh.wst[wv][1] += sm;
      }
      if (eedf_on && st < 3) {
        const double b = floor(s.energy_c * v2 * dd.eedf_inv_width);
        const int bin = b >= static_cast<double>(dd.eedf_bins) ? dd.eedf_bins : static_cast<int>(b);
        atomicAdd(&sh.eedf[bin], 1u);
      }
    }
    if (s.t_refl && __ballot(st == 1 || st == 2)) {  // electrons reaching an electrode
      const int st0 = st;
      if (st == 1 || st == 2) st = reflect_at_wall<P>(s, q.id, step32, st, d, pos, vxn);
      n_wall[2] += static_cast<uint32_t>(__popcll(__ballot(st0 == 1 && st == 0)));
      n_wall[3] += static_cast<uint32_t>(__popcll(__ballot(st0 == 2 && st == 0)));
    }
    const unsigned long long m_abs0 = __ballot(st == 1), m_abs1 = __ballot(st == 2);
    if (m_abs0 | m_abs1) {  // wave-uniform
      const double v1 = static_cast<double>(vxn);
      const double vyz = static_cast<double>(q.vy) * static_cast<double>(q.vy) +
                         static_cast<double>(q.vz) * static_cast<double>(q.vz);
      const double e = s.energy_c * (v1 * v1 + vyz);
      const double e0 = wave_sum(st == 1 ? e : 0.0), e1 = wave_sum(st == 2 ? e : 0.0);
      if (lane == 0) {
        sh.wst[wv][2] += e0;
        sh.wst[wv][3] += e1;
      }
      n_abs0 += static_cast<uint32_t>(__popcll(m_abs0));
      n_abs1 += static_cast<uint32_t>(__popcll(m_abs1));
      if (s.t_see) {
        // absorbed ions are listed at their place in this wave's list (input order, like
        // the MCC candidates); k_emit decides their secondary emission
        const unsigned long long am = m_abs0 | m_abs1;
        if (st == 1 || st == 2) {
          uint32_t e;
          if constexpr (kRev) e = wr.hi - 1u - n_em - static_cast<uint32_t>(__popcll(am & gt));
          else e = wr.lo + n_em + static_cast<uint32_t>(__popcll(am & lt));
          if (e < s.cap) s.ab_list[e] = make_uint2(q.id, static_cast<uint32_t>(st));
        }
        n_em += static_cast<uint32_t>(__popcll(am));
      }
    }
    n_pushed += static_cast<uint32_t>(__popcll(__ballot(st < 4)));
    n_alive += static_cast<uint32_t>(__popcll(__ballot(st == 0)));
    if (st == 3) atomicOr(&sh.err, kErrNonfinite);
    cand = false;
    if (st == 0 && s.t0 != 0u) cand = philox(q.id, step32, 0u, 0u, s.key0, s.key1).x < s.t0;
    return st;
  };
  // A candidate's entry (input order within the wave's piece) for k_collide; lanes that
  // are not candidates write the sink entry, so the stores are not branched over.
  // A deferred candidate (a far mover) keeps its place in the list but its entry is
  // written when its output index is known.
  // A backward wave fills its list from the end of its piece, so the list is always in
  // input order: [lo, lo + n) forwards, [hi - n, hi) backwards.
  auto list_candidate = [&](auto rev_tag, bool cand, bool defer, uint32_t dst, const Part<P>& q,
                            int d, real pos, real vxn) {
    constexpr bool kRev = decltype(rev_tag)::value;
    const unsigned long long cm = __ballot(cand);
    uint32_t e = sink;
    if (cand) {
      if constexpr (kRev)
        e = wr.hi - 1u - n_cand - static_cast<uint32_t>(__popcll(cm & gt));
      else
        e = wr.lo + n_cand + static_cast<uint32_t>(__popcll(cm & lt));
    }
    cand_store<P>(s.cand, defer ? sink : e, dst, q.id, d, pos, vxn, q.vy, q.vz);
    n_cand += static_cast<uint32_t>(__popcll(cm));
    return e;
  };
  auto write_candidate = [&](uint32_t e, uint32_t dst, uint32_t id, int d, real pos, real vx,
                             real vy, real vz) {
    cand_store<P>(s.cand, e, dst, id, d, pos, vx, vy, vz);
  };

  if (r.fine) {
    // Fine sort (the paper's pusher, Sec. 3.6 with Sec. 3.7 steps 1a/1b after it): every
    // particle stays in its slot; survivors get their new cell, offset and v_x, absorbed
    // ones a dead marker; k_fine_sort1..3 then move the ones that left the sorting cell.
    uint32_t alive = 0u;  // wave-uniform
    stream_range<Part<P>, MainU<P>::value>(
        wr.lo, wr.hi, load, [&](const Part<P>& q, uint32_t i, bool valid) {
          int d = 0;
          real pos = real(0), vxn = real(0);
          bool cand;
          const int st = push_and_test(std::false_type{}, std::false_type{}, q, valid, d, pos,
                                       vxn, cand, -1);
          store_in_place<P>(out, valid ? i : sink, st == 0, d, pos, vxn);
          list_candidate(std::false_type{}, cand, false, i, q, d, pos, vxn);
          if (st == 0) {
            const int k = window_slot(s, tile, d);
            if (k >= 0) {
              atomicAdd(&sh.cnt[k], 1u);
              atomicAdd(&sh.dep[lane & (kDepCopies - 1)][k], right_weight<P>(s, pos));
            } else {
              far_deposit<P>(s, d, pos);
            }
          }
          alive += static_cast<uint32_t>(__popcll(__ballot(st == 0)));
        });
    if (lane == 0 && alive) atomicAdd(&s.n_sorted[pq], alive);
  } else if (!r.tail) {
    // Far movers (beyond the window) wait in a per-wave LDS queue until the loop is
    // done: their output index is a global load, and a load inside the loop would make
    // the loop wait for the next chunk's loads too.
    uint32_t qn = 0;  // wave-uniform
    constexpr int kQid = std::is_same<P, P32>::value ? 6 : 2;  // id word (then candidate entry)
    auto flush = [&]() {  // one queue entry per lane (the queue holds at most 64)
      const uint32_t j = static_cast<uint32_t>(lane);
      if (j < qn) {
        const uint32_t* f = sh.fq[wv][j];
        const uint32_t i = f[0];
        const int d = static_cast<int>(f[1]);
        real pos, vx, vy, vz;
        if constexpr (std::is_same<P, P32>::value) {
          pos = __uint_as_float(f[2]);
          vx = __uint_as_float(f[3]);
          vy = __uint_as_float(f[4]);
          vz = __uint_as_float(f[5]);
        } else {
          pos = sh.fqd[wv][j][0];
          vx = sh.fqd[wv][j][1];
          vy = sh.fqd[wv][j][2];
          vz = sh.fqd[wv][j][3];
        }
        uint32_t dst = far_ok && i < s.cap ? s.far_dest[i] : kNoDest;
        if (dst != kNoDest && dst >= n_out) {
          atomicOr(&sh.err, kErrState);
          dst = kNoDest;
        }
        if (dst != kNoDest) {
          store_record<P>(out, dst, d, pos, vx, vy, vz, f[kQid]);
          if (!kLag) far_deposit<P>(s, d, pos);  // lagged: deposited in the loop
        }
        if (f[kQid + 1] != kNoDest) write_candidate(f[kQid + 1], dst, f[kQid], d, pos, vx, vy, vz);
      }
      qn = 0;
    };
    auto cell_body = [&](auto rev_tag, const Part<P>& q, uint32_t i, bool valid) {
      constexpr bool kRev = decltype(rev_tag)::value;
      int d = 0;
      real pos = real(0), vxn = real(0);
      bool cand;
      int key = 0;
      int k = -1;
      if constexpr (kLag) {
        key = valid ? stored_cell<P>(q) : -1;
        valid = key >= 0 && key < s.n_cells;  // dead records are skipped
        k = valid ? window_slot(s, tile, key) : -1;
      }
      const int st = push_and_test(std::false_type{}, rev_tag, q, valid, d, pos, vxn, cand, k);
      if constexpr (!kLag) k = st == 0 ? window_slot(s, tile, d) : -1;
      const bool near = k >= 0;
      // the record written: the post-push state, or a dead record (lagged sort only)
      int d_out = d;
      real pos_out = pos;
      if constexpr (kLag) {
        if (st != 0) {
          d_out = -1;
          if constexpr (std::is_same<P, P64>::value) pos_out = -1.0;
        }
      }
      // stable rank inside this wave's unit of the order (from the unit's end backwards
      // for a backward wave)
      const unsigned long long m = match_key_few(k, near);
      const int rank = __popcll(m & (kRev ? gt : lt));
      uint32_t dst = sink;
      if (near) {
        if constexpr (kRev) dst = sh.off[wv][k] - 1u - static_cast<uint32_t>(rank);
        else dst = sh.off[wv][k] + static_cast<uint32_t>(rank);
      }
      if (near && rank == 0) {
        if constexpr (kRev) sh.off[wv][k] = dst + 1u - static_cast<uint32_t>(__popcll(m));
        else sh.off[wv][k] = dst + static_cast<uint32_t>(__popcll(m));
      }
      if (near && dst >= n_out) {
        atomicOr(&sh.err, kErrState);
        dst = sink;
      }
      store_record<P>(out, dst, d_out, pos_out, vxn, q.vy, q.vz, q.id);
      const bool far = kLag ? (valid && !near) : (st == 0 && !near);
      const uint32_t e = list_candidate(rev_tag, cand, far, near ? dst : kNoDest, q, d, pos, vxn);
      const unsigned long long fm = __ballot(far);
      if (fm) {
        if (qn + static_cast<uint32_t>(__popcll(fm)) > static_cast<uint32_t>(kFarQ)) flush();
        if (far) {
          const uint32_t j = qn + static_cast<uint32_t>(__popcll(fm & lt));
          uint32_t* f = sh.fq[wv][j];
          f[0] = i;
          f[1] = static_cast<uint32_t>(d_out);
          if constexpr (std::is_same<P, P32>::value) {
            f[2] = __float_as_uint(pos_out);
            f[3] = __float_as_uint(vxn);
            f[4] = __float_as_uint(q.vy);
            f[5] = __float_as_uint(q.vz);
          } else {
            sh.fqd[wv][j][0] = pos_out;
            sh.fqd[wv][j][1] = vxn;
            sh.fqd[wv][j][2] = q.vy;
            sh.fqd[wv][j][3] = q.vz;
          }
          f[kQid] = q.id;
          f[kQid + 1] = cand ? e : kNoDest;
        }
        qn += static_cast<uint32_t>(__popcll(fm));
      }
      // deposit of the near particles: the right-node weight into the slot's sum (LDS
      // integer atomics: exact in any order; the LDS pipe absorbs the same-slot conflicts).
      // Lagged: the deposit slot is the post-push cell's, not the scatter slot.
      if constexpr (kLag) {
        // the slot's count: one LDS add per group of lanes that share the slot
        const int kd = st == 0 ? window_slot(s, tile, d) : -1;
        const bool dn = kd >= 0;
        const unsigned long long md = match_key_few(kd, dn);
        if (dn && (md & lt) == 0ull) atomicAdd(&sh.cnt[kd], static_cast<uint32_t>(__popcll(md)));
        if (dn) atomicAdd(&sh.dep[lane & (kDepCopies - 1)][kd], right_weight<P>(s, pos));
        else if (st == 0) far_deposit<P>(s, d, pos);
      } else {
        if (near) atomicAdd(&sh.dep[lane & (kDepCopies - 1)][k], right_weight<P>(s, pos));
      }
    };
    if (wave_reversed(r, wv)) {
      stream_range_rev<Part<P>, MainU<P>::value>(
          wr.lo, wr.hi, load, [&](const Part<P>& q, uint32_t i, bool valid) {
            cell_body(std::true_type{}, q, i, valid);
          });
    } else {
      stream_range<Part<P>, MainU<P>::value>(
          wr.lo, wr.hi, load, [&](const Part<P>& q, uint32_t i, bool valid) {
            cell_body(std::false_type{}, q, i, valid);
          });
    }
    if (qn) flush();
  } else if (s.mode == kModeNone) {
    // Unsorted (the variant of Sec. 3.2 without fine sorting): survivors keep their input
    // order, compacted after the survivors of the units before; every deposit goes
    // straight into the node array with integer atomics.
    uint32_t run = 0u;  // survivors written by this wave so far (wave-uniform)
    const uint32_t ubase = s.tilerel[tile * kWaves + wv];
    stream_range<Part<P>, MainU<P>::value>(
        wr.lo, wr.hi, load, [&](const Part<P>& q, uint32_t i, bool valid) {
          int d = 0;
          real pos = real(0), vxn = real(0);
          bool cand;
          const int st = push_and_test(std::true_type{}, std::false_type{}, q, valid, d, pos, vxn,
                                       cand, -1);
          const unsigned long long m = __ballot(st == 0);
          uint32_t dst = kNoDest;
          if (st == 0) {
            dst = ubase + run + static_cast<uint32_t>(__popcll(m & lt));
            if (dst >= n_out) {
              atomicOr(&sh.err, kErrState);
              dst = kNoDest;
            }
          }
          store_record<P>(out, dst == kNoDest ? sink : dst, d, pos, vxn, q.vy, q.vz, q.id);
          list_candidate(std::false_type{}, cand, false, dst, q, d, pos, vxn);
          if (dst != kNoDest) far_deposit<P>(s, d, pos);
          run += static_cast<uint32_t>(__popcll(m));
        });
  } else {
    // Tail tile: rank per cell against this wave's global tail row, one returning atomic
    // per (cell, chunk) by the group leader; deposits go to the far array.
    uint32_t GM* trow = s.trel + static_cast<size_t>((tile - s.n_tiles) * kWaves + wv) * s.n_cells;
    const int nbits = key_bits(s.n_cells);
    stream_range<Part<P>, MainU<P>::value>(
        wr.lo, wr.hi, load, [&](const Part<P>& q, uint32_t i, bool valid) {
          int d = 0;
          real pos = real(0), vxn = real(0);
          bool cand;
          int key = 0;
          if constexpr (kLag) {
            key = valid ? stored_cell<P>(q) : -1;
            valid = key >= 0 && key < s.n_cells;
          }
          const int st = push_and_test(std::true_type{}, std::false_type{}, q, valid, d, pos, vxn,
                                       cand, -1);
          const bool act = kLag ? valid : st == 0;
          if constexpr (!kLag) key = d;
          const unsigned long long mc = match_key(key, act, nbits);
          const int rank = __popcll(mc & lt);
          uint32_t old = 0u;
          if (act && rank == 0) old = atomicAdd(&trow[key], static_cast<uint32_t>(__popcll(mc)));
          const int leader = act ? __ffsll(static_cast<long long>(mc)) - 1 : lane;
          old = __shfl(old, leader, 64);
          uint32_t dst = kNoDest;
          if (act) {
            dst = s.base[key] + old + static_cast<uint32_t>(rank);
            if (dst >= n_out) {
              atomicOr(&sh.err, kErrState);
              dst = kNoDest;
            }
          }
          int d_out = d;
          real pos_out = pos;
          if constexpr (kLag) {
            if (st != 0) {
              d_out = -1;
              if constexpr (std::is_same<P, P64>::value) pos_out = -1.0;
            }
          }
          store_record<P>(out, dst == kNoDest ? sink : dst, d_out, pos_out, vxn, q.vy, q.vz, q.id);
          list_candidate(std::false_type{}, cand, false, st == 0 ? dst : kNoDest, q, d, pos, vxn);
          if (dst != kNoDest && st == 0) far_deposit<P>(s, d, pos);
        });
  }
  if (lane == 0) {
    s.cand_cnt[tile * kWaves + wv] = n_cand;
    sh.wcnt[wv][0] = n_abs0;
    sh.wcnt[wv][1] = n_abs1;
    for (int k = 0; k < 4; ++k) sh.wcnt[wv][2 + k] = n_wall[k];
    sh.wcnt[wv][6] = n_pushed;
    sh.wcnt[wv][7] = n_alive;
    if (s.t_see) {
      s.ab_cnt[tile * kWaves + wv] = n_em;
      s.em_lo[tile * kWaves + wv] = wave_reversed(r, wv) ? wr.hi - n_em : wr.lo;
    }
  }
  __syncthreads();
  // tile epilogue: node j of the window takes count(j) one - sumF(j) from slot j and
  // sumF(j - 1) from slot j - 1
  if (!r.tail) {
    unsigned long long GM* part = s.partial + static_cast<size_t>(tile) * (W + 1);
    const uint32_t GM* hrow = s.hist + static_cast<size_t>(tile) * kWaves * W;
    for (int j = tid; j <= W; j += kWG) {
      unsigned long long v = 0ull;
      if (j < W) {
        uint32_t cnt = 0u;
        if (lds_counts) {
          cnt = sh.cnt[j];
        } else {
#pragma unroll
          for (int w = 0; w < kWaves; ++w) cnt += hrow[w * W + j];
        }
        unsigned long long f = 0ull;
#pragma unroll
        for (int c = 0; c < kDepCopies; ++c) f += sh.dep[c][j];
        v = static_cast<unsigned long long>(cnt) * s.dep_one - f;
      }
      if (j > 0) {
#pragma unroll
        for (int c = 0; c < kDepCopies; ++c) v += sh.dep[c][j - 1];
      }
      part[j] = v;
    }
  }
  if (tid == 0) {
    if (sh.err) atomicOr(sim.error, sh.err);
    // the tile's sums, waves in order: energies on energy steps; pushed and surviving
    // counts; wall events (rare: tiles at the walls) into the tile's event record, marked
    // in the event bitmap
    TileStats ts{};
    double ke = 0.0, mom = 0.0;
    uint32_t pushed = 0u, alive = 0u;
    for (int w = 0; w < kWaves; ++w) {
      ke += sh.wst[w][0];
      mom += sh.wst[w][1];
      ts.abs_e[0] += sh.wst[w][2];
      ts.abs_e[1] += sh.wst[w][3];
      ts.abs_n[0] += sh.wcnt[w][0];
      ts.abs_n[1] += sh.wcnt[w][1];
      ts.refl[0] += sh.wcnt[w][4];
      ts.refl[1] += sh.wcnt[w][5];
      pushed += sh.wcnt[w][6];
      alive += sh.wcnt[w][7];
    }
    if (energy_on) {
      s.tke[2 * tile] = ke;
      s.tke[2 * tile + 1] = mom;
    }
    s.tcount[tile] = make_uint2(pushed, alive);
    if (ts.abs_n[0] | ts.abs_n[1] | ts.refl[0] | ts.refl[1]) {
      s.tstats[tile] = ts;  // emit[] is filled in by k_emit
      atomicOr(&s.ev_bits[tile >> 5], 1u << (tile & 31));
    }
  }
  if (eedf_on)
    for (int k = tid; k <= dd.eedf_bins; k += kWG)
      if (sh.eedf[k]) atomicAdd(&dd.eedf[k], static_cast<unsigned long long>(sh.eedf[k]));
}

// ====================================================================================
// k_collide: modified null-collision MCC (Sec. 3.8, eq. null_collision) of the candidates
// k_main found (word 0 of the particle's Philox block 0 below floor(P0 2^32)).  A
// workgroup of kT threads takes a part of the candidates in input order (the tiles' waves'
// lists one after the other), kT at a time, so the collision path runs on full waves:
// * an electron tile's list (up to a few thousand candidates) by one workgroup; with few
//   electron tiles it has eight waves: the pass is a long dependent chain per lane, and
//   eight waves per tile keep the SIMDs busier than four (splitting the list over
//   workgroups instead would need the births' parent order across workgroups);
// * the ion tiles' lists (a handful of candidates each) up to kIonGroup tiles at a time:
//   every workgroup pays the collision path's chain once per pass, however few lanes it
//   has.
// k_main stored each candidate's post-push state beside its sorted slot; the
// post-collision velocity is written to that slot.  (Carrying words 1 and 2 of block 0
// in the record instead of computing the block again was measured slower: `k_main`
// held them live and lost 9-13 us, the MCC pass gained under 1 us.)  Births
// (electron ionization) are staged in the order of their parents (= input order);
// k_finalize appends and deposits them.
// ====================================================================================
template <class P, int kT>
__global__ __launch_bounds__(kT) void k_collide(const SimDev* __restrict__ simp) {
  using real = typename Part<P>::real;
  const SimDev& sim = *simp;
  const int4 cw = sim.collide_table[blockIdx.x];  // (species, first tile, tiles, 0)
  const SpeciesDev s = sim.sp[cw.x];
  const unsigned long long step = *sim.step;
  const uint32_t step32 = static_cast<uint32_t>(step);
  const int p = static_cast<int>(step & 1ull), pq = p ^ 1;
  const int tile = cw.y;
  const bool electrons = s.sp == 0;
  const TileRange r = tile_range(s, tile, p);
  // the (tile, wave) list segments of this workgroup's tiles, in input order
  constexpr int kSeg = kIonGroup * kWaves;
  static_assert(kSeg <= kT, "one thread per list segment");
  __shared__ uint32_t sg_lo[kSeg], sg_pre[kSeg + 1];
  __shared__ uint32_t bq[kT / 64 + 1];
  __shared__ uint32_t coll[3];
  const int tid = threadIdx.x;
  const int nseg = cw.z * kWaves;
  {
    uint32_t nc = 0u, lo = 0u;
    if (tid < nseg) {
      const int g = tid / kWaves, w = tid - g * kWaves;
      const TileRange rg = tile_range(s, tile + g, p);
      const WaveRange wr = piece_range(rg, w);  // w differs between the lanes
      nc = s.cand_cnt[(tile + g) * kWaves + w];
      lo = wave_reversed(rg, w) ? wr.hi - nc : wr.lo;  // see list_candidate in k_main
    }
    uint32_t tot;
    const uint32_t pre = block_exclusive_scan<uint32_t>(nc, bq, tot);
    if (tid < kSeg) {
      sg_lo[tid] = lo;
      sg_pre[tid] = pre;
    }
    if (tid == 0) sg_pre[kSeg] = tot;
  }
  if (tid == 0) coll[0] = coll[1] = coll[2] = 0u;
  __syncthreads();
  const uint32_t n = sg_pre[kSeg];
  if (n == 0u) {
    if (tid == 0 && electrons) {
      s.birth_cnt[tile] = 0u;
      s.stage_first[tile] = r.lo;
    }
    return;
  }
  uint32_t births = 0u;  // births staged so far (the same in every thread)
  const RecPtr out = rec_buf(&sim.sp[cw.x], pq);
  const RecPtr stage_e = rec_stage(&sim.sp[cw.x], 0);
  const RecPtr stage_i = rec_stage(&sim.sp[cw.x], 1);
  for (uint32_t b = 0; b < n; b += kT) {
    const uint32_t e = b + tid;
    bool born = false;
    uint32_t parent = 0u;
    int d = 0;
    real pos = real(0);
    real vs[3] = {real(0), real(0), real(0)}, vi[3] = {real(0), real(0), real(0)};
    if (e < n) {
      int w = 0;  // the last segment that starts at or before e (a non-empty one)
#pragma unroll
      for (int st = kSeg / 2; st >= 1; st >>= 1)
        if (w + st < nseg && sg_pre[w + st] <= e) w += st;
      const uint32_t idx = sg_lo[w] + (e - sg_pre[w]);
      real v[3] = {real(0), real(0), real(0)};
      const uint4 c = idx < s.cap ? cand_load<P>(s.cand, idx, pos, v)
                                  : make_uint4(kNoDest, 0u, 0u, 0u);
      const uint32_t dst = c.x;
      if (dst != kNoDest && dst < s.cap) {
        if constexpr (std::is_same<P, P32>::value) {
          d = static_cast<int>(c.z);
        } else {
          d = static_cast<int>(floor(pos));
        }
        const uint4 b0 = philox(c.y, step32, 0u, 0u, s.key0, s.key1);
        const int ch = collide<P>(s, c.y, step32, b0.y, b0.z, v, vs, vi);
        if (ch > 0) {
          atomicAdd(&coll[ch - 1], 1u);
          store_velocity<P>(out, dst, v);
          born = s.sp == 0 && ch == 3;
          parent = c.y;
        }
      }
    }
    // ionizations are rare: most passes have none and need no scan for the staging order
    const uint32_t total = static_cast<uint32_t>(__syncthreads_count(born ? 1 : 0));
    uint32_t pre = 0u;
    if (total) {
      uint32_t t2;
      pre = block_exclusive_scan<uint32_t>(born ? 1u : 0u, bq, t2);
    }
    if (born) {
      const uint32_t si = r.lo + births + pre;
      if (si < s.cap) {
        // (deposited by k_finalize once it is known that the birth fits)
        store_record<P, false>(stage_e, si, d, pos, vs[0], vs[1], vs[2], 0u);
        store_record<P, false>(stage_i, si, d, pos, vi[0], vi[1], vi[2], 0u);
        if (s.mode == kModeFine) s.fpid[si] = parent;  // fine sort: ids by parent id
      } else {
        atomicOr(sim.error, kErrState);
      }
    }
    births += total;
  }
  if (tid == 0) {
    if (electrons) {
      s.birth_cnt[tile] = births;
      s.stage_first[tile] = r.lo;
    }
    for (int k = 0; k < 3; ++k)
      if (coll[k]) atomicAdd(&s.collisions[k], static_cast<unsigned long long>(coll[k]));
  }
}
// ====================================================================================
// k_emit: secondary emission (Sec. 2: electrons inserted at the boundaries).  One wave per
// ion tile walks the absorbed-ion lists k_main left in its (tile, wave) units: an ion emits
// iff word 0 of its Philox block 6 is below floor(gamma 2^32) and the electron's start
// position (blocks 7, 8; device_common.h, emitted_electron) is inside the box.  The
// electrons are stored compacted in list order at the front of the unit's list range, and
// each unit's count goes to k_birth_scan, which numbers them after the ionisation births.
// ====================================================================================
template <class P>
__global__ __launch_bounds__(kWG) void k_emit(const SimDev* __restrict__ simp) {
  using real = typename Part<P>::real;
  const SimDev& sim = *simp;
  const int g = blockIdx.x * kWaves + wave_id();  // one wave per tile
  if (g >= sim.total_tiles) return;
  const int2 tt = sim.tile_table[g];
  const SpeciesDev s = sim.sp[tt.x];
  if (!s.t_see) return;
  const uint32_t step32 = static_cast<uint32_t>(*sim.step);
  const int lane = threadIdx.x & 63;
  const unsigned long long lt = lanes_below();
  RecPtr out;
#pragma unroll
  for (int k = 0; k < 6; ++k) out.f[k] = s.em_stage[k];
  out.boff4 = out.boff8 = out.boffv = 0u;
  uint32_t n_wall[2] = {0u, 0u};
  for (int w = 0; w < kWaves; ++w) {
    const int unit = tt.y * kWaves + w;
    const uint32_t n = s.ab_cnt[unit], lo = s.em_lo[unit];
    uint32_t em = 0u;  // wave-uniform
    for (uint32_t b = 0; b < n; b += 64u) {
      const uint32_t k = b + static_cast<uint32_t>(lane);
      bool emit = false;
      int st = 0;
      double xe = 0.0, ve[3] = {0.0, 0.0, 0.0};
      if (k < n && lo + k < s.cap) {
        const uint2 a = s.ab_list[lo + k];
        st = static_cast<int>(a.y);
        if (philox(a.x, step32, 6u, 0u, s.key0, s.key1).x < s.t_see)
          emit = emitted_electron(s.n_cells, st, s.vth_see,
                                  philox(a.x, step32, 7u, 0u, s.key0, s.key1),
                                  philox(a.x, step32, 8u, 0u, s.key0, s.key1), xe, ve);
      }
      const unsigned long long m = __ballot(emit);
      if (emit) {
        const uint32_t e = lo + em + static_cast<uint32_t>(__popcll(m & lt));
        const double c = floor(xe);
        if constexpr (std::is_same<P, P32>::value)
          store_record<P, false>(out, e, static_cast<int>(c), __double2float_rz(xe - c),
                                 static_cast<float>(ve[0]), static_cast<float>(ve[1]),
                                 static_cast<float>(ve[2]), 0u);
        else
          store_record<P, false>(out, e, static_cast<int>(c), xe, static_cast<real>(ve[0]),
                                 static_cast<real>(ve[1]), static_cast<real>(ve[2]), 0u);
      }
      em += static_cast<uint32_t>(__popcll(m));
      n_wall[0] += static_cast<uint32_t>(__popcll(__ballot(emit && st == 1)));
      n_wall[1] += static_cast<uint32_t>(__popcll(__ballot(emit && st == 2)));
    }
    if (lane == 0) s.em_cnt[unit] = em;
  }
  if (lane == 0) {
    s.tstats[tt.y].emit[0] = n_wall[0];
    s.tstats[tt.y].emit[1] = n_wall[1];
  }
}

// ====================================================================================
// Births are appended after the sorted survivors in the order of their parents' input
// index (the electron tiles are in index order and each keeps its births in index
// order); the children take the next ids of their species.
// k_birth_scan (one workgroup per discharge) scans the electron tiles' birth counts,
// settles how many births fit and their first id, and advances the step counter;
// k_finalize (one wave per tile, all tiles) copies each electron tile's staged births --
// electrons and ions -- to their places and deposits those that fit (a birth dropped for
// want of capacity leaves no charge behind).
// ====================================================================================
__global__ __launch_bounds__(kSolveWG) void k_birth_scan(const SimDev* __restrict__ simp) {
  const SimDev& sim = *simp;
  const DischargeDev dd = sim.ds[blockIdx.x];
  const SpeciesDev se = sim.sp[dd.spec0];
  const SpeciesDev sion = sim.sp[dd.spec0 + 1];
  __shared__ uint32_t lds[kSolveWG / 64 + 1];
  const unsigned long long step = *sim.step;
  const int q = static_cast<int>((step + 1ull) & 1ull);
  const int nt = se.n_tiles + se.n_tail;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // The step's tallies of both species, each combined in a fixed order:
  // * pushed and surviving particles of every tile (integers: wave sums, then the waves);
  // * on energy steps, the kinetic energy and momentum of every tile: thread t takes tiles
  //   t, t + B, ... in order, a butterfly inside each wave, then the waves in order;
  // * wall events: only the tiles marked in the event bitmap (a few, at the walls).  Each
  //   event tile gets its rank in tile order from a scan of the bitmap words' bit counts,
  //   its record goes to that place of an LDS list, and the settling thread adds the list
  //   in order (past kEvCap entries it reads the rest from global memory in tile order).
  const bool energy = diag_step(dd, step);
  constexpr int kD = 2, kU = 2;  // ke, mom | pushed, alive
  constexpr int kEvCap = 128;
  __shared__ double wd[2][kSolveWG / 64][kD];
  __shared__ uint32_t wu[2][kSolveWG / 64][kU];
  __shared__ TileStats evl[2][kEvCap];
  __shared__ uint32_t ev_n[2];
  {
    const int B = static_cast<int>(blockDim.x);
    const int tid = static_cast<int>(threadIdx.x);
    const int ntl[2] = {se.n_tiles + se.n_tail, sion.n_tiles + sion.n_tail};
    const uint2 GM* tc[2] = {se.tcount, sion.tcount};
    const uint32_t GM* eb[2] = {se.ev_bits, sion.ev_bits};
    // the counts of both species and this thread's bitmap words, all loads issued at once
    constexpr int kT = 8;  // a thread's tiles read at once
    uint32_t pushed[2] = {0u, 0u}, alive[2] = {0u, 0u};
    uint32_t word[2] = {0u, 0u};  // bitmap word tid (one per thread up to 32 B tiles)
    const int nw[2] = {(ntl[0] + 31) / 32, (ntl[1] + 31) / 32};
    const bool one_word = nw[0] <= B && nw[1] <= B;
    {
      uint2 c[2][kT];
#pragma unroll
      for (int sp = 0; sp < 2; ++sp) {
#pragma unroll
        for (int k = 0; k < kT; ++k) {
          c[sp][k] = make_uint2(0u, 0u);
          if (tid + k * B < ntl[sp]) c[sp][k] = tc[sp][tid + k * B];
        }
        if (one_word && tid < nw[sp]) word[sp] = eb[sp][tid];
      }
#pragma unroll
      for (int sp = 0; sp < 2; ++sp) {
#pragma unroll
        for (int k = 0; k < kT; ++k) {
          pushed[sp] += c[sp][k].x;
          alive[sp] += c[sp][k].y;
        }
        for (int t = tid + kT * B; t < ntl[sp]; t += B) {  // more than kT tiles per thread
          const uint2 cc = tc[sp][t];
          pushed[sp] += cc.x;
          alive[sp] += cc.y;
        }
      }
    }
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
      const SpeciesDev s = sp == 0 ? se : sion;
      double ke = 0.0, mom = 0.0;
      if (energy)
        for (int t = tid; t < ntl[sp]; t += B) {
          ke += s.tke[2 * t];
          mom += s.tke[2 * t + 1];
        }
      const uint32_t ps = __reduce_add_sync(~0ull, pushed[sp]);
      const uint32_t al = __reduce_add_sync(~0ull, alive[sp]);
      if (energy) {
        ke = wave_sum(ke);
        mom = wave_sum(mom);
      }
      if (lane == 0) {
        wu[sp][wv][0] = ps;
        wu[sp][wv][1] = al;
        wd[sp][wv][0] = ke;
        wd[sp][wv][1] = mom;
      }
    }
    // event tiles: thread t takes bitmap words [t pw, (t + 1) pw) of each species; their
    // ranks in tile order come from one scan of both species' counts (packed in 16-bit
    // halves: a species has fewer than 2^16 tiles)
    const int pw[2] = {(nw[0] + B - 1) / B, (nw[1] + B - 1) / B};
    uint32_t cnt[2] = {0u, 0u};
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
      if (one_word) {
        cnt[sp] = static_cast<uint32_t>(__popc(word[sp]));
      } else {
        const int w0 = min(nw[sp], tid * pw[sp]), w1 = min(nw[sp], w0 + pw[sp]);
        for (int w = w0; w < w1; ++w) cnt[sp] += static_cast<uint32_t>(__popc(eb[sp][w]));
      }
    }
    uint32_t total;
    const uint32_t rr = block_exclusive_scan<uint32_t>(cnt[0] | (cnt[1] << 16), lds, total);
    if (tid == 0) {
      ev_n[0] = total & 0xFFFFu;
      ev_n[1] = total >> 16;
    }
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
      const SpeciesDev s = sp == 0 ? se : sion;
      uint32_t r = sp == 0 ? (rr & 0xFFFFu) : (rr >> 16);
      if (!cnt[sp]) continue;
      const int w0 = one_word ? tid : min(nw[sp], tid * pw[sp]);
      const int w1 = one_word ? tid + 1 : min(nw[sp], w0 + pw[sp]);
      for (int w = w0; w < w1; ++w) {
        uint32_t bits = one_word ? word[sp] : eb[sp][w];
        while (bits) {
          const int t = 32 * w + __ffs(bits) - 1;
          bits &= bits - 1u;
          if (r < static_cast<uint32_t>(kEvCap)) evl[sp][r] = s.tstats[t];
          ++r;
        }
      }
    }
  }
  // thread s (s < 2) settles species s: every counter it reads is loaded here, before the
  // births scan, so that their latency overlaps it (nothing in this kernel writes them
  // before they are used)
  uint32_t n_surv = 0u, nid = 0u, slots = 0u;
  unsigned long long c_births = 0ull, c_ab[2] = {0ull, 0ull}, c_em[2] = {0ull, 0ull};
  unsigned long long c_rf[2] = {0ull, 0ull}, c_ps = 0ull;
  double c_ae[2] = {0.0, 0.0};
  if (threadIdx.x < 2) {
    const SpeciesDev s = threadIdx.x == 0 ? se : sion;
    n_surv = s.n_sorted[q];
    nid = *s.next_id;
    c_births = *s.births;
    c_ab[0] = s.absorbed[0];
    c_ab[1] = s.absorbed[1];
    c_ae[0] = s.absorbed_energy[0];
    c_ae[1] = s.absorbed_energy[1];
    c_em[0] = s.emitted[0];
    c_em[1] = s.emitted[1];
    c_rf[0] = s.reflected[0];
    c_rf[1] = s.reflected[1];
    c_ps = *s.psteps;
    slots = n_surv;  // the slots of the output, dead records included
  }
  const uint32_t Bn = array_exclusive_scan_to(se.birth_cnt, se.birth_base, nt, lds);
  // electrons emitted by absorbed ions follow the ionisation births, in the order of their
  // parent ions' input index ((tile, wave) units in order, each list in input order)
  const int nu_i = (sion.n_tiles + sion.n_tail) * kWaves;
  uint32_t E = 0u;
  if (sion.t_see) E = array_exclusive_scan_to(sion.em_cnt, sion.em_base, nu_i, lds);
  if (threadIdx.x < 2) {
    const SpeciesDev s = threadIdx.x == 0 ? se : sion;
    if (threadIdx.x == 0) {
      se.birth_base[nt] = Bn;
      if (sion.t_see) sion.em_base[nu_i] = E;
    }
    uint32_t fit = threadIdx.x == 0 ? Bn + E : Bn;
    const uint32_t room = s.cap > n_surv ? s.cap - n_surv : 0u;
    if (fit > room) {
      fit = room;
      atomicOr(sim.error, kErrCapacity);
    }
    if (static_cast<unsigned long long>(nid) + fit > 0xFFFFFFFFull) {
      fit = 0xFFFFFFFFu - nid;
      atomicOr(sim.error, kErrIdOverflow);
    }
    s.fin[0] = fit;
    s.fin[1] = nid;
    s.n_total[q] = n_surv + fit;
    *s.next_id = nid + fit;
    *s.births = c_births + fit;
  }
  __syncthreads();
  __shared__ double mom_sp[2];
  if (threadIdx.x < 2) {
    // thread sp settles species sp: the waves' sums in order, the event list in order,
    // then the counters
    const int sp = static_cast<int>(threadIdx.x);
    const SpeciesDev s = sp == 0 ? se : sion;
    double ke = 0.0, mom = 0.0, ae[2] = {0.0, 0.0};
    unsigned long long pushed = 0ull, alive = 0ull;
    unsigned long long ab[2] = {0ull, 0ull}, em[2] = {0ull, 0ull}, rf[2] = {0ull, 0ull};
    for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) {
      ke += wd[sp][w][0];
      mom += wd[sp][w][1];
      pushed += wu[sp][w][0];
      alive += wu[sp][w][1];
    }
    auto add_event = [&](const TileStats& ts) {
      ae[0] += ts.abs_e[0];
      ae[1] += ts.abs_e[1];
      ab[0] += ts.abs_n[0];
      ab[1] += ts.abs_n[1];
      em[0] += ts.emit[0];
      em[1] += ts.emit[1];
      rf[0] += ts.refl[0];
      rf[1] += ts.refl[1];
    };
    const uint32_t m = ev_n[sp];
    for (uint32_t r = 0; r < m && r < static_cast<uint32_t>(kEvCap); ++r) add_event(evl[sp][r]);
    if (m > static_cast<uint32_t>(kEvCap)) {  // the rest, in tile order, from global memory
      const int ntiles = s.n_tiles + s.n_tail;
      uint32_t r = 0u;
      for (int w = 0; w < (ntiles + 31) / 32; ++w) {
        uint32_t bits = s.ev_bits[w];
        while (bits) {
          const int t = 32 * w + __ffs(bits) - 1;
          bits &= bits - 1u;
          if (r >= static_cast<uint32_t>(kEvCap)) add_event(s.tstats[t]);
          ++r;
        }
      }
    }
    s.absorbed[0] = c_ab[0] + ab[0];
    s.absorbed[1] = c_ab[1] + ab[1];
    s.absorbed_energy[0] = c_ae[0] + ae[0];
    s.absorbed_energy[1] = c_ae[1] + ae[1];
    s.emitted[0] = c_em[0] + em[0];
    s.emitted[1] = c_em[1] + em[1];
    s.reflected[0] = c_rf[0] + rf[0];
    s.reflected[1] = c_rf[1] + rf[1];
    *s.psteps = c_ps + pushed;
    // lagged sort: the output holds a dead record for every counted slot whose particle
    // did not survive the push
    s.n_holes[q] = s.mode == kModeLag && slots > alive ? slots - static_cast<uint32_t>(alive) : 0u;
    if (energy) {
      const double ak = fabs(s.kappa);
      dd.dstat[DS_KIN_E + sp] = ke / (2.0 * ak);
      mom_sp[sp] = mom / ak;
    }
  }
  __syncthreads();
  {
    // the event bitmaps start the next step empty
    const int tid = static_cast<int>(threadIdx.x), B = static_cast<int>(blockDim.x);
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
      const SpeciesDev s = sp == 0 ? se : sion;
      const int nw = (s.n_tiles + s.n_tail + 31) / 32;
      for (int w = tid; w < nw; w += B)
        if (s.ev_bits[w]) s.ev_bits[w] = 0u;
    }
  }
  // The last discharge's workgroup advances the step counter (every workgroup read it at
  // its start); the kernel boundary publishes it to k_finalize and the next step.
  if (threadIdx.x == 0) {
    if (energy) {
      dd.dstat[DS_MOM] = mom_sp[0] + mom_sp[1];
      *dd.energy_step = step;
    }
    if (gridDim.x == 1u) {
      *sim.step = step + 1ull;
    } else {
      const uint32_t done = atomicAdd(sim.fin_count, 1u);
      if (done == gridDim.x - 1u) {
        *sim.fin_count = 0u;
        *sim.step = step + 1ull;
      }
    }
  }
}

template <class P>
__global__ __launch_bounds__(kWG) void k_finalize(const SimDev* __restrict__ simp) {
  using real = typename Part<P>::real;
  const SimDev& sim = *simp;
  const int lane = threadIdx.x & 63;
  const int g = blockIdx.x * kWaves + wave_id();  // one wave per tile
  const int q = static_cast<int>(*sim.step & 1ull);  // k_birth_scan advanced the step
  if (g < sim.total_tiles) {
    const int2 tt = sim.tile_table[g];
    const SpeciesDev se = sim.sp[tt.x];
    if (se.mode == kModeFine) {
      // births of a fine-sorted species go to their sorting cells (k_fine_births)
    } else if (se.sp == 0) {
      const int u = tt.y;
      const uint32_t b0 = se.birth_base[u], b1 = se.birth_base[u + 1];
      const uint32_t first = se.stage_first[u];
#pragma unroll
      for (int sp = 0; sp < 2; ++sp) {
        const SpeciesDev s = sim.sp[tt.x + sp];
        const uint32_t fit = s.fin[0], nid = s.fin[1];
        const uint32_t n_surv = s.n_sorted[q];
        const RecPtr src = rec_stage(&sim.sp[tt.x], sp);
        const RecPtr dst = rec_buf(&sim.sp[tt.x + sp], q);
        const uint32_t end = min(b1, fit);
        for (uint32_t b = b0 + static_cast<uint32_t>(lane); b < end; b += 64u) {
          const uint32_t si = first + (b - b0);
          if (si >= se.cap) continue;
          int cell = 0;
          real pos;
          if constexpr (std::is_same<P, P32>::value) {
            cell = ldg<int>(src.f[F32_CELL], si);
            pos = ldg<float>(src.f[F32_OFF], si);
          } else {
            pos = ldg<double>(src.f[F64_X], si);
          }
          real v[3];
          load_velocity<P>(src, si, v);
          store_record<P>(dst, n_surv + b, cell, pos, v[0], v[1], v[2], nid + b);
          if constexpr (std::is_same<P, P64>::value) cell = static_cast<int>(floor(pos));
          if (cell >= 0 && cell < s.n_cells) far_deposit<P>(s, cell, pos);
        }
      }
    } else if (se.t_see) {
      // an ion tile's emitted electrons, after all ionisation births
      const int u = tt.y;
      const SpeciesDev el = sim.sp[tt.x - 1];
      const uint32_t B = el.birth_base[el.n_tiles + el.n_tail];
      const uint32_t fit = el.fin[0], nid = el.fin[1];
      const uint32_t n_surv = el.n_sorted[q];
      RecPtr src;
#pragma unroll
      for (int k = 0; k < 6; ++k) src.f[k] = se.em_stage[k];
      src.boff4 = src.boff8 = src.boffv = 0u;
      const RecPtr dst = rec_buf(&sim.sp[tt.x - 1], q);
      for (int w = 0; w < kWaves; ++w) {
        const int unit = u * kWaves + w;
        const uint32_t cnt = se.em_cnt[unit], lo = se.em_lo[unit], base = se.em_base[unit];
        for (uint32_t k = static_cast<uint32_t>(lane); k < cnt; k += 64u) {
          const uint32_t b = B + base + k;
          const uint32_t si = lo + k;
          if (b >= fit || si >= se.cap) continue;
          int cell = 0;
          real pos;
          if constexpr (std::is_same<P, P32>::value) {
            cell = ldg<int>(src.f[F32_CELL], si);
            pos = ldg<float>(src.f[F32_OFF], si);
          } else {
            pos = ldg<double>(src.f[F64_X], si);
            cell = static_cast<int>(floor(pos));
          }
          real v[3];
          load_velocity<P>(src, si, v);
          store_record<P>(dst, n_surv + b, cell, pos, v[0], v[1], v[2], nid + b);
          if (cell >= 0 && cell < el.n_cells) far_deposit<P>(el, cell, pos);
        }
      }
    }
  }
}

// ====================================================================================
// host launchers.  With events, a launch goes through hipExtLaunchKernelGGL, which
// records them around the kernel's own execution (used for per-kernel timing).
// ====================================================================================
template <typename K, typename... Args>
static void launch_lds(K kernel, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                       hipEvent_t e0, hipEvent_t e1, Args... args) {
  if (e0 || e1) hipExtLaunchKernelGGL(kernel, grid, block, lds, st, e0, e1, 0, args...);
  else kernel<<<grid, block, lds, st>>>(args...);
}

template <typename K, typename... Args>
static void launch(K kernel, dim3 grid, dim3 block, hipStream_t st, hipEvent_t e0,
                   hipEvent_t e1, Args... args) {
  launch_lds(kernel, grid, block, 0, st, e0, e1, args...);
}

void launch_combine(const LaunchInfo& li, const SimDev* sim, hipStream_t st, hipEvent_t e0,
                    hipEvent_t e1) {
  const dim3 grid(li.n_node_wgs), block(kCombineNodes * kCombineLanes);
  launch(k_combine, grid, block, st, e0, e1, sim);
}

void launch_solve(const LaunchInfo& li, const SimDev* sim, int init_mode, hipStream_t st,
                  hipEvent_t e0, hipEvent_t e1) {
  launch(k_solve, dim3(li.n_ds), dim3(kSolveWG), st, e0, e1, sim, init_mode);
}

void launch_hist(const LaunchInfo& li, const SimDev* sim, hipStream_t st, hipEvent_t e0,
                 hipEvent_t e1) {
  const size_t lds = sizeof(uint32_t) * kWaves * kHistCopies * li.max_window;
  const dim3 g(li.total_tiles), b(kWG);
  if (li.lag) {
    if (li.fp32) launch_lds(k_hist<P32, true>, g, b, lds, st, e0, e1, sim);
    else launch_lds(k_hist<P64, true>, g, b, lds, st, e0, e1, sim);
  } else {
    if (li.fp32) launch_lds(k_hist<P32, false>, g, b, lds, st, e0, e1, sim);
    else launch_lds(k_hist<P64, false>, g, b, lds, st, e0, e1, sim);
  }
}

void launch_scan(const LaunchInfo& li, const SimDev* sim, hipStream_t st, hipEvent_t e0,
                 hipEvent_t e1) {
  if (li.n_cell_wgs > 0)
    launch(k_scan_cells, dim3(li.n_cell_wgs), dim3(kScanCells * kScanLanes), st, e0,
           static_cast<hipEvent_t>(nullptr), sim);
  else if (e0)
    (void)hipEventRecord(e0, st);  // every species unsorted: no per-cell offsets
  launch(k_scan_base, dim3(li.n_spec), dim3(kSolveWG), st, static_cast<hipEvent_t>(nullptr),
         e1, sim);
}

void launch_main(const LaunchInfo& li, const SimDev* sim, hipStream_t st, hipEvent_t e0,
                 hipEvent_t e1) {
  const dim3 g(li.total_tiles), b(kWG);
  if (li.lag) {
    if (li.fp32) launch(k_main<P32, true>, g, b, st, e0, e1, sim);
    else launch(k_main<P64, true>, g, b, st, e0, e1, sim);
  } else {
    if (li.fp32) launch(k_main<P32, false>, g, b, st, e0, e1, sim);
    else launch(k_main<P64, false>, g, b, st, e0, e1, sim);
  }
}

void launch_collide(const LaunchInfo& li, const SimDev* sim, hipStream_t st, hipEvent_t e0,
                    hipEvent_t e1) {
  const dim3 grid(li.n_collide_wgs);
  hipEvent_t e1c = li.emission ? static_cast<hipEvent_t>(nullptr) : e1;
  const dim3 block(li.collide_wg);
  if (li.collide_wg == kCollideWide) {
    if (li.fp32) launch(k_collide<P32, kCollideWide>, grid, block, st, e0, e1c, sim);
    else launch(k_collide<P64, kCollideWide>, grid, block, st, e0, e1c, sim);
  } else {
    if (li.fp32) launch(k_collide<P32, kWG>, grid, block, st, e0, e1c, sim);
    else launch(k_collide<P64, kWG>, grid, block, st, e0, e1c, sim);
  }
  if (li.emission) {
    const dim3 eg((li.total_tiles + kWaves - 1) / kWaves);
    if (li.fp32) launch(k_emit<P32>, eg, dim3(kWG), st, static_cast<hipEvent_t>(nullptr), e1, sim);
    else launch(k_emit<P64>, eg, dim3(kWG), st, static_cast<hipEvent_t>(nullptr), e1, sim);
  }
}

void launch_finalize(const LaunchInfo& li, const SimDev* sim, hipStream_t st, hipEvent_t e0,
                     hipEvent_t e1) {
  launch(k_birth_scan, dim3(li.n_ds), dim3(kSolveWG), st, e0, static_cast<hipEvent_t>(nullptr),
         sim);
  const dim3 grid((li.total_tiles + kWaves - 1) / kWaves);
  if (li.fp32) launch(k_finalize<P32>, grid, dim3(kWG), st, static_cast<hipEvent_t>(nullptr), e1, sim);
  else launch(k_finalize<P64>, grid, dim3(kWG), st, static_cast<hipEvent_t>(nullptr), e1, sim);
}

}  // namespace fspic
