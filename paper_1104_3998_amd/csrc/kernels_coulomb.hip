// kernels_coulomb.hip -- binary Coulomb collisions between the particles of one grid cell,
// the collision process that a particle array kept sorted by cell makes straightforward
// (Sec. 3.2: the sorting cell must then not exceed a Debye length; here the pairing cell
// is one grid cell).
//
// Each pair's relative velocity u = v_a - v_b is turned by an angle Theta with
// tan(Theta / 2) = delta, delta normal with variance
//   q_a^2 q_b^2 n_L lnLambda dt / (8 pi eps0^2 m_ab^2 |u|^3)     (m_ab the reduced mass)
// about a uniformly drawn azimuth (Takizuka and Abe, J. Comput. Phys. 25, 205, 1977), and
// the change is shared in the ratio of the masses, so the pair's momentum and kinetic
// energy are unchanged.
//
// Pairing, after the step's sort and before the births are appended: in every cell the
// particles of a species pair up in array order (first with second, third with fourth;
// an odd one out does not collide), then the k-th electron of the cell pairs with its
// k-th ion.  Thread j of a cell owns electrons 2j, 2j+1 and ions 2j, 2j+1 of the cell, so
// the like pair and the two electron-ion pairs of those particles run in sequence in its
// registers, in FP64, and the result is rounded to the layout once.  n_L is the cell
// density of the species (like pairs) or the lower of the two (electron-ion pairs).
// Draws: Philox counter (id of particle a, step, block, tag 2) under particle a's species
// key: like pairs blocks 0 (delta, Box-Muller) and 1 (azimuth), electron-ion pairs 2 and 3.
#include <hip/hip_ext.h>

#include <type_traits>

#include "device_common.h"
#include "host_common.h"

namespace fspic {

namespace {

struct C32 {};
struct C64 {};

template <class P>
struct CReal;
template <>
struct CReal<C32> {
  using type = float;
};
template <>
struct CReal<C64> {
  using type = double;
};

// FP32: vx, vy, vz are words 0-2 of the particle's 16-byte velocity record, the id word 3;
// FP64: the three doubles of its 24-byte record
template <class P>
__device__ __forceinline__ void load_v(const SpeciesDev& s, int buf, uint32_t i, double v[3]) {
  if constexpr (std::is_same<P, C32>::value) {
    const uint32_t o = 4u * (i + (buf ? s.bstridev / 16u : 0u));
    for (int a = 0; a < 3; ++a) v[a] = static_cast<double>(ldg<float>(s.fld[0][F_VX], o + a));
  } else {
    const uint32_t o = 3u * (i + (buf ? s.bstridev / 24u : 0u));
    for (int a = 0; a < 3; ++a) v[a] = ldg<double>(s.fld[0][F_VX], o + a);
  }
}

template <class P>
__device__ __forceinline__ void store_v(const SpeciesDev& s, int buf, uint32_t i, const double v[3]) {
  if constexpr (std::is_same<P, C32>::value) {
    const uint32_t o = 4u * (i + (buf ? s.bstridev / 16u : 0u));
    for (int a = 0; a < 3; ++a) stg<float>(s.fld[0][F_VX], o + a, static_cast<float>(v[a]));
  } else {
    const uint32_t o = 3u * (i + (buf ? s.bstridev / 24u : 0u));
    for (int a = 0; a < 3; ++a) stg<double>(s.fld[0][F_VX], o + a, v[a]);
  }
}

template <class P>
__device__ __forceinline__ uint32_t load_id(const SpeciesDev& s, int buf, uint32_t i) {
  if constexpr (std::is_same<P, C32>::value)
    return ldg<uint32_t>(s.fld[0][F_VX], 4u * (i + (buf ? s.bstridev / 16u : 0u)) + 3u);
  else
    return ldg<uint32_t>(s.fld[0][F_ID], i + (buf ? s.bstride4 / 4u : 0u));
}

// One pair collision in SI-free form: velocities in cells / step, `coef` carries
// e^4 lnLambda dt / (8 pi eps0^2 m_ab^2), speeds are turned into m/s with vunit.
__device__ void pair_collide(double va[3], double vb[3], double coef, double n_l, double vunit,
                             double fa, double fb, uint4 b0, uint4 b1) {
  const double u[3] = {va[0] - vb[0], va[1] - vb[1], va[2] - vb[2]};
  const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  if (!(u2 > 0.0)) return;
  const double um = sqrt(u2);
  const double usi = um * vunit;
  const double var = coef * n_l / (usi * usi * usi);
  double z0, z1;
  normals64(b0, z0, z1);
  const double delta = sqrt(var) * z0;
  const double ph = kTwoPi * u53(b1.x, b1.y);
  const double den = 1.0 + delta * delta;
  const double sth = 2.0 * delta / den;          // sin Theta
  const double omc = 2.0 * delta * delta / den;  // 1 - cos Theta
  double sph, cph;
  sincos(ph, &sph, &cph);
  const double up = sqrt(u[0] * u[0] + u[1] * u[1]);
  double du[3];
  if (up > 0.0) {
    const double ex = u[0] / up, ey = u[1] / up;
    du[0] = ex * u[2] * sth * cph - ey * um * sth * sph - u[0] * omc;
    du[1] = ey * u[2] * sth * cph + ex * um * sth * sph - u[1] * omc;
    du[2] = -up * sth * cph - u[2] * omc;
  } else {  // u along the z axis
    du[0] = u[2] * sth * cph;
    du[1] = u[2] * sth * sph;
    du[2] = -u[2] * omc;
  }
  for (int a = 0; a < 3; ++a) {
    va[a] = va[a] + fa * du[a];
    vb[a] = vb[a] - fb * du[a];
  }
}

// Grid: (cell, discharge); 256 threads walk the cell's pair slots j.
template <class P>
__global__ __launch_bounds__(256) void k_coulomb(const SimDev* __restrict__ simp) {
  const SimDev& sim = *simp;
  const DischargeDev dd = sim.ds[blockIdx.y];
  const int c = blockIdx.x;
  if (!dd.coulomb || c >= dd.n_cells) return;
  const SpeciesDev se = sim.sp[dd.spec0];
  const SpeciesDev si = sim.sp[dd.spec0 + 1];
  const unsigned long long step = *sim.step;
  const uint32_t step32 = static_cast<uint32_t>(step);
  const int q = static_cast<int>((step + 1ull) & 1ull);  // the step's sorted output
  const int N = dd.n_cells;
  const uint32_t GM* cse = se.cell_start + q * (N + 1);
  const uint32_t GM* csi = si.cell_start + q * (N + 1);
  const uint32_t e0 = cse[c], ne = cse[c + 1] - e0;
  const uint32_t i0 = csi[c], ni = csi[c + 1] - i0;
  const bool ee = dd.coulomb & 1, ii = (dd.coulomb & 2) != 0, ei = (dd.coulomb & 4) != 0;
  const uint32_t nmax = ne > ni ? ne : ni;
  const uint32_t np = ne < ni ? ne : ni;  // electron-ion pairs
  for (uint32_t j = threadIdx.x; 2u * j < nmax; j += blockDim.x) {
    const uint32_t k0 = 2u * j;
    double v[2][2][3];  // [species][member][component]
    bool have[2][2];
    for (int s = 0; s < 2; ++s) {
      const uint32_t n = s == 0 ? ne : ni;
      const uint32_t base = s == 0 ? e0 : i0;
      const SpeciesDev& S = s == 0 ? se : si;
      for (int m = 0; m < 2; ++m) {
        have[s][m] = k0 + m < n;
        if (have[s][m]) load_v<P>(S, q, base + k0 + m, v[s][m]);
      }
    }
    bool touched[2][2] = {{false, false}, {false, false}};
    // like pairs
    if (ee && have[0][1]) {
      const uint32_t id = load_id<P>(se, q, e0 + k0);
      pair_collide(v[0][0], v[0][1], dd.coul_coef[0], static_cast<double>(ne) * dd.coul_dens,
                   dd.vunit, 0.5, 0.5, philox(id, step32, 0u, 2u, se.key0, se.key1),
                   philox(id, step32, 1u, 2u, se.key0, se.key1));
      touched[0][0] = touched[0][1] = true;
    }
    if (ii && have[1][1]) {
      const uint32_t id = load_id<P>(si, q, i0 + k0);
      pair_collide(v[1][0], v[1][1], dd.coul_coef[1], static_cast<double>(ni) * dd.coul_dens,
                   dd.vunit, 0.5, 0.5, philox(id, step32, 0u, 2u, si.key0, si.key1),
                   philox(id, step32, 1u, 2u, si.key0, si.key1));
      touched[1][0] = touched[1][1] = true;
    }
    // electron-ion pairs: electron k with ion k
    if (ei) {
      for (int m = 0; m < 2; ++m) {
        if (k0 + m >= np) break;
        const uint32_t id = load_id<P>(se, q, e0 + k0 + m);
        pair_collide(v[0][m], v[1][m], dd.coul_coef[2], static_cast<double>(np) * dd.coul_dens,
                     dd.vunit, dd.mfrac_e, dd.mfrac_i,
                     philox(id, step32, 2u, 2u, se.key0, se.key1),
                     philox(id, step32, 3u, 2u, se.key0, se.key1));
        touched[0][m] = touched[1][m] = true;
      }
    }
    for (int m = 0; m < 2; ++m) {
      if (touched[0][m]) store_v<P>(se, q, e0 + k0 + m, v[0][m]);
      if (touched[1][m]) store_v<P>(si, q, i0 + k0 + m, v[1][m]);
    }
  }
}

}  // namespace

void launch_coulomb(const LaunchInfo& li, const SimDev* sim, hipStream_t st, hipEvent_t e0,
                    hipEvent_t e1) {
  const dim3 grid(li.max_cells, li.n_ds);
  if (e0 || e1) {
    if (li.fp32) hipExtLaunchKernelGGL(k_coulomb<C32>, grid, dim3(256), 0, st, e0, e1, 0, sim);
    else hipExtLaunchKernelGGL(k_coulomb<C64>, grid, dim3(256), 0, st, e0, e1, 0, sim);
  } else {
    if (li.fp32) k_coulomb<C32><<<grid, 256, 0, st>>>(sim);
    else k_coulomb<C64><<<grid, 256, 0, st>>>(sim);
  }
}

}  // namespace fspic
