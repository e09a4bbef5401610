// Device-side layout and arithmetic shared by the LDS-resident, the
// one-workgroup and the grid kernels.  gfx950 only.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hdk {

enum : int { ROLE_MOBILE = 0, ROLE_FIXED = 1, ROLE_RIGID = 2 };
enum : int { FLAG_UNSTABLE = 1, FLAG_NBR_OVERFLOW = 2 };
// Per-system sums: E, d2, G, sumF_R[3], sumHu_R[3], sumU_R[3], and the count
// of atoms whose LJ force is non-finite or above kForceLimit.  The grid
// kernels' tile partials add u.Hu and sumT_R[3] (the third-derivative vector
// T[u,u] over the rigid layer) for systems biased on the curvature, and for
// systems biased on the eigenvalue w.Hw, sumT_R[3] (T[w,w]), the mobile
// atoms' |w|^2 and sumHw_R[3], w the mode estimate spread over the atoms.
enum : int { NRED = 13, NPART = 21 };
enum : int { P_XHX = 13, P_TR = 14, P_W2 = 17, P_HWR = 18 };
// Bias variables (eq. 5-7, eq. 15) and the extra pair-pass terms a plan
// compiles in.
enum : int { BVAR_SLOPE = 0, BVAR_CURV = 1, BVAR_DIST = 2, BVAR_EIG = 3 };
// EXT_NOE: a pair pass whose energy nobody reads (the steps before a
// captured sequence's last) leaves the pair energy out.
enum : int { EXT_BONDS = 1, EXT_CURV = 2, EXT_EIG = 4, EXT_NOE = 8 };
constexpr double kForceLimit2 = 1e12;  // (1e6 eps/sigma)^2

// Read-only description of one system (uploaded at finalize / parameter
// changes).  Per-atom arrays of the batch are concatenated; component k of
// batch atom a lives at k*ntot + a.
struct SysDesc {
  int32_t dim, n;
  int64_t off;                 // first batch atom of this system
  int32_t n_rigid, first_rigid;
  int32_t periodic[3];
  double box[3], hbox[3], inv_box[3];  // inv_box = 1/box on periodic axes, else 0
  double mass, inv_mass, massR, inv_massR;
  double eps[4], sig2[4], shift[4];      // [ta*2+tb]
  float eps_f[4], sig2_f[4], shift_f[4];
  double rc2, rl2, skin_half2;
  double dt, hdt, c1, c2, c2R, kT;
  uint64_t seed;
  double k_spring, f_normal, x_slider, v_slider;
  int32_t bias_on, m_b;
  double dv_max, g_lo, g_hi;
  // reciprocals used by the per-step scalars: 1/kT, 1/(g_L - g_U), 1/n_R,
  // k/n_R^2
  double inv_kT, inv_glh, inv_nR, k_nR2;
  // cell grid, fixed for the life of the context
  int32_t nc[3], ncell;
  double lo[3], inv_h[3];
  int64_t cell_off, cstart_off;
  // neighbour list: entry (j << 1 | type_j) of slot k of atom i at
  // nbr[nbr_off + k*n + i]; grid plans (i the sorted position) at
  // nbr[nbr_off + grid_list_index(k, n, i)], below
  int64_t nbr_off;
  int32_t maxnb, pad0;
  double XR0[3];
  // harmonic tip bonds (eq. 12; tip_bonds != 0): tip-tip pairs closer than
  // the bond cut (squared: rbc2) are springs k_bond (r - r_bond)^2 / 2,
  // farther tip-tip pairs do not interact
  int32_t tip_bonds, pad1;
  double k_bond, r_bond, rbc2;
  float k_bond_f, r_bond_f, rbc2_f, pad2;
  // bias variables: bias_var1 drives the switch with g_lo/g_hi, bias_var2
  // (-1: none) a second one with b2_lo/b2_hi, combined by eq. 13.  gen_bias:
  // anything but the slope alone (grid kernels only); curv: the curvature is
  // one of them (the pair pass then accumulates T[u,u])
  int32_t bias_var1, bias_var2, gen_bias, curv;
  double b2_lo, b2_hi, inv_glh2;
  // thermostat: 0 Langevin (BAOAB), 1 Nose-Hoover chain of nhc_len
  // thermostats, masses nhc_Q1 = N_f kT tau^2 and nhc_Q = kT tau^2, with
  // nhc_NfkT = N_f kT (grid kernels only)
  int32_t thermostat, nhc_len;
  double nhc_Q1, nhc_Q, nhc_NfkT;
  // eigenvalue variable (eq. 15; grid kernels only): eig != 0 when one of
  // the bias variables is it; the mode estimate's rotation step after each
  // step is q <- (q - mode_alpha (P^T H q - lambda q)) / |q|
  int32_t eig;
  // grid plans of LJ-only systems below 32768 atoms keep 16-bit list
  // entries ((sorted position << 1) | type in an unsigned short)
  int32_t list16;
  double mode_alpha;
};

// Mutable per-system state.
struct SysState {
  double XR[3], VR[3], FR[3];  // rigid body: centre of mass, velocity, force
  double t_md, t_hyper;
  int64_t step;
  double e_lj, v_drive, e_pot, e_kin, d, g, dv, dvp, x_slider, x_tip, f_lat;
  int32_t flags, n_rebuilds;
  int32_t rebuild, pad1;
  double kappa, dv1, dv2;
  double xi[4], eta[4];        // Nose-Hoover chain velocities and positions
  double e_nhc;                // the chain's energy (conserved with K + V + dV)
  double qR[3];                // eigenvalue variable: the rigid body's mode component
  double lambda;               // the eigenvalue variable of the last evaluation
  double eig_inv_q2;           // 1/|q|^2 of the mode that evaluation used
};

struct Arrays {
  int64_t ntot;
  int32_t rec_f32, pad_rec;               // pair records in the float32 layout (below)
  double *x, *v, *rO, *xb, *cofs, *ftot;  // [3][ntot]
  double *flj, *hu, *fb;                  // [3][ntot]
  float *flj_f, *hu_f;                    // [3][ntot] float32 runs' grid pair sums, read by the grid kick
  void *u;                                // [3][ntot] float or double
  uint8_t *tr;                            // type | role << 1
  int32_t *nbr, *nnb;
  int32_t *cell_count, *cell_start, *cell_atoms, *cidx;
  int32_t *sys_of;                        // [ntot] system of each batch atom
  double *partials;                       // grid kernels: per-tile sums
  double *XR_next;                        // grid kernels: [S][6] rigid body after drift
  int32_t *rebuild_flag;                  // grid kernels: [S]
  // grid kernels: atoms are visited in cell-sorted order.  pos[a] is the
  // sorted position of atom a within its system (cell_atoms is the inverse);
  // rec holds one 64-byte pair record per sorted position, refreshed by
  // every drift.  float64 runs: x (doubles 0-2), u (doubles 3-5) and
  // type | role << 1 (double 7).  float32 runs (rec_f32): x (doubles 0-2), u
  // as float32 (bytes 24-35), type | role << 1 (int32, bytes 36-39) and u as
  // float64 (doubles 5-7, for the atom's own per-system sums), so that a
  // neighbour is the record's first 40 bytes and needs no conversion.
  // Neighbour lists hold sorted positions, so a neighbour's data is one
  // aligned record, and the atoms of a wavefront share cells and read nearby
  // records.
  int32_t *pos;                           // [ntot]
  double *rec;                            // [ntot][8]
  // list build: the build positions (doubles 0-2) and type | role << 1
  // (integer bits of the fourth slot) of each sorted position, written by
  // the cell sort, so a stencil row's candidates are consecutive 32-byte
  // records
  double *brec;                           // [ntot][4]
  double *tuu;                            // [3][ntot] T[u,u] (curvature bias) or T[w,w] (eigenvalue)
  // eigenvalue bias: the mode estimate q of the mobile atoms (rigid atoms'
  // in SysState.qR), H w of the last pair pass, and per sorted position the
  // mode spread over the atoms (w: doubles 0-2 of a 32-byte record)
  double *qm, *hw;                        // [3][ntot]
  double *recw;                           // [ntot][4]
  // grid kernels: the tiles (indices into the plan's tiles) and systems
  // whose lists expire this step, and their counts (written by kg_compact
  // after the drift, cleared by kg_reduce)
  int32_t *rb_tiles, *rb_sys, *rb_count;
};

constexpr int kRecDoubles = 8;

// Write the pair record of one atom (layout above).
__device__ __forceinline__ void rec_store(const Arrays &A, double *rec, int dim, const double x[3],
                                          const double u[3], int tr) {
  for (int k = 0; k < dim; ++k) rec[k] = x[k];
  if (A.rec_f32) {
    float *uf = (float *)(rec + 3);
    for (int k = 0; k < dim; ++k) { uf[k] = (float)u[k]; rec[5 + k] = u[k]; }
    ((int32_t *)rec)[9] = tr;
  } else {
    for (int k = 0; k < dim; ++k) rec[3 + k] = u[k];
    rec[7] = (double)tr;
  }
}

// A neighbour's u component from its pair record (float32 kernels read the
// float32 layout, float64 kernels the float64 one).
template <typename T>
__device__ __forceinline__ T rec_u(const double *r, int k) {
  if constexpr (sizeof(T) == 4) return ((const float *)(r + 3))[k];
  else return r[3 + k];
}

// ---------------------------------------------------------------------------
// Small helpers
__device__ __forceinline__ double minimg(double dx, double L, double hL, int periodic) {
  if (periodic) {
    if (dx > hL) dx -= L;
    else if (dx < -hL) dx += L;
  }
  return dx;
}

__device__ __forceinline__ double wrapx(double x, double L, int periodic) {
  if (periodic) {
    if (x >= L) x -= L;
    else if (x < 0.0) x += L;
  }
  return x;
}

// Philox4x32-10 (Salmon et al., SC'11).
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0;
    const uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

// Standard normals for (step, particle, tag): uniforms (w + 1/2) 2^-32 and
// Box-Muller on (u0,u1) -> z0,z1 and (u2,u3) -> z2,z3.
__device__ __forceinline__ void normals4(uint64_t seed, int64_t step, uint32_t particle,
                                         uint32_t tag, double z[4]) {
  uint32_t c[4] = {(uint32_t)((uint64_t)step & 0xffffffffu), (uint32_t)((uint64_t)step >> 32),
                   particle, tag};
  philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
  const double s = 2.3283064365386963e-10;
  const double u0 = ((double)c[0] + 0.5) * s, u1 = ((double)c[1] + 0.5) * s;
  const double u2 = ((double)c[2] + 0.5) * s, u3 = ((double)c[3] + 0.5) * s;
  const double two_pi = 6.283185307179586;
  const double r0 = sqrt(-2.0 * log(u0)), r1 = sqrt(-2.0 * log(u2));
  z[0] = r0 * cos(two_pi * u1);
  z[1] = r0 * sin(two_pi * u1);
  z[2] = r1 * cos(two_pi * u3);
  z[3] = r1 * sin(two_pi * u3);
}

// The first NZ standard normals of (step, particle, tag): the same transform
// as normals4, evaluating only the components a DIM-dimensional update uses.
template <int NZ>
__device__ __forceinline__ void normals_n(uint64_t seed, int64_t step, uint32_t particle, uint32_t tag,
                                          double z[3]) {
  uint32_t c[4] = {(uint32_t)((uint64_t)step & 0xffffffffu), (uint32_t)((uint64_t)step >> 32),
                   particle, tag};
  philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
  const double s = 2.3283064365386963e-10;
  const double two_pi = 6.283185307179586;
  const double u0 = ((double)c[0] + 0.5) * s, u1 = ((double)c[1] + 0.5) * s;
  const double r0 = sqrt(-2.0 * log(u0));
  double sn, cs;
  sincos(two_pi * u1, &sn, &cs);
  z[0] = r0 * cs;
  z[1] = r0 * sn;
  if constexpr (NZ > 2) {
    const double u2 = ((double)c[2] + 0.5) * s, u3 = ((double)c[3] + 0.5) * s;
    z[2] = sqrt(-2.0 * log(u2)) * cos(two_pi * u3);
  }
}

// Float32 form of the same transform for the float32 pair-arithmetic mode:
// the same Philox words, the logarithm and the angle evaluated in float32.
// -2 ln u is taken from whichever of u and 1 - u is below one half, both
// formed from the integer word so that the small one is nearly exact; the
// angle 2 pi u is split into its quadrant (top two bits of the word) and a
// fraction of a quarter turn.  Relative error about 1e-7.
__device__ __forceinline__ float m2ln_u32(uint32_t c) {
  const float s = 2.3283064365386963e-10f;  // 2^-32
  if (c < 0x80000000u) return -2.0f * logf(((float)c + 0.5f) * s);
  return -2.0f * log1pf(-(((float)(0xffffffffu - c) + 0.5f) * s));
}

__device__ __forceinline__ void sincos_turn_u32(uint32_t c, float &sn, float &cs) {
  const float th = ((float)(c & 0x3fffffffu) + 0.5f) * (1.5707963267948966f * 9.313225746154785e-10f);
  float s0, c0;
  sincosf(th, &s0, &c0);
  const uint32_t q = c >> 30;
  sn = q == 0 ? s0 : (q == 1 ? c0 : (q == 2 ? -s0 : -c0));
  cs = q == 0 ? c0 : (q == 1 ? -s0 : (q == 2 ? -c0 : s0));
}

template <int NZ>
__device__ __forceinline__ void normals_nf(uint64_t seed, int64_t step, uint32_t particle, uint32_t tag,
                                           double z[3]) {
  uint32_t c[4] = {(uint32_t)((uint64_t)step & 0xffffffffu), (uint32_t)((uint64_t)step >> 32),
                   particle, tag};
  philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
  const float r0 = sqrtf(m2ln_u32(c[0]));
  float sn, cs;
  sincos_turn_u32(c[1], sn, cs);
  z[0] = (double)(r0 * cs);
  z[1] = (double)(r0 * sn);
  if constexpr (NZ > 2) {
    float s3, c3;
    sincos_turn_u32(c[3], s3, c3);
    z[2] = (double)(sqrtf(m2ln_u32(c[2])) * c3);
  }
}

// Langevin normals of a kernel computing pairs in T: float64 transform for
// float64, float32 transform for float32.
template <int NZ, typename T>
__device__ __forceinline__ void noise(uint64_t seed, int64_t step, uint32_t particle, double z[3]) {
  if constexpr (sizeof(T) == 4) normals_nf<NZ>(seed, step, particle, 0u, z);
  else normals_n<NZ>(seed, step, particle, 0u, z);
}

// The switch of eq. 14 (eq. 15 has the same form) of a bias variable v with
// critical values lo and hi (inv = 1/(lo - hi)) and its derivative in v:
// dV_max at or beyond hi, zero at or beyond lo, dV_max (1 - xi^m)^2 with
// xi = (v - hi)/(lo - hi) between.  With lo < hi (slope, curvature) the bias
// is full for large values, with lo > hi (distance) for small ones.
__device__ __forceinline__ void bias_switch(const SysDesc &D, double v, double lo, double hi, double inv,
                                            double &dv, double &dvp) {
  const bool up = lo < hi;
  if (up ? v >= hi : v <= hi) { dv = D.dv_max; dvp = 0.0; return; }
  if (up ? v <= lo : v >= lo) { dv = 0.0; dvp = 0.0; return; }
  const double xi = (v - hi) * inv;
  double xm1 = 1.0;
  for (int q = 0; q < D.m_b - 1; ++q) xm1 *= xi;
  const double xm = xm1 * xi;
  const double one = 1.0 - xm;
  dv = D.dv_max * one * one;
  dvp = -2.0 * D.m_b * D.dv_max * one * xm1 * inv;
}

// Nose-Hoover chain (Martyna, Klein, Tuckerman 1992) over half a step h =
// dt/2 given twice the kinetic energy K2 of the thermostatted degrees of
// freedom: the thermostat velocities xi from the chain's end inwards over
// h/2, the particle velocities' scale factor exp(-xi_1 h) (returned) and the
// thermostat positions eta advanced by h, then the thermostat velocities
// outwards over h/2; each inner update sits between exp(-xi_{j+1} h/4)
// factors (Trotter splitting of Martyna, Tuckerman, Tobias, Klein 1996).
__device__ __forceinline__ double nhc_force(const SysDesc &D, const double *xi, int j, double k2) {
  if (j == 0) return (k2 - D.nhc_NfkT) / D.nhc_Q1;
  const double Qp = j == 1 ? D.nhc_Q1 : D.nhc_Q;
  return (Qp * xi[j - 1] * xi[j - 1] - D.kT) / D.nhc_Q;
}

__device__ inline double nhc_half_step(const SysDesc &D, double *xi, double *eta, double K2) {
  const int M = D.nhc_len;
  const double h = D.hdt;
  xi[M - 1] += 0.5 * h * nhc_force(D, xi, M - 1, K2);
  for (int j = M - 2; j >= 0; --j) {
    const double e = exp(-0.25 * h * xi[j + 1]);
    xi[j] *= e;
    xi[j] += 0.5 * h * nhc_force(D, xi, j, K2);
    xi[j] *= e;
  }
  const double c = exp(-h * xi[0]);
  K2 *= c * c;
  for (int j = 0; j < M; ++j) eta[j] += h * xi[j];
  for (int j = 0; j < M - 1; ++j) {
    const double e = exp(-0.25 * h * xi[j + 1]);
    xi[j] *= e;
    xi[j] += 0.5 * h * nhc_force(D, xi, j, K2);
    xi[j] *= e;
  }
  xi[M - 1] += 0.5 * h * nhc_force(D, xi, M - 1, K2);
  return c;
}

// The chain's energy sum_j Q_j xi_j^2 / 2 + N_f kT eta_1 + kT sum_{j>1} eta_j.
__device__ inline double nhc_energy(const SysDesc &D, const double *xi, const double *eta) {
  double en = D.nhc_NfkT * eta[0];
  for (int j = 0; j < D.nhc_len; ++j) {
    en += 0.5 * (j == 0 ? D.nhc_Q1 : D.nhc_Q) * xi[j] * xi[j];
    if (j > 0) en += D.kT * eta[j];
  }
  return en;
}

// Per-system scalars derived from the reduced sums (LJ part) and the rigid
// body: drive energy and force, slope, bias.
struct Scal {
  double e_lj, v_drive, e_pot, d, g, dv, dvp, xs, x_tip, f_lat;
  double Fd[3];      // drive force on the rigid body
  double hud[3];     // drive Hessian term per rigid atom (k/nR^2) sum_R u
  double sumFb[3];   // bias force summed over rigid atoms
  double bad;        // atoms with a non-finite or runaway force
  double bias_a, bias_b;  // bias force = bias_a (Hu - F - bias_b u): -dV'/d, g/d
  // general bias (eq. 13 over any of slope, curvature, distance): the bias
  // force is cH Hu + cF F + cU u + cT T[u,u] where live
  double kappa, dv1, dv2, cH, cF, cU, cT;
  // eigenvalue variable: lambda = w.Hw/|q|^2 and eig_s = 1/|q| (0 without a
  // mode), |q| over the degrees of freedom
  double lambda, eig_s;
  int live;
};

template <int DIM, bool GEN = false>
__device__ __forceinline__ void eval_scalars(const SysDesc &D, const double *sums,
                                             const double XR[3], int64_t step, Scal &S,
                                             const double *qR = nullptr) {
  constexpr int dim = DIM;
  S.xs = D.x_slider + D.v_slider * ((double)step * D.dt);
  S.e_lj = sums[0];
  S.v_drive = 0.0; S.x_tip = 0.0; S.f_lat = 0.0;
  double G = sums[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) { S.Fd[k] = 0.0; S.hud[k] = 0.0; S.sumFb[k] = 0.0; }
  if (D.n_rigid > 0) {
    const int perp = dim - 1;
    S.x_tip = XR[0] - D.XR0[0];
    const double ext = S.xs - S.x_tip;
    S.f_lat = D.k_spring * ext;
    S.v_drive = 0.5 * D.k_spring * ext * ext;
    S.Fd[0] = D.k_spring * ext;
    if (dim == 3) {
      const double dy = XR[1] - D.XR0[1];
      S.v_drive += 0.5 * D.k_spring * dy * dy;
      S.Fd[1] = -D.k_spring * dy;
    }
    S.v_drive += D.f_normal * (XR[perp] - D.XR0[perp]);
    S.Fd[perp] += -D.f_normal;
    constexpr int nspring = dim == 3 ? 2 : 1;
#pragma unroll
    for (int k = 0; k < nspring; ++k) S.hud[k] = D.k_nR2 * sums[9 + k];
    // drive share of each rigid atom enters F.u
#pragma unroll
    for (int k = 0; k < dim; ++k) G += (S.Fd[k] * D.inv_nR) * sums[9 + k];
  }
  S.e_pot = S.e_lj + S.v_drive;
  S.bad = sums[12];
  // d = |u| and 1/d from one reciprocal square root refined by two Newton
  // steps (relative error ~1e-16)
  const double d2 = sums[1];
  double inv_d = 0.0;
  if (d2 > 0.0) {
    double y = __builtin_amdgcn_rsq(d2);
    y = y * __builtin_fma(-0.5 * d2 * y, y, 1.5);
    y = y * __builtin_fma(-0.5 * d2 * y, y, 1.5);
    inv_d = y;
  }
  S.d = d2 * inv_d;
  const bool has_d = S.d >= 1e-12;
  S.g = has_d ? -G * inv_d : 0.0;
  S.kappa = 0.0; S.dv2 = 0.0;
  S.cH = S.cF = S.cU = S.cT = 0.0;
  S.lambda = 0.0; S.eig_s = 0.0;
  S.live = 0;
  if constexpr (GEN) {
    if (D.gen_bias) {
      // the eigenvalue variable (eq. 15): lambda = w.Hw / |q|^2 along the
      // mode estimate q (w = P q spread over the atoms), |q|^2 over the
      // degrees of freedom (mobile atoms and the rigid body once), the
      // drive's Hessian adding k |q_R|^2 on its spring axes
      double inv_q2 = 0.0;
      if (D.eig) {
        double q2 = sums[P_W2], xhx = sums[P_XHX];
        if (D.n_rigid > 0 && qR) {
          constexpr int nspring = dim == 3 ? 2 : 1;
#pragma unroll
          for (int k = 0; k < dim; ++k) q2 += qR[k] * qR[k];
#pragma unroll
          for (int k = 0; k < nspring; ++k) xhx += D.k_spring * qR[k] * qR[k];
        }
        if (q2 > 0.0) {
          inv_q2 = 1.0 / q2;
          S.lambda = xhx * inv_q2;
          S.eig_s = sqrt(inv_q2);
        }
      }
      // curvature kappa = u.Hu/d^2 (eq. 6), the drive's Hessian included
      double uHu = D.eig ? 0.0 : sums[P_XHX];
      if (D.n_rigid > 0) {
        constexpr int nspring = dim == 3 ? 2 : 1;
#pragma unroll
        for (int k = 0; k < nspring; ++k) uHu += S.hud[k] * sums[9 + k];
      }
      const double inv_d2 = inv_d * inv_d;
      S.kappa = has_d ? uHu * inv_d2 : 0.0;
      double dv1 = 0.0, p1 = 0.0, dv2 = 0.0, p2 = 0.0;
      const int v1 = D.bias_var1, v2 = D.bias_var2;
      auto value = [&](int v) {
        return v == BVAR_SLOPE ? S.g : (v == BVAR_CURV ? S.kappa : (v == BVAR_DIST ? S.d : S.lambda));
      };
      if (D.bias_on) {
        bias_switch(D, value(v1), D.g_lo, D.g_hi, D.inv_glh, dv1, p1);
        if (v2 >= 0) bias_switch(D, value(v2), D.b2_lo, D.b2_hi, D.inv_glh2, dv2, p2);
      }
      // eq. 13 and the partial derivatives of dV in the two variables
      double w1 = p1, w2 = 0.0;
      S.dv = dv1;
      if (D.bias_on && v2 >= 0) {
        S.dv = dv1 + dv2 - dv1 * dv2 / D.dv_max;
        w1 = p1 * (1.0 - dv2 / D.dv_max);
        w2 = p2 * (1.0 - dv1 / D.dv_max);
      }
      S.dv1 = dv1; S.dv2 = dv2; S.dvp = w1;
      S.live = (D.bias_on && has_d && (w1 != 0.0 || w2 != 0.0)) ? 1 : 0;
      // -dV'(v) grad v for each variable, grad g = (Hu - F - g u/d)/d,
      // grad kappa = (2 Hu + T)/d^2 - 2 kappa u/d^2, grad d = u/d
      double cH = 0.0, cF = 0.0, cU = 0.0, cT = 0.0;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int v = q == 0 ? v1 : v2;
        const double w = q == 0 ? w1 : w2;
        if (v == BVAR_SLOPE) { cH -= w * inv_d; cF += w * inv_d; cU += w * S.g * inv_d2; }
        else if (v == BVAR_CURV) { cH -= 2.0 * w * inv_d2; cT -= w * inv_d2; cU += 2.0 * w * S.kappa * inv_d2; }
        else if (v == BVAR_DIST) { cU -= w * inv_d; }
        else if (v == BVAR_EIG) { cT -= w * inv_q2; }   // grad lambda = T[w,w]/|q|^2
      }
      if (S.live) { S.cH = cH; S.cF = cF; S.cU = cU; S.cT = cT; }
      S.bias_a = 0.0; S.bias_b = 0.0;
      if (S.live && D.n_rigid > 0) {
        const double nR = (double)D.n_rigid;
#pragma unroll
        for (int k = 0; k < dim; ++k) {
          const double sumHu = sums[6 + k] + nR * S.hud[k];
          const double sumF = sums[3 + k] + S.Fd[k];
          S.sumFb[k] = S.cH * sumHu + S.cF * sumF + S.cU * sums[9 + k] + S.cT * sums[P_TR + k];
        }
      }
      return;
    }
  }
  S.dv = 0.0; S.dvp = 0.0;
  if (D.bias_on) bias_switch(D, S.g, D.g_lo, D.g_hi, D.inv_glh, S.dv, S.dvp);
  S.dv1 = S.dv;
  S.bias_a = has_d ? -S.dvp * inv_d : 0.0;
  S.bias_b = has_d ? S.g * inv_d : 0.0;
  if (D.bias_on && has_d && S.dvp != 0.0 && D.n_rigid > 0) {
    const double nR = (double)D.n_rigid;
#pragma unroll
    for (int k = 0; k < dim; ++k) {
      const double sumHu = sums[6 + k] + nR * S.hud[k];
      const double sumF = sums[3 + k] + S.Fd[k];
      S.sumFb[k] = S.bias_a * (sumHu - sumF - S.bias_b * sums[9 + k]);
    }
  }
}

// ---------------------------------------------------------------------------
// Pair pass for one atom over its full neighbour list.
//
// FP64: everything in double.  FP32C: the displacement and the cutoff test
// are float64 (so the interacting set is decided exactly as in float64); the
// pair arithmetic is float32, and each atom's sums of the float32 terms are
// float64.  On gfx950 a float64 add issues at the rate of a float32 one, so
// the float64 sum costs two operations per term (convert, add) where a
// compensated float32 sum costs four, and is the more accurate of the two.

struct Sum64 {  // float32 terms summed in float64
  double s;
  __device__ __forceinline__ void init() { s = 0.0; }
  __device__ __forceinline__ void add(float x) { s += (double)x; }
  __device__ __forceinline__ double get() const { return s; }
};

template <typename T> struct PairAcc;

// F, H u, the half pair energy, T[u,u] (curvature bias) or T[w,w]
// (eigenvalue bias) and H w (eigenvalue bias)
template <> struct PairAcc<double> {
  double F[3], H[3], X[3], W[3], e;
  __device__ __forceinline__ void init() {
    for (int k = 0; k < 3; ++k) { F[k] = 0.0; H[k] = 0.0; X[k] = 0.0; W[k] = 0.0; }
    e = 0.0;
  }
};

template <> struct PairAcc<float> {
  Sum64 F[3], H[3], X[3], W[3], e;
  __device__ __forceinline__ void init() {
    for (int k = 0; k < 3; ++k) { F[k].init(); H[k].init(); X[k].init(); W[k].init(); }
    e.init();
  }
};

__device__ __forceinline__ float rcp_nr(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  const float e = __builtin_fmaf(-x, r, 1.0f);
  return __builtin_fmaf(r, e, r);
}

// The LJ parameters of atom i's type against both neighbour types (eq. 9 with
// the pair's epsilon and sigma, energy-shifted at rc), held in registers for
// the whole neighbour loop: the neighbour's type then selects between two
// registers instead of indexing a table in memory per pair.
template <typename T>
struct LJRow {
  T eps[2], sig2[2], shift[2];
  bool bond;          // atom i is a tip atom of a model with tip bonds
  T kb, rb, rbc2;     // its bond constants
  __device__ __forceinline__ void load(const SysDesc &D, int ti) {
    bond = D.tip_bonds != 0 && ti == 1;
    if constexpr (sizeof(T) == 8) { kb = D.k_bond; rb = D.r_bond; rbc2 = D.rbc2; }
    else { kb = D.k_bond_f; rb = D.r_bond_f; rbc2 = D.rbc2_f; }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      if constexpr (sizeof(T) == 8) {
        eps[b] = ti ? D.eps[2 + b] : D.eps[b];
        sig2[b] = ti ? D.sig2[2 + b] : D.sig2[b];
        shift[b] = ti ? D.shift[2 + b] : D.shift[b];
      } else {
        eps[b] = ti ? D.eps_f[2 + b] : D.eps_f[b];
        sig2[b] = ti ? D.sig2_f[2 + b] : D.sig2_f[b];
        shift[b] = ti ? D.shift_f[2 + b] : D.shift_f[b];
      }
    }
  }
};

// The pair's f = -phi'(r)/r (force on i: f dx), C = (phi'' - phi'/r)/r^2
// (H u contribution: C (dx.w) dx - f w) and energy phi, for a tip-tip pair
// of a model with tip bonds (eq. 12): a spring within the bond cut, nothing
// beyond.  Zero when the pair is outside the cut.
// 1/r from the hardware reciprocal square root, refined by Newton steps
// (two in float64: relative error ~1e-16; float32's is ~1 ulp as is).
template <typename T>
__device__ __forceinline__ T inv_sqrt(T q) {
  if constexpr (sizeof(T) == 8) {
    double y = __builtin_amdgcn_rsq(q);
    y = y * __builtin_fma(-0.5 * q * y, y, 1.5);
    return y * __builtin_fma(-0.5 * q * y, y, 1.5);
  } else {
    return __builtin_amdgcn_rsqf(q);
  }
}

// With the curvature bias also Dc = (dC/dr)/r = -3 k r0 / r^5.
template <typename T>
__device__ __forceinline__ void bond_terms(const LJRow<T> &R, double r2, T &f, T &C, T &e, T &Dc) {
  const bool in = r2 < (double)R.rbc2;
  const T m = in ? T(1) : T(0);
  const T q = in ? (T)r2 : T(1);
  const T ir = inv_sqrt<T>(q);
  const T dr = q * ir - R.rb;
  f = -R.kb * dr * ir * m;
  C = R.kb * R.rb * (ir * ir * ir) * m;
  e = T(0.5) * R.kb * dr * dr * m;
  Dc = T(-3) * C * ir * ir;
}

// One neighbour's contribution to F_i, (H u)_i and the half pair energy.
// dx = x_i - x_j (float64, minimum image), r2 its exactly rounded square
// norm.  The term is evaluated branch-free; a neighbour that is not `live`
// (outside rc) contributes exactly zero.  Tip-tip pairs of a model with tip
// bonds take the bond instead of the LJ terms (compiled in with EXT_BONDS
// only: kernels that never see such a model keep the LJ-only registers).
// With EXT_CURV also the pair's share of T[u,u], the gradient of u.H(r)u at
// fixed u: (C |w|^2 + Dc (dx.w)^2) dx + 2 C (dx.w) w with Dc = (dC/dr)/r.
// WITH_E = false, or EXT_NOE, leaves the energy out (a step whose energy
// nobody reads).
// With EXT_EIG also, for the eigenvalue bias, the pair's shares of H w and
// T[w,w] with w = wi - wj the mode estimate's difference (T[w,w] in the X
// accumulator: the curvature and the eigenvalue bias are not combined).
template <int DIM, typename T, int EXT = 0, bool WITH_E = true>
__device__ __forceinline__ void pair_term(const LJRow<T> &R, int tj, bool live, const double dx[3], double r2,
                                          const T ui[3], const T uj[3], PairAcc<T> &acc,
                                          const T *wi = nullptr, const T *wj = nullptr) {
  constexpr bool BONDS = (EXT & EXT_BONDS) != 0, CURV = (EXT & EXT_CURV) != 0, EIG = (EXT & EXT_EIG) != 0;
  constexpr bool WE = WITH_E && (EXT & EXT_NOE) == 0;
  if constexpr (sizeof(T) == 8) {
    double f, C, e, Dc = 0.0;
    if (BONDS && R.bond && tj) {
      bond_terms<double>(R, r2, f, C, e, Dc);
    } else {
      // outside the cut: epsilon and the shift are zero, r2 stands in as 1
      const double r2i = 1.0 / (live ? r2 : 1.0);
      const double eps = live ? (tj ? R.eps[1] : R.eps[0]) : 0.0;
      const double sr2 = (tj ? R.sig2[1] : R.sig2[0]) * r2i;
      const double sr6 = sr2 * sr2 * sr2;
      f = eps * r2i * sr6 * (48.0 * sr6 - 24.0);
      C = eps * r2i * r2i * sr6 * (672.0 * sr6 - 192.0);
      e = 4.0 * eps * (sr6 * sr6 - sr6) - (live ? (tj ? R.shift[1] : R.shift[0]) : 0.0);
      if constexpr (CURV || EIG) Dc = eps * r2i * r2i * r2i * sr6 * (-10752.0 * sr6 + 1920.0);
    }
    if constexpr (EIG) {
      double om[3], Do = 0.0, o2 = 0.0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        om[k] = wi[k] - wj[k];
        Do += dx[k] * om[k];
        o2 += om[k] * om[k];
      }
      const double CDo = C * Do, a = C * o2 + Dc * Do * Do, b = 2.0 * CDo;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        acc.W[k] += CDo * dx[k] - f * om[k];
        acc.X[k] += a * dx[k] + b * om[k];
      }
    }
    double w[3], Dw = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      w[k] = ui[k] - uj[k];
      Dw += dx[k] * w[k];
    }
    const double CDw = C * Dw;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      acc.F[k] += f * dx[k];
      acc.H[k] += CDw * dx[k] - f * w[k];
    }
    if constexpr (WE) acc.e += 0.5 * e;
    if constexpr (CURV) {
      double w2 = 0.0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) w2 += w[k] * w[k];
      const double a = C * w2 + Dc * Dw * Dw, b = 2.0 * CDw;
#pragma unroll
      for (int k = 0; k < DIM; ++k) acc.X[k] += a * dx[k] + b * w[k];
    }
  } else {
    float f, C, e, Dc = 0.0f;
    if (BONDS && R.bond && tj) {
      bond_terms<float>(R, r2, f, C, e, Dc);
    } else {
      // outside the cut: epsilon and the shift are zero, r2 stands in as 1
      const float r2i = rcp_nr(live ? (float)r2 : 1.0f);
      const float eps = live ? (tj ? R.eps[1] : R.eps[0]) : 0.0f;
      const float sr2 = (tj ? R.sig2[1] : R.sig2[0]) * r2i;
      const float sr6 = sr2 * sr2 * sr2;
      const float epsr = eps * r2i * sr6;
      f = epsr * (48.0f * sr6 - 24.0f);
      C = epsr * r2i * (672.0f * sr6 - 192.0f);
      e = 4.0f * eps * sr6 * (sr6 - 1.0f) - (live ? (tj ? R.shift[1] : R.shift[0]) : 0.0f);
      if constexpr (CURV || EIG) Dc = epsr * r2i * r2i * (-10752.0f * sr6 + 1920.0f);
    }
    float d[3], w[3], Dw = 0.0f;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      d[k] = (float)dx[k];
      w[k] = ui[k] - uj[k];
      Dw = __builtin_fmaf(d[k], w[k], Dw);
    }
    if constexpr (EIG) {
      float om[3], Do = 0.0f, o2 = 0.0f;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        om[k] = wi[k] - wj[k];
        Do = __builtin_fmaf(d[k], om[k], Do);
        o2 = __builtin_fmaf(om[k], om[k], o2);
      }
      const float CDo = C * Do, a = __builtin_fmaf(Dc * Do, Do, C * o2), b = 2.0f * CDo;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        acc.W[k].add(__builtin_fmaf(CDo, d[k], -f * om[k]));
        acc.X[k].add(__builtin_fmaf(a, d[k], b * om[k]));
      }
    }
    const float CDw = C * Dw;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      acc.F[k].add(f * d[k]);
      acc.H[k].add(__builtin_fmaf(CDw, d[k], -f * w[k]));
    }
    if constexpr (WE) acc.e.add(0.5f * e);
    if constexpr (CURV) {
      float w2 = 0.0f;
#pragma unroll
      for (int k = 0; k < DIM; ++k) w2 = __builtin_fmaf(w[k], w[k], w2);
      const float a = __builtin_fmaf(Dc * Dw, Dw, C * w2), b = 2.0f * CDw;
#pragma unroll
      for (int k = 0; k < DIM; ++k) acc.X[k].add(__builtin_fmaf(a, d[k], b * w[k]));
    }
  }
}

// Float32 pair vectors for a half list: f_ij Delta (force on i), h_ij (the
// pair's H u contribution to i) and the pair energy; j receives the negatives.
template <int DIM, bool BONDS = false>
__device__ __forceinline__ void pair_vals_f(const LJRow<float> &R, int tj, bool live, const double dx[3], double r2,
                                            const float ui[3], const float uj[3], float fv[3], float hv[3],
                                            float &e) {
  float f, C;
  if (BONDS && R.bond && tj) {
    float Dc;
    bond_terms<float>(R, r2, f, C, e, Dc);
  } else {
    const float m = live ? 1.0f : 0.0f;
    const float r2i = rcp_nr(live ? (float)r2 : 1.0f);
    const float eps = (tj ? R.eps[1] : R.eps[0]) * m;
    const float sr2 = (tj ? R.sig2[1] : R.sig2[0]) * r2i;
    const float sr6 = sr2 * sr2 * sr2;
    const float epsr = eps * r2i * sr6;
    f = epsr * (48.0f * sr6 - 24.0f);
    C = epsr * r2i * (672.0f * sr6 - 192.0f);
    e = 4.0f * eps * sr6 * (sr6 - 1.0f) - (tj ? R.shift[1] : R.shift[0]) * m;
  }
  float d[3], w[3], Dw = 0.0f;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    d[k] = (float)dx[k];
    w[k] = ui[k] - uj[k];
    Dw = __builtin_fmaf(d[k], w[k], Dw);
  }
  const float CDw = C * Dw;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    fv[k] = f * d[k];
    hv[k] = __builtin_fmaf(CDw, d[k], -f * w[k]);
  }
}

// Displacement x_i - x_j (minimum image) and r^2 = (dx*dx + dy*dy) + dz*dz,
// rounded operation by operation so that the cutoff decision is exactly the
// float64 one.
//
// r2 + d*d rounded twice, as the float64 rule has it: no fused multiply-add
// (the pragma keeps the compiler from contracting the pair).
__device__ __forceinline__ double add_sq_exact(double r2, double d) {
#pragma clang fp contract(off)
  const double p = d * d;
  return r2 + p;
}

// Branch-free minimum image: dx - L rint(dx/L) (inv_box is 0 on open axes).
// Every pair of a list is closer than rc + skin <= L/2, and for those this
// equals the strict rule (subtract/add L beyond +-L/2) exactly: the shift is
// an exact multiple of L and the single rounding matches.
template <int DIM>
__device__ __forceinline__ double pair_disp(const SysDesc &D, const double xi[3], const double xj[3],
                                            double dx[3]) {
  double r2 = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const double raw = xi[k] - xj[k];
    dx[k] = __builtin_fma(-D.box[k], __builtin_rint(raw * D.inv_box[k]), raw);
    r2 = add_sq_exact(r2, dx[k]);
  }
  return r2;
}

// Pair pass of atom i over its full list in global memory.
template <int DIM, typename T>
__device__ __forceinline__ void pair_atom(const SysDesc &D, const Arrays &A, int i,
                                          const double xi[3], const T ui[3], int ti,
                                          PairAcc<T> &acc) {
  const int64_t off = D.off, N = A.ntot;
  const int n = D.n;
  const T *__restrict__ u = (const T *)A.u;
  const double *__restrict__ x = A.x;
  const int32_t *__restrict__ nbr = A.nbr + D.nbr_off;
  const int nn = A.nnb[off + i];
  LJRow<T> R;
  R.load(D, ti);
#pragma unroll 2
  for (int q = 0; q < nn; ++q) {
    const int ent = nbr[(int64_t)q * n + i];
    const int64_t aj = off + (ent >> 1);
    double xj[3], dx[3];
    T uj[3];
#pragma unroll
    for (int k = 0; k < DIM; ++k) { xj[k] = x[k * N + aj]; uj[k] = u[k * N + aj]; }
    const double r2 = pair_disp<DIM>(D, xi, xj, dx);
    pair_term<DIM, T>(R, ent & 1, r2 < D.rc2, dx, r2, ui, uj, acc);
  }
}

// pair_disp with the last axis known periodic (LASTP) or open: on an open
// axis the minimum image is an exact no-op (inv_box = box = 0), so skipping it
// changes no bit and saves three float64 operations per neighbour.
template <int DIM, bool LASTP>
__device__ __forceinline__ double pair_disp_l(const SysDesc &D, const double xi[3], const double xj[3],
                                              double dx[3]) {
  double r2 = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const double raw = xi[k] - xj[k];
    if (LASTP || k < DIM - 1) dx[k] = __builtin_fma(-D.box[k], __builtin_rint(raw * D.inv_box[k]), raw);
    else dx[k] = raw;
    r2 = add_sq_exact(r2, dx[k]);
  }
  return r2;
}

// Grid-plan neighbour lists: the entries of a sorted position come in
// blocks of four consecutive slots, block b of position i in the four entries
// from (b n + i) 4, so that the four lanes of an atom's quad (slots s, s + 4,
// ... for lane s) read one contiguous piece per load, and a wavefront's
// lanes (16 consecutive positions) one contiguous run.  Capacity: the
// per-system region holds roundup4(maxnb) n entries.
__host__ __device__ inline int64_t grid_list_index(int64_t k, int64_t n, int64_t i) {
  return ((k >> 2) * n + i) * 4 + (k & 3);
}
// Byte offsets of a sorted position's grid-list entries.
struct ListAddr {
  uint32_t base, row;   // the position's first entry; one block row (4 n entries)
  uint32_t esz;         // bytes per entry
  __device__ __forceinline__ uint32_t at(int k) const {
    return ((uint32_t)k >> 2) * row + base + ((uint32_t)k & 3u) * esz;
  }
};

// List entries gathered together in the bonded pair loop.
constexpr int kGatherBlock = 4;

// The neighbour loop of pair_atom_rec (one or two lanes per atom): lane q0 of
// qstep takes entries q0, q0 + qstep, ... of the grid list, addressed by
// 32-bit byte offsets like the records (offsets from the system's uniform
// bases, so that both loads take a scalar base).
template <int DIM, typename T, int EXT, bool LASTP, bool E16 = false>
__device__ __forceinline__ void pair_loop_rec(const SysDesc &D, const LJRow<T> &R, const char *__restrict__ recb,
                                              const char *__restrict__ nbrb, const ListAddr la, int q0, int qstep,
                                              int cnt, const double xi[3], const T ui[3], PairAcc<T> &acc,
                                              const char *__restrict__ recwb = nullptr, const T *wi = nullptr) {
  if constexpr ((EXT & EXT_EIG) != 0) {
    // eigenvalue bias: the neighbour's mode estimate comes from its 32-byte
    // mode record beside the pair record
    for (int c = 0; c < cnt; ++c) {
      const int ent = __builtin_nontemporal_load((const int32_t *)(nbrb + la.at(q0 + c * qstep)));
      const uint32_t pj = (uint32_t)ent >> 1;
      const double *r = (const double *)(recb + (pj << 6));
      const double *rw = (const double *)(recwb + (pj << 5));
      double xj[3], dx[3];
      T uj[3], wj[3];
#pragma unroll
      for (int k = 0; k < DIM; ++k) { xj[k] = r[k]; uj[k] = rec_u<T>(r, k); wj[k] = (T)rw[k]; }
      const double r2 = pair_disp_l<DIM, LASTP>(D, xi, xj, dx);
      pair_term<DIM, T, EXT>(R, ent & 1, r2 < D.rc2, dx, r2, ui, uj, acc, wi, wj);
    }
  } else if constexpr ((EXT & EXT_BONDS) != 0) {
    // With tip bonds the pair term branches (bond or LJ), which keeps the
    // compiler from hoisting the next neighbours' gathers over it: a block of
    // kGatherBlock list entries and their records is loaded before the
    // block's arithmetic (entries past the end repeat the block's first), and
    // the terms are then added in list order as below.
    for (int c0 = 0; c0 < cnt; c0 += kGatherBlock) {
      int ent[kGatherBlock];
#pragma unroll
      for (int u4 = 0; u4 < kGatherBlock; ++u4) {
        const uint32_t o = la.at(q0 + (c0 + u4 < cnt ? c0 + u4 : c0) * qstep);
        ent[u4] = __builtin_nontemporal_load((const int32_t *)(nbrb + o));
      }
      double xj[kGatherBlock][3];
      T uj[kGatherBlock][3];
#pragma unroll
      for (int u4 = 0; u4 < kGatherBlock; ++u4) {
        const double *r = (const double *)(recb + (((uint32_t)ent[u4] >> 1) << 6));
#pragma unroll
        for (int k = 0; k < DIM; ++k) { xj[u4][k] = r[k]; uj[u4][k] = rec_u<T>(r, k); }
      }
#pragma unroll
      for (int u4 = 0; u4 < kGatherBlock; ++u4) {
        if (c0 + u4 < cnt) {
          double dx[3];
          const double r2 = pair_disp_l<DIM, LASTP>(D, xi, xj[u4], dx);
          pair_term<DIM, T, EXT>(R, ent[u4] & 1, r2 < D.rc2, dx, r2, ui, uj[u4], acc);
        }
      }
    }
  } else {
#pragma unroll 4
    for (int c = 0; c < cnt; ++c) {
      // the list is read once per step: a streaming load, so that it does not
      // evict the records the neighbouring atoms share
      const uint32_t o = la.at(q0 + c * qstep);
      const int ent = E16 ? (int)__builtin_nontemporal_load((const uint16_t *)(nbrb + o))
                          : __builtin_nontemporal_load((const int32_t *)(nbrb + o));
      const double *r = (const double *)(recb + (((uint32_t)ent >> 1) << 6));
      double xj[3], dx[3];
      T uj[3];
#pragma unroll
      for (int k = 0; k < DIM; ++k) { xj[k] = r[k]; uj[k] = rec_u<T>(r, k); }
      const double r2 = pair_disp_l<DIM, LASTP>(D, xi, xj, dx);
      pair_term<DIM, T, EXT>(R, ent & 1, r2 < D.rc2, dx, r2, ui, uj, acc);
    }
  }
}

// Quad gather for four lanes per atom.  The plain loop has every lane load its
// neighbour's record itself, in three loads whose lanes touch up to 64
// different cache lines each.  Here the quad of an atom fetches the records
// of its four lanes' neighbours one after the other, lane s bringing bytes
// 16s..16s+15 of the record straight into LDS, so that each load touches one
// line per quad (about half the vector-L1 lookups per pair); every lane then
// reads its own neighbour (x and u, the record's first 36 or 48 bytes) from
// LDS.  The next round's list entries are requested behind the records, so
// that their memory latency overlaps the round's arithmetic.  The LDS slot of
// a load is 1024 + 16 bytes per wavefront: with that stride the 16 lanes
// served together by an LDS read take 16 different bank groups.  With the
// eigenvalue bias each lane also loads its neighbour's mode record itself.
// Two neighbours per lane per round: larger rounds take more
// LDS than they gain (the LDS then bounds the workgroups per CU).
constexpr int kQuadUnroll = 2;               // neighbours per lane per round
constexpr int kQuadSlot = 1040;              // bytes per load in a wavefront's LDS area
constexpr int kQuadWaveBytes = kQuadUnroll * 4 * kQuadSlot;

template <int Q>
__device__ __forceinline__ int quad_bcast(int v) {   // lane Q's value to its whole quad
  return __builtin_amdgcn_update_dpp(0, v, Q * 0x55, 0xf, 0xf, true);
}

// One 16-byte chunk of a record into a lane's place in an LDS slot.
__device__ __forceinline__ void lds_chunk(const char *__restrict__ src, char *slot) {
  __builtin_amdgcn_global_load_lds((const void *)src, (__attribute__((address_space(3))) void *)slot, 16, 0, 0);
}

// The neighbour loop of one lane of a quad: cnt is the lane's entry count,
// rounds the quad's (every lane of the quad runs them, so that the quad's
// loads are complete; entries past a lane's count are its own position,
// masked).  lds is this wavefront's kQuadWaveBytes area (wave-uniform).
template <int DIM, typename T, int EXT, bool LASTP, bool E16>
__device__ __forceinline__ void pair_loop_quad(const SysDesc &D, const LJRow<T> &R, const char *__restrict__ recb,
                                               const char *__restrict__ nbrb, uint32_t lo, uint32_t lstep, int cnt,
                                               int rounds, int self, const double xi[3], const T ui[3],
                                               PairAcc<T> &acc, char *lds, const char *__restrict__ recwb = nullptr,
                                               const T *wi = nullptr) {
  constexpr bool EIG = (EXT & EXT_EIG) != 0;
  const uint32_t chunk = (threadIdx.x & 3) * 16;
  const int rd = (threadIdx.x & 3) * kQuadSlot + ((threadIdx.x & 63) >> 2) * 64;   // own record in a round's slot
  // the system's constants in registers: the waits below are compiler
  // barriers, across which loads through D would be repeated
  const double rc2 = D.rc2;
  double box[3], ibox[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) { box[k] = D.box[k]; ibox[k] = D.inv_box[k]; }
  const uint32_t lo0 = lo;
  // list entries c .. c + kQuadUnroll - 1 of this lane, as loaded (past its
  // count: from an address inside its list, replaced by use() with its own
  // position)
  auto entries = [&](int c, int (&ent)[kQuadUnroll]) {
#pragma unroll
    for (int j = 0; j < kQuadUnroll; ++j) {
      const uint32_t o = c + j < cnt ? lo + (uint32_t)j * lstep : lo0;
      ent[j] = E16 ? (int)__builtin_nontemporal_load((const uint16_t *)(nbrb + o))
                   : __builtin_nontemporal_load((const int32_t *)(nbrb + o));
    }
    lo += (uint32_t)kQuadUnroll * lstep;
  };
  auto use = [&](int c, int (&ent)[kQuadUnroll]) {
#pragma unroll
    for (int j = 0; j < kQuadUnroll; ++j) ent[j] = c + j < cnt ? ent[j] : self << 1;
  };
  int ent[kQuadUnroll];
  entries(0, ent);
  use(0, ent);
  for (int c = 0; c < rounds * kQuadUnroll; c += kQuadUnroll) {
    // the last round's LDS reads are complete before its slots are refilled
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    // each lane's record offset to its whole quad, plus the lane's chunk
    // (DPP adds, with every lane of the quad active)
    uint32_t o[kQuadUnroll][4];
#pragma unroll
    for (int j = 0; j < kQuadUnroll; ++j) {
      const uint32_t roff = ((uint32_t)ent[j] >> 1) << 6;
      o[j][0] = (uint32_t)quad_bcast<0>((int)roff) + chunk;
      o[j][1] = (uint32_t)quad_bcast<1>((int)roff) + chunk;
      o[j][2] = (uint32_t)quad_bcast<2>((int)roff) + chunk;
      o[j][3] = (uint32_t)quad_bcast<3>((int)roff) + chunk;
    }
    // a neighbour needs the record's first 48 bytes: the quad's fourth lane
    // loads nothing
    if (chunk < 48) {
#pragma unroll
      for (int j = 0; j < kQuadUnroll; ++j)
#pragma unroll
        for (int t = 0; t < 4; ++t) lds_chunk(recb + o[j][t], lds + (j * 4 + t) * kQuadSlot);
    }
    // eigenvalue bias: each lane loads its neighbour's mode component itself
    // (32-byte mode records beside the pair records)
    T wj[kQuadUnroll][3];
    if constexpr (EIG) {
#pragma unroll
      for (int j = 0; j < kQuadUnroll; ++j) {
        const double *rw = (const double *)(recwb + (((uint32_t)ent[j] >> 1) << 5));
#pragma unroll
        for (int k = 0; k < DIM; ++k) wj[j][k] = (T)rw[k];
      }
    }
    // the next round's entries are requested after this round's records (a
    // compiler barrier keeps that order), so that the wait below, which
    // leaves the last kQuadUnroll loads in flight, covers the records only;
    // the loads write LDS behind the compiler's back, hence the explicit wait
    int nxt[kQuadUnroll];
    asm volatile("" ::: "memory");
    entries(c + kQuadUnroll, nxt);
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(kQuadUnroll) : "memory");
#pragma unroll
    for (int j = 0; j < kQuadUnroll; ++j) {
      const double *r = (const double *)(lds + j * 4 * kQuadSlot + rd);
      double xj[3], dx[3];
      T uj[3];
#pragma unroll
      for (int k = 0; k < DIM; ++k) { xj[k] = r[k]; uj[k] = rec_u<T>(r, k); }
      double r2 = 0.0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        const double raw = xi[k] - xj[k];
        if (LASTP || k < DIM - 1) dx[k] = __builtin_fma(-box[k], __builtin_rint(raw * ibox[k]), raw);
        else dx[k] = raw;
        r2 = add_sq_exact(r2, dx[k]);
      }
      pair_term<DIM, T, EXT>(R, ent[j] & 1, c + j < cnt && r2 < rc2, dx, r2, ui, uj, acc, wi, EIG ? wj[j] : nullptr);
    }
#pragma unroll
    for (int j = 0; j < kQuadUnroll; ++j) ent[j] = nxt[j];
    use(c + kQuadUnroll, ent);
  }
}

// Pair pass of the atom at sorted position p over its full list (entries
// hold sorted positions), neighbours read from the packed records; same
// arithmetic as pair_atom.  Lane q0 of qstep lanes takes entries q0,
// q0 + qstep, ...  With QUAD (four lanes per atom) the quad gather above, in
// the wavefront's LDS area quad_lds.
template <int DIM, typename T, int EXT = 0, bool E16 = false, bool QUAD = false>
__device__ __forceinline__ void pair_atom_rec(const SysDesc &D, const Arrays &A, int p,
                                              const double xi[3], const T ui[3], int ti,
                                              PairAcc<T> &acc, int q0 = 0, int qstep = 1,
                                              const T *wi = nullptr, char *quad_lds = nullptr) {
  static_assert(!E16 || (EXT & ~EXT_NOE) == 0, "16-bit lists serve the LJ-only pass");
  static_assert(kRecDoubles == 8, "records are 64 bytes");
  const int64_t off = D.off;
  const int n = D.n;
  const char *recb = (const char *)(A.rec + off * kRecDoubles);
  const char *nbrb = (const char *)(A.nbr + D.nbr_off);
  const int nn = A.nnb[off + p];
  const int cnt = nn > q0 ? (nn - q0 + qstep - 1) / qstep : 0;
  constexpr uint32_t esz = E16 ? 2u : 4u;   // bytes per list entry
  const ListAddr la{(uint32_t)p * 4u * esz, (uint32_t)n * 4u * esz, esz};
  const char *recwb = (EXT & EXT_EIG) != 0 ? (const char *)(A.recw + off * 4) : nullptr;
  LJRow<T> R;
  R.load(D, ti);
  if constexpr (QUAD) {
    // (qstep == 4) every lane of the quad runs the rounds of its first lane;
    // lane q0's entries q0 + 4c are one block row apart
    const uint32_t lo = la.at(q0), lstep = la.row;
    const int rounds = ((nn + 3) / 4 + kQuadUnroll - 1) / kQuadUnroll;
    if (D.periodic[DIM - 1])
      pair_loop_quad<DIM, T, EXT, true, E16>(D, R, recb, nbrb, lo, lstep, cnt, rounds, p, xi, ui, acc, quad_lds,
                                             recwb, wi);
    else
      pair_loop_quad<DIM, T, EXT, false, E16>(D, R, recb, nbrb, lo, lstep, cnt, rounds, p, xi, ui, acc, quad_lds,
                                              recwb, wi);
    return;
  }
  if (D.periodic[DIM - 1])
    pair_loop_rec<DIM, T, EXT, true, E16>(D, R, recb, nbrb, la, q0, qstep, cnt, xi, ui, acc, recwb, wi);
  else
    pair_loop_rec<DIM, T, EXT, false, E16>(D, R, recb, nbrb, la, q0, qstep, cnt, xi, ui, acc, recwb, wi);
}

// ---------------------------------------------------------------------------
// Workgroup reductions (wavefront 64).  Deterministic: fixed shuffle tree and
// fixed order over waves.  lds must hold NV * 16 doubles.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double x = v[k];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    v[k] = x;
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) lds[k * 16 + wave] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += lds[k * 16 + w];
    v[k] = s;
  }
  __syncthreads();
}

// Cross-lane move of a double by a DPP control (both 32-bit halves move the
// same way; lanes without a source read 0).
template <int CTRL>
__device__ __forceinline__ double dpp_mov_f64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  int lo = (int)(unsigned)(b & 0xffffffffull), hi = (int)(unsigned)(b >> 32);
  lo = __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xf, 0xf, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

// Sum over the 64 lanes of a wavefront with DPP (quad permutes, row shifts,
// row broadcasts), fixed order; every lane receives the total (read from lane
// 63).
// Wavefront totals of NP values at once (NP a power of two, at most 64):
// a reduce-scatter butterfly.  At stage s each lane keeps one half of its
// current values (lower or upper half by lane bit s) and adds the partner's
// (lane ^ 2^s) copy of that half, so the work shrinks by half per stage
// instead of staying NP; after log2(NP) stages the remaining stages add one
// value.  On return every lane holds the total
// of value index wave_scatter_index<NP>(lane).  Fixed order: deterministic.
template <int NP>
__device__ __forceinline__ double wave_sums_scatter(double (&v)[NP], int lane) {
  static_assert((NP & (NP - 1)) == 0 && NP <= 64, "NP must be a power of two");
  constexpr int LOG = NP >= 64 ? 6 : NP >= 32 ? 5 : NP >= 16 ? 4 : NP >= 8 ? 3 : NP >= 4 ? 2 : NP >= 2 ? 1 : 0;
#pragma unroll
  for (int s = 0; s < LOG; ++s) {
    const int half = NP >> (s + 1);
    const bool upper = (lane >> s) & 1;
#pragma unroll
    for (int j = 0; j < half; ++j) {
      // the partner's share of the half this lane keeps arrives in
      // (lower lanes keep j, upper lanes keep j + half)
      const double from_lo = __shfl_xor(v[j], 1 << s, 64);
      const double from_hi = __shfl_xor(v[j + half], 1 << s, 64);
      const double sum_lo = v[j] + from_lo, sum_hi = v[j + half] + from_hi;
      v[j] = upper ? sum_hi : sum_lo;
    }
  }
  double t = v[0];
#pragma unroll
  for (int s = LOG; s < 6; ++s) t += __shfl_xor(t, 1 << s, 64);
  return t;
}

// The value index whose total lane holds after wave_sums_scatter<NP>.
template <int NP>
__device__ __forceinline__ int wave_scatter_index(int lane) {
  int q = 0;
#pragma unroll
  for (int s = 0; (NP >> (s + 1)) >= 1; ++s) q += ((lane >> s) & 1) * (NP >> (s + 1));
  return q;
}

// Value of v in lane l, returned to every lane (uniform).
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ __forceinline__ double wave_sum_f64(double v) {
  v += dpp_mov_f64<0xb1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov_f64<0x4e>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov_f64<0x114>(v);  // row_shr:4
  v += dpp_mov_f64<0x118>(v);  // row_shr:8
  v += dpp_mov_f64<0x142>(v);  // row_bcast:15
  v += dpp_mov_f64<0x143>(v);  // row_bcast:31
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), 63);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Workgroup sum of NV doubles: DPP within each wavefront, then the wave
// totals added in wave order.  lds must hold NV * 16 doubles.
template <int NV>
__device__ __forceinline__ void block_sum_dpp(double (&v)[NV], double *lds) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum_f64(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) lds[k * 16 + wave] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double t[16];
#pragma unroll
    for (int w = 0; w < 16; ++w) t[w] = lds[k * 16 + w];  // all loads in flight at once
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < 16; ++w) s += (w < nw) ? t[w] : 0.0;
    v[k] = s;
  }
  __syncthreads();
}

// Workgroup OR of one flag per thread with a single barrier: each wavefront
// writes its ballot to its own slot (slots alternate between two banks so the
// next call needs no clearing barrier).  lds_int holds >= 32 ints.
__device__ __forceinline__ int block_any(int v, int *lds_int, int &parity) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int nw = (blockDim.x + 63) >> 6;
  const unsigned long long b = __ballot(v != 0);
  int *slot = lds_int + 16 * parity;
  if (lane == 0) slot[wave] = b != 0ull ? 1 : 0;
  __syncthreads();
  int r = 0;
#pragma unroll
  for (int w = 0; w < 16; ++w) r |= (w < nw) ? slot[w] : 0;
  parity ^= 1;
  return r;
}

__device__ __forceinline__ int block_or(int v, int *lds_int) {
  if (threadIdx.x == 0) *lds_int = 0;
  __syncthreads();
  if (v) atomicOr(lds_int, 1);
  __syncthreads();
  const int r = *lds_int;
  __syncthreads();
  return r;
}

// Exclusive prefix sum of one int per thread across the workgroup; returns
// the exclusive prefix and writes the total.  lds_int holds >= 17 ints.
__device__ __forceinline__ int block_exscan(int v, int *lds_int, int &total) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds_int[wave] = x;
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int w = 0; w < nw; ++w) { const int t = lds_int[w]; lds_int[w] = run; run += t; }
    lds_int[16] = run;
  }
  __syncthreads();
  const int r = lds_int[wave] + x - v;
  total = lds_int[16];
  __syncthreads();
  return r;
}

}  // namespace hdk
