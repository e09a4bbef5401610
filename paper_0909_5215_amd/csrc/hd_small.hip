// LDS-resident batched kernel for systems that fit one workgroup: one thread
// per atom, the atom's own x, v and total force in registers, and the
// system's positions, displacements u = r - r_O, references r_O, build
// positions, cell list and neighbour list in LDS for the whole chunk of
// steps.  A step touches no global memory: the neighbour gathers of the pair
// pass are LDS reads, and the per-system reductions and barriers stay inside
// the workgroup.  State is loaded at the start of a launch and written back
// at its end.
//
// The method is the one of the grid and one-workgroup kernels (BAOAB, LJ +
// H u pair terms, slope bias of eq. 13-14, boosted clock of eq. 3); the
// per-system sums are taken in a different fixed order.
#include <type_traits>

#include "hd_device.h"
#include "hd_launch.h"

namespace hdk {

// Fixed point of the half-list partner sums: units of 2^-32.  A float32
// term rounds once (to nearest) onto the grid; the sum of a pair list's
// terms (each below 2^31 in magnitude, far beyond the instability limit
// on forces) is then exact in 64 bits.
constexpr double kFixScale = 4294967296.0;   // 2^32
__device__ __forceinline__ unsigned long long to_fixed(float v) {
  return (unsigned long long)(long long)__builtin_rint((double)v * kFixScale);
}
__device__ __forceinline__ double from_fixed(unsigned long long a) {
  return (double)(long long)a * (1.0 / kFixScale);
}

struct SmallLayout {
  int nmax, maxnb, cellmax;
  size_t off_x, off_acc, off_ref, off_u, off_nbr, off_cnt, off_cst, off_cat, bytes;
};

// Pair-pass variants ("kind"): 0 float64 with full lists; 1 float32 with half
// lists (each pair once; the partner's share of F, H u and the energy is
// accumulated in LDS, the acc region, as 64-bit fixed point: integer
// addition does not depend on the order the atomics land in); 2 float32
// with full lists.
__host__ __device__ inline SmallLayout small_layout(int dim, int kind, int nmax, int maxnb, int cellmax) {
  const int tsize = kind == 0 ? 8 : 4;
  SmallLayout L;
  L.nmax = nmax; L.maxnb = maxnb; L.cellmax = cellmax;
  size_t o = 0;
  L.off_x = o; o += (size_t)8 * dim * nmax;
  L.off_acc = o; if (kind == 1) o += (size_t)8 * (2 * dim + 1) * nmax;
  // per-atom reference r_O and positions at the last build
  L.off_ref = o; o += (size_t)8 * 2 * dim * nmax;
  L.off_u = o; o += (size_t)tsize * dim * nmax; o = (o + 7) & ~(size_t)7;
  L.off_nbr = o; o += (size_t)2 * maxnb * nmax; o = (o + 7) & ~(size_t)7;
  L.off_cnt = o; o += (size_t)4 * cellmax;
  L.off_cst = o; o += (size_t)4 * (cellmax + 1);
  L.off_cat = o; o += (size_t)4 * nmax; o = (o + 15) & ~(size_t)15;
  L.bytes = o;
  return L;
}

size_t small_lds_bytes(int dim, int kind, int nmax, int maxnb, int cellmax) {
  return small_layout(dim, kind, nmax, maxnb, cellmax).bytes;
}

// Rebuild the cell list and every atom's neighbour list in LDS from the LDS
// positions.  Same cell rule, pair test (r^2 summed axis by axis without
// contraction, strict < (rc+skin)^2) and exclusions as the global version.
template <int DIM, bool HALF>
__device__ int lds_rebuild(const SysDesc &D, const double *__restrict__ xs, uint16_t *__restrict__ nbr,
                           int *__restrict__ cnt, int *__restrict__ cst, int *__restrict__ cat,
                           const uint8_t *__restrict__ tr_all, int stride, int *lds_int, int &nn_own,
                           const double xi[3], int i, int ri) {
  const int tid = threadIdx.x, B = blockDim.x, n = D.n, ncell = D.ncell;
  for (int c = tid; c < ncell; c += B) cnt[c] = 0;
  __syncthreads();
  int my_cell = 0;
  if (i < n) {
    int c3[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      int ck = (int)floor((xi[k] - D.lo[k]) * D.inv_h[k]);
      c3[k] = ck < 0 ? 0 : (ck >= D.nc[k] ? D.nc[k] - 1 : ck);
    }
    my_cell = (c3[2] * D.nc[1] + c3[1]) * D.nc[0] + c3[0];
    atomicAdd(&cnt[my_cell], 1);
  }
  __syncthreads();
  const int chunk = (ncell + B - 1) / B;
  const int c0 = tid * chunk, c1 = min(ncell, c0 + chunk);
  int local = 0;
  for (int c = c0; c < c1; ++c) local += cnt[c];
  int total = 0;
  int run = block_exscan(local, lds_int, total);
  for (int c = c0; c < c1; ++c) { const int k = cnt[c]; cst[c] = run; run += k; cnt[c] = 0; }
  if (tid == 0) cst[ncell] = total;
  __syncthreads();
  if (i < n) {
    const int slot = atomicAdd(&cnt[my_cell], 1);
    cat[cst[my_cell] + slot] = i;
  }
  __syncthreads();
  for (int c = tid; c < ncell; c += B) {
    const int b = cst[c], e = cst[c + 1];
    for (int p = b + 1; p < e; ++p) {
      const int key = cat[p];
      int q = p - 1;
      while (q >= b && cat[q] > key) { cat[q + 1] = cat[q]; --q; }
      cat[q + 1] = key;
    }
  }
  __syncthreads();
  int ov = 0;
  if (i < n) {
    int cc[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      int ck = (int)floor((xi[k] - D.lo[k]) * D.inv_h[k]);
      cc[k] = ck < 0 ? 0 : (ck >= D.nc[k] ? D.nc[k] - 1 : ck);
    }
    int lo3[3] = {0, 0, 0}, hi3[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < DIM; ++k)
      if (D.nc[k] > 1) { lo3[k] = -1; hi3[k] = 1; }
    int count = 0;
    for (int oz = lo3[2]; oz <= hi3[2]; ++oz)
      for (int oy = lo3[1]; oy <= hi3[1]; ++oy)
        for (int ox = lo3[0]; ox <= hi3[0]; ++ox) {
          int q3[3] = {cc[0] + ox, cc[1] + oy, cc[2] + oz};
          bool skip = false;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            if (q3[k] < 0 || q3[k] >= D.nc[k]) {
              if (k < DIM && D.periodic[k]) q3[k] = (q3[k] + D.nc[k]) % D.nc[k];
              else skip = true;
            }
          }
          if (skip) continue;
          const int q = (q3[2] * D.nc[1] + q3[1]) * D.nc[0] + q3[0];
          for (int p = cst[q]; p < cst[q + 1]; ++p) {
            const int j = cat[p];
            // half lists: each pair once, owned by i when (j > i) xor (i + j odd),
            // which gives every atom about half of its neighbours
            if (j == i || (HALF && ((j > i) == (((i + j) & 1) != 0)))) continue;
            const int trj = tr_all[j];
            const int rj = trj >> 1;
            if ((ri == ROLE_FIXED && rj == ROLE_FIXED) || (ri == ROLE_RIGID && rj == ROLE_RIGID)) continue;
            double r2 = 0.0;
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
              const double d = minimg(xs[k * stride + j] - xi[k], D.box[k], D.hbox[k], D.periodic[k]);
              r2 = add_sq_exact(r2, d);
            }
            if (r2 < D.rl2) {
              if (count < D.maxnb) nbr[count * stride + i] = (uint16_t)((j << 1) | (trj & 1));
              ++count;
            }
          }
        }
    nn_own = count < D.maxnb ? count : D.maxnb;
    if (count > D.maxnb) ov = 1;
  }
  return block_or(ov, lds_int + 20);
}

// The scalars of a step that every thread needs for its bias force and
// final half-kick (written by wave 0, read by all after a barrier).
struct Bcast {
  double Fd_n[3];   // drive force per rigid atom
  double hud[3];    // drive Hessian term per rigid atom
  double FR[3];     // total force on the rigid body
  double bias_a, bias_b;
  int bias_live, bad;
};

template <int DIM, typename T, bool HALF, int BLOCK, bool NHC, bool FIRE = false>
__device__ void run_small(const SysDesc &D, SysState *__restrict__ stg, const Arrays &A,
                          int64_t nsteps, int mode, char *lds, const SmallLayout L,
                          FireSys *__restrict__ fire = nullptr, double ftol2 = 0.0) {
  constexpr int NW = BLOCK / 64;       // wavefronts per workgroup
  static_assert(!HALF || sizeof(T) == 4, "half lists are a float32 variant");
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int n = D.n, stride = L.nmax;
  const int64_t N = A.ntot, off = D.off;
  double *xs = (double *)(lds + L.off_x);
  // [2*DIM+1][stride]: F, H u, e of the j side, fixed point (kFixScale units)
  unsigned long long *jacc = (unsigned long long *)(lds + L.off_acc);
  double *rOs = (double *)(lds + L.off_ref);    // [DIM][stride] r_O
  double *xbs = rOs + DIM * stride;             // [DIM][stride] positions at the last build
  T *us = (T *)(lds + L.off_u);
  uint16_t *nbr = (uint16_t *)(lds + L.off_nbr);
  int *cnt = (int *)(lds + L.off_cnt);
  int *cst = (int *)(lds + L.off_cst);
  int *cat = (int *)(lds + L.off_cat);

  constexpr int NV = 4 + 3 * DIM;      // per-system sums of a step
  __shared__ double red[2][NV * 16];  // wave partials, alternating by step
  __shared__ Bcast bc[2];             // the step's scalars for every thread
  __shared__ int lds_int[32];
  __shared__ int vote[32];
  __shared__ uint8_t tr_all[1024];
  __shared__ double sh_zR[2][3];      // rigid-body noise, drawn one step ahead
  __shared__ Scal sh_out;
  __shared__ double sh_xi[4], sh_eta[4], sh_scale;   // Nose-Hoover chain
  __shared__ double red_k[16];

  const int i = tid;
  const bool own = i < n;
  const int64_t a = off + i;
  int tr = 0, role = ROLE_FIXED;
  double x[3] = {0, 0, 0}, v[3] = {0, 0, 0}, ft[3] = {0, 0, 0}, cof[3] = {0, 0, 0};
  if (own) {
    tr = A.tr[a];
    role = tr >> 1;
    tr_all[i] = (uint8_t)tr;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      x[k] = A.x[k * N + a]; v[k] = A.v[k * N + a]; ft[k] = A.ftot[k * N + a];
      cof[k] = A.cofs[k * N + a];
      rOs[k * stride + i] = A.rO[k * N + a];
      xbs[k * stride + i] = A.xb[k * N + a];
    }
  }
  // the rigid body, the step counter and the clock are kept by every thread
  // (identical arithmetic everywhere, so no broadcast barrier is needed)
  double XR[3], VR[3], FR[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) { XR[k] = stg->XR[k]; VR[k] = stg->VR[k]; FR[k] = stg->FR[k]; }
  int64_t step = stg->step;
  double t_md = stg->t_md, t_hyper = stg->t_hyper;
  int flags = stg->flags, rebuilds = stg->n_rebuilds;
  const int rebuild_state = stg->rebuild;
  if (flags & FLAG_UNSTABLE) return;
  const bool compute_only = (mode & 1) != 0;
  const bool rigid_body = D.n_rigid > 0;
  const bool wave_rigid = __ballot(own && role == ROLE_RIGID) != 0;   // uniform per wavefront
  // Nose-Hoover chain in place of the Langevin O step (D.thermostat == 1):
  // the chain lives in LDS and is advanced by thread 0; every step ends with
  // its closing half step and, within the launch, the next step's opening
  // one (one reduction of 2K); the launch opens the first step itself
  // (compiled in only with NHC: the Langevin instantiations stay as they were)
  const bool nhc = NHC && !compute_only && D.thermostat == 1;
  auto nhc_k2 = [&]() -> double {
    double k2[1] = {0.0};
    if (own && role == ROLE_MOBILE)
#pragma unroll
      for (int k = 0; k < DIM; ++k) k2[0] += D.mass * v[k] * v[k];
    block_sum<1>(k2, red_k);
    double K2 = k2[0];
    if (rigid_body)
#pragma unroll
      for (int k = 0; k < DIM; ++k) K2 += D.massR * VR[k] * VR[k];
    return K2;
  };
  if (nhc) {
    if (tid == 0)
      for (int j = 0; j < 4; ++j) { sh_xi[j] = stg->xi[j]; sh_eta[j] = stg->eta[j]; }
    const double K2 = nhc_k2();
    if (tid == 0) sh_scale = nhc_half_step(D, sh_xi, sh_eta, K2);
    __syncthreads();
    const double c = sh_scale;
#pragma unroll
    for (int k = 0; k < DIM; ++k) { v[k] *= c; VR[k] *= c; }
  }
  if (!FIRE && !compute_only && !nhc && rigid_body && tid == 0) {
    double z[3];
    noise<DIM, T>(D.seed, step, (uint32_t)n, z);
#pragma unroll
    for (int k = 0; k < DIM; ++k) sh_zR[step & 1][k] = z[k];
  }
  __syncthreads();   // the first step's rigid-body noise and the atom table are in LDS
  // FIRE (quench mode): the minimiser's state, kept by every thread
  // (identical arithmetic everywhere, like the rigid body)
  double f_dt = 0.0, f_alpha = 0.0;
  int f_since = 0, f_done = 0;
  int64_t f_iters = 0;
  if constexpr (FIRE) {
    f_dt = fire->dt;
    f_alpha = fire->alpha;
    f_since = fire->since_neg;
    // the read-out scalars of the evaluation before the launch, kept when
    // the starting point has already converged
    if (tid == 0) {
      sh_out.e_lj = stg->e_lj; sh_out.v_drive = stg->v_drive; sh_out.e_pot = stg->e_pot;
      sh_out.d = stg->d; sh_out.g = stg->g; sh_out.dv = stg->dv; sh_out.dvp = stg->dvp;
      sh_out.xs = stg->x_slider; sh_out.x_tip = stg->x_tip; sh_out.f_lat = stg->f_lat;
    }
  }

  const int64_t iters = compute_only ? 1 : nsteps;
  // the list lives in LDS only for this launch: rebuild at the start, from
  // the recorded build positions unless an evaluation was requested (an
  // evaluation right after a restored checkpoint also rebuilds from them, so
  // that it leaves the restored run's build positions as they are)
  int rebuild_req = compute_only ? (rebuild_state == 2 ? 2 : 1) : (rebuild_state == 1 ? 1 : 2);
  int vote_parity = 0;
  int nn = 0;
  double F[3] = {0, 0, 0}, H[3] = {0, 0, 0}, e_own = 0.0, fbv[3] = {0, 0, 0};
  // this atom's normals for the coming step, when already drawn
  double zn[3] = {0, 0, 0};
  bool have_zn = false;

  for (int64_t it = 0; it < iters; ++it) {
    int moved = 0;
    if constexpr (FIRE) {
      // ---- FIRE iteration at the current forces: power P = F.v, |v|, |F|
      // over the mobile atoms and the rigid body; converged when no degree
      // of freedom feels |F| >= ftol; else velocity mixing, step-size
      // control and a semi-implicit Euler step (the values of Bitzek et al.)
      double q4[4] = {0.0, 0.0, 0.0, 0.0};
      if (own && role == ROLE_MOBILE) {
        double a2 = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          q4[0] += ft[k] * v[k];
          q4[1] += v[k] * v[k];
          q4[2] += ft[k] * ft[k];
          a2 += ft[k] * ft[k];
        }
        q4[3] = a2 < ftol2 ? 0.0 : 1.0;
      }
      block_sum<4>(q4, red[(step + 1) & 1]);
      double P = q4[0], vv = q4[1], ff = q4[2];
      bool big = q4[3] > 0.0;
      if (rigid_body) {
        double r2 = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          P += FR[k] * VR[k];
          vv += VR[k] * VR[k];
          ff += FR[k] * FR[k];
          r2 += FR[k] * FR[k];
        }
        big = big || !(r2 < ftol2);
      }
      if (!big) {
        f_done = 1;
        f_iters = it;
        break;
      }
      const double vn = sqrt(vv), fn = sqrt(ff);
      double mixv = 0.0, mixf = 0.0;
      const bool reset = !(P > 0.0);
      if (!reset) {
        mixv = 1.0 - f_alpha;
        mixf = fn > 0.0 ? f_alpha * vn / fn : 0.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) VR[k] = mixv * VR[k] + mixf * FR[k];
        if (f_since > kFireNmin) {
          f_dt = fmin(f_dt * kFireFinc, 10.0 * D.dt);
          f_alpha *= kFireFalpha;
        }
        f_since += 1;
      } else {
        f_dt *= kFireFdec;
        f_alpha = kFireAlpha0;
        f_since = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) VR[k] = 0.0;
      }
      if (rigid_body) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          VR[k] += f_dt * FR[k] * D.inv_massR;
          XR[k] += f_dt * VR[k];
        }
      }
      f_iters = it + 1;
      if (own && role == ROLE_MOBILE) {
        double d2 = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          double vk = reset ? 0.0 : mixv * v[k] + mixf * ft[k];
          vk += f_dt * ft[k] * D.inv_mass;
          v[k] = vk;
          x[k] = wrapx(x[k] + f_dt * vk, D.box[k], D.periodic[k]);
          const double dd = minimg(x[k] - xbs[k * stride + i], D.box[k], D.hbox[k], D.periodic[k]);
          d2 += dd * dd;
        }
        if (d2 > D.skin_half2) moved = 1;
      }
    }
    // ---- B A O A: mobile atoms, and the rigid body in every thread --------
    if (!FIRE && !compute_only) {
      if (own && role == ROLE_MOBILE && nhc) {
        // velocity Verlet: half kick, full drift
        double d2 = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          const double vv = v[k] + D.hdt * ft[k] * D.inv_mass;
          x[k] = wrapx(x[k] + D.dt * vv, D.box[k], D.periodic[k]);
          v[k] = vv;
          const double dd = minimg(x[k] - xbs[k * stride + i], D.box[k], D.hbox[k], D.periodic[k]);
          d2 += dd * dd;
        }
        if (d2 > D.skin_half2) moved = 1;
      } else if (own && role == ROLE_MOBILE) {
        double z[3] = {zn[0], zn[1], zn[2]};
        if (!have_zn) noise<DIM, T>(D.seed, step, (uint32_t)i, z);
        have_zn = false;
        double d2 = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          double vv = v[k], xx = x[k];
          vv = vv + D.hdt * ft[k] * D.inv_mass;
          xx = xx + D.hdt * vv;
          vv = D.c1 * vv + D.c2 * z[k];
          xx = xx + D.hdt * vv;
          x[k] = wrapx(xx, D.box[k], D.periodic[k]);
          v[k] = vv;
          const double dd = minimg(x[k] - xbs[k * stride + i], D.box[k], D.hbox[k], D.periodic[k]);
          d2 += dd * dd;
        }
        if (d2 > D.skin_half2) moved = 1;
      }
      if (rigid_body && nhc) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          VR[k] = VR[k] + D.hdt * FR[k] * D.inv_massR;
          XR[k] = XR[k] + D.dt * VR[k];
        }
      } else if (rigid_body) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          double vv = VR[k], xx = XR[k];
          vv = vv + D.hdt * FR[k] * D.inv_massR;
          xx = xx + D.hdt * vv;
          vv = D.c1 * vv + D.c2R * sh_zR[step & 1][k];
          xx = xx + D.hdt * vv;
          XR[k] = xx;
          VR[k] = vv;
        }
      }
    }
    // ---- rigid atoms at X_R + c_i; u = r - r_O (eq. 7); publish to LDS -----
    double u64[3] = {0, 0, 0};
    if (own) {
      if (role == ROLE_RIGID) {
        double d2 = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          x[k] = wrapx(XR[k] + cof[k], D.box[k], D.periodic[k]);
          const double dd = minimg(x[k] - xbs[k * stride + i], D.box[k], D.hbox[k], D.periodic[k]);
          d2 += dd * dd;
        }
        if ((FIRE || !compute_only) && d2 > D.skin_half2) moved = 1;
      }
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        if (role != ROLE_FIXED) u64[k] = minimg(x[k] - rOs[k * stride + i], D.box[k], D.hbox[k], D.periodic[k]);
        xs[k * stride + i] = x[k];
        us[k * stride + i] = (T)u64[k];
      }
      if constexpr (HALF) {
#pragma unroll
        for (int k = 0; k < 2 * DIM + 1; ++k) jacc[k * stride + i] = 0ull;
      }
    }
    const int need = block_any(moved, vote, vote_parity);   // barrier A
    if (need || rebuild_req) {
      // at a launch start the list is rebuilt from the recorded build
      // positions, which reproduces the list of an uninterrupted run
      const bool from_xb = !need && rebuild_req == 2;
      double xsrc[3] = {0, 0, 0};
      if (own)
#pragma unroll
        for (int k = 0; k < DIM; ++k) xsrc[k] = from_xb ? xbs[k * stride + i] : x[k];
      if (from_xb) {
        if (own)
#pragma unroll
          for (int k = 0; k < DIM; ++k) xs[k * stride + i] = xsrc[k];
        __syncthreads();
      }
      const int ov = lds_rebuild<DIM, HALF>(D, xs, nbr, cnt, cst, cat, tr_all, stride, lds_int, nn, xsrc, i, role);
      if (own) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) xbs[k * stride + i] = xsrc[k];
      }
      if (!from_xb) ++rebuilds;
      if (ov) flags |= FLAG_NBR_OVERFLOW;
      if (from_xb) {
        if (own)
#pragma unroll
          for (int k = 0; k < DIM; ++k) xs[k * stride + i] = x[k];
        __syncthreads();
      }
      rebuild_req = 0;
    }
    // ---- pair pass from LDS ------------------------------------------------
    if (own) {
      PairAcc<T> acc;
      acc.init();
      const int ti = tr & 1;
      LJRow<T> R;
      R.load(D, ti);
      T ui[3];
#pragma unroll
      for (int k = 0; k < DIM; ++k) ui[k] = (T)u64[k];
      // versions of the loop for a periodic and an open last axis (the open
      // axis skips its minimum image, an exact no-op: no bit changes), with
      // and without the pair energy: within a launch only the last step's
      // energy is read (the per-step instability test also counts forces
      // beyond the limit, NaN included), so the other steps leave it out
      auto pair_pass = [&](auto last_periodic, auto with_energy) {
        constexpr bool LP = decltype(last_periodic)::value;
        constexpr bool WE = decltype(with_energy)::value;
        if constexpr (HALF) {
          // half list: the pair's vectors go to i (float64 sums, registers) and,
          // negated, to j (fixed-point LDS atomics: each float32 term rounded
          // once to a multiple of 2^-32, then summed exactly, so the j side's
          // total does not depend on the order of the atomics).  The next
          // neighbour's data are loaded before this pair's atomics are issued,
          // so that LDS latency overlaps the arithmetic.
          int ent = nn > 0 ? nbr[i] : 0;
          double xj[3];
          float uj[3];
  #pragma unroll
          for (int k = 0; k < DIM; ++k) { xj[k] = xs[k * stride + (ent >> 1)]; uj[k] = (float)us[k * stride + (ent >> 1)]; }
          for (int q = 0; q < nn; ++q) {
            const int j = ent >> 1, tj = ent & 1;
            double dx[3];
            const double r2 = pair_disp_l<DIM, LP>(D, x, xj, dx);
            const bool live = r2 < D.rc2;
            float fv[3], hv[3], e;
            pair_vals_f<DIM>(R, tj, live, dx, r2, (const float *)ui, uj, fv, hv, e);
            if (q + 1 < nn) {
              ent = nbr[(q + 1) * stride + i];
  #pragma unroll
              for (int k = 0; k < DIM; ++k) { xj[k] = xs[k * stride + (ent >> 1)]; uj[k] = (float)us[k * stride + (ent >> 1)]; }
            }
  #pragma unroll
            for (int k = 0; k < DIM; ++k) { acc.F[k].add(fv[k]); acc.H[k].add(hv[k]); }
            if constexpr (WE) acc.e.add(0.5f * e);
            if (live) {
  #pragma unroll
              for (int k = 0; k < DIM; ++k) {
                atomicAdd(&jacc[k * stride + j], to_fixed(-fv[k]));
                atomicAdd(&jacc[(DIM + k) * stride + j], to_fixed(-hv[k]));
              }
              if constexpr (WE) atomicAdd(&jacc[2 * DIM * stride + j], to_fixed(0.5f * e));
            }
          }
        } else {
  #pragma unroll 4
          for (int q = 0; q < nn; ++q) {
            const int ent = nbr[q * stride + i];
            const int j = ent >> 1;
            double xj[3], dx[3];
            T uj[3];
  #pragma unroll
            for (int k = 0; k < DIM; ++k) { xj[k] = xs[k * stride + j]; uj[k] = us[k * stride + j]; }
            const double r2 = pair_disp_l<DIM, LP>(D, x, xj, dx);
            pair_term<DIM, T, 0, WE>(R, ent & 1, r2 < D.rc2, dx, r2, ui, uj, acc);
          }
        }
      };
      const bool want_e = compute_only || it + 1 == iters;
      if (D.periodic[DIM - 1]) {
        if (want_e) pair_pass(std::true_type{}, std::true_type{});
        else pair_pass(std::true_type{}, std::false_type{});
      } else {
        if (want_e) pair_pass(std::false_type{}, std::true_type{});
        else pair_pass(std::false_type{}, std::false_type{});
      }
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        if constexpr (sizeof(T) == 8) { F[k] = acc.F[k]; H[k] = acc.H[k]; }
        else { F[k] = acc.F[k].get(); H[k] = acc.H[k].get(); }
      }
      if constexpr (sizeof(T) == 8) e_own = acc.e; else e_own = acc.e.get();
    }
    // the rigid body's noise for the next step, drawn while others finish
    if (!FIRE && !compute_only && !nhc && rigid_body && tid == 0) {
      double z[3];
      noise<DIM, T>(D.seed, step + 1, (uint32_t)n, z);
#pragma unroll
      for (int k = 0; k < DIM; ++k) sh_zR[(step + 1) & 1][k] = z[k];
    }
    if constexpr (HALF) {
      __syncthreads();   // barrier B: every pair's j-side share has landed
      if (own) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          F[k] += from_fixed(jacc[k * stride + i]);
          H[k] += from_fixed(jacc[(DIM + k) * stride + i]);
        }
        e_own += from_fixed(jacc[2 * DIM * stride + i]);
      }
    }
    // ---- per-system sums (eq. 5, 7 and the rigid layer): DPP within each
    // wavefront, partials to LDS (barrier C); wave 0 adds them in wave order,
    // evaluates the scalars (eq. 13-14 and the drive) and broadcasts them
    // (barrier D) ---------------------------------------------------------
    double vals[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) vals[q] = 0.0;
    if (own) {
      vals[0] = e_own;
      double f2 = 0.0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) f2 += F[k] * F[k];
      vals[3] = (f2 <= kForceLimit2) ? 0.0 : 1.0;
      if (role != ROLE_FIXED) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) { vals[1] += u64[k] * u64[k]; vals[2] += F[k] * u64[k]; }
      }
      if (role == ROLE_RIGID) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) { vals[4 + k] = F[k]; vals[4 + DIM + k] = H[k]; vals[4 + 2 * DIM + k] = u64[k]; }
      }
    }
    double *rb = red[step & 1];
    if (wave_rigid) {
      // all NV sums, padded to 16 values
      double w16[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) w16[q] = q < NV ? vals[q] : 0.0;
      const double tot = wave_sums_scatter<16>(w16, lane);
      const int q = wave_scatter_index<16>(lane);
      if (lane < 16 && q < NV) rb[q * 16 + wave] = tot;
    } else {
      // the rigid-layer sums are exact zeros in wavefronts without rigid atoms
      double w4[4] = {vals[0], vals[1], vals[2], vals[3]};
      const double tot = wave_sums_scatter<4>(w4, lane);
      if (lane < 4) rb[wave_scatter_index<4>(lane) * 16 + wave] = tot;
      else if (lane < NV) rb[lane * 16 + wave] = 0.0;
    }
    __syncthreads();   // barrier C
    // while wave 0 evaluates the scalars, the other wavefronts draw their
    // atoms' normals for the next step (they depend on the counter only)
    if (!FIRE && wave != 0 && !compute_only && !nhc && own && role == ROLE_MOBILE && it + 1 < iters) {
      noise<DIM, T>(D.seed, step + 1, (uint32_t)i, zn);
      have_zn = true;
    }
    const int64_t estep = compute_only ? step : step + 1;
    Bcast &B = bc[step & 1];
    Scal S;
    if (wave == 0) {
      // lane q adds sum q over the waves in wave order (all loads in flight
      // at once)
      double t = 0.0;
      if (lane < NV) {
        double pw[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) pw[w] = rb[lane * 16 + w];
#pragma unroll
        for (int w = 0; w < NW; ++w) t += pw[w];
      }
      double sums[NRED];
#pragma unroll
      for (int q = 0; q < NRED; ++q) sums[q] = 0.0;
      sums[0] = readlane_f64(t, 0);
      sums[1] = readlane_f64(t, 1);
      sums[2] = readlane_f64(t, 2);
      sums[12] = readlane_f64(t, 3);
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        sums[3 + k] = readlane_f64(t, 4 + k);
        sums[6 + k] = readlane_f64(t, 4 + DIM + k);
        sums[9 + k] = readlane_f64(t, 4 + 2 * DIM + k);
      }
      eval_scalars<DIM>(D, sums, XR, estep, S);
      if (lane == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          B.Fd_n[k] = S.Fd[k] * D.inv_nR;
          B.hud[k] = S.hud[k];
          B.FR[k] = sums[3 + k] + S.Fd[k] + S.sumFb[k];
        }
        B.bias_a = S.bias_a;
        B.bias_b = S.bias_b;
        B.bias_live = (D.bias_on && S.d >= 1e-12 && S.dvp != 0.0) ? 1 : 0;
        B.bad = (!isfinite(S.e_pot) || S.bad > 0.0) ? 1 : 0;
      }
    }
    __syncthreads();   // barrier D
    // the boosted clock (eq. 3) is wave 0's alone, off the others' path
    if (!FIRE && wave == 0 && !compute_only) t_hyper += D.dt * exp(S.dv * D.inv_kT);
    // ---- bias force, total force, final B ------------------------------------
    // one batch of LDS reads, then branch-free arithmetic
    const Bcast Bl = B;
    {
      const bool rigid = own && role == ROLE_RIGID;
      const bool biased = own && role != ROLE_FIXED && Bl.bias_live;
      const bool kick = !FIRE && !compute_only && own && role == ROLE_MOBILE;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        const double f = F[k] + (rigid ? Bl.Fd_n[k] : 0.0);
        const double h = H[k] + (rigid ? Bl.hud[k] : 0.0);
        const double fb = biased ? Bl.bias_a * (h - f - Bl.bias_b * u64[k]) : 0.0;
        F[k] = f;
        H[k] = h;
        fbv[k] = fb;
        ft[k] = f + fb;
        v[k] = kick ? v[k] + D.hdt * ft[k] * D.inv_mass : v[k];
      }
    }
#pragma unroll
    for (int k = 0; k < DIM; ++k) FR[k] = Bl.FR[k];
    if (!FIRE && !compute_only) {
      if (rigid_body)
#pragma unroll
        for (int k = 0; k < DIM; ++k) VR[k] = VR[k] + D.hdt * FR[k] * D.inv_massR;
      t_md += D.dt;
      step = step + 1;
    }
    const bool bad = Bl.bad != 0;
    if (nhc && !bad) {
      // closing half step of this step, opening one of the next
      const double K2 = nhc_k2();
      if (tid == 0) {
        double c = nhc_half_step(D, sh_xi, sh_eta, K2);
        if (it + 1 < iters) c *= nhc_half_step(D, sh_xi, sh_eta, K2 * c * c);
        sh_scale = c;
      }
      __syncthreads();
      const double c = sh_scale;
#pragma unroll
      for (int k = 0; k < DIM; ++k) { v[k] *= c; VR[k] *= c; }
    }
    if (bad) flags |= FLAG_UNSTABLE;
    if ((FIRE || it == iters - 1 || bad) && tid == 0) sh_out = S;
    if (bad) break;
  }
  // ---- write back ----------------------------------------------------------
  double ek[1] = {0.0};
  if (own) {
    T *u = (T *)A.u;
    if (role == ROLE_RIGID) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) v[k] = VR[k];
    }
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      A.x[k * N + a] = x[k]; A.v[k * N + a] = v[k]; A.ftot[k * N + a] = ft[k];
      A.xb[k * N + a] = xbs[k * stride + i];
      A.flj[k * N + a] = F[k]; A.hu[k * N + a] = H[k]; A.fb[k * N + a] = fbv[k];
      u[k * N + a] = us[k * stride + i];
    }
    A.nnb[a] = nn;
    // the list itself lives in LDS; leave a copy in the global list so that
    // read-outs (hd_debug_pairs) see the list the last step used
    int32_t *gl = A.nbr + D.nbr_off;
    for (int q = 0; q < nn; ++q) gl[(int64_t)q * n + i] = (int32_t)nbr[q * stride + i];
    if (role == ROLE_MOBILE)
#pragma unroll
      for (int k = 0; k < DIM; ++k) ek[0] += 0.5 * D.mass * v[k] * v[k];
  }
  __syncthreads();
  block_sum<1>(ek, red[0]);
  if (tid == 0) {
    const Scal &S = sh_out;
    double ekr = 0.0;
    for (int k = 0; k < DIM; ++k) ekr += 0.5 * D.massR * VR[k] * VR[k];
    for (int k = 0; k < 3; ++k) { stg->XR[k] = XR[k]; stg->VR[k] = VR[k]; stg->FR[k] = FR[k]; }
    stg->t_md = t_md;
    stg->t_hyper = t_hyper;
    stg->step = step;
    stg->e_lj = S.e_lj; stg->v_drive = S.v_drive; stg->e_pot = S.e_pot;
    stg->e_kin = ek[0] + (D.n_rigid > 0 ? ekr : 0.0);
    stg->d = S.d; stg->g = S.g; stg->dv = S.dv; stg->dvp = S.dvp;
    stg->kappa = 0.0; stg->dv1 = S.dv; stg->dv2 = 0.0;
    stg->x_slider = S.xs; stg->x_tip = S.x_tip; stg->f_lat = S.f_lat;
    stg->flags = flags;
    stg->n_rebuilds = rebuilds;
    stg->rebuild = 0;
    if (nhc) {
      for (int j = 0; j < 4; ++j) { stg->xi[j] = sh_xi[j]; stg->eta[j] = sh_eta[j]; }
      stg->e_nhc = nhc_energy(D, sh_xi, sh_eta);
    }
    if constexpr (FIRE) {
      fire->dt = f_dt;
      fire->alpha = f_alpha;
      fire->since_neg = f_since;
      fire->done = f_done;
      fire->iters = f_iters;
    }
  }
}

// MODE 0: nsteps BAOAB steps (MODE 2: the same for groups holding a system
// with the Nose-Hoover chain); MODE 1: one evaluation at the current
// positions (separate instantiation so the two never share a profile row).
// One instantiation per dimension and workgroup size, so that the register
// budget follows the launch size.
template <typename T, int DIM, int MODE, int BLOCK, bool HALF>
__global__ __launch_bounds__(BLOCK) void k_small(const SysDesc *__restrict__ descs,
                                                 SysState *__restrict__ states, Arrays A,
                                                 const int32_t *__restrict__ sys_list, int64_t nsteps,
                                                 SmallLayout L) {
  extern __shared__ __align__(16) char lds[];
  const int s = sys_list[blockIdx.x];
  run_small<DIM, T, HALF, BLOCK, MODE == 2>(descs[s], states + s, A, nsteps, MODE & 1, lds, L);
}

// FIRE quench of the listed systems (fire[b] belongs to sys_list[b]): up to
// max_iters iterations in one launch, each one an LDS pair pass at the
// stepping kernel's evaluation (one workgroup of 512 or 1024 threads per
// system: 512 keeps the register budget of the stepping kernel's 512-thread
// variant, without spills).
template <typename T, int DIM, int BLOCK, bool HALF>
__global__ __launch_bounds__(BLOCK) void k_small_fire(const SysDesc *__restrict__ descs,
                                                     SysState *__restrict__ states, Arrays A,
                                                     const int32_t *__restrict__ sys_list, int64_t max_iters,
                                                     SmallLayout L, FireSys *__restrict__ fire, double ftol2) {
  extern __shared__ __align__(16) char lds[];
  const int s = sys_list[blockIdx.x];
  run_small<DIM, T, HALF, BLOCK, false, true>(descs[s], states + s, A, max_iters, 0, lds, L, fire + blockIdx.x,
                                              ftol2);
}

template <typename T, int DIM, int MODE, int BLOCK, bool HALF>
static hipError_t launch_small_t(const SysDesc *descs, SysState *states, const Arrays &A,
                                 const int32_t *sys_list, int nsys, size_t bytes, int64_t nsteps,
                                 SmallLayout L, hipStream_t stream) {
  hipLaunchKernelGGL((k_small<T, DIM, MODE, BLOCK, HALF>), dim3(nsys), dim3(BLOCK), bytes, stream, descs, states,
                     A, sys_list, nsteps, L);
  return hipGetLastError();
}

template <typename T, int DIM, bool HALF>
static hipError_t allow_lds_d(int bytes) {
  const void *fns[9] = {(const void *)k_small<T, DIM, 1, 1024, HALF>, (const void *)k_small<T, DIM, 0, 256, HALF>,
                        (const void *)k_small<T, DIM, 0, 512, HALF>, (const void *)k_small<T, DIM, 0, 1024, HALF>,
                        (const void *)k_small<T, DIM, 2, 256, HALF>, (const void *)k_small<T, DIM, 2, 512, HALF>,
                        (const void *)k_small<T, DIM, 2, 1024, HALF>, (const void *)k_small_fire<T, DIM, 512, HALF>,
                        (const void *)k_small_fire<T, DIM, 1024, HALF>};
  for (const void *f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Allow `bytes` of dynamic LDS for every LDS-resident kernel of this variant
// and dimension (done once per schedule, outside any graph capture).
hipError_t small_allow_lds(int kind, int dim, size_t bytes) {
  if (kind == 0) return dim == 2 ? allow_lds_d<double, 2, false>((int)bytes) : allow_lds_d<double, 3, false>((int)bytes);
  if (kind == 1) return dim == 2 ? allow_lds_d<float, 2, true>((int)bytes) : allow_lds_d<float, 3, true>((int)bytes);
  return dim == 2 ? allow_lds_d<float, 2, false>((int)bytes) : allow_lds_d<float, 3, false>((int)bytes);
}

size_t small_group_bytes(int kind, int dim, int nmax, int maxnb, int cellmax) {
  return small_layout(dim, kind, nmax, maxnb, cellmax).bytes;
}

template <typename T, int DIM, bool HALF>
static hipError_t launch_small_d(const SysDesc *descs, SysState *states, const Arrays &A,
                                 const int32_t *sys_list, int nsys, int block, size_t bytes, int64_t nsteps,
                                 int mode, SmallLayout L, hipStream_t stream) {
  if (mode == 1)
    return launch_small_t<T, DIM, 1, 1024, HALF>(descs, states, A, sys_list, nsys, bytes, nsteps, L, stream);
  if (mode == 2) {
    if (block <= 256)
      return launch_small_t<T, DIM, 2, 256, HALF>(descs, states, A, sys_list, nsys, bytes, nsteps, L, stream);
    if (block <= 512)
      return launch_small_t<T, DIM, 2, 512, HALF>(descs, states, A, sys_list, nsys, bytes, nsteps, L, stream);
    return launch_small_t<T, DIM, 2, 1024, HALF>(descs, states, A, sys_list, nsys, bytes, nsteps, L, stream);
  }
  if (block <= 256)
    return launch_small_t<T, DIM, 0, 256, HALF>(descs, states, A, sys_list, nsys, bytes, nsteps, L, stream);
  if (block <= 512)
    return launch_small_t<T, DIM, 0, 512, HALF>(descs, states, A, sys_list, nsys, bytes, nsteps, L, stream);
  return launch_small_t<T, DIM, 0, 1024, HALF>(descs, states, A, sys_list, nsys, bytes, nsteps, L, stream);
}

hipError_t launch_small(int kind, int dim, const SysDesc *descs, SysState *states, const Arrays &A,
                        const int32_t *sys_list, int nsys, int nmax, int maxnb, int cellmax,
                        int block, int64_t nsteps, int mode, hipStream_t stream) {
  if (nsys <= 0) return hipSuccess;
  // one thread per atom: the workgroup must cover the largest system
  if (nmax > 1024 || block < nmax || (block != 256 && block != 512 && block != 1024)) return hipErrorInvalidValue;
  if (kind < 0 || kind > 2 || (dim != 2 && dim != 3)) return hipErrorInvalidValue;
  const SmallLayout L = small_layout(dim, kind, nmax, maxnb, cellmax);
  const size_t b = L.bytes;
  if (kind == 0)
    return dim == 2 ? launch_small_d<double, 2, false>(descs, states, A, sys_list, nsys, block, b, nsteps, mode, L, stream)
                    : launch_small_d<double, 3, false>(descs, states, A, sys_list, nsys, block, b, nsteps, mode, L, stream);
  if (kind == 1)
    return dim == 2 ? launch_small_d<float, 2, true>(descs, states, A, sys_list, nsys, block, b, nsteps, mode, L, stream)
                    : launch_small_d<float, 3, true>(descs, states, A, sys_list, nsys, block, b, nsteps, mode, L, stream);
  return dim == 2 ? launch_small_d<float, 2, false>(descs, states, A, sys_list, nsys, block, b, nsteps, mode, L, stream)
                  : launch_small_d<float, 3, false>(descs, states, A, sys_list, nsys, block, b, nsteps, mode, L, stream);
}

template <typename T, int DIM, bool HALF>
static hipError_t launch_fire_d(const SysDesc *descs, SysState *states, const Arrays &A, const int32_t *sys_list,
                                int nsys, size_t bytes, int64_t max_iters, SmallLayout L, FireSys *fire,
                                double ftol2, hipStream_t stream) {
  if (L.nmax <= 512)
    hipLaunchKernelGGL((k_small_fire<T, DIM, 512, HALF>), dim3(nsys), dim3(512), bytes, stream, descs, states, A,
                       sys_list, max_iters, L, fire, ftol2);
  else
    hipLaunchKernelGGL((k_small_fire<T, DIM, 1024, HALF>), dim3(nsys), dim3(1024), bytes, stream, descs, states, A,
                       sys_list, max_iters, L, fire, ftol2);
  return hipGetLastError();
}

hipError_t launch_small_fire(int kind, int dim, const SysDesc *descs, SysState *states, const Arrays &A,
                             const int32_t *sys_list, int nsys, int nmax, int maxnb, int cellmax, int64_t max_iters,
                             FireSys *fire, double ftol, hipStream_t stream) {
  if (nsys <= 0) return hipSuccess;
  if (nmax > 1024 || kind < 0 || kind > 2 || (dim != 2 && dim != 3) || max_iters < 1) return hipErrorInvalidValue;
  const SmallLayout L = small_layout(dim, kind, nmax, maxnb, cellmax);
  const size_t b = L.bytes;
  const double f2 = ftol * ftol;
  if (kind == 0)
    return dim == 2 ? launch_fire_d<double, 2, false>(descs, states, A, sys_list, nsys, b, max_iters, L, fire, f2, stream)
                    : launch_fire_d<double, 3, false>(descs, states, A, sys_list, nsys, b, max_iters, L, fire, f2, stream);
  if (kind == 1)
    return dim == 2 ? launch_fire_d<float, 2, true>(descs, states, A, sys_list, nsys, b, max_iters, L, fire, f2, stream)
                    : launch_fire_d<float, 3, true>(descs, states, A, sys_list, nsys, b, max_iters, L, fire, f2, stream);
  return dim == 2 ? launch_fire_d<float, 2, false>(descs, states, A, sys_list, nsys, b, max_iters, L, fire, f2, stream)
                  : launch_fire_d<float, 3, false>(descs, states, A, sys_list, nsys, b, max_iters, L, fire, f2, stream);
}

}  // namespace hdk
