// One-workgroup global-memory kernel of the hyperdynamics-for-sliding hot
// path (gfx950), and the Maxwell-Boltzmann velocity initialisation.
//
// k_batched: one workgroup owns one system for a whole chunk of steps
// (persistent), state and lists in global memory; all synchronisation is
// workgroup barriers, so independent slider positions never wait on each
// other (the parallel slider-position scheme of Sec. 2.3 maps onto the batch
// dimension of the GPU).  It is one of the launch shapes of the autotuner;
// the LDS-resident kernel (hd_small.hip) and the grid kernels (hd_grid.hip)
// share the per-atom arithmetic of hd_device.h with it.
//
// A step is Langevin BAOAB: B-A-O-A on the integrated degrees of freedom
// (mobile atoms, the rigid top layer as one body), neighbour-list refresh when
// an atom has moved more than skin/2, the pair pass (LJ forces, energy and the
// Hessian-vector product H u), per-system reductions, the slope bias
// (eq. 5, eq. 7, eq. 13-14) with its force, the final B, and the boosted clock
// (eq. 3, eq. 8).
#include "hd_device.h"
#include "hd_launch.h"

namespace hdk {

// ---------------------------------------------------------------------------
// Cell grid and neighbour lists
template <int DIM>
__device__ __forceinline__ int cell_of(const SysDesc &D, const double *__restrict__ x, int64_t N, int64_t a) {
  int c3[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    int ck = (int)floor((x[k * N + a] - D.lo[k]) * D.inv_h[k]);
    ck = ck < 0 ? 0 : (ck >= D.nc[k] ? D.nc[k] - 1 : ck);
    c3[k] = ck;
  }
  return (c3[2] * D.nc[1] + c3[1]) * D.nc[0] + c3[0];
}

// Full Verlet list of atom i: all j != i with r^2 < (rc + skin)^2 in the 3^DIM
// neighbouring cells, without fixed-fixed and rigid-rigid pairs.  r^2 is
// summed axis by axis with no contraction.  Returns the number of entries
// (entries beyond maxnb are counted but not stored).
template <int DIM>
__device__ int build_list_atom(const SysDesc &D, const Arrays &A, const double *__restrict__ xs, int i) {
  const int64_t N = A.ntot, off = D.off;
  const int n = D.n;
  const int64_t ai = off + i;
  double xi[3];
#pragma unroll
  for (int k = 0; k < DIM; ++k) xi[k] = xs[k * N + ai];
  const int ri = A.tr[ai] >> 1;
  int cc[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    int ck = (int)floor((xi[k] - D.lo[k]) * D.inv_h[k]);
    cc[k] = ck < 0 ? 0 : (ck >= D.nc[k] ? D.nc[k] - 1 : ck);
  }
  int lo3[3] = {0, 0, 0}, hi3[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    if (D.nc[k] > 1) { lo3[k] = -1; hi3[k] = 1; }
  }
  const int32_t *cstart = A.cell_start + D.cstart_off;
  const int32_t *catoms = A.cell_atoms + off;
  int32_t *list = A.nbr + D.nbr_off;
  int cnt = 0;
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
        const int b = cstart[q], e = cstart[q + 1];
        for (int p = b; p < e; ++p) {
          const int j = catoms[p];
          if (j == i) continue;
          const int64_t aj = off + j;
          const int trj = A.tr[aj];
          const int rj = trj >> 1;
          if ((ri == ROLE_FIXED && rj == ROLE_FIXED) || (ri == ROLE_RIGID && rj == ROLE_RIGID)) continue;
          double r2 = 0.0;
#pragma unroll
          for (int k = 0; k < DIM; ++k) {
            const double d = minimg(xs[k * N + aj] - xi[k], D.box[k], D.hbox[k], D.periodic[k]);
            r2 = add_sq_exact(r2, d);
          }
          if (r2 < D.rl2) {
            if (cnt < D.maxnb) list[(int64_t)cnt * n + i] = (j << 1) | (trj & 1);
            ++cnt;
          }
        }
      }
  return cnt;
}

// Workgroup-wide rebuild of one system's cell list and neighbour lists.
// Counting sort into cells (global atomics, read back with atomic loads),
// exclusive scan, scatter, per-cell sort by index (deterministic order), then
// one list per atom.  Records x at build time for the skin test.
template <int DIM>
__device__ void wg_rebuild(const SysDesc &D, const Arrays &A, const double *__restrict__ xs,
                           int *lds_int, int &overflow) {
  const int tid = threadIdx.x, B = blockDim.x;
  const int n = D.n, ncell = D.ncell;
  const int64_t N = A.ntot, off = D.off;
  int32_t *cnt = A.cell_count + D.cell_off;
  int32_t *cst = A.cell_start + D.cstart_off;
  int32_t *cat = A.cell_atoms + off;
  for (int c = tid; c < ncell; c += B) cnt[c] = 0;
  __syncthreads();
  for (int i = tid; i < n; i += B) {
    const int c = cell_of<DIM>(D, xs, N, off + i);
    A.cidx[off + i] = c;
    atomicAdd(&cnt[c], 1);
  }
  __syncthreads();
  // exclusive scan over cells, in contiguous chunks per thread
  const int chunk = (ncell + B - 1) / B;
  const int c0 = tid * chunk, c1 = min(ncell, c0 + chunk);
  int local = 0;
  for (int c = c0; c < c1; ++c) local += __hip_atomic_load(&cnt[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  int total = 0;
  int run = block_exscan(local, lds_int, total);
  for (int c = c0; c < c1; ++c) {
    const int k = __hip_atomic_load(&cnt[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    cst[c] = run;
    run += k;
  }
  if (tid == 0) cst[ncell] = total;
  __syncthreads();
  for (int c = tid; c < ncell; c += B)
    __hip_atomic_store(&cnt[c], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  for (int i = tid; i < n; i += B) {
    const int c = A.cidx[off + i];
    const int slot = atomicAdd(&cnt[c], 1);
    cat[cst[c] + slot] = i;
  }
  __syncthreads();
  // sort each cell by index, then clear its count: counts are zero outside a
  // rebuild, which the grid kernels' counting sort relies on
  for (int c = tid; c < ncell; c += B) {
    const int b = cst[c], e = cst[c + 1];
    for (int p = b + 1; p < e; ++p) {
      const int key = cat[p];
      int q = p - 1;
      while (q >= b && cat[q] > key) { cat[q + 1] = cat[q]; --q; }
      cat[q + 1] = key;
    }
    __hip_atomic_store(&cnt[c], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  int ov = 0;
  for (int i = tid; i < n; i += B) {
    const int c = build_list_atom<DIM>(D, A, xs, i);
    A.nnb[off + i] = c < D.maxnb ? c : D.maxnb;
    if (c > D.maxnb) ov = 1;
#pragma unroll
    for (int k = 0; k < DIM; ++k) A.xb[k * N + off + i] = xs[k * N + off + i];
  }
  overflow = block_or(ov, lds_int + 20);
}

// ---------------------------------------------------------------------------
// Batched persistent kernel: blockIdx.x -> system sys_list[blockIdx.x].
//
// mode bit 0 (COMPUTE): evaluate at the current positions without stepping.
template <int DIM, typename T>
__device__ void run_system(const SysDesc &D, SysState *__restrict__ stg, const Arrays &A,
                           int64_t nsteps, int mode) {
  const int tid = threadIdx.x, B = blockDim.x;
  const int n = D.n;
  const int64_t N = A.ntot, off = D.off;
  T *__restrict__ u = (T *)A.u;

  __shared__ double red[NRED * 16];
  __shared__ int lds_int[32];
  __shared__ double sh_XR[3], sh_VR[3], sh_FR[3];
  __shared__ double sh_clock[2];
  __shared__ int64_t sh_step;
  __shared__ int sh_flags, sh_rebuilds;
  __shared__ Scal sh_out;

  if (tid == 0) {
    for (int k = 0; k < 3; ++k) { sh_XR[k] = stg->XR[k]; sh_VR[k] = stg->VR[k]; sh_FR[k] = stg->FR[k]; }
    sh_clock[0] = stg->t_md; sh_clock[1] = stg->t_hyper;
    sh_step = stg->step;
    sh_flags = stg->flags;
    sh_rebuilds = stg->n_rebuilds;
  }
  __syncthreads();
  if (sh_flags & FLAG_UNSTABLE) return;  // frozen system

  const bool compute_only = (mode & 1) != 0;
  const int64_t iters = compute_only ? 1 : nsteps;
  // list requests: 1 = rebuild from the current positions, 2 = rebuild from
  // the recorded build positions (checkpoint restore); evaluations rebuild
  int rebuild_req = compute_only ? 1 : stg->rebuild;

  for (int64_t it = 0; it < iters; ++it) {
    const int64_t step = sh_step;
    int moved = 0;
    // ---- B A O A on mobile atoms; the rigid body on thread 0 -------------
    if (!compute_only) {
      for (int i = tid; i < n; i += B) {
        const int64_t a = off + i;
        if ((A.tr[a] >> 1) != ROLE_MOBILE) continue;
        double z[3];
        noise<DIM, T>(D.seed, step, (uint32_t)i, z);
        double d2 = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          double v = A.v[k * N + a], x = A.x[k * N + a];
          v = v + D.hdt * A.ftot[k * N + a] * D.inv_mass;
          x = x + D.hdt * v;
          v = D.c1 * v + D.c2 * z[k];
          x = x + D.hdt * v;
          x = wrapx(x, D.box[k], D.periodic[k]);
          A.x[k * N + a] = x;
          A.v[k * N + a] = v;
          const double dd = minimg(x - A.xb[k * N + a], D.box[k], D.hbox[k], D.periodic[k]);
          d2 += dd * dd;
        }
        if (d2 > D.skin_half2) moved = 1;
      }
      if (tid == 0 && D.n_rigid > 0) {
        double z[3];
        noise<DIM, T>(D.seed, step, (uint32_t)n, z);
        for (int k = 0; k < DIM; ++k) {
          double v = sh_VR[k], x = sh_XR[k];
          v = v + D.hdt * sh_FR[k] * D.inv_massR;
          x = x + D.hdt * v;
          v = D.c1 * v + D.c2R * z[k];
          x = x + D.hdt * v;
          sh_XR[k] = x;
          sh_VR[k] = v;
        }
      }
      __syncthreads();
    }
    // ---- rigid atoms at X_R + c_i; u = r - r_O (eq. 7) ---------------------
    for (int i = tid; i < n; i += B) {
      const int64_t a = off + i;
      const int role = A.tr[a] >> 1;
      if (role == ROLE_FIXED) continue;
      double d2 = 0.0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        double x;
        if (role == ROLE_RIGID) {
          x = wrapx(sh_XR[k] + A.cofs[k * N + a], D.box[k], D.periodic[k]);
          A.x[k * N + a] = x;
          const double dd = minimg(x - A.xb[k * N + a], D.box[k], D.hbox[k], D.periodic[k]);
          d2 += dd * dd;
        } else {
          x = A.x[k * N + a];
        }
        u[k * N + a] = (T)minimg(x - A.rO[k * N + a], D.box[k], D.hbox[k], D.periodic[k]);
      }
      if (role == ROLE_RIGID && d2 > D.skin_half2) moved = 1;
    }
    const int need = block_or(moved, lds_int + 24);
    if (need || rebuild_req) {
      int overflow = 0;
      wg_rebuild<DIM>(D, A, (rebuild_req == 2 && !need) ? A.xb : A.x, lds_int, overflow);
      if (tid == 0) { sh_rebuilds++; if (overflow) sh_flags |= FLAG_NBR_OVERFLOW; }
      rebuild_req = 0;
    }
    // ---- pair pass -----------------------------------------------------------
    double sums[NRED];
#pragma unroll
    for (int q = 0; q < NRED; ++q) sums[q] = 0.0;
    for (int i = tid; i < n; i += B) {
      const int64_t a = off + i;
      const int tr = A.tr[a];
      const int role = tr >> 1;
      double xi[3] = {0, 0, 0}, u64[3] = {0, 0, 0};
      T ui[3] = {0, 0, 0};
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        xi[k] = A.x[k * N + a];
        if (role != ROLE_FIXED) u64[k] = minimg(xi[k] - A.rO[k * N + a], D.box[k], D.hbox[k], D.periodic[k]);
        ui[k] = (T)u64[k];
      }
      PairAcc<T> acc;
      acc.init();
      pair_atom<DIM, T>(D, A, i, xi, ui, tr & 1, acc);
      double F[3], H[3];
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        if constexpr (sizeof(T) == 8) { F[k] = acc.F[k]; H[k] = acc.H[k]; }
        else { F[k] = acc.F[k].get(); H[k] = acc.H[k].get(); }
        A.flj[k * N + a] = F[k];
        A.hu[k * N + a] = H[k];
      }
      double e;
      if constexpr (sizeof(T) == 8) e = acc.e; else e = acc.e.get();
      sums[0] += e;
      {
        double f2 = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) f2 += F[k] * F[k];
        if (!(f2 <= kForceLimit2)) sums[12] += 1.0;
      }
      if (role != ROLE_FIXED) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          sums[1] += u64[k] * u64[k];
          sums[2] += F[k] * u64[k];
        }
      }
      if (role == ROLE_RIGID) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) { sums[3 + k] += F[k]; sums[6 + k] += H[k]; sums[9 + k] += u64[k]; }
      }
    }
    block_sum<NRED>(sums, red);
    const int64_t estep = compute_only ? step : step + 1;
    double XRl[3] = {sh_XR[0], sh_XR[1], sh_XR[2]};
    Scal S;
    eval_scalars<DIM>(D, sums, XRl, estep, S);
    // ---- bias force, total force, final B --------------------------------
    for (int i = tid; i < n; i += B) {
      const int64_t a = off + i;
      const int role = A.tr[a] >> 1;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        double f = A.flj[k * N + a], h = A.hu[k * N + a], fb = 0.0;
        if (role != ROLE_FIXED) {
          if (role == ROLE_RIGID) { f += S.Fd[k] * D.inv_nR; h += S.hud[k]; }
          if (D.bias_on && S.d >= 1e-12 && S.dvp != 0.0) {
            const double uk = minimg(A.x[k * N + a] - A.rO[k * N + a], D.box[k], D.hbox[k], D.periodic[k]);
            fb = S.bias_a * (h - f - S.bias_b * uk);
          }
        }
        const double ft = f + fb;
        if (compute_only || role == ROLE_RIGID) {
          A.flj[k * N + a] = f;
          A.hu[k * N + a] = h;
        }
        A.fb[k * N + a] = fb;
        A.ftot[k * N + a] = ft;
        if (!compute_only && role == ROLE_MOBILE)
          A.v[k * N + a] = A.v[k * N + a] + D.hdt * ft * D.inv_mass;
      }
    }
    if (tid == 0) {
      for (int k = 0; k < DIM; ++k) sh_FR[k] = sums[3 + k] + S.Fd[k] + S.sumFb[k];
      if (!compute_only) {
        for (int k = 0; k < DIM; ++k) sh_VR[k] = sh_VR[k] + D.hdt * sh_FR[k] * D.inv_massR;
        sh_clock[0] += D.dt;
        sh_clock[1] += D.dt * exp(S.dv * D.inv_kT);
        sh_step = step + 1;
      }
      if (!isfinite(S.e_pot) || S.bad > 0.0) sh_flags |= FLAG_UNSTABLE;
      sh_out = S;
    }
    __syncthreads();
    if (sh_flags & FLAG_UNSTABLE) break;
  }
  const Scal &S = sh_out;
  // ---- write back: rigid atom velocities, kinetic energy, scalars ----------
  double ek[1] = {0.0};
  for (int i = tid; i < n; i += B) {
    const int64_t a = off + i;
    const int role = A.tr[a] >> 1;
    if (role == ROLE_RIGID) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) A.v[k * N + a] = sh_VR[k];
    } else if (role == ROLE_MOBILE) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) { const double v = A.v[k * N + a]; ek[0] += 0.5 * D.mass * v * v; }
    }
  }
  block_sum<1>(ek, red);
  if (tid == 0) {
    double ekr = 0.0;
    for (int k = 0; k < DIM; ++k) ekr += 0.5 * D.massR * sh_VR[k] * sh_VR[k];
    for (int k = 0; k < 3; ++k) { stg->XR[k] = sh_XR[k]; stg->VR[k] = sh_VR[k]; stg->FR[k] = sh_FR[k]; }
    stg->t_md = sh_clock[0];
    stg->t_hyper = sh_clock[1];
    stg->step = sh_step;
    stg->e_lj = S.e_lj; stg->v_drive = S.v_drive; stg->e_pot = S.e_pot;
    stg->e_kin = ek[0] + (D.n_rigid > 0 ? ekr : 0.0);
    stg->d = S.d; stg->g = S.g; stg->dv = S.dv; stg->dvp = S.dvp;
    stg->kappa = 0.0; stg->dv1 = S.dv; stg->dv2 = 0.0;
    stg->x_slider = S.xs; stg->x_tip = S.x_tip; stg->f_lat = S.f_lat;
    stg->flags = sh_flags;
    stg->n_rebuilds = sh_rebuilds;
    stg->rebuild = 0;
  }
}

// MODE 0: nsteps BAOAB steps; MODE 1: one evaluation (own instantiation).
// One instantiation per dimension and workgroup size.
template <typename T, int DIM, int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_batched(const SysDesc *__restrict__ descs,
                                                   SysState *__restrict__ states, Arrays A,
                                                   const int32_t *__restrict__ sys_list,
                                                   int64_t nsteps) {
  const int s = sys_list[blockIdx.x];
  run_system<DIM, T>(descs[s], states + s, A, nsteps, MODE);
}

// Maxwell-Boltzmann velocities v = sqrt(kT/m) z, Philox tag 1 at step 0; the
// rigid body (particle index n) with its total mass.
__global__ void k_init_velocities(const SysDesc *__restrict__ descs, SysState *__restrict__ states,
                                  Arrays A, int s) {
  const SysDesc &D = descs[s];
  const int64_t N = A.ntot;
  const double sm = sqrt(D.kT * D.inv_mass), sR = sqrt(D.kT * D.inv_massR);
  double zR[4];
  normals4(D.seed, 0, (uint32_t)D.n, 1u, zR);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < D.n; i += gridDim.x * blockDim.x) {
    const int64_t a = D.off + i;
    const int role = A.tr[a] >> 1;
    double z[4] = {0, 0, 0, 0};
    if (role == ROLE_MOBILE) normals4(D.seed, 0, (uint32_t)i, 1u, z);
    for (int k = 0; k < D.dim; ++k) {
      double v = 0.0;
      if (role == ROLE_MOBILE) v = sm * z[k];
      else if (role == ROLE_RIGID) v = sR * zR[k];
      A.v[k * N + a] = v;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) states[s].VR[k] = (D.n_rigid > 0 && k < D.dim) ? sR * zR[k] : 0.0;
}

// ---------------------------------------------------------------------------
// Host launchers
hipError_t launch_init_velocities(const SysDesc *descs, SysState *states, const Arrays &A, int sys,
                                  int n, int block, hipStream_t stream) {
  const int grid = (n + block - 1) / block;
  hipLaunchKernelGGL(k_init_velocities, dim3(grid > 0 ? grid : 1), dim3(block), 0, stream, descs, states, A, sys);
  return hipGetLastError();
}

template <typename T, int DIM>
static hipError_t launch_batched_d(const SysDesc *descs, SysState *states, const Arrays &A,
                                   const int32_t *sys_list, int nsys, int block, int64_t nsteps, int mode,
                                   hipStream_t stream) {
  if (mode)
    hipLaunchKernelGGL((k_batched<T, DIM, 1, 1024>), dim3(nsys), dim3(1024), 0, stream, descs, states, A, sys_list, nsteps);
  else if (block <= 256)
    hipLaunchKernelGGL((k_batched<T, DIM, 0, 256>), dim3(nsys), dim3(256), 0, stream, descs, states, A, sys_list, nsteps);
  else if (block <= 512)
    hipLaunchKernelGGL((k_batched<T, DIM, 0, 512>), dim3(nsys), dim3(512), 0, stream, descs, states, A, sys_list, nsteps);
  else
    hipLaunchKernelGGL((k_batched<T, DIM, 0, 1024>), dim3(nsys), dim3(1024), 0, stream, descs, states, A, sys_list, nsteps);
  return hipGetLastError();
}

hipError_t launch_batched(int prec, int dim, const SysDesc *descs, SysState *states, const Arrays &A,
                          const int32_t *sys_list, int nsys, int block, int64_t nsteps, int mode,
                          hipStream_t stream) {
  if (nsys <= 0) return hipSuccess;
  if (prec == 0)
    return dim == 2 ? launch_batched_d<double, 2>(descs, states, A, sys_list, nsys, block, nsteps, mode, stream)
                    : launch_batched_d<double, 3>(descs, states, A, sys_list, nsys, block, nsteps, mode, stream);
  return dim == 2 ? launch_batched_d<float, 2>(descs, states, A, sys_list, nsys, block, nsteps, mode, stream)
                  : launch_batched_d<float, 3>(descs, states, A, sys_list, nsys, block, nsteps, mode, stream);
}

}  // namespace hdk
