// Grid scheduler: a step is a short sequence of kernels over tiles, each tile
// a contiguous range of one system's atoms (atom order for drift and kick,
// cell-sorted order for the list build and the pair pass).  Used for the
// plain single-system path (one system per graph) and for systems too large
// for one workgroup.  Kernel boundaries are the per-system barriers; the pair
// pass leaves per-tile partial sums that a separate launch reduces per system
// in a fixed tile order.
#include "hd_device.h"
#include "hd_launch.h"

namespace hdk {

// Scalars of the last evaluation, consumed by the kick kernel.
struct GridScal {
  Scal S;
  double XRn[3], VRn[3];
};

// Tile of this workgroup.  Workgroups are dealt round-robin to the 8 XCDs;
// consecutive tiles (spatial neighbours) are given to the same XCD so that
// their halo data shares one L2.
__device__ __forceinline__ int xcd_tile(int b, int nt) {
  const int q = nt >> 3, r = nt & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

template <int DIM, typename T>
__device__ void rigid_advance(const SysDesc &D, const SysState &st, int64_t step, double XRn[3],
                              double VRn[3]) {
  if (D.thermostat == 1) {   // Nose-Hoover chain: B and a full A
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const double v = st.VR[k] + D.hdt * st.FR[k] * D.inv_massR;
      XRn[k] = st.XR[k] + D.dt * v;
      VRn[k] = v;
    }
    return;
  }
  double z[3];
  noise<DIM, T>(D.seed, step, (uint32_t)D.n, z);
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    double v = st.VR[k], x = st.XR[k];
    v = v + D.hdt * st.FR[k] * D.inv_massR;
    x = x + D.hdt * v;
    v = D.c1 * v + D.c2R * z[k];
    x = x + D.hdt * v;
    XRn[k] = x;
    VRn[k] = v;
  }
}

// Half kick v + (dt/2) F/m, with one explicit rounding pattern wherever it is
// taken (a step's closing kick and the next step's opening one, in separate
// kernels or in the fused one), so that a run split across calls is the
// same bit for bit as one call.
__device__ __forceinline__ double half_kick(const SysDesc &D, double v, double f) {
  return __builtin_fma(D.hdt * f, D.inv_mass, v);
}

// B A O A for one atom (B and a full A under the Nose-Hoover chain, whose
// velocity scalings are separate launches); rigid atoms follow the rigid
// body, which each of their threads advances identically.  A mobile atom's
// velocity, total force and mode estimate come from memory, or (FUSED) from
// the fused kick's registers vr, fr, qr.  Writes the atom's pair record and
// mode record, and raises the system's rebuild flag when the atom has left
// its skin.
template <int DIM, typename T, bool FUSED = false>
__device__ __forceinline__ void drift_atom(const SysDesc &D, const SysState &st, const Arrays &A, int i,
                                           bool compute_only, const double (&vr)[3], const double (&fr)[3],
                                           const double (&qr)[3]) {
  const int64_t N = A.ntot, a = D.off + i;
  const int tr = A.tr[a], role = tr >> 1;
  double *rec = A.rec + (D.off + A.pos[a]) * kRecDoubles;
  if (role == ROLE_FIXED) {
    // fixed atoms: position as is, u = 0 (and no mode component)
    double xf[3] = {0, 0, 0};
    const double zero[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < DIM; ++k) xf[k] = A.x[k * N + a];
    rec_store(A, rec, DIM, xf, zero, tr);
    if (D.eig) {
      double *rw = A.recw + (D.off + A.pos[a]) * 4;
#pragma unroll
      for (int k = 0; k < DIM; ++k) rw[k] = 0.0;
    }
    return;
  }
  const int64_t step = st.step;
  double xn[3] = {0, 0, 0};
  if (role == ROLE_MOBILE) {
    if (!compute_only && D.thermostat == 1) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        const double v = half_kick(D, FUSED ? vr[k] : A.v[k * N + a], FUSED ? fr[k] : A.ftot[k * N + a]);
        const double x = wrapx(A.x[k * N + a] + D.dt * v, D.box[k], D.periodic[k]);
        A.x[k * N + a] = x;
        A.v[k * N + a] = v;
        xn[k] = x;
      }
    } else if (!compute_only) {
      double z[3];
      noise<DIM, T>(D.seed, step, (uint32_t)i, z);
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        double v = FUSED ? vr[k] : A.v[k * N + a], x = A.x[k * N + a];
        v = half_kick(D, v, FUSED ? fr[k] : A.ftot[k * N + a]);
        x = x + D.hdt * v;
        v = D.c1 * v + D.c2 * z[k];
        x = x + D.hdt * v;
        x = wrapx(x, D.box[k], D.periodic[k]);
        A.x[k * N + a] = x;
        A.v[k * N + a] = v;
        xn[k] = x;
      }
    } else {
#pragma unroll
      for (int k = 0; k < DIM; ++k) xn[k] = A.x[k * N + a];
    }
  } else {
    double XRn[3], VRn[3];
    if (!compute_only) {
      rigid_advance<DIM, T>(D, st, step, XRn, VRn);
    } else {
#pragma unroll
      for (int k = 0; k < DIM; ++k) { XRn[k] = st.XR[k]; VRn[k] = st.VR[k]; }
    }
    const int s = A.sys_of[a];
    if (i == D.first_rigid) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) { A.XR_next[s * 6 + k] = XRn[k]; A.XR_next[s * 6 + 3 + k] = VRn[k]; }
    }
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      xn[k] = wrapx(XRn[k] + A.cofs[k * N + a], D.box[k], D.periodic[k]);
      A.x[k * N + a] = xn[k];
    }
  }
  // the pair record (the grid kernels read u there only)
  double d2 = 0.0, un[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    un[k] = minimg(xn[k] - A.rO[k * N + a], D.box[k], D.hbox[k], D.periodic[k]);
    const double dd = minimg(xn[k] - A.xb[k * N + a], D.box[k], D.hbox[k], D.periodic[k]);
    d2 += dd * dd;
  }
  rec_store(A, rec, DIM, xn, un, tr);
  if (D.eig) {
    // the mode estimate spread over the atoms, beside the pair record
    double *rw = A.recw + (D.off + A.pos[a]) * 4;
#pragma unroll
    for (int k = 0; k < DIM; ++k)
      rw[k] = role == ROLE_MOBILE ? (FUSED ? qr[k] : A.qm[k * N + a]) : st.qR[k];
  }
  // an atom outside its skin forces a rebuild from the current positions
  // (value 1), superseding a pending rebuild from build positions (value 2)
  if (d2 > D.skin_half2) atomicExch(&A.rebuild_flag[A.sys_of[a]], 1);
}

template <typename T>
__global__ __launch_bounds__(1024) void kg_drift(const SysDesc *__restrict__ descs,
                                                 const SysState *__restrict__ states, Arrays A,
                                                 const Tile *__restrict__ tiles, int ntiles,
                                                 int compute_only) {
  const Tile t = tiles[xcd_tile(blockIdx.x, ntiles)];
  if (threadIdx.x >= t.count) return;
  const SysDesc &D = descs[t.sys];
  const int i = t.first + threadIdx.x;
  const double none[3] = {0, 0, 0};
  if (D.dim == 2) drift_atom<2, T>(D, states[t.sys], A, i, compute_only != 0, none, none, none);
  else drift_atom<3, T>(D, states[t.sys], A, i, compute_only != 0, none, none, none);
}

// ---- neighbour-list rebuild, only for systems whose flag is raised --------
// After the drift has raised the flags, kg_compact lists the raised tiles and
// systems (in any order: the rebuild's results do not depend on it); the
// rebuild kernels then run fixed grids that walk only those lists, so a step
// in which no list expired costs a few empty launches.  The lists' counts are
// cleared by kg_reduce, after the rebuild of the step has read them.
__global__ void kg_set_flags(int32_t *flags, const int32_t *sys_ids, int nsys, int value) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nsys) flags[sys_ids[k]] = value;
}

__global__ __launch_bounds__(256) void kg_compact(Arrays A, const Tile *__restrict__ tiles, int ntiles,
                                                  const int32_t *__restrict__ sys_ids, int nsys) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < ntiles && A.rebuild_flag[tiles[k].sys]) A.rb_tiles[atomicAdd(&A.rb_count[0], 1)] = k;
  if (k < nsys && A.rebuild_flag[sys_ids[k]]) A.rb_sys[atomicAdd(&A.rb_count[1], 1)] = sys_ids[k];
}

template <int DIM>
__device__ int cell_of_g(const SysDesc &D, const double *x, int64_t N, int64_t a) {
  int c3[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    int ck = (int)floor((x[k * N + a] - D.lo[k]) * D.inv_h[k]);
    ck = ck < 0 ? 0 : (ck >= D.nc[k] ? D.nc[k] - 1 : ck);
    c3[k] = ck;
  }
  return (c3[2] * D.nc[1] + c3[1]) * D.nc[0] + c3[0];
}

__global__ __launch_bounds__(1024) void kg_cell_count(const SysDesc *__restrict__ descs, Arrays A,
                                                      const Tile *__restrict__ tiles) {
  const int nw = __hip_atomic_load(&A.rb_count[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int w = blockIdx.x; w < nw; w += gridDim.x) {
    const Tile t = tiles[A.rb_tiles[w]];
    if (threadIdx.x >= t.count) continue;
    const int flag = A.rebuild_flag[t.sys];
    const SysDesc &D = descs[t.sys];
    const int64_t a = D.off + t.first + threadIdx.x;
    const double *xs = flag == 2 ? A.xb : A.x;  // 2: from the recorded build positions
    const int c = D.dim == 2 ? cell_of_g<2>(D, xs, A.ntot, a) : cell_of_g<3>(D, xs, A.ntot, a);
    A.cidx[a] = c;
    atomicAdd(&A.cell_count[D.cell_off + c], 1);
  }
}

__global__ __launch_bounds__(1024) void kg_cell_scan(const SysDesc *__restrict__ descs, Arrays A) {
  __shared__ int lds_int[32];
  const int nw = __hip_atomic_load(&A.rb_count[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int w = blockIdx.x; w < nw; w += gridDim.x) {
    const int s = A.rb_sys[w];
    const SysDesc &D = descs[s];
    const int tid = threadIdx.x, B = blockDim.x, ncell = D.ncell;
    int32_t *cnt = A.cell_count + D.cell_off;
    int32_t *cst = A.cell_start + D.cstart_off;
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
      __hip_atomic_store(&cnt[c], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tid == 0) cst[ncell] = total;
  }
}

__global__ __launch_bounds__(1024) void kg_cell_scatter(const SysDesc *__restrict__ descs, Arrays A,
                                                        const Tile *__restrict__ tiles) {
  const int nw = __hip_atomic_load(&A.rb_count[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int w = blockIdx.x; w < nw; w += gridDim.x) {
    const Tile t = tiles[A.rb_tiles[w]];
    if (threadIdx.x >= t.count) continue;
    const SysDesc &D = descs[t.sys];
    const int i = t.first + threadIdx.x;
    const int64_t a = D.off + i;
    const int c = A.cidx[a];
    const int slot = atomicAdd(&A.cell_count[D.cell_off + c], 1);
    A.cell_atoms[D.off + A.cell_start[D.cstart_off + c] + slot] = i;
  }
}

// Build record of sorted position p (atom i): build position and type/role.
__device__ __forceinline__ void put_brec(const SysDesc &D, const Arrays &A, const double *__restrict__ xs,
                                         int p, int i) {
  const int64_t a = D.off + i, N = A.ntot;
  double *b = A.brec + (D.off + p) * 4;
  b[0] = xs[a];
  b[1] = xs[N + a];
  b[2] = D.dim == 3 ? xs[2 * N + a] : 0.0;
  ((int64_t *)b)[3] = (int64_t)A.tr[a];   // type/role as integer bits
}

// Sort each cell's atoms by index (so that lists are built in a fixed order),
// write their build records, and clear the cell's count.  One wavefront per
// cell: the cell's atoms are staged in LDS and each lane places its own atoms
// at their rank (the number of smaller indices in the cell).  Cells of more
// than kSortMax atoms, which only clamping at an open boundary can produce,
// are sorted by insertion.
constexpr int kSortMax = 256;
__global__ __launch_bounds__(256) void kg_cell_sort(const SysDesc *__restrict__ descs, Arrays A) {
  __shared__ int keys[4][kSortMax];
  const int nw = __hip_atomic_load(&A.rb_count[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int ws = blockIdx.y; ws < nw; ws += gridDim.y) {
  const int s = A.rb_sys[ws];
  const SysDesc &D = descs[s];
  const double *xs = A.rebuild_flag[s] == 2 ? A.xb : A.x;  // 2: from the recorded build positions
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int32_t *cat = A.cell_atoms + D.off;
  const int32_t *cst = A.cell_start + D.cstart_off;
  for (int c0 = blockIdx.x * 4; c0 < D.ncell; c0 += gridDim.x * 4) {
    const int c = c0 + wave;
    const bool have = c < D.ncell;
    const int b = have ? cst[c] : 0, m = have ? cst[c + 1] - b : 0;
    const bool staged = m > 1 && m <= kSortMax;
    if (staged)
      for (int k = lane; k < m; k += 64) keys[wave][k] = cat[b + k];
    __syncthreads();
    if (staged) {
      for (int k = lane; k < m; k += 64) {
        const int key = keys[wave][k];
        int r = 0;
        for (int j = 0; j < m; ++j) r += keys[wave][j] < key ? 1 : 0;
        cat[b + r] = key;
        put_brec(D, A, xs, b + r, key);
      }
    } else if (m == 1 && lane == 0) {
      put_brec(D, A, xs, b, cat[b]);
    } else if (m > kSortMax && lane == 0) {
      for (int p = b + 1; p < b + m; ++p) {
        const int key = cat[p];
        int q = p - 1;
        while (q >= b && cat[q] > key) { cat[q + 1] = cat[q]; --q; }
        cat[q + 1] = key;
      }
      for (int p = b; p < b + m; ++p) put_brec(D, A, xs, p, cat[p]);
    }
    if (have && lane == 0) __hip_atomic_store(&A.cell_count[D.cell_off + c], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
  }
  }
}

// List of the atom at sorted position p, one lane: candidates cell by cell in
// stencil order, within a cell in index order (the cells are sorted); each
// entry holds the neighbour's sorted position and type.  Positions are the
// build records the cell sort wrote.
template <int DIM>
__device__ int list_atom_g(const SysDesc &D, const Arrays &A, int p) {
  const int64_t off = D.off;
  const int n = D.n;
  const double *__restrict__ brec = A.brec + off * 4;
  double xi[3];
#pragma unroll
  for (int k = 0; k < DIM; ++k) xi[k] = brec[(int64_t)p * 4 + k];
  const int ri = (int)((const int64_t *)brec)[(int64_t)p * 4 + 3] >> 1;
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
  const int32_t *cstart = A.cell_start + D.cstart_off;
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
        const int pb = cstart[q], pe = cstart[q + 1];
        // candidates four at a time: all their loads are issued before any
        // is tested, so memory latency overlaps across them
        for (int p0 = pb; p0 < pe; p0 += 4) {
          int trj[4];
          double xj[4][3];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int pp = p0 + u < pe ? p0 + u : p0;
            const double *cr = brec + (int64_t)pp * 4;
            trj[u] = (int)((const int64_t *)cr)[3];
#pragma unroll
            for (int k = 0; k < DIM; ++k) xj[u][k] = cr[k];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int pp = p0 + u;
            if (pp >= pe || pp == p) continue;
            const int rj = trj[u] >> 1;
            if ((ri == ROLE_FIXED && rj == ROLE_FIXED) || (ri == ROLE_RIGID && rj == ROLE_RIGID)) continue;
            // r^2 exactly as the float64 rule: minimum image, then the sum of
            // squares axis by axis without contraction
            double dx[3];
            const double r2 = pair_disp<DIM>(D, xi, xj[u], dx);
            if (r2 < D.rl2) {
              if (cnt < D.maxnb) {
                const int e = (pp << 1) | (trj[u] & 1);
                if (D.list16) ((uint16_t *)list)[grid_list_index(cnt, n, p)] = (uint16_t)e;
                else list[grid_list_index(cnt, n, p)] = e;
              }
              ++cnt;
            }
          }
        }
      }
  return cnt;
}

// List build with one lane per stencil row: the 3^(DIM-1) rows (dy, dz) of
// an atom's cell stencil are scanned by separate lanes into LDS sub-lists,
// which are then concatenated in row order.  The result is the list
// list_atom_g builds (same entries, same order) with 3 or 9 times the
// parallelism, which a system whose skin expired needs to hide memory
// latency.  A row with more than kRowCap entries sends its atom to
// list_atom_g.  Blocks of kBuildThreads threads, kBuildThreads / 9 atoms
// each (3D), lanes ordered atoms-fastest within a row.  The sub-lists take
// 16-bit entries for systems with 16-bit lists: half the LDS, twice the
// workgroups per CU.
constexpr int kBuildThreads = 256;
constexpr int kRowCap = 48;

template <int DIM, typename SubT, bool SHIFT>
__device__ int scan_row(const SysDesc &D, const Arrays &A, int p,
                        const double xi[3], int ri, const int cc[3], int oy, int oz, SubT *sub) {
  const int32_t *cstart = A.cell_start + D.cstart_off;
  const double *__restrict__ brec = A.brec + D.off * 4;
  int lo0 = 0, hi0 = 0;
  if (D.nc[0] > 1) { lo0 = -1; hi0 = 1; }
  int cnt = 0;
  for (int ox = lo0; ox <= hi0; ++ox) {
    int q3[3] = {cc[0] + ox, cc[1] + oy, cc[2] + oz};
    bool skip = false;
    // SHIFT: the image of a wrapped stencil cell is the box length away
    // (every periodic axis has at least three cells, so for each pair within
    // the list radius this is the minimum image, rounded as the general rule
    // rounds it)
    double sh[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (q3[k] < 0 || q3[k] >= D.nc[k]) {
        if (k < DIM && D.periodic[k]) {
          sh[k] = q3[k] < 0 ? D.box[k] : -D.box[k];
          q3[k] = (q3[k] + D.nc[k]) % D.nc[k];
        } else {
          skip = true;
        }
      }
    }
    if (skip) continue;
    const int q = (q3[2] * D.nc[1] + q3[1]) * D.nc[0] + q3[0];
    const int pb = cstart[q], pe = cstart[q + 1];
    for (int p0 = pb; p0 < pe; p0 += 4) {
      int trj[4];
      double xj[4][3];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int pp = p0 + u < pe ? p0 + u : p0;
        const double *cr = brec + (int64_t)pp * 4;
        trj[u] = (int)((const int64_t *)cr)[3];
#pragma unroll
        for (int k = 0; k < DIM; ++k) xj[u][k] = cr[k];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int pp = p0 + u;
        const int rj = trj[u] >> 1;
        const bool excl = pp >= pe || pp == p || (ri == ROLE_FIXED && rj == ROLE_FIXED) ||
                          (ri == ROLE_RIGID && rj == ROLE_RIGID);
        double r2;
        if constexpr (SHIFT) {
          r2 = 0.0;
#pragma unroll
          for (int k = 0; k < DIM; ++k) r2 = add_sq_exact(r2, (xi[k] - xj[u][k]) + sh[k]);
        } else {
          double dx[3];
          r2 = pair_disp<DIM>(D, xi, xj[u], dx);
        }
        if (!excl && r2 < D.rl2) {
          if (cnt < kRowCap) sub[cnt * kBuildThreads] = (SubT)((pp << 1) | (trj[u] & 1));
          ++cnt;
        }
      }
    }
  }
  return cnt;
}

template <int DIM, typename SubT>
__device__ void build_rows(const SysDesc &D, SysState &st, const Arrays &A, int first, int count, int flag,
                           SubT *sub_all, int *counts, int *pre) {
  constexpr int S = DIM == 3 ? 9 : 3;        // stencil rows per atom
  constexpr int APB = kBuildThreads / S;     // atoms per block
  // lane (row r, atom la), atoms fastest: a quad of lanes scans one stencil
  // row for four consecutive positions, which share a cell, so its candidate
  // loads hit the same cache lines (the vector L1 looks lines up per quad)
  const int tid = threadIdx.x, r = tid / APB, la = tid % APB;
  const bool active = r < S && la < count;
  const int64_t off = D.off, N = A.ntot;
  const int p = first + la;
  int i = 0, ri = 0;
  double xi[3] = {0, 0, 0};
  int cc[3] = {0, 0, 0};
  int cnt = 0;
  if (active) {
    i = A.cell_atoms[off + p];
    const double *b = A.brec + (off + p) * 4;
#pragma unroll
    for (int k = 0; k < DIM; ++k) xi[k] = b[k];
    ri = (int)((const int64_t *)b)[3] >> 1;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const int ck = (int)floor((xi[k] - D.lo[k]) * D.inv_h[k]);
      cc[k] = ck < 0 ? 0 : (ck >= D.nc[k] ? D.nc[k] - 1 : ck);
    }
    const int oy = DIM == 3 ? r % 3 - 1 : r - 1, oz = DIM == 3 ? r / 3 - 1 : 0;
    const bool in_y = D.nc[1] > 1 || oy == 0, in_z = DIM < 3 || D.nc[2] > 1 || oz == 0;
    bool shift = true;   // every periodic axis has at least three cells
#pragma unroll
    for (int k = 0; k < DIM; ++k) shift = shift && (!D.periodic[k] || D.nc[k] >= 3);
    if (in_y && in_z)
      cnt = shift ? scan_row<DIM, SubT, true>(D, A, p, xi, ri, cc, oy, oz, sub_all + tid)
                  : scan_row<DIM, SubT, false>(D, A, p, xi, ri, cc, oy, oz, sub_all + tid);
  }
  counts[tid] = cnt;
  __syncthreads();
  // per atom (its first lane): where each row's entries start in its list,
  // and how many entries the block writes for it (none when a row is crowded:
  // the one-lane build below writes that atom's whole list)
  constexpr int PS = S + 1;
  int total = 0;
  bool over = false;
  if (active && r == 0) {
    for (int q = 0; q < S; ++q) {
      const int c = counts[q * APB + la];
      pre[la * PS + q] = total;
      total += c;
      over = over || c > kRowCap;
    }
    pre[la * PS + S] = over ? 0 : (total < D.maxnb ? total : D.maxnb);
  }
  __syncthreads();
  // The block writes its atoms' lists together: entry q of consecutive sorted
  // positions is four entries apart in memory, so thread (g, a) takes
  // entries g, g + G, ... of atom a, and a wavefront writes short-strided
  // runs over consecutive positions instead of one entry per line.  Same
  // entries in the same places as row-by-row writes.
  int32_t *list = A.nbr + D.nbr_off;
  const int n = D.n;
  {
    const int nb = count < APB ? count : APB;
    const int G = kBuildThreads / nb;
    if (tid < G * nb) {
      const int a = tid % nb, g = tid / nb;
      const int *pa = pre + a * PS;
      const int lim = pa[S];
      int rr = 0;
      for (int q = g; q < lim; q += G) {
        while (rr + 1 < S && pa[rr + 1] <= q) ++rr;   // the row that holds entry q
        const SubT e = sub_all[(q - pa[rr]) * kBuildThreads + rr * APB + a];
        if (D.list16) ((uint16_t *)list)[grid_list_index(q, n, first + a)] = (uint16_t)e;
        else list[grid_list_index(q, n, first + a)] = (int32_t)e;
      }
    }
  }
  if (!active || r != 0) return;
  if (over) total = list_atom_g<DIM>(D, A, p);   // a crowded row: the one-lane build
  const int64_t a = off + i;
  A.nnb[off + p] = total < D.maxnb ? total : D.maxnb;
  if (total > D.maxnb) atomicOr(&st.flags, FLAG_NBR_OVERFLOW);
  // the atom's record moves to its new sorted position (current x and u)
  A.pos[a] = p;
  double *rec = A.rec + (off + p) * kRecDoubles;
  const int tr = A.tr[a];
  {
    double xr[3] = {0, 0, 0}, ur[3] = {0, 0, 0};
    for (int k = 0; k < DIM; ++k) {
      xr[k] = A.x[k * N + a];
      ur[k] = (tr >> 1) == ROLE_FIXED ? 0.0 : minimg(xr[k] - A.rO[k * N + a], D.box[k], D.hbox[k], D.periodic[k]);
    }
    rec_store(A, rec, DIM, xr, ur, tr);
  }
  if (D.eig) {
    double *rw = A.recw + (off + p) * 4;
    for (int k = 0; k < DIM; ++k)
      rw[k] = (tr >> 1) == ROLE_MOBILE ? A.qm[k * N + a] : ((tr >> 1) == ROLE_RIGID ? st.qR[k] : 0.0);
  }
  if (flag != 2)
    for (int k = 0; k < DIM; ++k) A.xb[k * N + a] = A.x[k * N + a];
  if (p == 0 && flag != 2) atomicAdd(&st.n_rebuilds, 1);
}

// Work item w = chunk * (flagged systems) + k: a chunk of kBuildThreads / 9
// (3D) or / 3 (2D) consecutive sorted positions of the k-th system whose
// list expired, independent of the tile size (every lane of a chunk but a
// system's last has an atom); consecutive items are chunks of different
// systems, and consecutive workgroups go to different XCDs, so the few
// systems that rebuild in a step spread over the whole chip.
template <bool E16>
__global__ __launch_bounds__(kBuildThreads) __attribute__((amdgpu_waves_per_eu(5))) void kg_build_list(const SysDesc *__restrict__ descs,
                                                               SysState *__restrict__ states, Arrays A,
                                                               int chunks) {
  using SubT = typename std::conditional<E16, uint16_t, int32_t>::type;
  __shared__ SubT sub[kRowCap * kBuildThreads];
  __shared__ int counts[kBuildThreads];
  __shared__ int pre[(kBuildThreads / 3) * 4];   // per atom: row starts and entries to write
  const int nrb = __hip_atomic_load(&A.rb_count[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int w = blockIdx.x; w < nrb * chunks; w += gridDim.x) {
    const int c = w / nrb;
    const int s = A.rb_sys[w - c * nrb];
    const SysDesc &D = descs[s];
    const int apb = D.dim == 2 ? kBuildThreads / 3 : kBuildThreads / 9;
    const int first = c * apb;
    if (first >= D.n) continue;   // the same for every thread of the workgroup
    const int count = D.n - first < apb ? D.n - first : apb;
    const int flag = A.rebuild_flag[s];
    if (D.dim == 2) build_rows<2, SubT>(D, states[s], A, first, count, flag, sub, counts, pre);
    else build_rows<3, SubT>(D, states[s], A, first, count, flag, sub, counts, pre);
    __syncthreads();   // sub and counts are reused by the next item
  }
}

// ---- pair pass with per-tile partial sums ---------------------------------
// LPA adjacent lanes per atom: lane s of an atom takes list entries s,
// s + LPA, ...; the lanes' sums are then combined by quad permutes (a + b on
// both lanes, the same bits).  More wavefronts per tile hide more gather
// latency.
template <int DIM, typename T, int LPA, int EXT, bool E16 = false>
__device__ void pairs_tile(const SysDesc &D, const Arrays &A, const Tile &t, int tile_index) {
  constexpr bool CURV = (EXT & EXT_CURV) != 0, EIG = (EXT & EXT_EIG) != 0;
  static_assert(!(CURV && EIG), "the curvature and the eigenvalue bias share the X accumulator");
  // partial slots this instantiation fills
  constexpr int NVALID = EIG ? NPART : (CURV ? NRED + 4 : NRED);
  __shared__ double red[NPART * 16];
  const int64_t N = A.ntot;
  double sums[NRED];
#pragma unroll
  for (int q = 0; q < NRED; ++q) sums[q] = 0.0;
  const int la = threadIdx.x / LPA, sub = threadIdx.x % LPA;
  const bool valid = la < t.count;
  // one atom per sorted position; results go to the atom's own index
  const int p = t.first + (valid ? la : 0);
  const double *r = A.rec + (D.off + p) * kRecDoubles;
  constexpr bool F32 = sizeof(T) == 4;   // float32 record layout
  const int tr = F32 ? ((const int32_t *)r)[9] : (int)r[7], role = tr >> 1;
  double xi[3] = {0, 0, 0}, u64[3] = {0, 0, 0};
  T ui[3] = {0, 0, 0};
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    xi[k] = r[k];
    u64[k] = F32 ? r[5 + k] : r[3 + k];
    ui[k] = (T)u64[k];
  }
  double w64[3] = {0, 0, 0};
  T wi[3] = {0, 0, 0};
  if constexpr (EIG) {
    const double *rw = A.recw + (D.off + p) * 4;
#pragma unroll
    for (int k = 0; k < DIM; ++k) { w64[k] = rw[k]; wi[k] = (T)w64[k]; }
  }
  PairAcc<T> acc;
  acc.init();
  if constexpr (LPA == 4) {
    // the quad gather, in this wavefront's share of the dynamic LDS
    extern __shared__ __attribute__((aligned(16))) char quad_area[];
    char *ql = quad_area + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) * kQuadWaveBytes;
    if (valid) pair_atom_rec<DIM, T, EXT, E16, true>(D, A, p, xi, ui, tr & 1, acc, sub, LPA, wi, ql);
  } else {
    if (valid) pair_atom_rec<DIM, T, EXT, E16>(D, A, p, xi, ui, tr & 1, acc, sub, LPA, wi);
  }
  double F[3] = {0, 0, 0}, H[3] = {0, 0, 0}, X[3] = {0, 0, 0}, W[3] = {0, 0, 0}, e;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    if constexpr (sizeof(T) == 8) { F[k] = acc.F[k]; H[k] = acc.H[k]; }
    else { F[k] = acc.F[k].get(); H[k] = acc.H[k].get(); }
    if constexpr (CURV || EIG) {
      if constexpr (sizeof(T) == 8) X[k] = acc.X[k]; else X[k] = acc.X[k].get();
    }
    if constexpr (EIG) {
      if constexpr (sizeof(T) == 8) W[k] = acc.W[k]; else W[k] = acc.W[k].get();
    }
  }
  if constexpr (sizeof(T) == 8) e = acc.e; else e = acc.e.get();
  // every lane takes part in the permutes (no divergence around them)
  if constexpr (LPA >= 2) {
#pragma unroll
    for (int k = 0; k < DIM; ++k) { F[k] += dpp_mov_f64<0xb1>(F[k]); H[k] += dpp_mov_f64<0xb1>(H[k]); }
    e += dpp_mov_f64<0xb1>(e);   // lanes 0<->1, 2<->3
    if constexpr (CURV || EIG) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) X[k] += dpp_mov_f64<0xb1>(X[k]);
    }
    if constexpr (EIG) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) W[k] += dpp_mov_f64<0xb1>(W[k]);
    }
  }
  if constexpr (LPA >= 4) {
#pragma unroll
    for (int k = 0; k < DIM; ++k) { F[k] += dpp_mov_f64<0x4e>(F[k]); H[k] += dpp_mov_f64<0x4e>(H[k]); }
    e += dpp_mov_f64<0x4e>(e);   // lanes 0<->2, 1<->3
    if constexpr (CURV || EIG) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) X[k] += dpp_mov_f64<0x4e>(X[k]);
    }
    if constexpr (EIG) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) W[k] += dpp_mov_f64<0x4e>(W[k]);
    }
  }
  double ext[4] = {0.0, 0.0, 0.0, 0.0};   // u.Hu, sum over the rigid layer of T
  // eigenvalue bias: w.Hw, the rigid layer's T[w,w], the mobile atoms' |w|^2
  // and the rigid layer's H w (slots P_XHX ... P_HWR + 2)
  double ext8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  static_assert(LPA == 1 || LPA == 2 || LPA == 4, "one, two or four lanes per atom");
  if (valid && sub == 0) {
    const int64_t a = D.off + A.cell_atoms[D.off + p];
    // float32 runs hand the kick float32 sums (rounded once, from float64)
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      if constexpr (sizeof(T) == 8) {
        A.flj[k * N + a] = F[k];
        A.hu[k * N + a] = H[k];
      } else {
        A.flj_f[k * N + a] = (float)F[k];
        A.hu_f[k * N + a] = (float)H[k];
      }
    }
    sums[0] = e;
    double f2 = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) f2 += F[k] * F[k];
    sums[12] = (f2 <= kForceLimit2) ? 0.0 : 1.0;
    if (role != ROLE_FIXED) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) { sums[1] += u64[k] * u64[k]; sums[2] += F[k] * u64[k]; }
    }
    if (role == ROLE_RIGID) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) { sums[3 + k] = F[k]; sums[6 + k] = H[k]; sums[9 + k] = u64[k]; }
    }
    if constexpr (CURV) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) A.tuu[k * N + a] = X[k];
      if (role != ROLE_FIXED) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) ext[0] += u64[k] * H[k];
      }
      if (role == ROLE_RIGID) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) ext[1 + k] = X[k];
      }
    }
    if constexpr (EIG) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) { A.tuu[k * N + a] = X[k]; A.hw[k * N + a] = W[k]; }
      if (role != ROLE_FIXED) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) ext8[0] += w64[k] * W[k];
      }
      if (role == ROLE_MOBILE) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) ext8[4] += w64[k] * w64[k];
      }
      if (role == ROLE_RIGID) {
#pragma unroll
        for (int k = 0; k < DIM; ++k) { ext8[1 + k] = X[k]; ext8[5 + k] = W[k]; }
      }
    }
  }
  // the tile's sums: a reduce-scatter butterfly within each wavefront (the
  // rigid-layer sums only in wavefronts holding rigid atoms; elsewhere they
  // are exact zeros), then the first NRED threads add the wave totals in
  // wave order
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const bool wave_rigid = __ballot(valid && sub == 0 && role == ROLE_RIGID) != 0;
  if (wave_rigid) {
    double w16[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) w16[q] = q < NRED ? sums[q] : 0.0;
    const double tot = wave_sums_scatter<16>(w16, lane);
    const int q = wave_scatter_index<16>(lane);
    if (lane < 16 && q < NRED) red[q * 16 + wave] = tot;
  } else {
    double w4[4] = {sums[0], sums[1], sums[2], sums[12]};
    const double tot = wave_sums_scatter<4>(w4, lane);
    if (lane < 4) {
      const int q = wave_scatter_index<4>(lane);
      red[(q == 3 ? 12 : q) * 16 + wave] = tot;
    } else if (lane < NRED) {
      red[(lane - 1) * 16 + wave] = 0.0;   // the rigid-layer slots 3..11
    }
  }
  if constexpr (CURV) {
    const double tot = wave_sums_scatter<4>(ext, lane);
    if (lane < 4) red[(NRED + wave_scatter_index<4>(lane)) * 16 + wave] = tot;
  }
  if constexpr (EIG) {
    const double tot = wave_sums_scatter<8>(ext8, lane);
    if (lane < 8) red[(NRED + wave_scatter_index<8>(lane)) * 16 + wave] = tot;
  }
  __syncthreads();
  if (threadIdx.x < NPART) {
    double s = 0.0;
    if (threadIdx.x < NVALID)
      for (int w = 0; w < nw; ++w) s += red[threadIdx.x * 16 + w];
    A.partials[(int64_t)tile_index * NPART + threadIdx.x] = s;
  }
}

// Per-system sums of the tile partials in tile order (one workgroup per
// system), then the scalars (eq. 5, 7, 13-14, the drive), the rigid body's
// final half-kick and the boosted clock (eq. 3).  A separate launch: the
// kernel boundary makes every tile's partials visible without device-wide
// fences inside the pair kernel.
template <int DIM>
__device__ void reduce_system(const SysDesc &D, SysState &st, const Arrays &A, int s, int first_tile,
                              int ntiles_s, GridScal *gs, bool compute_only) {
  __shared__ double red[NPART * 16];
  double tot[NPART];
#pragma unroll
  for (int q = 0; q < NPART; ++q) tot[q] = 0.0;
  for (int k = threadIdx.x; k < ntiles_s; k += blockDim.x) {
    const double *p = A.partials + (int64_t)(first_tile + k) * NPART;
#pragma unroll
    for (int q = 0; q < NPART; ++q) tot[q] += p[q];
  }
  block_sum<NPART>(tot, red);
  if (threadIdx.x == 0) {
    double XRn[3] = {st.XR[0], st.XR[1], st.XR[2]};
    double VRn[3] = {st.VR[0], st.VR[1], st.VR[2]};
    if (!compute_only && D.n_rigid > 0) {
      for (int k = 0; k < DIM; ++k) { XRn[k] = A.XR_next[s * 6 + k]; VRn[k] = A.XR_next[s * 6 + 3 + k]; }
    }
    const int64_t estep = compute_only ? st.step : st.step + 1;
    Scal S;
    eval_scalars<DIM, true>(D, tot, XRn, estep, S, st.qR);
    st.lambda = S.lambda;
    st.eig_inv_q2 = S.eig_s * S.eig_s;
    if (!compute_only && D.eig && S.eig_s > 0.0 && D.n_rigid > 0) {
      // the rigid body's row of the mode's rotation step: its atoms' H w and
      // the drive's Hessian k q_R on the spring axes
      constexpr int nspring = DIM == 3 ? 2 : 1;
      double qn[3] = {0, 0, 0};
      for (int k = 0; k < DIM; ++k) {
        const double HR = tot[P_HWR + k] + (k < nspring ? D.k_spring * st.qR[k] : 0.0);
        qn[k] = S.eig_s * (st.qR[k] - D.mode_alpha * (HR - S.lambda * st.qR[k]));
      }
      for (int k = 0; k < DIM; ++k) st.qR[k] = qn[k];
    }
    double FR[3] = {0, 0, 0};
    for (int k = 0; k < DIM; ++k) FR[k] = tot[3 + k] + S.Fd[k] + S.sumFb[k];
    if (!compute_only) {
      for (int k = 0; k < DIM; ++k) { st.XR[k] = XRn[k]; st.VR[k] = VRn[k] + D.hdt * FR[k] * D.inv_massR; }
      st.t_md += D.dt;
      st.t_hyper += D.dt * exp(S.dv * D.inv_kT);
      st.step = st.step + 1;
    }
    for (int k = 0; k < DIM; ++k) st.FR[k] = FR[k];
    st.e_lj = S.e_lj; st.v_drive = S.v_drive; st.e_pot = S.e_pot;
    st.d = S.d; st.g = S.g; st.dv = S.dv; st.dvp = S.dvp;
    st.kappa = S.kappa; st.dv1 = S.dv1; st.dv2 = S.dv2;
    st.x_slider = S.xs; st.x_tip = S.x_tip; st.f_lat = S.f_lat;
    if (!isfinite(S.e_pot) || S.bad > 0.0) st.flags |= FLAG_UNSTABLE;
    gs[s].S = S;
    for (int k = 0; k < 3; ++k) { gs[s].VRn[k] = st.VR[k]; gs[s].XRn[k] = st.XR[k]; }
    A.rebuild_flag[s] = 0;
  }
}

__global__ __launch_bounds__(256) void kg_reduce(const SysDesc *__restrict__ descs,
                                                 SysState *__restrict__ states, Arrays A,
                                                 const int32_t *__restrict__ sys_ids,
                                                 const int32_t *__restrict__ sys_tile0,
                                                 const Tile *__restrict__ tiles, GridScal *gs,
                                                 int compute_only) {
  const int s = sys_ids[blockIdx.x];
  const int first = sys_tile0[blockIdx.x];
  const int nts = tiles[first].tiles_in_sys;
  const SysDesc &D = descs[s];
  if (D.dim == 2) reduce_system<2>(D, states[s], A, s, first, nts, gs, compute_only != 0);
  else reduce_system<3>(D, states[s], A, s, first, nts, gs, compute_only != 0);
  // this step's rebuild lists have been used: empty them for the next one
  if (blockIdx.x == 0 && threadIdx.x == 0) { A.rb_count[0] = 0; A.rb_count[1] = 0; }
}

// EXT: the extra pair terms the plan's systems need -- EXT_BONDS for models
// with harmonic tip bonds, EXT_CURV for a curvature bias (T[u,u]) -- each
// combination a separate instantiation, so that LJ-only plans keep their
// register budget; EXT_NOE for the steps whose pair energy is not read.
template <typename T, int LPA, int EXT, bool E16 = false>
__global__ __launch_bounds__(1024) void kg_pairs(const SysDesc *__restrict__ descs, Arrays A,
                                                 const Tile *__restrict__ tiles, int ntiles) {
  const int ti = xcd_tile(blockIdx.x, ntiles);
  const Tile t = tiles[ti];
  const SysDesc &D = descs[t.sys];
  if (D.dim == 2) pairs_tile<2, T, LPA, EXT, E16>(D, A, t, ti);
  else pairs_tile<3, T, LPA, EXT, E16>(D, A, t, ti);
}

// ---- bias force, total force and final B -----------------------------------
// One atom's closing kick of a step: the drive's share on rigid atoms, the
// bias force, the total force ft and the final B (mobile atoms; rigid atoms
// take the rigid body's velocity), and the eigenvalue variable's mode
// rotation.  store: write the forces and the velocity (a step that closes a
// call, or an evaluation); the fused kick-drift keeps them in registers.
template <int DIM, typename T>
__device__ __forceinline__ void kick_atom(const SysDesc &D, const GridScal &G, const Arrays &A, int64_t a,
                                          int role, bool compute_only, bool store, double (&ft)[3],
                                          double (&vn)[3], double (&qn)[3]) {
  const Scal &S = G.S;
  const int64_t N = A.ntot;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    double f, h, fb = 0.0;
    if constexpr (sizeof(T) == 8) { f = A.flj[k * N + a]; h = A.hu[k * N + a]; }
    else { f = A.flj_f[k * N + a]; h = A.hu_f[k * N + a]; }
    if (role != ROLE_FIXED) {
      if (role == ROLE_RIGID) { f += S.Fd[k] * D.inv_nR; h += S.hud[k]; }
      if (D.gen_bias) {
        if (S.live) {
          const double uk = minimg(A.x[k * N + a] - A.rO[k * N + a], D.box[k], D.hbox[k], D.periodic[k]);
          fb = S.cH * h + S.cF * f + S.cU * uk;
          if (D.curv || D.eig) fb += S.cT * A.tuu[k * N + a];
        }
      } else if (D.bias_on && S.d >= 1e-12 && S.dvp != 0.0) {
        const double uk = minimg(A.x[k * N + a] - A.rO[k * N + a], D.box[k], D.hbox[k], D.periodic[k]);
        fb = S.bias_a * (h - f - S.bias_b * uk);
      }
    }
    ft[k] = f + fb;
    if (store) {
      A.flj[k * N + a] = f;
      A.hu[k * N + a] = h;
      A.fb[k * N + a] = fb;
      A.ftot[k * N + a] = ft[k];
    }
    if (!compute_only) {
      if (role == ROLE_MOBILE) vn[k] = half_kick(D, A.v[k * N + a], ft[k]);
      else vn[k] = G.VRn[k];
      if (store && role != ROLE_FIXED) A.v[k * N + a] = vn[k];
      // the mode estimate's rotation step towards the lowest mode
      if (D.eig && role == ROLE_MOBILE) {
        const double q = A.qm[k * N + a];
        qn[k] = S.eig_s > 0.0 ? S.eig_s * (q - D.mode_alpha * (A.hw[k * N + a] - S.lambda * q)) : q;
        A.qm[k * N + a] = qn[k];
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void kg_kick(const SysDesc *__restrict__ descs, Arrays A,
                                                const Tile *__restrict__ tiles, int ntiles,
                                                const GridScal *__restrict__ gs, int compute_only) {
  const Tile t = tiles[xcd_tile(blockIdx.x, ntiles)];
  if (threadIdx.x >= t.count) return;
  const SysDesc &D = descs[t.sys];
  const int64_t a = D.off + t.first + threadIdx.x;
  const int role = A.tr[a] >> 1;
  double ft[3], vn[3], qn[3];
  if (D.dim == 2) kick_atom<2, T>(D, gs[t.sys], A, a, role, compute_only != 0, true, ft, vn, qn);
  else kick_atom<3, T>(D, gs[t.sys], A, a, role, compute_only != 0, true, ft, vn, qn);
}

// A step's closing kick fused with the next step's B A O A (Langevin plans
// only: the Nose-Hoover chain scales the velocities in between): the total
// force, velocity and mode stay in registers between the two, so the forces
// are not written and read back, and x, v and r_O are read once.
template <typename T>
__global__ __launch_bounds__(1024) void kg_kick_drift(const SysDesc *__restrict__ descs,
                                                      const SysState *__restrict__ states, Arrays A,
                                                      const Tile *__restrict__ tiles, int ntiles,
                                                      const GridScal *__restrict__ gs) {
  const Tile t = tiles[xcd_tile(blockIdx.x, ntiles)];
  if (threadIdx.x >= t.count) return;
  const SysDesc &D = descs[t.sys];
  const int i = t.first + threadIdx.x;
  const int64_t a = D.off + i;
  const int role = A.tr[a] >> 1;
  double ft[3] = {0, 0, 0}, vn[3] = {0, 0, 0}, qn[3] = {0, 0, 0};
  if (D.dim == 2) {
    kick_atom<2, T>(D, gs[t.sys], A, a, role, false, false, ft, vn, qn);
    drift_atom<2, T, true>(D, states[t.sys], A, i, false, vn, ft, qn);
  } else {
    kick_atom<3, T>(D, gs[t.sys], A, a, role, false, false, ft, vn, qn);
    drift_atom<3, T, true>(D, states[t.sys], A, i, false, vn, ft, qn);
  }
}

// Nose-Hoover chain over half a step (nhc_half_step), one workgroup per
// system, before the drift and after the kick: 2K of the mobile atoms and the
// rigid body, the chain advanced by one thread, the velocities scaled.
__global__ __launch_bounds__(256) void kg_nhc_half(const SysDesc *__restrict__ descs,
                                                   SysState *__restrict__ states, Arrays A,
                                                   const int32_t *__restrict__ sys_ids) {
  __shared__ double red[16];
  __shared__ double scale_sh;
  const int s = sys_ids[blockIdx.x];
  const SysDesc &D = descs[s];
  if (D.thermostat != 1) return;
  SysState &st = states[s];
  const int64_t N = A.ntot;
  double k2[1] = {0.0};
  for (int i = threadIdx.x; i < D.n; i += blockDim.x) {
    const int64_t a = D.off + i;
    if ((A.tr[a] >> 1) != ROLE_MOBILE) continue;
    for (int k = 0; k < D.dim; ++k) { const double v = A.v[k * N + a]; k2[0] += D.mass * v * v; }
  }
  block_sum<1>(k2, red);
  if (threadIdx.x == 0) {
    double K2 = k2[0];
    if (D.n_rigid > 0)
      for (int k = 0; k < D.dim; ++k) K2 += D.massR * st.VR[k] * st.VR[k];
    const double c = nhc_half_step(D, st.xi, st.eta, K2);
    for (int k = 0; k < D.dim; ++k) st.VR[k] *= c;
    st.e_nhc = nhc_energy(D, st.xi, st.eta);
    scale_sh = c;
  }
  __syncthreads();
  const double c = scale_sh;
  for (int i = threadIdx.x; i < D.n; i += blockDim.x) {
    const int64_t a = D.off + i;
    if ((A.tr[a] >> 1) == ROLE_FIXED) continue;
    for (int k = 0; k < D.dim; ++k) A.v[k * N + a] *= c;
  }
}

// Kinetic energy per system (mobile atoms + rigid body), one workgroup each.
__global__ __launch_bounds__(256) void kg_ekin(const SysDesc *__restrict__ descs,
                                               SysState *__restrict__ states, Arrays A,
                                               const int32_t *__restrict__ sys_ids) {
  __shared__ double red[16];
  const int s = sys_ids[blockIdx.x];
  const SysDesc &D = descs[s];
  double ek[1] = {0.0};
  for (int i = threadIdx.x; i < D.n; i += blockDim.x) {
    const int64_t a = D.off + i;
    if ((A.tr[a] >> 1) != ROLE_MOBILE) continue;
    for (int k = 0; k < D.dim; ++k) { const double v = A.v[k * A.ntot + a]; ek[0] += 0.5 * D.mass * v * v; }
  }
  block_sum<1>(ek, red);
  if (threadIdx.x == 0) {
    double ekr = 0.0;
    if (D.n_rigid > 0)
      for (int k = 0; k < D.dim; ++k) ekr += 0.5 * D.massR * states[s].VR[k] * states[s].VR[k];
    states[s].e_kin = ek[0] + ekr;
  }
}

// ---------------------------------------------------------------------------
size_t grid_scal_bytes() { return sizeof(GridScal); }

hipError_t grid_allow_lds() {
  // the largest quad-gather workgroup: 256 atoms, 1024 threads
  const int bytes = 16 * kQuadWaveBytes;
  const void *fns[28] = {
      (const void *)kg_pairs<float, 4, 0, true>,   (const void *)kg_pairs<float, 4, 0, false>,
      (const void *)kg_pairs<float, 4, 1, false>,  (const void *)kg_pairs<float, 4, 2, false>,
      (const void *)kg_pairs<float, 4, 3, false>,  (const void *)kg_pairs<float, 4, 4, false>,
      (const void *)kg_pairs<float, 4, 5, false>,  (const void *)kg_pairs<double, 4, 0, true>,
      (const void *)kg_pairs<double, 4, 0, false>, (const void *)kg_pairs<double, 4, 1, false>,
      (const void *)kg_pairs<double, 4, 2, false>, (const void *)kg_pairs<double, 4, 3, false>,
      (const void *)kg_pairs<double, 4, 4, false>, (const void *)kg_pairs<double, 4, 5, false>,
      (const void *)kg_pairs<float, 4, 8, true>,   (const void *)kg_pairs<float, 4, 8, false>,
      (const void *)kg_pairs<float, 4, 9, false>,  (const void *)kg_pairs<float, 4, 10, false>,
      (const void *)kg_pairs<float, 4, 11, false>, (const void *)kg_pairs<float, 4, 12, false>,
      (const void *)kg_pairs<float, 4, 13, false>, (const void *)kg_pairs<double, 4, 8, true>,
      (const void *)kg_pairs<double, 4, 8, false>, (const void *)kg_pairs<double, 4, 9, false>,
      (const void *)kg_pairs<double, 4, 10, false>, (const void *)kg_pairs<double, 4, 11, false>,
      (const void *)kg_pairs<double, 4, 12, false>, (const void *)kg_pairs<double, 4, 13, false>};
  for (const void *f : fns) {
    const hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

namespace {

// The rebuild of the lists that expired: compaction of the raised flags,
// then the cell count, scan, scatter and sort and the list build over the
// listed tiles and systems only (fixed grids).
int launch_rebuild(const SysDesc *descs, SysState *states, const Arrays &A, const GridPlan &P,
                   hipStream_t stream) {
  const int nt = P.ntiles, B = P.block;
  const int nc = nt > P.nsys ? nt : P.nsys;
  hipLaunchKernelGGL(kg_compact, dim3((nc + 255) / 256), dim3(256), 0, stream, A, P.tiles, nt, P.sys_ids, P.nsys);
  const int gt = nt < 2048 ? nt : 2048;
  hipLaunchKernelGGL(kg_cell_count, dim3(gt), dim3(B), 0, stream, descs, A, P.tiles);
  hipLaunchKernelGGL(kg_cell_scan, dim3(P.nsys < 256 ? P.nsys : 256), dim3(256), 0, stream, descs, A);
  hipLaunchKernelGGL(kg_cell_scatter, dim3(gt), dim3(B), 0, stream, descs, A, P.tiles);
  const int sort_blocks = (P.max_ncell + 3) / 4 < 1024 ? (P.max_ncell + 3) / 4 : 1024;
  hipLaunchKernelGGL(kg_cell_sort, dim3(sort_blocks > 0 ? sort_blocks : 1, P.nsys < 64 ? P.nsys : 64), dim3(256), 0,
                     stream, descs, A);
  // work items: chunks of a system's sorted positions (kBuildThreads / 9
  // atoms each in 3D, / 3 in 2D), for every system whose list expired
  const int chunks = (P.max_n + kBuildThreads / 9 - 1) / (kBuildThreads / 9);
  const int64_t items = (int64_t)P.nsys * chunks;
  const int gb = items < 4096 ? (int)items : 4096;
  if (P.list16)
    hipLaunchKernelGGL(kg_build_list<true>, dim3(gb), dim3(kBuildThreads), 0, stream, descs, states, A, chunks);
  else
    hipLaunchKernelGGL(kg_build_list<false>, dim3(gb), dim3(kBuildThreads), 0, stream, descs, states, A, chunks);
  return 6;
}

// The pair pass (four or two lanes per atom where the workgroup allows it)
// and the per-system reduction.  with_e = false leaves the pair energy out.
int launch_pairs_reduce(int prec, const SysDesc *descs, SysState *states, const Arrays &A, const GridPlan &P,
                        bool compute_only, hipStream_t stream, bool with_e = true) {
  const int nt = P.ntiles, B = P.block, co = compute_only ? 1 : 0;
  GridScal *gs = (GridScal *)P.gscal;
  const int lpa = B <= 256 ? 4 : (B <= 512 ? 2 : 1);
  // dynamic LDS of the quad gather (four lanes per atom)
  const size_t qb = (size_t)(4 * B / 64) * kQuadWaveBytes;
#define HD_PAIRS(TT, L, BB)                                                                      \
  hipLaunchKernelGGL((kg_pairs<TT, L, BB>), dim3(nt), dim3(L * B), L == 4 ? qb : 0, stream, descs, A, P.tiles, nt)
#define HD_PAIRS16(TT, L, NE)                                                                    \
  hipLaunchKernelGGL((kg_pairs<TT, L, NE, true>), dim3(nt), dim3(L * B), L == 4 ? qb : 0, stream, descs, A, \
                     P.tiles, nt)
#define HD_PAIRS_B(TT, L, NE)                                                                    \
  do {                                                                                           \
    if (P.any_eig) { if (P.any_bonds) HD_PAIRS(TT, L, 5 | NE); else HD_PAIRS(TT, L, 4 | NE); }   \
    else if (P.any_curv) { if (P.any_bonds) HD_PAIRS(TT, L, 3 | NE); else HD_PAIRS(TT, L, 2 | NE); } \
    else if (P.any_bonds) HD_PAIRS(TT, L, 1 | NE);                                               \
    else if (P.list16) HD_PAIRS16(TT, L, NE);                                                    \
    else HD_PAIRS(TT, L, NE);                                                                    \
  } while (0)
#define HD_PAIRS_E(TT, NE)                                                                       \
  do {                                                                                           \
    if (lpa == 4) HD_PAIRS_B(TT, 4, NE); else if (lpa == 2) HD_PAIRS_B(TT, 2, NE); else HD_PAIRS_B(TT, 1, NE); \
  } while (0)
  if (prec == 0) {
    if (with_e) HD_PAIRS_E(double, 0); else HD_PAIRS_E(double, EXT_NOE);
  } else {
    if (with_e) HD_PAIRS_E(float, 0); else HD_PAIRS_E(float, EXT_NOE);
  }
#undef HD_PAIRS_E
#undef HD_PAIRS_B
#undef HD_PAIRS16
#undef HD_PAIRS
  hipLaunchKernelGGL(kg_reduce, dim3(P.nsys), dim3(256), 0, stream, descs, states, A, P.sys_ids, P.sys_tile0,
                     P.tiles, gs, co);
  return 2;
}

int launch_drift(int prec, const SysDesc *descs, SysState *states, const Arrays &A, const GridPlan &P,
                 bool compute_only, hipStream_t stream) {
  const int nt = P.ntiles, co = compute_only ? 1 : 0;
  if (prec == 0)
    hipLaunchKernelGGL(kg_drift<double>, dim3(nt), dim3(P.block), 0, stream, descs, states, A, P.tiles, nt, co);
  else
    hipLaunchKernelGGL(kg_drift<float>, dim3(nt), dim3(P.block), 0, stream, descs, states, A, P.tiles, nt, co);
  return 1;
}

int launch_nhc(const SysDesc *descs, SysState *states, const Arrays &A, const GridPlan &P, hipStream_t stream) {
  hipLaunchKernelGGL(kg_nhc_half, dim3(P.nsys), dim3(256), 0, stream, descs, states, A, P.sys_ids);
  return 1;
}

}  // namespace

hipError_t grid_step(int prec, const SysDesc *descs, SysState *states, const Arrays &A,
                     const GridPlan &P, bool compute_only, hipStream_t stream, int *launches,
                     bool force_rebuild) {
  if (!compute_only) return grid_steps(prec, descs, states, A, P, 1, stream, launches);
  int nl = 0;
  if (force_rebuild) {
    hipLaunchKernelGGL(kg_set_flags, dim3((P.nsys + 255) / 256), dim3(256), 0, stream,
                       A.rebuild_flag, P.sys_ids, P.nsys, 1);
    ++nl;
  }
  nl += launch_drift(prec, descs, states, A, P, true, stream);
  nl += launch_rebuild(descs, states, A, P, stream);
  nl += launch_pairs_reduce(prec, descs, states, A, P, true, stream);
  if (prec == 0)
    hipLaunchKernelGGL(kg_kick<double>, dim3(P.ntiles), dim3(P.block), 0, stream, descs, A, P.tiles, P.ntiles,
                       (const GridScal *)P.gscal, 1);
  else
    hipLaunchKernelGGL(kg_kick<float>, dim3(P.ntiles), dim3(P.block), 0, stream, descs, A, P.tiles, P.ntiles,
                       (const GridScal *)P.gscal, 1);
  ++nl;
  if (launches) *launches += nl;
  return hipGetLastError();
}

hipError_t grid_steps(int prec, const SysDesc *descs, SysState *states, const Arrays &A, const GridPlan &P,
                      int nsteps, hipStream_t stream, int *launches) {
  const int nt = P.ntiles, B = P.block;
  const GridScal *gs = (const GridScal *)P.gscal;
  // Langevin plans fuse each step's closing kick with the next step's drift
  const bool fuse = !P.any_nhc;
  int nl = 0;
  for (int s = 0; s < nsteps; ++s) {
    if (!fuse || s == 0) {
      if (P.any_nhc) nl += launch_nhc(descs, states, A, P, stream);
      nl += launch_drift(prec, descs, states, A, P, false, stream);
    }
    nl += launch_rebuild(descs, states, A, P, stream);
    // the pair energy only where a caller can read it: the sequence's last step
    nl += launch_pairs_reduce(prec, descs, states, A, P, false, stream, s + 1 == nsteps);
    if (fuse && s + 1 < nsteps) {
      if (prec == 0)
        hipLaunchKernelGGL(kg_kick_drift<double>, dim3(nt), dim3(B), 0, stream, descs, states, A, P.tiles, nt, gs);
      else
        hipLaunchKernelGGL(kg_kick_drift<float>, dim3(nt), dim3(B), 0, stream, descs, states, A, P.tiles, nt, gs);
      ++nl;
    } else {
      if (prec == 0) hipLaunchKernelGGL(kg_kick<double>, dim3(nt), dim3(B), 0, stream, descs, A, P.tiles, nt, gs, 0);
      else hipLaunchKernelGGL(kg_kick<float>, dim3(nt), dim3(B), 0, stream, descs, A, P.tiles, nt, gs, 0);
      ++nl;
      if (P.any_nhc) nl += launch_nhc(descs, states, A, P, stream);
    }
  }
  if (launches) *launches += nl;
  return hipGetLastError();
}

hipError_t grid_ekin(const SysDesc *descs, SysState *states, const Arrays &A, const GridPlan &P,
                     hipStream_t stream) {
  hipLaunchKernelGGL(kg_ekin, dim3(P.nsys), dim3(256), 0, stream, descs, states, A, P.sys_ids);
  return hipGetLastError();
}

}  // namespace hdk
