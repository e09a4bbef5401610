// Host-side launchers of the kernels in hd_kernels.hip / hd_grid.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "hd_device.h"

namespace hdk {

struct FireSys;   // a listed system's FIRE state (below)

// One workgroup of `block` threads (256, 512 or 1024) per listed system, all
// of dimension `dim`; nsteps BAOAB steps (mode 1: evaluate only, 1024
// threads).  prec 0 = float64, 1 = float32 pair terms summed in float64.
hipError_t launch_batched(int prec, int dim, const SysDesc *descs, SysState *states, const Arrays &A,
                          const int32_t *sys_list, int nsys, int block, int64_t nsteps, int mode,
                          hipStream_t stream);

// LDS-resident variant for systems of at most 1024 atoms whose positions,
// displacements, cell list and neighbour list fit in one workgroup's LDS.
// All listed systems have dimension `dim`; nmax (<= 1024) is the LDS row
// stride and bounds every listed n; maxnb is their neighbour capacity;
// cellmax bounds every listed ncell.  mode 0: nsteps steps; 1: one
// evaluation; 2: steps with the Nose-Hoover chain compiled in (for groups
// holding a system that uses it).
hipError_t launch_small(int kind, int dim, const SysDesc *descs, SysState *states, const Arrays &A,
                        const int32_t *sys_list, int nsys, int nmax, int maxnb, int cellmax,
                        int block, int64_t nsteps, int mode, hipStream_t stream);
// The FIRE quench of the listed LDS-resident systems in one launch (fire[b]
// is sys_list[b]'s minimiser state, set up as for fire_iteration): up to
// max_iters iterations, each testing convergence (no degree of freedom with
// |F| >= ftol) at the current forces, then mixing and stepping, then an
// evaluation in LDS.  Starts from the forces and rigid-body force of an
// unbiased evaluation at the current positions.
hipError_t launch_small_fire(int kind, int dim, const SysDesc *descs, SysState *states, const Arrays &A,
                             const int32_t *sys_list, int nsys, int nmax, int maxnb, int cellmax, int64_t max_iters,
                             FireSys *fire, double ftol, hipStream_t stream);
size_t small_lds_bytes(int dim, int kind, int nmax, int maxnb, int cellmax);
// Dynamic LDS bytes of one LDS-resident group, and the one-time permission to
// use that much (call outside graph capture, before the first launch).
size_t small_group_bytes(int kind, int dim, int nmax, int maxnb, int cellmax);
hipError_t small_allow_lds(int kind, int dim, size_t bytes);

// FIRE minimisation state of one listed system (hd_fire.hip).
struct FireSys {
  double dt, alpha;    // current step and mixing weight
  double mixv, mixf;   // this iteration's velocity mixing: v <- mixv v + mixf F
  double fmax;         // largest force on a degree of freedom at the last test
  int64_t iters;       // iterations done (at convergence: the iteration that met it)
  int32_t since_neg;   // iterations since the power was last non-positive
  int32_t done;        // converged
  int32_t reset;       // this iteration zeroes the velocities (P <= 0)
  int32_t pad;
};

// One FIRE iteration of the listed systems (count of them, nmax bounds their
// atom counts) from the forces in A.ftot and the rigid-body force in the
// state: convergence test on the largest force (< ftol), velocity mixing and
// semi-implicit Euler step.  Forces must be re-evaluated before the next one.
// partials: device scratch of fire_partials_doubles(count, nmax) doubles.
constexpr int kFireChunk = 2048;   // atoms per first-level reduction block
// FIRE constants (the values of Bitzek et al.)
constexpr double kFireAlpha0 = 0.1, kFireFinc = 1.1, kFireFdec = 0.5, kFireFalpha = 0.99;
constexpr int kFireNmin = 5;
inline size_t fire_partials_doubles(int count, int nmax) {
  return (size_t)count * (size_t)((nmax + kFireChunk - 1) / kFireChunk) * 4;
}
hipError_t fire_iteration(const SysDesc *descs, SysState *states, const Arrays &A, const int32_t *sys_list,
                          int count, int nmax, FireSys *fire, double ftol, int64_t iter, double *partials,
                          hipStream_t stream);

// Tiles of the grid scheduler: each tile is a contiguous atom range of one
// system (tiles never straddle systems).
struct Tile {
  int32_t sys, first, count, tile_in_sys, tiles_in_sys, pad;
};

struct GridPlan {
  const Tile *tiles;       // device
  int ntiles;
  int block;               // threads per tile (== max atoms per tile)
  const int32_t *sys_ids;  // device, systems covered
  const int32_t *sys_tile0;  // device, first tile of each covered system
  int nsys;
  int max_ncell;           // largest cell count among the covered systems
  int max_n;               // largest atom count among the covered systems
  void *gscal;             // device, per-system scalars of the last evaluation
  int any_bonds;           // some covered system has harmonic tip bonds
  int any_curv;            // some covered system is biased on the curvature
  int any_nhc;             // some covered system has the Nose-Hoover chain
  int any_eig;             // some covered system is biased on the eigenvalue
  int list16;              // LJ-only systems below 32768 atoms: 16-bit list entries
};

size_t grid_scal_bytes();
// Allow the pair kernels with the quad gather their dynamic LDS (up to
// 1024-thread workgroups; once per schedule, outside any graph capture).
hipError_t grid_allow_lds();

// One full step (or an evaluation when compute_only) of the grid scheduler.
// Enqueues several kernels on `stream`; safe to capture in a HIP graph (no
// memset or host synchronisation inside).  An evaluation rebuilds every list
// from the current positions unless force_rebuild is false; then, as in a
// step, only lists whose atoms left half the skin are rebuilt.
hipError_t grid_step(int prec, const SysDesc *descs, SysState *states, const Arrays &A,
                     const GridPlan &P, bool compute_only, hipStream_t stream, int *launches,
                     bool force_rebuild = true);
// nsteps full steps in one sequence of launches (graph-capturable): plans
// without the Nose-Hoover chain fuse each step's closing kick with the next
// step's drift, so only the last step writes the force arrays.
hipError_t grid_steps(int prec, const SysDesc *descs, SysState *states, const Arrays &A, const GridPlan &P,
                      int nsteps, hipStream_t stream, int *launches);
// Kinetic energy of the covered systems.
hipError_t grid_ekin(const SysDesc *descs, SysState *states, const Arrays &A, const GridPlan &P,
                     hipStream_t stream);

}  // namespace hdk
