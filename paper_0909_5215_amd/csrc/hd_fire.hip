// Energy minimisation of listed systems: FIRE (Bitzek, Koskinen, Gaehler,
// Moseler, Gumbsch, PRL 97, 170201 (2006)) on the unbiased potential.  It
// gives the basin minimum r_O that the bias of eq. 7 and eq. 13-14 measures
// from, and the quench-and-compare check for a transition between basins
// that the parallel slider-position algorithm of §2.3 needs.
//
// The degrees of freedom are the mobile atoms and the rigid body (fixed atoms
// stay put).  One iteration: chunks of every system's atoms reduce the power
// P = F.v, |v|, |F| and the largest force across the chip, a control kernel
// per system adds the chunks, tests convergence, chooses the velocity mixing
// and the step (the rigid body is advanced there, by one thread); a move
// kernel mixes and advances the mobile atoms (semi-implicit Euler); then the
// forces are evaluated by the stepping kernels in evaluation mode.  The host
// runtime drives the iterations.
#include "hd_device.h"
#include "hd_launch.h"

namespace hdk {

namespace {

constexpr int kFireThreads = 256;

// First level of the reductions, spread over the chip: blockIdx.y is the
// listed system, blockIdx.x a chunk of kFireChunk of its atoms.  Writes the
// chunk's P = F.v, |v|^2, |F|^2 over mobile atoms and its largest |F|^2.
__global__ __launch_bounds__(kFireThreads) void k_fire_partial(const SysDesc *__restrict__ descs, Arrays A,
                                                               const int32_t *__restrict__ sys_list,
                                                               const FireSys *__restrict__ fire,
                                                               double *__restrict__ partials, int maxchunks) {
  __shared__ double red[3 * 16];
  __shared__ double redm[16];
  if (fire[blockIdx.y].done) return;
  const SysDesc &D = descs[sys_list[blockIdx.y]];
  const int first = blockIdx.x * kFireChunk;
  if (first >= D.n) return;
  const int last = min(D.n, first + kFireChunk);
  const int64_t N = A.ntot, off = D.off;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double v3[3] = {0.0, 0.0, 0.0};
  double fm = 0.0;
  for (int i = first + tid; i < last; i += kFireThreads) {
    const int64_t a = off + i;
    if ((A.tr[a] >> 1) != ROLE_MOBILE) continue;
    double a2 = 0.0;
    for (int k = 0; k < D.dim; ++k) {
      const double F = A.ftot[k * N + a], v = A.v[k * N + a];
      v3[0] += F * v;
      v3[1] += v * v;
      v3[2] += F * F;
      a2 += F * F;
    }
    fm = fmax(fm, a2);
  }
  block_sum<3>(v3, red);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) fm = fmax(fm, __shfl_xor(fm, o, 64));
  if (lane == 0) redm[wave] = fm;
  __syncthreads();
  if (tid != 0) return;
  for (int w = 0; w < kFireThreads / 64; ++w) fm = fmax(fm, redm[w]);
  double *p = partials + ((int64_t)blockIdx.y * maxchunks + blockIdx.x) * 4;
  p[0] = v3[0]; p[1] = v3[1]; p[2] = v3[2]; p[3] = fm;
}

// Second level and the FIRE control, one workgroup per listed system: the
// chunks' partials in chunk order, convergence, mixing, step size, and the
// rigid body's step (one thread).
__global__ __launch_bounds__(kFireThreads) void k_fire_control(const SysDesc *__restrict__ descs,
                                                               SysState *__restrict__ states, Arrays A,
                                                               const int32_t *__restrict__ sys_list,
                                                               FireSys *__restrict__ fire, double ftol,
                                                               int64_t iter, const double *__restrict__ partials,
                                                               int maxchunks) {
  __shared__ double red[3 * 16];
  __shared__ double redm[16];
  const int b = blockIdx.x;
  FireSys &f = fire[b];
  if (f.done) return;
  const int s = sys_list[b];
  const SysDesc &D = descs[s];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nchunks = (D.n + kFireChunk - 1) / kFireChunk;
  double v3[3] = {0.0, 0.0, 0.0};   // P, |v|^2, |F|^2 over the mobile atoms
  double fm = 0.0;                  // largest |F|^2 of a mobile atom
  for (int c = tid; c < nchunks; c += kFireThreads) {
    const double *p = partials + ((int64_t)b * maxchunks + c) * 4;
    v3[0] += p[0]; v3[1] += p[1]; v3[2] += p[2];
    fm = fmax(fm, p[3]);
  }
  block_sum<3>(v3, red);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) fm = fmax(fm, __shfl_xor(fm, o, 64));
  if (lane == 0) redm[wave] = fm;
  __syncthreads();
  if (tid != 0) return;
  for (int w = 0; w < kFireThreads / 64; ++w) fm = fmax(fm, redm[w]);
  SysState &st = states[s];
  double P = v3[0], vv = v3[1], ff = v3[2];
  if (D.n_rigid > 0) {
    double r2 = 0.0;
    for (int k = 0; k < D.dim; ++k) {
      P += st.FR[k] * st.VR[k];
      vv += st.VR[k] * st.VR[k];
      ff += st.FR[k] * st.FR[k];
      r2 += st.FR[k] * st.FR[k];
    }
    fm = fmax(fm, r2);
  }
  f.fmax = sqrt(fm);
  if (f.fmax < ftol) {   // converged at the positions of this iteration
    f.done = 1;
    f.iters = iter;
    return;
  }
  const double vn = sqrt(vv), fn = sqrt(ff);
  double VR[3] = {st.VR[0], st.VR[1], st.VR[2]};
  if (P > 0.0) {
    f.mixv = 1.0 - f.alpha;
    f.mixf = fn > 0.0 ? f.alpha * vn / fn : 0.0;
    f.reset = 0;
    for (int k = 0; k < D.dim; ++k) VR[k] = f.mixv * VR[k] + f.mixf * st.FR[k];
    if (f.since_neg > kFireNmin) {
      f.dt = fmin(f.dt * kFireFinc, 10.0 * D.dt);
      f.alpha *= kFireFalpha;
    }
    f.since_neg += 1;
  } else {
    f.dt *= kFireFdec;
    f.alpha = kFireAlpha0;
    f.since_neg = 0;
    f.reset = 1;
    for (int k = 0; k < 3; ++k) VR[k] = 0.0;
  }
  // the rigid body's semi-implicit Euler step; its atoms follow it at the
  // next evaluation
  if (D.n_rigid > 0) {
    for (int k = 0; k < D.dim; ++k) {
      VR[k] += f.dt * st.FR[k] * D.inv_massR;
      st.XR[k] += f.dt * VR[k];
    }
  }
  for (int k = 0; k < 3; ++k) st.VR[k] = VR[k];
  f.iters = iter + 1;
}

// Mixing and semi-implicit Euler step of the mobile atoms: blockIdx.y is the
// listed system, blockIdx.x a chunk of its atoms.
__global__ __launch_bounds__(kFireThreads) void k_fire_move(const SysDesc *__restrict__ descs, Arrays A,
                                                            const int32_t *__restrict__ sys_list,
                                                            const FireSys *__restrict__ fire) {
  const FireSys &f = fire[blockIdx.y];
  if (f.done) return;
  const SysDesc &D = descs[sys_list[blockIdx.y]];
  const int i = blockIdx.x * kFireThreads + threadIdx.x;
  if (i >= D.n) return;
  const int64_t N = A.ntot, a = D.off + i;
  if ((A.tr[a] >> 1) != ROLE_MOBILE) return;
  for (int k = 0; k < D.dim; ++k) {
    const double F = A.ftot[k * N + a];
    double v = f.reset ? 0.0 : f.mixv * A.v[k * N + a] + f.mixf * F;
    v += f.dt * F * D.inv_mass;
    A.v[k * N + a] = v;
    A.x[k * N + a] = wrapx(A.x[k * N + a] + f.dt * v, D.box[k], D.periodic[k]);
  }
}

}  // namespace

hipError_t fire_iteration(const SysDesc *descs, SysState *states, const Arrays &A, const int32_t *sys_list,
                          int count, int nmax, FireSys *fire, double ftol, int64_t iter, double *partials,
                          hipStream_t stream) {
  if (count <= 0) return hipSuccess;
  const int maxchunks = (nmax + kFireChunk - 1) / kFireChunk;
  hipLaunchKernelGGL(k_fire_partial, dim3(maxchunks > 0 ? maxchunks : 1, count), dim3(kFireThreads), 0, stream,
                     descs, A, sys_list, fire, partials, maxchunks);
  hipLaunchKernelGGL(k_fire_control, dim3(count), dim3(kFireThreads), 0, stream, descs, states, A, sys_list, fire,
                     ftol, iter, partials, maxchunks);
  const int chunks = (nmax + kFireThreads - 1) / kFireThreads;
  hipLaunchKernelGGL(k_fire_move, dim3(chunks > 0 ? chunks : 1, count), dim3(kFireThreads), 0, stream, descs, A,
                     sys_list, fire);
  return hipGetLastError();
}

}  // namespace hdk
