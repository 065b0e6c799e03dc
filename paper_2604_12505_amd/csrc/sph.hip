// Body-frame weakly compressible SPH step for gfx950 (MI355X), coupled to
// planar rigid-body dynamics, behind the C ABI of include/slosh.h.
//
// One step (the paper's state-transition algorithm, Section 3.4, followed by
// first-order symplectic Euler) is five kernels, captured into HIP graphs
// for rollouts:
//
//   sph_bin      apply the previous step's fluid update (deferred so that it
//                can use the rigid accelerations of that step), compute each
//                particle's cell key, count particles per cell (atomics on
//                integer counters only), latch escape / non-finite flags;
//   sph_scan     exclusive scan of the cell counts (one workgroup), which
//                also clears the counters for the next step;
//   sph_place    stable counting-sort placement: one thread per destination
//                cell walks the 3x3 block of source cells in ascending key
//                order and copies the particles that now belong to it, so the
//                new order is deterministic and particle state is rewritten
//                cell-contiguously (coalesced reads in the neighbour loops);
//   sph_density  density with the gamma1 ghost term (eq. density_update) and
//                the equation of state (eq. EOS, or its Tait form), stored as
//                (rho, P/rho^2);
//   sph_force    fluid-fluid pressure (eq. momentum) and viscosity (eq.
//                viscous), ghost-to-fluid pressure and viscosity with the
//                spiky kernel (eqs. pressure_b2f, viscous_b2f), per-particle
//                reaction wrench reduced per workgroup, then the last
//                workgroup to finish reduces the partials in a fixed order,
//                applies the zero-order-hold attitude law, the rigid-body
//                equations (eq. tankdynamics) and writes the logs.
//
// Neighbours are found on a body-frame cell grid of side 2h (1 + 1e-6): the
// support of every pair sum, so candidates of a particle lie in the three
// contiguous key ranges of its 3x3 cell block.  Ghost particles are fixed in
// the body frame, so their cell list is built once.  No floating-point
// atomics are used: repeated runs are bitwise identical.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "slosh.h"

namespace {

constexpr int kBlock = 256;       // threads per workgroup of the particle kernels
constexpr int kScanThreads = 1024;
constexpr int kChunk = 64;        // steps per captured graph (even: parity returns)

// --------------------------------------------------------------------------
// device-side structures
// --------------------------------------------------------------------------

struct Grid {
  double x0, y0, inv_cell;  // key = floor((x - x0) * inv_cell), in double
  int ncx, ncy;
};

struct Consts {
  float inv_h, R2;          // cubic-spline support (2h)^2, binary32
  float Rs2, hs;            // spiky support h_s and h_s^2
  float wc;                 // cubic constant sigma
  float dwc;                // sigma / h^2: grad W = dwc * f(q) * r_ij
  float dws;                // spiky -30 / (pi h_s^5)
  float mass, gamma1, rho0, rho0_inv, B, k_lin;
  float a2h;                // 2 alpha h
  float beta2;              // 2 beta
  float eps_h2;             // eps h^2
  float dt;
  int eos, tgamma;          // tgamma > 0: integer Tait exponent
  float tgamma_f;
};

struct DevRigid {
  double r[2], theta, rdot[2], thetadot;  // state at global step `step`
  double tau_ctrl;                        // torque held by the zero-order hold
  double wrench[3];                       // body-frame wrench of the last evaluation
  double acc[3];                          // r''_x, r''_y, theta'' of the last evaluation
  double th_eval, thd_eval;               // theta, thetadot used by the last evaluation
  double wsum[3];                         // running sum for the mean-wrench log
  long long step;
  int wcount, pad0;
  // binary32 coefficients of the fluid update of the last evaluated step
  float c, s, abx, aby, thd, thdd, pad1[2];
};

struct DevRollout {
  const float* u;           // [n_steps][3] or null
  const double* theta_ref;  // [n_ref] or null
  float* y_log;
  float* w_log;
  float* u_log;
  float* wm_log;
  long long step0;          // global step of local step 0
  long long n_steps;
  int n_ref, log_stride;
};

enum Mode { kStep = 0, kEval = 1 };

// --------------------------------------------------------------------------
// small device helpers
// --------------------------------------------------------------------------

__device__ __forceinline__ int cell_coord(float x, double x0, double inv, int n) {
  double f = floor(((double)x - x0) * inv);
  if (!(f == f)) f = 0.0;   // NaN: flagged elsewhere
  f = f < 0.0 ? 0.0 : f;
  f = f > (double)(n - 1) ? (double)(n - 1) : f;
  return (int)f;
}

__device__ __forceinline__ void cell_of(float2 s, const Grid& g, int& cx, int& cy) {
  cx = cell_coord(s.x, g.x0, g.inv_cell, g.ncx);
  cy = cell_coord(s.y, g.y0, g.inv_cell, g.ncy);
}

// Squared distance exactly as fmaf(dy, dy, dx*dx) in binary32.
__device__ __forceinline__ float dist2(float dx, float dy) {
  return __builtin_fmaf(dy, dy, dx * dx);
}

// Cubic spline (eq. cubicspline) shape without its constant, q = r/h < 2.
__device__ __forceinline__ float cubic_shape(float q) {
  float a = 2.0f - q;
  float w = a * a * a;
  if (q < 1.0f) {
    float b = 1.0f - q;
    w -= 4.0f * b * b * b;
  }
  return w;
}

// (dW/dr)/r of the cubic spline divided by sigma/h^2:
//   q < 1:  -12 + 9 q;   1 <= q < 2:  -3 (2 - q)^2 / q.
__device__ __forceinline__ float cubic_grad_f(float q) {
  if (q < 1.0f) return 9.0f * q - 12.0f;
  float a = 2.0f - q;
  return -3.0f * a * a / q;
}

__device__ __forceinline__ float eos_over_rho2(float rho, const Consts& k, float* P_out) {
  float P;
  if (k.eos == SPH_EOS_LINEAR) {
    P = k.k_lin * (rho - k.rho0);
  } else {
    float x = rho * k.rho0_inv;
    float xp;
    if (k.tgamma > 0) {
      xp = 1.0f;
      float b = x;
      int e = k.tgamma;
      while (e) {
        if (e & 1) xp *= b;
        b *= b;
        e >>= 1;
      }
    } else {
      xp = powf(x, k.tgamma_f);
    }
    P = k.B * (xp - 1.0f);
  }
  if (P_out) *P_out = P;
  return P / (rho * rho);
}

// Visits every fluid particle j in the 3x3 cell block of position s, in
// ascending sorted order per grid row: f(j, s_j).
template <class F>
__device__ __forceinline__ void for_each_in_block(float2 s, const Grid& g, const int* __restrict__ start,
                                                  const float2* __restrict__ pos, F&& f) {
  int cx, cy;
  cell_of(s, g, cx, cy);
  int xa = cx > 0 ? cx - 1 : 0;
  int xb = cx < g.ncx - 1 ? cx + 1 : g.ncx - 1;
  for (int oy = -1; oy <= 1; ++oy) {
    int yy = cy + oy;
    if (yy < 0 || yy >= g.ncy) continue;
    int j0 = start[yy * g.ncx + xa];
    int j1 = start[yy * g.ncx + xb + 1];
    for (int j = j0; j < j1; ++j) f(j, pos[j]);
  }
}

// Body-frame fluid acceleration with the fictitious terms of the rotating,
// accelerating tank frame (x = r + R(theta) s differentiated twice):
//   dw/dt = a_sph - R^T r'' - 2 thetadot J w - theta'' J s + thetadot^2 s,  J v = (-v_y, v_x).
__device__ __forceinline__ float2 body_frame_accel(float2 s, float2 w, float2 a,
                                                   const DevRigid* __restrict__ rb) {
  float thd = rb->thd, thdd = rb->thdd, om2 = thd * thd;
  return make_float2(a.x - rb->abx + 2.0f * thd * w.y + thdd * s.y + om2 * s.x,
                     a.y - rb->aby - 2.0f * thd * w.x - thdd * s.x + om2 * s.y);
}

// First-order symplectic Euler: velocity first, then position with the new velocity.
__device__ __forceinline__ void fluid_update(float2& s, float2& w, float2 a,
                                             const DevRigid* __restrict__ rb, float dt) {
  float2 dw = body_frame_accel(s, w, a, rb);
  w.x += dt * dw.x;
  w.y += dt * dw.y;
  s.x += dt * w.x;
  s.y += dt * w.y;
}

__device__ __forceinline__ void flag(unsigned* status, unsigned bits) {
  if (bits) atomicOr(status, bits);
}

// --------------------------------------------------------------------------
// cell-list kernels
// --------------------------------------------------------------------------

// Deferred fluid update of the previous step (fictitious accelerations and
// symplectic Euler, velocity first), then cell key and count.
//   dw/dt = a_sph - R^T r'' - 2 thetadot J w - theta'' J s + thetadot^2 s
__global__ void __launch_bounds__(kBlock) sph_bin(float2* __restrict__ pos, float2* __restrict__ vel,
                                                  const float2* __restrict__ acc, int n, int integrate,
                                                  const DevRigid* __restrict__ rb, Grid g,
                                                  float dt, double lo_x, double lo_y, double hi_x,
                                                  double hi_y, int* __restrict__ key,
                                                  int* __restrict__ count, int* __restrict__ slot,
                                                  unsigned* __restrict__ status) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float2 s = pos[i];
  if (integrate) {
    float2 w = vel[i];
    fluid_update(s, w, acc[i], rb, dt);
    pos[i] = s;
    vel[i] = w;
    unsigned bad = 0;
    if (!isfinite(s.x) || !isfinite(s.y) || !isfinite(w.x) || !isfinite(w.y)) bad |= SPH_ST_NONFINITE;
    flag(status, bad);
  }
  unsigned bad = 0;
  if (!((double)s.x >= lo_x && (double)s.x < hi_x && (double)s.y >= lo_y && (double)s.y < hi_y))
    bad |= (isfinite(s.x) && isfinite(s.y)) ? SPH_ST_ESCAPED : SPH_ST_NONFINITE;
  flag(status, bad);
  int cx, cy;
  cell_of(s, g, cx, cy);
  int k = cy * g.ncx + cx;
  key[i] = k;
  int sl = atomicAdd(&count[k], 1);
  if (slot) slot[i] = sl;
}

// Exclusive scan of count[0..nc) into start[0..nc]; clears count.  One
// workgroup: each thread scans a contiguous slice, slice totals are scanned
// in LDS.
__global__ void __launch_bounds__(kScanThreads) sph_scan(int* __restrict__ count, int nc,
                                                         int* __restrict__ start, int expect,
                                                         unsigned* __restrict__ status) {
  __shared__ int part[kScanThreads];
  int t = threadIdx.x;
  int per = (nc + kScanThreads - 1) / kScanThreads;
  int b = t * per;
  int e = b + per < nc ? b + per : nc;
  int sum = 0;
  for (int c = b; c < e; ++c) sum += count[c];
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - sum;
  for (int c = b; c < e; ++c) {
    start[c] = run;
    run += count[c];
    count[c] = 0;
  }
  if (t == kScanThreads - 1) {
    start[nc] = part[t];
    if (part[t] != expect) atomicOr(status, SPH_ST_SORT);
  }
}

// Stable placement after a step: thread c gathers, in ascending source
// position, the particles of the 3x3 source block whose new key is c.
__global__ void __launch_bounds__(kBlock) sph_place(const int* __restrict__ key,
                                                    const int* __restrict__ start_old,
                                                    const int* __restrict__ start_new, Grid g,
                                                    const float2* __restrict__ pos_in,
                                                    const float2* __restrict__ vel_in,
                                                    const int* __restrict__ id_in,
                                                    float2* __restrict__ pos_out,
                                                    float2* __restrict__ vel_out,
                                                    int* __restrict__ id_out,
                                                    unsigned* __restrict__ status) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  int nc = g.ncx * g.ncy;
  if (c >= nc) return;
  int cy = c / g.ncx, cx = c - cy * g.ncx;
  int dst = start_new[c], end = start_new[c + 1];
  int xa = cx > 0 ? cx - 1 : 0;
  int xb = cx < g.ncx - 1 ? cx + 1 : g.ncx - 1;
  for (int oy = -1; oy <= 1; ++oy) {
    int yy = cy + oy;
    if (yy < 0 || yy >= g.ncy) continue;
    int i0 = start_old[yy * g.ncx + xa];
    int i1 = start_old[yy * g.ncx + xb + 1];
    for (int i = i0; i < i1; ++i) {
      if (key[i] != c) continue;
      if (dst < end) {
        pos_out[dst] = pos_in[i];
        vel_out[dst] = vel_in[i];
        id_out[dst] = id_in[i];
      }
      ++dst;
    }
  }
  if (dst != end) atomicOr(status, SPH_ST_SORT);
}

// General (first) sort: scatter by (key, atomic slot), then order each cell by
// source index, which makes the result a stable counting sort.
__global__ void sph_scatter(const int* __restrict__ key, const int* __restrict__ slot, int n,
                            const int* __restrict__ start, int* __restrict__ order) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  order[start[key[i]] + slot[i]] = i;
}

__global__ void sph_cell_order(const int* __restrict__ start, int nc, int* __restrict__ order) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  int b = start[c], e = start[c + 1];
  for (int i = b + 1; i < e; ++i) {
    int v = order[i];
    int j = i - 1;
    while (j >= b && order[j] > v) {
      order[j + 1] = order[j];
      --j;
    }
    order[j + 1] = v;
  }
}

__global__ void sph_gather(const int* __restrict__ order, int n, const float2* __restrict__ pos_in,
                           const float2* __restrict__ vel_in, const int* __restrict__ id_in,
                           float2* __restrict__ pos_out, float2* __restrict__ vel_out,
                           int* __restrict__ id_out) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int i = order[p];
  pos_out[p] = pos_in[i];
  if (vel_in) vel_out[p] = vel_in[i];
  if (id_out) id_out[p] = id_in ? id_in[i] : i;
}

// --------------------------------------------------------------------------
// particle sums
// --------------------------------------------------------------------------

// rho_i = m sigma (sum_f shape + gamma1 sum_g shape), then P and P/rho^2.
__global__ void __launch_bounds__(kBlock) sph_density(const float2* __restrict__ pos,
                                                      const int* __restrict__ start,
                                                      const float2* __restrict__ gpos,
                                                      const int* __restrict__ gstart, int n, Grid g,
                                                      Consts k, float2* __restrict__ rp) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  float2 s = pos[p];
  float sf = 0.0f, sg = 0.0f;
  for_each_in_block(s, g, start, pos, [&](int, float2 sj) {
    float dx = s.x - sj.x, dy = s.y - sj.y;
    float d2 = dist2(dx, dy);
    if (d2 < k.R2) sf += cubic_shape(sqrtf(d2) * k.inv_h);
  });
  for_each_in_block(s, g, gstart, gpos, [&](int, float2 gj) {
    float dx = s.x - gj.x, dy = s.y - gj.y;
    float d2 = dist2(dx, dy);
    if (d2 < k.R2) sg += cubic_shape(sqrtf(d2) * k.inv_h);
  });
  float rho = k.mass * k.wc * (sf + k.gamma1 * sg);
  float pr = eos_over_rho2(rho, k, nullptr);
  rp[p] = make_float2(rho, pr);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Rigid-body part of a step, run by one thread after the wrench is reduced:
// zero-order-hold attitude law, eq. tankdynamics, logs, symplectic Euler.
__device__ void rigid_step(DevRigid* rb, const DevRollout* ro, const double F[3], int mode,
                           double dt, double body_mass, double body_inertia, int motion, int ctrl,
                           int ctrl_period, double kp, double kd, double sine_amp,
                           double sine_freq) {
  long long n = rb->step;
  long long loc = n - ro->step0;
  double u[3] = {0.0, 0.0, 0.0};
  if (mode == kStep && ro->u && loc >= 0 && loc < ro->n_steps) {
    u[0] = ro->u[3 * loc];
    u[1] = ro->u[3 * loc + 1];
    u[2] = ro->u[3 * loc + 2];
  } else if (mode == kEval && ro->u) {
    u[0] = ro->u[0];
    u[1] = ro->u[1];
    u[2] = ro->u[2];
  }
  if (mode == kStep && ctrl == SPH_CTRL_PD_ZOH && ctrl_period > 0 && n % ctrl_period == 0) {
    long long kk = n / ctrl_period;
    double ref = 0.0;
    if (ro->theta_ref && ro->n_ref > 0) ref = ro->theta_ref[kk < ro->n_ref ? kk : ro->n_ref - 1];
    rb->tau_ctrl = kp * (ref - rb->theta) - kd * rb->thetadot;
  }
  double th, thd, acc[3];
  if (motion == SPH_MOTION_SINE) {
    double w = 2.0 * M_PI * sine_freq, t = (double)n * dt;
    th = sine_amp * sin(w * t);
    thd = sine_amp * w * cos(w * t);
    acc[0] = acc[1] = 0.0;
    acc[2] = -sine_amp * w * w * sin(w * t);
  } else {
    th = rb->theta;
    thd = rb->thetadot;
    double c = cos(th), s = sin(th);
    acc[0] = (c * F[0] - s * F[1] + u[0]) / body_mass;
    acc[1] = (s * F[0] + c * F[1] + u[1]) / body_mass;
    acc[2] = (F[2] + u[2] + rb->tau_ctrl) / body_inertia;
  }
  for (int d = 0; d < 3; ++d) {
    rb->wrench[d] = F[d];
    rb->acc[d] = acc[d];
  }
  rb->th_eval = th;
  rb->thd_eval = thd;
  double c = cos(th), s = sin(th);
  rb->c = (float)c;
  rb->s = (float)s;
  rb->abx = (float)(c * acc[0] + s * acc[1]);    // R^T r''
  rb->aby = (float)(-s * acc[0] + c * acc[1]);
  rb->thd = (float)thd;
  rb->thdd = (float)acc[2];
  if (mode != kStep) return;

  if (ro->log_stride > 0 && loc >= 0 && loc < ro->n_steps) {
    long long kk = loc / ro->log_stride;
    if (loc % ro->log_stride == 0) {
      if (ro->y_log) {
        float* y = ro->y_log + 6 * kk;
        y[0] = (float)rb->r[0];
        y[1] = (float)rb->r[1];
        y[2] = (float)rb->theta;
        y[3] = (float)rb->rdot[0];
        y[4] = (float)rb->rdot[1];
        y[5] = (float)rb->thetadot;
      }
      if (ro->w_log)
        for (int d = 0; d < 3; ++d) ro->w_log[3 * kk + d] = (float)F[d];
      if (ro->u_log) {
        ro->u_log[3 * kk] = (float)u[0];
        ro->u_log[3 * kk + 1] = (float)u[1];
        ro->u_log[3 * kk + 2] = (float)(u[2] + rb->tau_ctrl);
      }
    }
    for (int d = 0; d < 3; ++d) rb->wsum[d] += F[d];
    rb->wcount += 1;
    if (loc % ro->log_stride == ro->log_stride - 1 || loc == ro->n_steps - 1) {
      if (ro->wm_log)
        for (int d = 0; d < 3; ++d) ro->wm_log[3 * kk + d] = (float)(rb->wsum[d] / rb->wcount);
      rb->wsum[0] = rb->wsum[1] = rb->wsum[2] = 0.0;
      rb->wcount = 0;
    }
  }
  if (motion == SPH_MOTION_SINE) {
    double w = 2.0 * M_PI * sine_freq, t = (double)(n + 1) * dt;
    rb->theta = sine_amp * sin(w * t);
    rb->thetadot = sine_amp * w * cos(w * t);
    rb->r[0] = rb->r[1] = rb->rdot[0] = rb->rdot[1] = 0.0;
  } else {
    rb->rdot[0] += dt * acc[0];
    rb->rdot[1] += dt * acc[1];
    rb->thetadot += dt * acc[2];
    rb->r[0] += dt * rb->rdot[0];
    rb->r[1] += dt * rb->rdot[1];
    rb->theta += dt * rb->thetadot;
  }
  rb->step = n + 1;
}

struct RigidArgs {
  double dt, body_mass, body_inertia, kp, kd, sine_amp, sine_freq;
  int motion, ctrl, ctrl_period, mode;
};

// Forces and the slosh wrench.  a_i = m sum_j [-(P_i/rho_i^2 + P_j/rho_j^2)
//   + 2 alpha h (w_ij . s_ij) / ((rho_i + rho_j)(r^2 + eps h^2))] grad_i W_ij
//   + sum_g m [-2 P_i/rho_i^2 + (2 beta / (2 rho_i)) min(w_i . s_ig, 0)/(r^2 + eps h^2)] grad_i W_s3
// The tank receives -m * (wall term) per pair, with torque arm g.
__global__ void __launch_bounds__(kBlock) sph_force(const float2* __restrict__ pos,
                                                    const float2* __restrict__ vel,
                                                    const float2* __restrict__ rp,
                                                    const int* __restrict__ start,
                                                    const float2* __restrict__ gpos,
                                                    const int* __restrict__ gstart, int n, Grid g,
                                                    Consts k, float2* __restrict__ acc,
                                                    double* __restrict__ partials,
                                                    unsigned* __restrict__ ticket, DevRigid* rb,
                                                    const DevRollout* __restrict__ ro, RigidArgs ra) {
  __shared__ double red[3][kBlock / 64];
  __shared__ int last;
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  float fx = 0.0f, fy = 0.0f, tq = 0.0f;
  if (p < n) {
    float2 s = pos[p];
    float2 w = vel[p];
    float2 me = rp[p];
    float rho_i = me.x, Pi = me.y;
    float axf = 0.0f, ayf = 0.0f;
    for_each_in_block(s, g, start, pos, [&](int j, float2 sj) {
      float dx = s.x - sj.x, dy = s.y - sj.y;
      float d2 = dist2(dx, dy);
      if (d2 < k.R2 && d2 > 0.0f) {
        float2 wj = vel[j];
        float2 o = rp[j];
        float q = sqrtf(d2) * k.inv_h;
        float gW = k.dwc * cubic_grad_f(q);
        float vr = (w.x - wj.x) * dx + (w.y - wj.y) * dy;
        float coef = (-(Pi + o.y) + k.a2h * vr / ((rho_i + o.x) * (d2 + k.eps_h2))) * gW;
        axf += coef * dx;
        ayf += coef * dy;
      }
    });
    float axg = 0.0f, ayg = 0.0f;
    for_each_in_block(s, g, gstart, gpos, [&](int, float2 gj) {
      float dx = s.x - gj.x, dy = s.y - gj.y;
      float d2 = dist2(dx, dy);
      if (d2 < k.Rs2 && d2 > 0.0f) {
        float r = sqrtf(d2);
        float t = k.hs - r;
        float gW = k.dws * t * t / r;
        float vr = w.x * dx + w.y * dy;
        float coef = k.mass * (-2.0f * Pi + k.beta2 / (2.0f * rho_i) * fminf(vr, 0.0f) / (d2 + k.eps_h2)) * gW;
        float ax = coef * dx, ay = coef * dy;   // wall force on the fluid / m
        axg += ax;
        ayg += ay;
        float Fx = k.mass * ax, Fy = k.mass * ay;
        fx -= Fx;
        fy -= Fy;
        tq -= gj.x * Fy - gj.y * Fx;
      }
    });
    acc[p] = make_float2(k.mass * axf + axg, k.mass * ayf + ayg);
  }
  // workgroup reduction of the wrench, in double, fixed order
  double v[3] = {(double)fx, (double)fy, (double)tq};
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int d = 0; d < 3; ++d) {
    double t = wave_sum(v[d]);
    if (lane == 0) red[d][wv] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int d = 0; d < 3; ++d) {
      double t = 0.0;
      for (int q = 0; q < kBlock / 64; ++q) t += red[d][q];
      partials[3 * blockIdx.x + d] = t;
    }
    __threadfence();
    unsigned tk = atomicAdd(ticket, 1u);
    last = (tk == gridDim.x - 1);
  }
  __syncthreads();
  if (!last) return;
  // last workgroup: reduce all partials in a fixed order
  __threadfence();
  double acc3[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < (int)gridDim.x; b += blockDim.x)
    for (int d = 0; d < 3; ++d) acc3[d] += partials[3 * b + d];
  for (int d = 0; d < 3; ++d) {
    double t = wave_sum(acc3[d]);
    if (lane == 0) red[d][wv] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double F[3];
    for (int d = 0; d < 3; ++d) {
      double t = 0.0;
      for (int q = 0; q < kBlock / 64; ++q) t += red[d][q];
      F[d] = t;
    }
    rigid_step(rb, ro, F, ra.mode, ra.dt, ra.body_mass, ra.body_inertia, ra.motion, ra.ctrl,
               ra.ctrl_period, ra.kp, ra.kd, ra.sine_amp, ra.sine_freq);
    *ticket = 0u;
  }
}

// Final fluid update at the end of a rollout (the same update sph_bin defers).
__global__ void __launch_bounds__(kBlock) sph_integrate(float2* __restrict__ pos, float2* __restrict__ vel,
                                                        const float2* __restrict__ acc, int n,
                                                        const DevRigid* __restrict__ rb, float dt,
                                                        unsigned* __restrict__ status) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float2 s = pos[i], w = vel[i];
  fluid_update(s, w, acc[i], rb, dt);
  pos[i] = s;
  vel[i] = w;
  if (!isfinite(s.x) || !isfinite(s.y) || !isfinite(w.x) || !isfinite(w.y)) flag(status, SPH_ST_NONFINITE);
}

// Outputs of sph_rhs in caller order.
__global__ void sph_rhs_out(const float2* __restrict__ pos, const float2* __restrict__ vel,
                            const float2* __restrict__ acc, const float2* __restrict__ rp,
                            const int* __restrict__ id, int n, const DevRigid* __restrict__ rb,
                            Consts k, float* rho_o, float* p_o, float2* a_o, float2* wd_o) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  int i = id[q];
  float rho = rp[q].x;
  float P;
  eos_over_rho2(rho, k, &P);
  if (rho_o) rho_o[i] = rho;
  if (p_o) p_o[i] = P;
  float2 a = acc[q], s = pos[q], w = vel[q];
  if (a_o) a_o[i] = a;
  if (wd_o) wd_o[i] = body_frame_accel(s, w, a, rb);
}

__global__ void sph_small_out(const DevRigid* __restrict__ rb, float* wrench, float* acc3, int frame) {
  if (threadIdx.x != 0) return;
  double F0 = rb->wrench[0], F1 = rb->wrench[1];
  if (frame == SPH_FRAME_WORLD) {
    double c = cos(rb->th_eval), s = sin(rb->th_eval);
    double a = c * F0 - s * F1, b = s * F0 + c * F1;
    F0 = a;
    F1 = b;
  }
  if (wrench) {
    wrench[0] = (float)F0;
    wrench[1] = (float)F1;
    wrench[2] = (float)rb->wrench[2];
  }
  if (acc3)
    for (int d = 0; d < 3; ++d) acc3[d] = (float)rb->acc[d];
}

__global__ void sph_unpermute(const float2* __restrict__ src, const int* __restrict__ id, int n,
                              float2* __restrict__ dst) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  dst[id[q]] = src[q];
}

__global__ void sph_set_rollout(DevRollout* ro, DevRollout v, const DevRigid* rb) {
  if (threadIdx.x != 0) return;
  v.step0 = rb->step;
  *ro = v;
}

// Test hook: neighbour ids (caller order) of every particle, ascending.
__global__ void sph_nbr_list(const float2* __restrict__ pos, const int* __restrict__ start,
                             const int* __restrict__ id, int n, Grid g, Consts k, int max_nbr,
                             int* __restrict__ nbr, int* __restrict__ cnt) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  float2 s = pos[p];
  int i = id[p];
  int c = 0;
  int* row = nbr + (size_t)i * max_nbr;
  for_each_in_block(s, g, start, pos, [&](int j, float2 sj) {
    if (j == p) return;
    float dx = s.x - sj.x, dy = s.y - sj.y;
    if (dist2(dx, dy) < k.R2) {
      if (c < max_nbr) row[c] = id[j];
      ++c;
    }
  });
  cnt[i] = c;
  int m = c < max_nbr ? c : max_nbr;
  for (int a = 1; a < m; ++a) {
    int v = row[a], b = a - 1;
    while (b >= 0 && row[b] > v) {
      row[b + 1] = row[b];
      --b;
    }
    row[b + 1] = v;
  }
}

// --------------------------------------------------------------------------
// host side
// --------------------------------------------------------------------------

thread_local char g_err[512];

int hip_fail(hipError_t e, const char* what) {
  snprintf(g_err, sizeof g_err, "%s: %s", what, hipGetErrorString(e));
  return SPH_E_HIP;
}

#define HIPCHK(x)                                  \
  do {                                             \
    hipError_t e_ = (x);                           \
    if (e_ != hipSuccess) return hip_fail(e_, #x); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
  size_t pos[2], vel[2], id[2], acc, rp, key, slot, order, count, cstart[2], gpos, graw, gstart,
      partials, rigid, rollout, ticket, status, total;
};

bool make_grid(const sph_params* p, Grid* g) {
  double support = 2.0 * p->h > p->h_spiky ? 2.0 * p->h : p->h_spiky;
  double cell = support * (1.0 + 1e-6);
  double w = p->domain_max[0] - p->domain_min[0], hh = p->domain_max[1] - p->domain_min[1];
  if (!(w > 0 && hh > 0 && cell > 0)) return false;
  double nx = std::ceil(w / cell), ny = std::ceil(hh / cell);
  if (nx < 1) nx = 1;
  if (ny < 1) ny = 1;
  if (nx * ny > double(1 << 26)) return false;
  g->x0 = p->domain_min[0];
  g->y0 = p->domain_min[1];
  g->inv_cell = 1.0 / cell;
  g->ncx = (int)nx;
  g->ncy = (int)ny;
  return true;
}

int nblocks(int n) { return n > 0 ? (n + kBlock - 1) / kBlock : 1; }

Layout make_layout(int N, int G, int nc) {
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes > 0 ? bytes : 1);
    return at;
  };
  size_t n = (size_t)N, gg = (size_t)G;
  for (int b = 0; b < 2; ++b) {
    L.pos[b] = take(n * 8);
    L.vel[b] = take(n * 8);
    L.id[b] = take(n * 4);
  }
  L.acc = take(n * 8);
  L.rp = take(n * 8);
  L.key = take((n > gg ? n : gg) * 4);
  L.slot = take((n > gg ? n : gg) * 4);
  L.order = take((n > gg ? n : gg) * 4);
  L.count = take((size_t)nc * 4);
  L.cstart[0] = take(((size_t)nc + 1) * 4);
  L.cstart[1] = take(((size_t)nc + 1) * 4);
  L.gpos = take(gg * 8);
  L.graw = take(gg * 8);
  L.gstart = take(((size_t)nc + 1) * 4);
  L.partials = take((size_t)nblocks(N) * 3 * 8);
  L.rigid = take(sizeof(DevRigid));
  L.rollout = take(sizeof(DevRollout));
  L.ticket = take(4);
  L.status = take(4);
  L.total = o;
  return L;
}

bool params_ok(const sph_params* p) {
  if (!p) return false;
  if (!(p->h > 0 && p->h_spiky > 0 && p->mass > 0 && p->dt > 0 && p->rho0 > 0)) return false;
  if (p->eos != SPH_EOS_TAIT && p->eos != SPH_EOS_LINEAR) return false;
  if (p->eos == SPH_EOS_TAIT && !(p->c0 > 0 && p->tait_gamma > 0)) return false;
  if (p->motion != SPH_MOTION_FREE && p->motion != SPH_MOTION_SINE) return false;
  if (p->ctrl != SPH_CTRL_NONE && p->ctrl != SPH_CTRL_PD_ZOH) return false;
  if (p->kernel_norm != SPH_KNORM_UNIT && p->kernel_norm != SPH_KNORM_PRINTED) return false;
  if (p->motion == SPH_MOTION_FREE && !(p->body_mass > 0 && p->body_inertia > 0)) return false;
  if (p->ctrl == SPH_CTRL_PD_ZOH && p->ctrl_period <= 0) return false;
  return true;
}

Consts make_consts(const sph_params* p) {
  Consts k;
  double h = p->h, hs = p->h_spiky;
  double sigma = (p->kernel_norm == SPH_KNORM_PRINTED ? 15.0 : 5.0) / (14.0 * M_PI * h * h);
  k.inv_h = (float)(1.0 / h);
  float r = (float)(2.0 * h);
  k.R2 = r * r;
  float rs = (float)hs;
  k.Rs2 = rs * rs;
  k.hs = rs;
  k.wc = (float)sigma;
  k.dwc = (float)(sigma / (h * h));
  k.dws = (float)(-30.0 / (M_PI * std::pow(hs, 5)));
  k.mass = (float)p->mass;
  k.gamma1 = (float)p->gamma1;
  k.rho0 = (float)p->rho0;
  k.rho0_inv = (float)(1.0 / p->rho0);
  k.B = (float)(p->eos == SPH_EOS_TAIT ? p->rho0 * p->c0 * p->c0 / p->tait_gamma : 0.0);
  k.k_lin = (float)p->k_lin;
  k.a2h = (float)(2.0 * p->visc_alpha * h);
  k.beta2 = (float)(2.0 * p->visc_beta);
  k.eps_h2 = (float)(p->eps * h * h);
  k.dt = (float)p->dt;
  k.eos = p->eos;
  double gi = std::round(p->tait_gamma);
  k.tgamma = (std::fabs(gi - p->tait_gamma) < 1e-12 && gi >= 1 && gi <= 64) ? (int)gi : 0;
  k.tgamma_f = (float)p->tait_gamma;
  return k;
}

}  // namespace

struct sph_handle {
  sph_params p;
  int N, G, nc;
  Grid grid;
  Consts k;
  RigidArgs ra;
  hipStream_t stream;
  char* ws;
  Layout L;
  int cur;
  hipGraphExec_t graph[2];   // kChunk steps starting from buffer 0 / 1
  bool graph_ok[2];

  template <class T>
  T* at(size_t off) { return reinterpret_cast<T*>(ws + off); }
};

namespace {

// Enqueues one step (first: the state is already integrated, skip the deferred
// update).  ev, if given, holds 6 events recorded around the 5 kernels.
void enqueue_step(sph_handle* h, bool first, int mode, hipEvent_t* ev = nullptr) {
  int src = h->cur, dst = 1 - h->cur;
  const sph_params& p = h->p;
  auto mark = [&](int i) {
    if (ev) (void)hipEventRecord(ev[i], h->stream);
  };
  mark(0);
  hipLaunchKernelGGL(sph_bin, dim3(nblocks(h->N)), dim3(kBlock), 0, h->stream,
                     h->at<float2>(h->L.pos[src]), h->at<float2>(h->L.vel[src]),
                     h->at<float2>(h->L.acc), h->N, first ? 0 : 1, h->at<DevRigid>(h->L.rigid),
                     h->grid, h->k.dt, p.domain_min[0], p.domain_min[1], p.domain_max[0],
                     p.domain_max[1], h->at<int>(h->L.key), h->at<int>(h->L.count), (int*)nullptr,
                     h->at<unsigned>(h->L.status));
  mark(1);
  hipLaunchKernelGGL(sph_scan, dim3(1), dim3(kScanThreads), 0, h->stream, h->at<int>(h->L.count),
                     h->nc, h->at<int>(h->L.cstart[dst]), h->N, h->at<unsigned>(h->L.status));
  mark(2);
  hipLaunchKernelGGL(sph_place, dim3(nblocks(h->nc)), dim3(kBlock), 0, h->stream,
                     h->at<int>(h->L.key), h->at<int>(h->L.cstart[src]),
                     h->at<int>(h->L.cstart[dst]), h->grid, h->at<float2>(h->L.pos[src]),
                     h->at<float2>(h->L.vel[src]), h->at<int>(h->L.id[src]),
                     h->at<float2>(h->L.pos[dst]), h->at<float2>(h->L.vel[dst]),
                     h->at<int>(h->L.id[dst]), h->at<unsigned>(h->L.status));
  mark(3);
  hipLaunchKernelGGL(sph_density, dim3(nblocks(h->N)), dim3(kBlock), 0, h->stream,
                     h->at<float2>(h->L.pos[dst]), h->at<int>(h->L.cstart[dst]),
                     h->at<float2>(h->L.gpos), h->at<int>(h->L.gstart), h->N, h->grid, h->k,
                     h->at<float2>(h->L.rp));
  mark(4);
  RigidArgs ra = h->ra;
  ra.mode = mode;
  hipLaunchKernelGGL(sph_force, dim3(nblocks(h->N)), dim3(kBlock), 0, h->stream,
                     h->at<float2>(h->L.pos[dst]), h->at<float2>(h->L.vel[dst]),
                     h->at<float2>(h->L.rp), h->at<int>(h->L.cstart[dst]), h->at<float2>(h->L.gpos),
                     h->at<int>(h->L.gstart), h->N, h->grid, h->k, h->at<float2>(h->L.acc),
                     h->at<double>(h->L.partials), h->at<unsigned>(h->L.ticket),
                     h->at<DevRigid>(h->L.rigid), h->at<DevRollout>(h->L.rollout), ra);
  mark(5);
  h->cur = dst;
}

void enqueue_integrate(sph_handle* h) {
  hipLaunchKernelGGL(sph_integrate, dim3(nblocks(h->N)), dim3(kBlock), 0, h->stream,
                     h->at<float2>(h->L.pos[h->cur]), h->at<float2>(h->L.vel[h->cur]),
                     h->at<float2>(h->L.acc), h->N, h->at<DevRigid>(h->L.rigid), h->k.dt,
                     h->at<unsigned>(h->L.status));
}

// Full stable sort of the raw fluid arrays (caller order) into buffer 0.
int sort_fluid(sph_handle* h, const float2* s, const float2* w) {
  int nb = nblocks(h->N);
  const sph_params& p = h->p;
  // the raw arrays go through buffer 1 so that s/w may alias nothing of ours
  if (h->N > 0) {
    HIPCHK(hipMemcpyAsync(h->at<float2>(h->L.pos[1]), s, (size_t)h->N * 8, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->at<float2>(h->L.vel[1]), w, (size_t)h->N * 8, hipMemcpyDeviceToDevice, h->stream));
  }
  HIPCHK(hipMemsetAsync(h->at<int>(h->L.count), 0, (size_t)h->nc * 4, h->stream));
  hipLaunchKernelGGL(sph_bin, dim3(nb), dim3(kBlock), 0, h->stream, h->at<float2>(h->L.pos[1]),
                     h->at<float2>(h->L.vel[1]), h->at<float2>(h->L.acc), h->N, 0,
                     h->at<DevRigid>(h->L.rigid), h->grid, h->k.dt, p.domain_min[0],
                     p.domain_min[1], p.domain_max[0], p.domain_max[1], h->at<int>(h->L.key),
                     h->at<int>(h->L.count), h->at<int>(h->L.slot), h->at<unsigned>(h->L.status));
  hipLaunchKernelGGL(sph_scan, dim3(1), dim3(kScanThreads), 0, h->stream, h->at<int>(h->L.count),
                     h->nc, h->at<int>(h->L.cstart[0]), h->N, h->at<unsigned>(h->L.status));
  if (h->N > 0) {
    hipLaunchKernelGGL(sph_scatter, dim3(nb), dim3(kBlock), 0, h->stream, h->at<int>(h->L.key),
                       h->at<int>(h->L.slot), h->N, h->at<int>(h->L.cstart[0]), h->at<int>(h->L.order));
    hipLaunchKernelGGL(sph_cell_order, dim3(nblocks(h->nc)), dim3(kBlock), 0, h->stream,
                       h->at<int>(h->L.cstart[0]), h->nc, h->at<int>(h->L.order));
    hipLaunchKernelGGL(sph_gather, dim3(nb), dim3(kBlock), 0, h->stream, h->at<int>(h->L.order), h->N,
                       h->at<float2>(h->L.pos[1]), h->at<float2>(h->L.vel[1]), (const int*)nullptr,
                       h->at<float2>(h->L.pos[0]), h->at<float2>(h->L.vel[0]), h->at<int>(h->L.id[0]));
  }
  HIPCHK(hipGetLastError());
  h->cur = 0;
  return SPH_OK;
}

int sort_ghosts(sph_handle* h, const float2* graw) {
  int nb = nblocks(h->G);
  HIPCHK(hipMemsetAsync(h->at<int>(h->L.count), 0, (size_t)h->nc * 4, h->stream));
  unsigned* scratch_status = h->at<unsigned>(h->L.ticket);  // ghost escapes are not fluid errors
  hipLaunchKernelGGL(sph_bin, dim3(nb), dim3(kBlock), 0, h->stream, const_cast<float2*>(graw),
                     (float2*)nullptr, (const float2*)nullptr, h->G, 0, h->at<DevRigid>(h->L.rigid),
                     h->grid, h->k.dt, -1e300, -1e300, 1e300, 1e300, h->at<int>(h->L.key),
                     h->at<int>(h->L.count), h->at<int>(h->L.slot), scratch_status);
  hipLaunchKernelGGL(sph_scan, dim3(1), dim3(kScanThreads), 0, h->stream, h->at<int>(h->L.count),
                     h->nc, h->at<int>(h->L.gstart), h->G, scratch_status);
  if (h->G > 0) {
    hipLaunchKernelGGL(sph_scatter, dim3(nb), dim3(kBlock), 0, h->stream, h->at<int>(h->L.key),
                       h->at<int>(h->L.slot), h->G, h->at<int>(h->L.gstart), h->at<int>(h->L.order));
    hipLaunchKernelGGL(sph_cell_order, dim3(nblocks(h->nc)), dim3(kBlock), 0, h->stream,
                       h->at<int>(h->L.gstart), h->nc, h->at<int>(h->L.order));
    hipLaunchKernelGGL(sph_gather, dim3(nb), dim3(kBlock), 0, h->stream, h->at<int>(h->L.order), h->G,
                       graw, (const float2*)nullptr, (const int*)nullptr, h->at<float2>(h->L.gpos),
                       (float2*)nullptr, (int*)nullptr);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemsetAsync(h->at<unsigned>(h->L.ticket), 0, 4, h->stream));
  return SPH_OK;
}

int set_rigid(sph_handle* h, const double* rigid, double tau_ctrl, long long step) {
  DevRigid r;
  memset(&r, 0, sizeof r);
  r.r[0] = rigid[0];
  r.r[1] = rigid[1];
  r.theta = rigid[2];
  r.rdot[0] = rigid[3];
  r.rdot[1] = rigid[4];
  r.thetadot = rigid[5];
  r.tau_ctrl = tau_ctrl;
  r.step = step;
  HIPCHK(hipMemcpyAsync(h->at<DevRigid>(h->L.rigid), &r, sizeof r, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return SPH_OK;
}

int set_rollout(sph_handle* h, const float* u, const double* ref, int n_ref, int stride,
                long long n_steps, float* y, float* wl, float* ul, float* wm) {
  DevRollout v;
  memset(&v, 0, sizeof v);
  v.u = u;
  v.theta_ref = ref;
  v.n_ref = n_ref;
  v.log_stride = stride;
  v.n_steps = n_steps;
  v.y_log = y;
  v.w_log = wl;
  v.u_log = ul;
  v.wm_log = wm;
  hipLaunchKernelGGL(sph_set_rollout, dim3(1), dim3(64), 0, h->stream, h->at<DevRollout>(h->L.rollout),
                     v, h->at<DevRigid>(h->L.rigid));
  HIPCHK(hipGetLastError());
  return SPH_OK;
}

int build_graph(sph_handle* h, int parity) {
  if (h->graph_ok[parity]) return SPH_OK;
  int saved = h->cur;
  h->cur = parity;
  hipGraph_t gr;
  HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  for (int s = 0; s < kChunk; ++s) enqueue_step(h, s == 0, kStep);
  enqueue_integrate(h);
  hipError_t e = hipStreamEndCapture(h->stream, &gr);
  h->cur = saved;
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&h->graph[parity], gr, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gr);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  h->graph_ok[parity] = true;
  return SPH_OK;
}

}  // namespace

extern "C" {

int sph_workspace_bytes(const sph_params* p, int32_t n_fluid, int32_t n_ghost, size_t* bytes) {
  if (!params_ok(p) || n_fluid < 0 || n_ghost < 0 || !bytes) return SPH_E_INVAL;
  Grid g;
  if (!make_grid(p, &g)) return SPH_E_INVAL;
  *bytes = make_layout(n_fluid, n_ghost, g.ncx * g.ncy).total;
  return SPH_OK;
}

int sph_init(const sph_params* p, int32_t n_fluid, const float* s0_dev, const float* w0_dev,
             int32_t n_ghost, const float* g_dev, const double* rigid0, void* ws_dev,
             size_t ws_bytes, void* stream, sph_handle** out) {
  if (!out || !params_ok(p) || n_fluid < 0 || n_ghost < 0 || !rigid0 || !ws_dev) return SPH_E_INVAL;
  if ((n_fluid > 0 && (!s0_dev || !w0_dev)) || (n_ghost > 0 && !g_dev)) return SPH_E_INVAL;
  if (reinterpret_cast<uintptr_t>(ws_dev) & 255) return SPH_E_INVAL;
  Grid g;
  if (!make_grid(p, &g)) return SPH_E_INVAL;
  Layout L = make_layout(n_fluid, n_ghost, g.ncx * g.ncy);
  if (ws_bytes < L.total) return SPH_E_CAPACITY;
  sph_handle* h = new (std::nothrow) sph_handle();
  if (!h) return SPH_E_INVAL;
  h->p = *p;
  h->N = n_fluid;
  h->G = n_ghost;
  h->grid = g;
  h->nc = g.ncx * g.ncy;
  h->k = make_consts(p);
  h->ra = RigidArgs{p->dt, p->body_mass, p->body_inertia, p->kp, p->kd, p->sine_amp, p->sine_freq,
                    p->motion, p->ctrl, p->ctrl_period, kStep};
  h->stream = reinterpret_cast<hipStream_t>(stream);
  h->ws = reinterpret_cast<char*>(ws_dev);
  h->L = L;
  h->cur = 0;
  h->graph_ok[0] = h->graph_ok[1] = false;
  int rc = SPH_OK;
  auto fail = [&](int code) {
    delete h;
    return code;
  };
  hipError_t e = hipMemsetAsync(h->ws, 0, L.total, h->stream);
  if (e != hipSuccess) return fail(hip_fail(e, "hipMemsetAsync"));
  if ((rc = set_rigid(h, rigid0, 0.0, 0)) != SPH_OK) return fail(rc);
  if (n_ghost > 0) {
    e = hipMemcpyAsync(h->at<float2>(L.graw), g_dev, (size_t)n_ghost * 8, hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) return fail(hip_fail(e, "hipMemcpyAsync"));
  }
  if ((rc = sort_ghosts(h, h->at<float2>(L.graw))) != SPH_OK) return fail(rc);
  if ((rc = sort_fluid(h, reinterpret_cast<const float2*>(s0_dev), reinterpret_cast<const float2*>(w0_dev))) != SPH_OK)
    return fail(rc);
  e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return fail(hip_fail(e, "hipStreamSynchronize"));
  unsigned st = 0;
  e = hipMemcpy(&st, h->at<unsigned>(L.status), 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail(hip_fail(e, "hipMemcpy"));
  if (st) {
    snprintf(g_err, sizeof g_err, "sph_init: initial state outside the domain box or not finite (status %u)", st);
    return fail(SPH_E_INVAL);
  }
  *out = h;
  return SPH_OK;
}

int sph_destroy(sph_handle* h) {
  if (!h) return SPH_E_INVAL;
  for (int b = 0; b < 2; ++b)
    if (h->graph_ok[b]) (void)hipGraphExecDestroy(h->graph[b]);
  delete h;
  return SPH_OK;
}

int sph_rollout(sph_handle* h, int32_t n_steps, const float* u_seq_dev, const double* theta_ref_dev,
                int32_t n_ref, int32_t log_stride, float* y_log_dev, float* wrench_log_dev,
                float* u_log_dev, float* wmean_log_dev) {
  if (!h || n_steps < 0 || log_stride < 0 || n_ref < 0) return SPH_E_INVAL;
  if (n_steps == 0) return SPH_OK;
  int rc = set_rollout(h, u_seq_dev, theta_ref_dev, n_ref, log_stride, n_steps, y_log_dev,
                       wrench_log_dev, u_log_dev, wmean_log_dev);
  if (rc) return rc;
  // graphs need a capturable stream; on the legacy default stream steps are launched directly
  int full = h->stream ? n_steps / kChunk : 0;
  int rem = n_steps - full * kChunk;
  for (int c = 0; c < full; ++c) {
    if ((rc = build_graph(h, h->cur)) != SPH_OK) return rc;
    HIPCHK(hipGraphLaunch(h->graph[h->cur], h->stream));
  }
  if (rem) {
    for (int s = 0; s < rem; ++s) enqueue_step(h, s == 0, kStep);
    enqueue_integrate(h);
    HIPCHK(hipGetLastError());
  }
  return SPH_OK;
}

int sph_time_kernels(sph_handle* h, int32_t n_steps, const float* u_seq_dev,
                     const double* theta_ref_dev, int32_t n_ref, float* avg_us) {
  if (!h || n_steps < 1 || !avg_us || n_ref < 0) return SPH_E_INVAL;
  int rc = set_rollout(h, u_seq_dev, theta_ref_dev, n_ref, 0, n_steps, nullptr, nullptr, nullptr,
                       nullptr);
  if (rc) return rc;
  hipEvent_t ev[6];
  for (int i = 0; i < 6; ++i) HIPCHK(hipEventCreate(&ev[i]));
  double sum[5] = {0, 0, 0, 0, 0};
  for (int st = 0; st < n_steps; ++st) {
    enqueue_step(h, st == 0, kStep, ev);
    HIPCHK(hipEventSynchronize(ev[5]));
    for (int k = 0; k < 5; ++k) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
      sum[k] += ms;
    }
  }
  enqueue_integrate(h);
  HIPCHK(hipStreamSynchronize(h->stream));
  for (int i = 0; i < 6; ++i) (void)hipEventDestroy(ev[i]);
  for (int k = 0; k < 5; ++k) avg_us[k] = (float)(sum[k] * 1000.0 / n_steps);
  return SPH_OK;
}

int sph_step(sph_handle* h, const float* u_dev) {
  return sph_rollout(h, 1, u_dev, nullptr, 0, 0, nullptr, nullptr, nullptr, nullptr);
}

int sph_rhs(sph_handle* h, const float* u_dev, float* rho_dev, float* p_dev, float* a_sph_dev,
            float* wdot_dev, float* wrench_dev, float* acc_dev) {
  if (!h) return SPH_E_INVAL;
  int rc = set_rollout(h, u_dev, nullptr, 0, 0, 0, nullptr, nullptr, nullptr, nullptr);
  if (rc) return rc;
  enqueue_step(h, true, kEval);
  hipLaunchKernelGGL(sph_rhs_out, dim3(nblocks(h->N)), dim3(kBlock), 0, h->stream,
                     h->at<float2>(h->L.pos[h->cur]), h->at<float2>(h->L.vel[h->cur]),
                     h->at<float2>(h->L.acc), h->at<float2>(h->L.rp), h->at<int>(h->L.id[h->cur]),
                     h->N, h->at<DevRigid>(h->L.rigid), h->k, rho_dev, p_dev,
                     reinterpret_cast<float2*>(a_sph_dev), reinterpret_cast<float2*>(wdot_dev));
  hipLaunchKernelGGL(sph_small_out, dim3(1), dim3(64), 0, h->stream, h->at<DevRigid>(h->L.rigid),
                     wrench_dev, acc_dev, (int)SPH_FRAME_BODY);
  HIPCHK(hipGetLastError());
  return SPH_OK;
}

int sph_slosh_wrench(sph_handle* h, int32_t frame, float* out_dev) {
  if (!h || !out_dev || (frame != SPH_FRAME_BODY && frame != SPH_FRAME_WORLD)) return SPH_E_INVAL;
  hipLaunchKernelGGL(sph_small_out, dim3(1), dim3(64), 0, h->stream, h->at<DevRigid>(h->L.rigid),
                     out_dev, (float*)nullptr, (int)frame);
  HIPCHK(hipGetLastError());
  return SPH_OK;
}

int sph_get_state(sph_handle* h, float* s_dev, float* w_dev, double* rigid, double* tau_ctrl,
                  int64_t* step) {
  if (!h) return SPH_E_INVAL;
  int nb = nblocks(h->N);
  if (s_dev && h->N > 0)
    hipLaunchKernelGGL(sph_unpermute, dim3(nb), dim3(kBlock), 0, h->stream, h->at<float2>(h->L.pos[h->cur]),
                       h->at<int>(h->L.id[h->cur]), h->N, reinterpret_cast<float2*>(s_dev));
  if (w_dev && h->N > 0)
    hipLaunchKernelGGL(sph_unpermute, dim3(nb), dim3(kBlock), 0, h->stream, h->at<float2>(h->L.vel[h->cur]),
                       h->at<int>(h->L.id[h->cur]), h->N, reinterpret_cast<float2*>(w_dev));
  HIPCHK(hipGetLastError());
  DevRigid r;
  HIPCHK(hipMemcpyAsync(&r, h->at<DevRigid>(h->L.rigid), sizeof r, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (rigid) {
    rigid[0] = r.r[0];
    rigid[1] = r.r[1];
    rigid[2] = r.theta;
    rigid[3] = r.rdot[0];
    rigid[4] = r.rdot[1];
    rigid[5] = r.thetadot;
  }
  if (tau_ctrl) *tau_ctrl = r.tau_ctrl;
  if (step) *step = r.step;
  return SPH_OK;
}

int sph_set_state(sph_handle* h, const float* s_dev, const float* w_dev, const double* rigid,
                  double tau_ctrl, int64_t step) {
  if (!h || !rigid || (h->N > 0 && (!s_dev || !w_dev))) return SPH_E_INVAL;
  HIPCHK(hipMemsetAsync(h->at<unsigned>(h->L.status), 0, 4, h->stream));
  int rc = set_rigid(h, rigid, tau_ctrl, step);
  if (rc) return rc;
  rc = sort_fluid(h, reinterpret_cast<const float2*>(s_dev), reinterpret_cast<const float2*>(w_dev));
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(h->stream));
  return SPH_OK;
}

int sph_status(sph_handle* h, uint32_t* flags) {
  if (!h || !flags) return SPH_E_INVAL;
  unsigned st = 0;
  HIPCHK(hipMemcpyAsync(&st, h->at<unsigned>(h->L.status), 4, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  *flags = st;
  return st ? SPH_E_STATE : SPH_OK;
}

int sph_neighbours(sph_handle* h, int32_t max_nbr, int32_t* nbr_dev, int32_t* count_dev) {
  if (!h || max_nbr < 1 || !nbr_dev || !count_dev) return SPH_E_INVAL;
  // re-sort so the cell structure matches the current positions
  int rc = set_rollout(h, nullptr, nullptr, 0, 0, 0, nullptr, nullptr, nullptr, nullptr);
  if (rc) return rc;
  enqueue_step(h, true, kEval);
  hipLaunchKernelGGL(sph_nbr_list, dim3(nblocks(h->N)), dim3(kBlock), 0, h->stream,
                     h->at<float2>(h->L.pos[h->cur]), h->at<int>(h->L.cstart[h->cur]),
                     h->at<int>(h->L.id[h->cur]), h->N, h->grid, h->k, max_nbr, nbr_dev, count_dev);
  HIPCHK(hipGetLastError());
  return SPH_OK;
}

const char* sph_strerror(int code) {
  switch (code) {
    case SPH_OK: return "ok";
    case SPH_E_INVAL: return g_err[0] ? g_err : "invalid argument";
    case SPH_E_HIP: return g_err[0] ? g_err : "HIP runtime error";
    case SPH_E_CAPACITY: return "workspace too small";
    case SPH_E_STATE: return "device status flags set (escaped / non-finite / sort)";
    default: return "unknown error";
  }
}

}  // extern "C"
