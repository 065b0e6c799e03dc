// Body-frame weakly compressible SPH step for gfx950 (MI355X), coupled to
// planar rigid-body dynamics, behind the C ABI of include/slosh.h.  One
// handle advances one tank or a batch of independent tanks of any sizes in
// the same launches.
//
// A step (the paper's state-transition algorithm, Section 3.4, followed by
// first-order symplectic Euler) is three kernels; rollouts replay them from
// captured HIP graphs:
//
//   sph_density  applies the previous step's fluid update (fictitious
//                accelerations + symplectic Euler; it needs the rigid-body
//                accelerations of that step, known only once its wrench was
//                reduced), stores the updated state, and computes the density
//                with the gamma1 ghost term (eq. density_update) and the
//                equation of state (eq. EOS, or its Tait form).  Neighbour
//                positions are updated on the fly with the same arithmetic,
//                so no separate integration pass is needed;
//   sph_force    fluid-fluid pressure (eq. momentum) and viscosity (eq.
//                viscous), ghost-to-fluid pressure and viscosity with the
//                spiky kernel (eqs. pressure_b2f, viscous_b2f); the tank's
//                reactions are reduced per workgroup;
//   sph_wrench   one workgroup per tank sums that tank's partials in a fixed
//                order and runs the zero-order-hold attitude law, the
//                rigid-body equations (eq. tankdynamics) and the logs.
//                (A separate launch, not a last-workgroup handoff: on this
//                chip a device-scope fence writes back and invalidates the
//                L2 of the issuing XCD, once per workgroup.)
//
// Both neighbour kernels work on tiles of 256/G consecutive particles of one
// tank (in cell order), G lanes per particle.  A tile is cut into row
// segments (its particles that share a grid row); for each segment the
// workgroup stages in LDS, with one coalesced pass, every fluid and ghost
// candidate of the three neighbouring rows over the segment's cell span, then
// each particle's G lanes walk its own 3x3 block from LDS and combine their
// sums with cross-lane shuffles.  A segment too large for the LDS stage
// reads its candidates from global memory instead.  G is 4, 8, 16 or 32, chosen
// by sph_autotune (8 by default).
//
// Neighbours come from a body-frame cell grid of side (S + skin)(1 + 1e-6),
// S = max(2h, h_spiky) the widest support, rebuilt every few steps (4 by
// default, sph_set_rebuild_interval) by
// a stable counting sort (sph_bin, sph_scan, sph_place) that also rewrites
// the particle state in cell order.  A particle is searched from the cell it
// was sorted into; while every particle stays within skin/2 of its position at
// the rebuild, every pair closer than S is in adjacent cells.  The density
// kernel checks that bound each step and latches SPH_ST_SORT if it fails.
// Ghost particles are fixed in the body frame: their cell list is built once.
// No floating-point atomics are used: repeated runs are bitwise identical, and
// a tank gives the same bits alone or in a batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "slosh.h"

namespace {

constexpr int kBlock = 256;       // threads per workgroup of the particle kernels
constexpr int kPlaceGroup = 8;    // lanes per cell in the placement
constexpr int kPlaceAhead = 4;    // source keys per lane loaded ahead in the placement
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 8;       // cells per thread per scan chunk
// one workgroup per tank sums its tile partials; one wave per SIMD, so that
// thread 0's FP64 tail has every register
constexpr int kWrenchThreads = 256;
constexpr int kSortEvery = 4;     // default steps between cell-list rebuilds
constexpr int kChunk = 64;        // steps per captured graph (a multiple of every rebuild interval, even)
constexpr double kSkinOverH = 1.0;  // skin = h: a particle may move h/2 between rebuilds
// Candidates staged in LDS per row segment: fluid (by tile size) and ghosts.
// A tile's segment covers its cells of one grid row and the cells around
// them in three rows: with ~15 particles per cell (cell side 3h at
// h = 1.3 dx) that is ~320 fluid candidates for 64-particle tiles (at most
// ~520 in the random tanks, 1 in 1,000 above 385) and under 300 for 32 or
// fewer; ghosts ~130 at the 99.9th percentile.  A larger segment reads its
// candidates from global memory instead.  Sized so that the 4-lane force
// kernel fits six workgroups per CU.
template <int TP>
constexpr int stage_f() { return TP >= 64 ? 416 : 384; }
constexpr int kStageG = 128;
// In-support neighbours listed per particle and pass in the force kernel's
// LDS.  With the near-list radius 1.5 times the support, a near list that
// fits (64) holds about 28 fluid neighbours inside the support at most, and
// at h_s = h a particle has a few walls inside the wall support; more take
// the per-lane path over the marked entries (or list in several passes
// without near lists).
constexpr int kListF = 48;        // fluid
constexpr int kListG = 16;        // ghost
// A variant's list capacity: at least one ballot round of its G lanes
template <int G>
constexpr int list_cap_f() { return kListF > G ? kListF : G; }
template <int G>
constexpr int list_cap_g() { return kListG > G ? kListG : G; }
// Near lists, built at the first step after each rebuild: for every particle
// the ordinals (positions in its candidate enumeration, one byte each) of
// the candidates that can come within the support before the next rebuild.
constexpr int kNearF = 64;        // capacity of a fluid near list
constexpr int kNearG = 32;        // capacity of a ghost near list
constexpr int kNearNone = 255;    // list length meaning "not listed: walk all candidates"
// Marks: for the force kernel of the same step, the density kernel records
// which listed candidates lie inside the support, one 32-bit word per lane
// of a particle's group: bit 4q + b for the lane's q-th list word, byte b
// (fluid list, bits 0-15), bit 16 + 4q + b likewise for the ghost list.
constexpr int kMarkGhostShift = 16;
constexpr int kNumVariants = 4;   // lanes per particle: 4, 8, 16, 32
constexpr int kLanes[kNumVariants] = {4, 8, 16, 32};
constexpr int kDefaultVariant = 1;

static_assert(kChunk % kSortEvery == 0 && kChunk % 2 == 0, "graph chunk");

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
  float half_skin2;         // (skin / 2)^2: allowed squared displacement between rebuilds
  float RL2;                // near-list radius^2 for fluid pairs: (2h + skin)^2, both move
  float RG2;                // near-list radius^2 for ghosts: (S + skin/2)^2, ghosts are fixed
  float cfl_w2;             // largest squared speed that keeps the step's Courant number within its limit
  int eos, tgamma;          // tgamma > 0: integer Tait exponent
  float tgamma_f;
};

struct Box {
  double lo_x, lo_y, hi_x, hi_y;
};

struct RigidArgs {
  double dt, body_mass, body_inertia, kp, kd, sine_amp, sine_freq;
  int motion, ctrl, ctrl_period, pad;
};

// Everything a kernel needs to know about one tank.
struct Tank {
  Grid g;
  Grid g2;        // cells of side 2h (no skin) for the LDS-resident rollout
  Consts k;
  Box box;
  RigidArgs ra;
  int p0, n;      // particles [p0, p0 + n) of the global arrays
  int c0, nc;     // cells [c0, c0 + nc) of the global cell arrays
  int q0, ng;     // ghosts [q0, q0 + ng)
  int pad[2];
};

struct DevRigid {
  double r[2], theta, rdot[2], thetadot;  // state at global step `step`
  double tau_ctrl;                        // torque held by the zero-order hold
  double wrench[3];                       // body-frame wrench of the last evaluation
  double acc[3];                          // r''_x, r''_y, theta'' of the last evaluation
  double th_eval, thd_eval;               // theta, thetadot used by the last evaluation
  double wsum[3];                         // running sum for the mean-wrench log
  long long step;
  long long step0;                        // global step of the current rollout's local step 0
  int wcount, pad0;
  // binary32 coefficients of the fluid update of the last evaluated step
  float c, s, abx, aby, thd, thdd, pad1[2];
};

// Rollout inputs and logs, tank-major: tank t uses u + t * n_steps * 3, ...
struct DevRollout {
  const float* u;           // [T][n_steps][3] or null
  const double* theta_ref;  // [T][n_ref] or null
  float* y_log;             // [T][n_log][6]
  float* w_log;             // [T][n_log][3]
  float* u_log;             // [T][n_log][3]
  float* wm_log;            // [T][n_log][3]
  long long n_steps;
  int n_ref, log_stride, n_log, pad;
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

// Hardware square root and reciprocal (1 ulp), for the pair terms.
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }

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

// The same shape without a branch: zero unless `in` (the support test);
// selects, so every candidate costs the same instructions.
__device__ __forceinline__ float cubic_shape_clamped(float q, bool in) {
  const float a = 2.0f - q, b = fmaxf(1.0f - q, 0.0f);
  const float w = a * a * a - 4.0f * (b * b * b);
  return in ? w : 0.0f;
}

// (dW/dr)/r of the cubic spline divided by sigma/h^2:
//   q < 1:  -12 + 9 q;   1 <= q < 2:  -3 (2 - q)^2 / q.
__device__ __forceinline__ float cubic_grad_f(float q) {
  if (q < 1.0f) return 9.0f * q - 12.0f;
  float a = 2.0f - q;
  return -3.0f * a * a * frcp(q);
}

__device__ __forceinline__ float eos_over_rho2(float rho, const Consts& k, float* P_out) {
  float P;
  if (k.eos == SPH_EOS_LINEAR || k.eos == SPH_EOS_LINEAR_CLAMPED) {
    P = k.k_lin * (rho - k.rho0);
    if (k.eos == SPH_EOS_LINEAR_CLAMPED) P = fmaxf(P, 0.0f);
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
    if (k.eos == SPH_EOS_TAIT_CLAMPED) P = fmaxf(P, 0.0f);
  }
  if (P_out) *P_out = P;
  return P / (rho * rho);
}

// Coefficients of the body-frame fluid update of the last evaluated step.
struct Frame {
  float abx, aby, thd, thdd;
};

__device__ __forceinline__ Frame load_frame(const DevRigid* __restrict__ rb) {
  return Frame{rb->abx, rb->aby, rb->thd, rb->thdd};
}

// Body-frame fluid acceleration with the fictitious terms of the rotating,
// accelerating tank frame (x = r + R(theta) s differentiated twice):
//   dw/dt = a_sph - R^T r'' - 2 thetadot J w - theta'' J s + thetadot^2 s,  J v = (-v_y, v_x).
__device__ __forceinline__ float2 body_frame_accel(float2 s, float2 w, float2 a, const Frame& f) {
  float om2 = f.thd * f.thd;
  return make_float2(a.x - f.abx + 2.0f * f.thd * w.y + f.thdd * s.y + om2 * s.x,
                     a.y - f.aby - 2.0f * f.thd * w.x - f.thdd * s.x + om2 * s.y);
}

// First-order symplectic Euler: velocity first, then position with the new velocity.
__device__ __forceinline__ void fluid_update(float2& s, float2& w, float2 a, const Frame& f, float dt) {
  float2 dw = body_frame_accel(s, w, a, f);
  w.x += dt * dw.x;
  w.y += dt * dw.y;
  s.x += dt * w.x;
  s.y += dt * w.y;
}

// DPP controls of the cross-lane moves (rows of 16 lanes).
constexpr int kDppQuadXor1 = 0xB1;       // quad_perm [1, 0, 3, 2]
constexpr int kDppQuadXor2 = 0x4E;       // quad_perm [2, 3, 0, 1]
constexpr int kDppRowMirror = 0x140;     // lane i of a row reads lane 15 - i
constexpr int kDppRowHalfMirror = 0x141; // lane i of a half-row reads lane 7 - i

template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)((unsigned long long)hi << 32 | lo));
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)((unsigned long long)hi << 32 | lo));
}

template <int G>
__device__ __forceinline__ float group_sum(float v) {
  // butterfly inside aligned groups of G lanes with DPP moves (VALU, no trip
  // through the LDS crossbar): xor 1 and xor 2 inside each quad, then the
  // mirrored half of the 8-lane half-row and of the 16-lane row; every lane
  // of the group ends with the same sum (each addition is commutative)
  v += dpp_f<kDppQuadXor1>(v);
  v += dpp_f<kDppQuadXor2>(v);
  if (G >= 8) v += dpp_f<kDppRowHalfMirror>(v);
  if (G >= 16) v += dpp_f<kDppRowMirror>(v);
  if (G >= 32) v += __shfl_xor(v, 16, 64);
  return v;
}

__device__ __forceinline__ void flag(unsigned* status, unsigned bits) {
  if (bits) atomicOr(status, bits);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// The same wavefront sum, valid in lane 0, in a fixed order with DPP moves
// inside each 16-lane row and three lane reads across the rows.  Every lane
// must be active.
__device__ __forceinline__ double wave_sum0(double v) {
  v += dpp_d<kDppQuadXor1>(v);
  v += dpp_d<kDppQuadXor2>(v);
  v += dpp_d<kDppRowHalfMirror>(v);
  v += dpp_d<kDppRowMirror>(v);
  return (v + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

// Workgroup -> tile, XCD-aware.  The dispatcher deals consecutive
// workgroups out to the 8 XCDs in turn, and each XCD has its own L2; this
// gives every XCD one contiguous run of tiles (cell-ordered particles), so
// the candidate rows that neighbouring tiles share are fetched into one L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  constexpr int kXcd = 8;
  const int x = b % kXcd, i = b / kXcd, q = n / kXcd, r = n % kXcd;
  return x * q + (x < r ? x : r) + i;
}

// --------------------------------------------------------------------------
// cell-list kernels
// --------------------------------------------------------------------------

// Adds one to count[k] for every valid lane, with one atomic per run of
// equal keys: the keys sit on lanes 0, S, 2S, ... of the wavefront and the
// valid ones form a prefix of them.
template <int S>
__device__ __forceinline__ void add_runs(int* __restrict__ count, int k, bool valid) {
  const int lane = threadIdx.x & 63;
  const int kprev = __shfl_up(k, S, 64);
  const bool head = valid && (lane < S || kprev != k);
  const unsigned long long heads = __ballot(head);
  const unsigned long long vm = __ballot(valid);
  if (head) {
    const unsigned long long after = heads & ~((2ull << lane) - 1ull);
    const int last = 63 - __clzll((long long)vm);
    const int end = after ? __ffsll((unsigned long long)after) - 1 : last + S;
    atomicAdd(&count[k], (end - lane) / S);
  }
}

// Global cell key and per-cell count (integer atomics); slot, if given,
// receives the order of arrival (used by the first, general sort only).
// owner[i] is the tank of element i.  Without slots, lanes of a wavefront
// that hold a run of equal keys (the common case: the input is in cell order
// since the last rebuild) add their run length with one atomic.
__global__ void __launch_bounds__(kBlock) sph_bin(const float2* __restrict__ pos, int n,
                                                  const int* __restrict__ owner,
                                                  const Tank* __restrict__ tanks, int* __restrict__ key,
                                                  int* __restrict__ count, int* __restrict__ slot) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < n;
  int k = -1;
  if (valid) {
    const Tank& tk = tanks[owner[i]];
    int cx, cy;
    cell_of(pos[i], tk.g, cx, cy);
    k = tk.c0 + cy * tk.g.ncx + cx;
    key[i] = k;
  }
  if (slot) {
    if (valid) slot[i] = atomicAdd(&count[k], 1);
    return;
  }
  add_runs<1>(count, k, valid);
}

// Exclusive scan of each tank's cell counts into start (global indices,
// first element of the tank at p0 / q0); clears the counts.  One workgroup
// per tank takes its cells in chunks of kScanThreads * kScanPer: a coalesced
// load into LDS, a sequential scan of kScanPer cells per thread, a
// workgroup scan of the per-thread sums (wave shuffles, wave totals in LDS),
// a coalesced write back, and a running carry between chunks.
// ghosts = 1 scans the ghost layout (base q0, count ng).
__device__ __forceinline__ int scan_slot(int i) { return i + i / kScanPer; }   // padded: no bank conflicts

constexpr int kChunkCells = kScanThreads * kScanPer;

struct ScanLds {
  int buf[kChunkCells + kScanThreads];
  int wsum[kScanThreads / 64];
};

// The counts of the chunk from `base` into registers (coalesced: v[q] is
// cell base + q * kScanThreads + thread; 0 past the tank's last cell).
__device__ __forceinline__ void scan_load(int (&v)[kScanPer], const int* __restrict__ count, const Tank& tk,
                                          int base) {
  for (int q = 0; q < kScanPer; ++q) {
    const int i = q * kScanThreads + threadIdx.x;
    v[q] = base + i < tk.nc ? count[tk.c0 + base + i] : 0;
  }
}

// One chunk of kChunkCells cells from `base`, its counts v loaded by
// scan_load: exclusive scan of the counts plus `carry` written to start
// (offset by base0), counts cleared; returns the chunk's total.  The counts
// into LDS, a sequential scan of kScanPer cells per thread, a workgroup scan
// of the per-thread sums (wave shuffles, wave totals in LDS), a coalesced
// write back.
__device__ int scan_chunk(ScanLds& S, const int (&v)[kScanPer], int* __restrict__ count, const Tank& tk,
                          int base, int carry, int base0, int* __restrict__ start) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  for (int q = 0; q < kScanPer; ++q) S.buf[scan_slot(q * kScanThreads + t)] = v[q];
  __syncthreads();
  int sum = 0;
  for (int q = 0; q < kScanPer; ++q) {
    const int k = scan_slot(t * kScanPer + q);
    const int v = S.buf[k];
    S.buf[k] = sum;
    sum += v;
  }
  int x = sum;   // inclusive scan of the per-thread sums
  for (int off = 1; off < 64; off <<= 1) {
    int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) S.wsum[wave] = x;
  __syncthreads();
  if (wave == 0) {
    int w = lane < kScanThreads / 64 ? S.wsum[lane] : 0;
    for (int off = 1; off < kScanThreads / 64; off <<= 1) {
      int y = __shfl_up(w, off, 64);
      if (lane >= off) w += y;
    }
    if (lane < kScanThreads / 64) S.wsum[lane] = w;
  }
  __syncthreads();
  const int excl = carry + (wave > 0 ? S.wsum[wave - 1] : 0) + x - sum;
  for (int q = 0; q < kScanPer; ++q) S.buf[scan_slot(t * kScanPer + q)] += excl;
  const int total = S.wsum[kScanThreads / 64 - 1];
  __syncthreads();
  for (int q = 0; q < kScanPer; ++q) {
    const int i = q * kScanThreads + t;
    if (base + i < tk.nc) {
      start[tk.c0 + base + i] = base0 + S.buf[scan_slot(i)];
      count[tk.c0 + base + i] = 0;
    }
  }
  __syncthreads();
  return total;
}

__global__ void __launch_bounds__(kScanThreads) sph_scan(int* __restrict__ count,
                                                         const Tank* __restrict__ tanks, int n_tanks,
                                                         int ghosts, int* __restrict__ start,
                                                         unsigned* __restrict__ status) {
  __shared__ ScanLds S;
  const Tank& tk = tanks[blockIdx.x];
  const int base0 = ghosts ? tk.q0 : tk.p0, expect = ghosts ? tk.ng : tk.n;
  int carry = 0;
  int v[kScanPer], nx[kScanPer] = {};
  scan_load(v, count, tk, 0);
  for (int base = 0; base < tk.nc; base += kChunkCells) {
    // the next chunk's counts are in flight while this chunk is scanned
    if (base + kChunkCells < tk.nc) scan_load(nx, count, tk, base + kChunkCells);
    carry += scan_chunk(S, v, count, tk, base, carry, base0, start);
    for (int q = 0; q < kScanPer; ++q) v[q] = nx[q];
  }
  if (threadIdx.x == 0) {
    // the entry past a tank's last cell is the next tank's first; the last
    // tank writes the final one
    if ((int)blockIdx.x == n_tanks - 1) start[tk.c0 + tk.nc] = base0 + carry;
    if (carry != expect && status) atomicOr(status, SPH_ST_SORT);
  }
}

// The same scan for one tank with many cells, in three launches instead of
// one workgroup walking every chunk: per-chunk totals, an exclusive scan of
// the totals (part[n_parts] = the grand total), then every chunk's scan
// from its offset.  The starts are identical to sph_scan's.
__global__ void __launch_bounds__(kScanThreads) sph_scan_sums(const int* __restrict__ count,
                                                              const Tank* __restrict__ tanks,
                                                              int* __restrict__ part) {
  __shared__ int wsum[kScanThreads / 64];
  const Tank& tk = tanks[0];
  const int base = blockIdx.x * kChunkCells;
  int v = 0;
  for (int q = 0; q < kScanPer; ++q) {
    const int i = base + q * kScanThreads + threadIdx.x;
    if (i < tk.nc) v += count[tk.c0 + i];
  }
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int tsum = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) tsum += wsum[w];
    part[blockIdx.x] = tsum;
  }
}

__global__ void __launch_bounds__(kScanThreads) sph_scan_tops(int* __restrict__ part, int n_parts) {
  __shared__ int wsum[kScanThreads / 64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  int carry = 0;
  for (int b0 = 0; b0 < n_parts; b0 += kScanThreads) {
    const int i = b0 + t;
    const int v = i < n_parts ? part[i] : 0;
    int x = v;
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    if (wave == 0) {
      int w = lane < kScanThreads / 64 ? wsum[lane] : 0;
      for (int off = 1; off < kScanThreads / 64; off <<= 1) {
        const int y = __shfl_up(w, off, 64);
        if (lane >= off) w += y;
      }
      if (lane < kScanThreads / 64) wsum[lane] = w;
    }
    __syncthreads();
    const int ex = carry + (wave > 0 ? wsum[wave - 1] : 0) + x - v;
    const int tot = wsum[kScanThreads / 64 - 1];
    __syncthreads();
    if (i < n_parts) part[i] = ex;
    carry += tot;
  }
  if (t == 0) part[n_parts] = carry;
}

__global__ void __launch_bounds__(kScanThreads) sph_scan_chunks(int* __restrict__ count,
                                                                const Tank* __restrict__ tanks, int ghosts,
                                                                const int* __restrict__ part, int n_parts,
                                                                int* __restrict__ start,
                                                                unsigned* __restrict__ status) {
  __shared__ ScanLds S;
  const Tank& tk = tanks[0];
  const int base0 = ghosts ? tk.q0 : tk.p0, expect = ghosts ? tk.ng : tk.n;
  int v[kScanPer];
  scan_load(v, count, tk, blockIdx.x * kChunkCells);
  scan_chunk(S, v, count, tk, blockIdx.x * kChunkCells, part[blockIdx.x], base0, start);
  if (threadIdx.x == 0 && (int)blockIdx.x == n_parts - 1) {
    const int total = part[n_parts];
    start[tk.c0 + tk.nc] = base0 + total;
    if (total != expect && status) atomicOr(status, SPH_ST_SORT);
  }
}

// Stable placement after a rebuild: a group of kPlaceGroup lanes per
// destination cell c walks the 3x3 block of source cells in ascending key
// (= ascending source position) and compacts the particles whose new key is
// c with a ballot, so their order is preserved.  Also records each particle's
// position at the rebuild.
// The candidate ranges of a particle in cell (cx, cy): for the rows cy-1,
// cy, cy+1, the fluid index range [lo, hi) and the ghost range covering
// cells cx-1 .. cx+1 (empty for rows outside the grid), packed as three int4:
// {f_lo0, f_hi0, f_lo1, f_hi1}, {f_lo2, f_hi2, g_lo0, g_hi0}, {g_lo1, g_hi1, g_lo2, g_hi2}.
__device__ __forceinline__ void cell_ranges(const Tank& tk, int cx, int cy, const int* __restrict__ start,
                                            const int* __restrict__ gstart, int v[12]) {
  const int ncx = tk.g.ncx;
  const int xa = cx > 0 ? cx - 1 : 0;
  const int xb = cx < ncx - 1 ? cx + 1 : ncx - 1;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int yy = cy - 1 + r;
    const bool in = yy >= 0 && yy < tk.g.ncy;
    const int c = tk.c0 + (in ? yy : 0) * ncx;
    v[2 * r] = in ? start[c + xa] : 0;
    v[2 * r + 1] = in ? start[c + xb + 1] : 0;
    v[6 + 2 * r] = in ? gstart[c + xa] : 0;
    v[6 + 2 * r + 1] = in ? gstart[c + xb + 1] : 0;
  }
}

__device__ __forceinline__ void store_ranges(int4* __restrict__ rng, int d, const int v[12]) {
  rng[3 * d] = make_int4(v[0], v[1], v[2], v[3]);
  rng[3 * d + 1] = make_int4(v[4], v[5], v[6], v[7]);
  rng[3 * d + 2] = make_int4(v[8], v[9], v[10], v[11]);
}

__global__ void __launch_bounds__(kBlock) sph_place(const int* __restrict__ key,
                                                    const int* __restrict__ cell_owner,
                                                    const Tank* __restrict__ tanks, int n_cells,
                                                    const int* __restrict__ start_old,
                                                    const int* __restrict__ start_new,
                                                    const int* __restrict__ gstart,
                                                    int4* __restrict__ rng, int* __restrict__ pkey,
                                                    const float2* __restrict__ pos_in,
                                                    const float2* __restrict__ vel_in,
                                                    const float2* __restrict__ acc_in,
                                                    const int* __restrict__ id_in,
                                                    float2* __restrict__ pos_out,
                                                    float2* __restrict__ vel_out,
                                                    float2* __restrict__ acc_out,
                                                    int* __restrict__ id_out,
                                                    float2* __restrict__ pos_sort,
                                                    unsigned* __restrict__ status) {
  constexpr int G = kPlaceGroup, A = kPlaceAhead;
  const int t = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int c = t / G, l = t % G;
  if (c >= n_cells) return;
  int dst = start_new[c];
  const int end = start_new[c + 1];
  if (dst == end) return;   // no particle has key c (most cells of the gas region)
  const Tank& tk = tanks[cell_owner[c]];
  const int ncx = tk.g.ncx, ncy = tk.g.ncy;
  const int shift = (threadIdx.x & 63) & ~(G - 1);   // first lane of this group in the wave
  const int lc = c - tk.c0;
  const int cy = lc / ncx, cx = lc - cy * ncx;
  const int xa = cx > 0 ? cx - 1 : 0;
  const int xb = cx < ncx - 1 ? cx + 1 : ncx - 1;
  int rv[12];
  cell_ranges(tk, cx, cy, start_new, gstart, rv);
  // the source rows' bounds, then the first A keys per lane of all three
  // rows at once (one memory round trip for the common case of rows of at
  // most A * G particles); longer rows load the rest as they go.  The
  // visiting order, and so the placement, is that of the rows in turn.
  int r0[3], r1[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int yy = cy - 1 + r;
    const bool in = yy >= 0 && yy < ncy;
    r0[r] = in ? start_old[tk.c0 + yy * ncx + xa] : 0;
    r1[r] = in ? start_old[tk.c0 + yy * ncx + xb + 1] : 0;
  }
  int kk[3][A];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int u = 0; u < A; ++u) {
      const int i = r0[r] + u * G + l;
      kk[r][u] = i < r1[r] ? key[i] : -1;
    }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int i1 = r1[r];
    for (int b = r0[r]; b < i1; b += A * G) {
      if (b != r0[r])
#pragma unroll
        for (int u = 0; u < A; ++u) {
          const int i = b + u * G + l;
          kk[r][u] = i < i1 ? key[i] : -1;
        }
      // destinations of the batch first, then its loads, then its stores
      int dd[A];
#pragma unroll
      for (int u = 0; u < A; ++u) {
        const bool match = kk[r][u] == c;   // c >= 0: lanes past the row never match
        const unsigned long long m = __ballot(match);
        const unsigned gm = (unsigned)(m >> shift) & ((1u << G) - 1u);
        const int d = dst + __popc(gm & ((1u << l) - 1u));
        dd[u] = match && d < end ? d : -1;
        dst += __popc(gm);
      }
      float2 sp[A], sv[A], sa[A];
      int sid[A];
#pragma unroll
      for (int u = 0; u < A; ++u)
        if (dd[u] >= 0) {
          const int i = b + u * G + l;
          sp[u] = pos_in[i];
          sv[u] = vel_in[i];
          sa[u] = acc_in[i];
          sid[u] = id_in[i];
        }
#pragma unroll
      for (int u = 0; u < A; ++u)
        if (dd[u] >= 0) {
          const int d = dd[u];
          pos_out[d] = sp[u];
          vel_out[d] = sv[u];
          acc_out[d] = sa[u];
          id_out[d] = sid[u];
          pos_sort[d] = sp[u];
          pkey[d] = c;
          store_ranges(rng, d, rv);
        }
    }
  }
  if (l == 0 && dst != end) atomicOr(status, SPH_ST_SORT);
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
                           const float2* __restrict__ vel_in, float2* __restrict__ pos_out,
                           float2* __restrict__ vel_out, int* __restrict__ id_out,
                           float2* __restrict__ pos_sort) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int i = order[p];
  float2 s = pos_in[i];
  pos_out[p] = s;
  if (vel_in) vel_out[p] = vel_in[i];
  if (id_out) id_out[p] = i;
  if (pos_sort) pos_sort[p] = s;
}

// Cell key and candidate ranges of every particle after the general sort.
__global__ void sph_ranges(const float2* __restrict__ pos_sort, int n, const int* __restrict__ owner,
                           const Tank* __restrict__ tanks, const int* __restrict__ start,
                           const int* __restrict__ gstart, int4* __restrict__ rng, int* __restrict__ pkey) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const Tank& tk = tanks[owner[p]];
  int cx, cy;
  cell_of(pos_sort[p], tk.g, cx, cy);
  int v[12];
  cell_ranges(tk, cx, cy, start, gstart, v);
  pkey[p] = tk.c0 + cy * tk.g.ncx + cx;
  store_ranges(rng, p, v);
}

// Marks escaped or non-finite particles of a state handed in by the caller.
__global__ void sph_check(const float2* __restrict__ pos, const float2* __restrict__ vel, int n,
                          const int* __restrict__ owner, const Tank* __restrict__ tanks,
                          unsigned* __restrict__ status) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Box& box = tanks[owner[i]].box;
  float2 s = pos[i], w = vel[i];
  unsigned bad = 0;
  if (!isfinite(s.x) || !isfinite(s.y) || !isfinite(w.x) || !isfinite(w.y)) bad |= SPH_ST_NONFINITE;
  else if (!((double)s.x >= box.lo_x && (double)s.x < box.hi_x && (double)s.y >= box.lo_y &&
             (double)s.y < box.hi_y))
    bad |= SPH_ST_ESCAPED;
  flag(status, bad);
}

// --------------------------------------------------------------------------
// tiles and row segments
// --------------------------------------------------------------------------

// A tile is (tank, first particle, count); tiles never cross a tank.
struct TileRef {
  int tank, p0, np, pad;
};

// Per-tile data in LDS: each particle's grid row and its candidate ranges.
template <int TP>
struct TileLds {
  int cy[TP];
  int rng[TP][12];
  int near[TP];   // fluid near-list length | ghost near-list length << 8
};

// One row segment of a tile: slots [first, last] share grid row cy[first];
// their candidates (rows cy-1 .. cy+1) are staged contiguously row after row:
// fluid index j of row r sits at LDS index off[r] + j - lo[r].  The cells of
// a segment are non-decreasing along the row, so its staged span of row r is
// [lo of its first particle, hi of its last].
// The candidates staged for one pass over a tile: the row ranges of one
// row segment, or of two consecutive ones back to back when both fit in the
// stage (a tile whose particles span two grid rows then takes one staging
// round trip and one compute pass instead of two).  Slots first .. split-1
// use ranges 0-2, slots split .. last ranges 3-5; unused ranges start at nf.
struct Seg {
  int lo[6], off[6], glo[6], goff[6];
  int nf, ng, first, last, split;
};

// The row segment that starts at tile slot `first`: the run of slots from
// `first` in the same grid row, found with one ballot of wavefront 0 (a tile
// holds at most 64 slots), and its candidate ranges.  Called by the threads
// of wavefront 0; thread 0 writes sg.
// Last slot of the run of slots from `first` in first's grid row, found with
// one ballot (a tile holds at most 64 slots).  All lanes of wavefront 0.
template <int TP>
__device__ __forceinline__ int seg_run_end(const TileLds<TP>& tl, int first) {
  static_assert(TP <= 64, "one wavefront covers the tile");
  const int lane = threadIdx.x;
  const int row = tl.cy[first];
  const unsigned long long same = __ballot(lane < TP && tl.cy[lane] == row);
  // slots first, first + 1, ... while the row stays the same (bit 0 of
  // `from` is slot first itself)
  const unsigned long long from = same >> first;
  const int len = ~from == 0ull ? 64 - first : __builtin_ctzll(~from);
  return first + len - 1;
}

// The stage that starts at tile slot `first`: its row segment, and the next
// one if `merge` and both fit in stage_f fluid / stage_g ghost slots.  Called
// by the threads of wavefront 0; thread 0 writes sg.
template <int TP>
__device__ void make_segment(Seg& sg, const TileLds<TP>& tl, int first, bool merge = false, int stage_f = 0,
                             int stage_g = 0) {
  const int last = seg_run_end<TP>(tl, first);
  const bool more = merge && last + 1 < TP && tl.cy[last + 1] >= 0;   // the same on every lane
  const int last2 = more ? seg_run_end<TP>(tl, last + 1) : last;
  if (threadIdx.x != 0) return;
  int nf = 0, ng = 0;
  auto ranges = [&](int a, int b, int r0) {   // slots a .. b of one row into ranges r0 .. r0 + 2
    for (int r = 0; r < 3; ++r) {
      sg.off[r0 + r] = nf;
      sg.goff[r0 + r] = ng;
      sg.lo[r0 + r] = tl.rng[a][2 * r];
      sg.glo[r0 + r] = tl.rng[a][6 + 2 * r];
      nf += tl.rng[b][2 * r + 1] - sg.lo[r0 + r];
      ng += tl.rng[b][6 + 2 * r + 1] - sg.glo[r0 + r];
    }
  };
  ranges(first, last, 0);
  const int nf1 = nf, ng1 = ng;
  int end = last;
  if (more) {
    ranges(last + 1, last2, 3);
    if (nf <= stage_f && ng <= stage_g) end = last2;
  }
  if (end == last) {
    nf = nf1;
    ng = ng1;
    for (int r = 3; r < 6; ++r) {
      sg.off[r] = nf;
      sg.goff[r] = ng;
      sg.lo[r] = sg.glo[r] = 0;
    }
  }
  sg.nf = nf;
  sg.ng = ng;
  sg.first = first;
  sg.last = end;
  sg.split = last + 1;
}

// Global index of staged element e (row ranges stored back to back).
__device__ __forceinline__ int seg_src(const int* lo, const int* off, int e) {
  if (e < off[1]) return lo[0] + e - off[0];
  if (e < off[2]) return lo[1] + e - off[1];
  return lo[2] + e - off[2];
}

// The same over the six ranges of a stage (empty and unused ranges are
// skipped: a later range that starts at the same offset takes precedence).
__device__ __forceinline__ int seg_src6(const int* lo, const int* off, int e) {
  int r = 0;
#pragma unroll
  for (int q = 1; q < 6; ++q) r += e >= off[q] ? 1 : 0;
  return lo[r] + e - off[r];
}

// The tile a workgroup works on.  A single-tank handle (single_n = its
// particle count, else -1) has tiles of TP consecutive particles from 0, so
// the record is computed instead of loaded: one dependent round trip less.
template <int TP>
__device__ __forceinline__ TileRef tile_ref(const TileRef* __restrict__ tiles, int tile, int single_n) {
  if (single_n >= 0) {
    const int p0 = tile * TP, left = single_n - p0;
    return TileRef{0, p0, left < TP ? left : TP, 0};
  }
  return tiles[tile];
}

// Rows and candidate ranges of the tile's particles into LDS; -1 marks slots
// past the end.
template <int TP>
__device__ __forceinline__ void tile_load(int p0, int np, const Tank& tk, const int* __restrict__ pkey,
                                          const int4* __restrict__ rng, TileLds<TP>& tl,
                                          const int* __restrict__ near_n = nullptr) {
  const int t = threadIdx.x;
  if (t < TP) {
    if (t < np) {
      tl.near[t] = near_n ? near_n[p0 + t] : (kNearNone | kNearNone << 8);
      tl.cy[t] = (pkey[p0 + t] - tk.c0) / tk.g.ncx;
      const int4 a = rng[3 * (p0 + t)], b = rng[3 * (p0 + t) + 1], c = rng[3 * (p0 + t) + 2];
      int* v = tl.rng[t];
      v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
      v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
      v[8] = c.x; v[9] = c.y; v[10] = c.z; v[11] = c.w;
    } else {
      tl.cy[t] = -1;
    }
  }
}

// Visits the candidates of tile slot `pl` for lane l of its group (ghosts if
// `ghost`): f(j, e) with global index j and LDS index e (valid when staged).
template <int G, int TP, class F>
__device__ __forceinline__ void visit(const TileLds<TP>& tl, int pl, bool ghost, const int* lo,
                                      const int* off, int l, F&& f) {
  const int* v = tl.rng[pl] + (ghost ? 6 : 0);
  for (int r = 0; r < 3; ++r) {
    const int a = v[2 * r], b = v[2 * r + 1];
    const int shift = off[r] - lo[r];
    for (int j = a + l; j < b; j += G) f(j, j + shift);
  }
}


// Orders LDS accesses of one wavefront (a compiler fence; no hardware barrier).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lanes of a G-lane group: the mask of the group's bits in a wavefront ballot.
template <int G>
__device__ __forceinline__ unsigned group_bits() {
  return G == 32 ? 0xffffffffu : ((1u << G) - 1u);
}

// Candidate ordinal (position in the enumeration row 0, row 1, row 2 of a
// tile slot's candidate ranges) -> LDS index of the staged candidate.
struct OrdMap {
  int n0, n01, e0, d1, d2;   // d1 = e1 - e0, d2 = e2 - e1: offsets added past each row boundary
  __device__ __forceinline__ int operator()(int c) const {
    return c + e0 + (d1 & -(int)(c >= n0)) + (d2 & -(int)(c >= n01));
  }
};

template <int TP>
__device__ __forceinline__ OrdMap ord_map(const TileLds<TP>& tl, int pl, bool ghost, const int* lo, const int* off,
                                          int* total) {
  const int* v = tl.rng[pl] + (ghost ? 6 : 0);
  OrdMap m;
  m.n0 = v[1] - v[0];
  m.n01 = m.n0 + v[3] - v[2];
  *total = m.n01 + v[5] - v[4];
  const int e0 = v[0] + off[0] - lo[0];
  const int e1 = v[2] + off[1] - lo[1] - m.n0;
  const int e2 = v[4] + off[2] - lo[2] - m.n01;
  m.e0 = e0;
  m.d1 = e1 - e0;
  m.d2 = e2 - e1;
  return m;
}

// One listing pass over the staged candidates of a tile slot, in ordinal
// order from c on: the G lanes of the particle test G candidates at a time
// and append the LDS indices of those that pass `keep` to `lst` (ballot
// compaction, order kept).  Stops before the list could overflow; returns
// its length and advances c (both the same on the G lanes).
template <int G, int CAP, class F>
__device__ __forceinline__ int list_pass(const OrdMap& m, int total, int l, int& c, unsigned short* lst, F&& keep) {
  static_assert(CAP >= G, "a pass must hold one ballot round, or it never advances");
  constexpr int cap = CAP;
  const int base = (int)(threadIdx.x & 63) - l;
  const unsigned below = (1u << l) - 1u;
  int cnt = 0;
  while (c < total && cnt <= cap - G) {
    const int cc = c + l;
    int e = 0;
    bool in = false;
    if (cc < total) {
      e = m(cc);
      in = keep(e);
    }
    const unsigned msk = (unsigned)(__ballot(in) >> base) & group_bits<G>();
    if (in) lst[cnt + __popc(msk & below)] = (unsigned short)e;
    cnt += __popc(msk);
    c += G;
  }
  return cnt;
}

// Near-list build: the ordinals of the candidates that pass `keep`, in
// order, as bytes into lst (capacity cap).  Returns the number that passed,
// which may exceed cap (the list is then not used).  total <= 255.  Walks
// the three rows one after the other, where a candidate's LDS index is its
// ordinal plus the row's offset (no per-candidate row search).
template <int G, class F>
__device__ __forceinline__ int near_build(const OrdMap& m, int total, int l, unsigned char* lst, int cap,
                                          F&& keep) {
  const int base = (int)(threadIdx.x & 63) - l;
  const unsigned below = (1u << l) - 1u;
  int cnt = 0;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int c0 = r == 0 ? 0 : (r == 1 ? m.n0 : m.n01);
    const int c1 = r == 0 ? m.n0 : (r == 1 ? m.n01 : total);
    const int sh = m.e0 + (r >= 1 ? m.d1 : 0) + (r >= 2 ? m.d2 : 0);
    for (int c = c0; c < c1; c += G) {
      const int cc = c + l;
      const bool in = cc < c1 && keep(cc + sh);
      const unsigned msk = (unsigned)(__ballot(in) >> base) & group_bits<G>();
      if (in) {
        const int at = cnt + __popc(msk & below);
        if (at < cap) lst[at] = (unsigned char)cc;
      }
      cnt += __popc(msk);
    }
  }
  return cnt;
}

// A near list is CAP one-byte ordinals in CAP/4 words; lane l of a
// particle's group takes words l, l + G, l + 2G, ... (at most kMaxW <= 4).
// The words do not depend on the list length, so they are fetched at the
// start of a kernel, in the same round trip as the tile's other loads, and
// consumed by rotation (an indexed array would be placed in scratch memory).
template <int G, int CAP>
struct NearWords {
  static constexpr int kWords = CAP / 4;
  static constexpr int kMaxW = (kWords + G - 1) / G;
  static_assert(kMaxW <= 4, "more than four near-list words per lane");
  unsigned w0 = 0u, w1 = 0u, w2 = 0u, w3 = 0u;
  __device__ __forceinline__ void load(const unsigned* __restrict__ row, int l) {
    if (l < kWords) w0 = row[l];
    if (kMaxW > 1 && l + G < kWords) w1 = row[l + G];
    if (kMaxW > 2 && l + 2 * G < kWords) w2 = row[l + 2 * G];
    if (kMaxW > 3 && l + 3 * G < kWords) w3 = row[l + 3 * G];
  }
  __device__ __forceinline__ unsigned pop() {
    const unsigned w = w0;
    w0 = w1;
    w1 = w2;
    w2 = w3;
    return w;
  }
  __device__ __forceinline__ unsigned word(int q) const { return q == 0 ? w0 : q == 1 ? w1 : q == 2 ? w2 : w3; }
};

// For every entry of lane l's share of a near list of n entries (lane l
// holds words l, l + G, ...; the words are consumed): calls f(e) with the
// LDS index of the staged candidate, which returns whether the candidate
// lies inside the support, and returns the lane's marks (bit 4q + b for
// entry 4(l + qG) + b).
template <int G, int CAP, class F>
__device__ __forceinline__ unsigned near_visit_marks(NearWords<G, CAP>& nw, int n, int l, const OrdMap& m, F&& f) {
  unsigned marks = 0u;
#pragma unroll
  for (int q = 0; q < NearWords<G, CAP>::kMaxW; ++q) {
    unsigned word = nw.pop();
    const int i0 = 4 * (l + q * G);
    if (i0 < n)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if (i0 + b < n && f(m((int)(word & 255u)))) marks |= 1u << (4 * q + b);
        word >>= 8;
      }
  }
  return marks;
}

// The same over a list of n ordinals held in LDS (the list the density
// kernel just built), in the lanes' word order of NearWords.
template <int G, int CAP, class F>
__device__ __forceinline__ unsigned lds_list_marks(const unsigned char* lst, int n, int l, const OrdMap& m, F&& f) {
  unsigned marks = 0u;
#pragma unroll
  for (int q = 0; q < NearWords<G, CAP>::kMaxW; ++q) {
    const int i0 = 4 * (l + q * G);
    if (i0 < n)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (i0 + b < n && f(m((int)lst[i0 + b]))) marks |= 1u << (4 * q + b);
  }
  return marks;
}

// Lists, from a near list and the marks the density kernel wrote for it at
// the same positions, the ordinals of the candidates inside the support:
// lane l writes its own marked entries, in bit order, from the sum of the
// counts of the group's lanes before it on (an exclusive scan over the G
// lanes); the group's total is the caller's.  No candidate is loaded or
// tested, and the words are not consumed.
template <int G, int CAP>
__device__ __forceinline__ void near_list_marked(const NearWords<G, CAP>& nw, unsigned marks, int l,
                                                 unsigned short* lst) {
  const int n = __popc(marks);
  int incl = n;
#pragma unroll
  for (int off = 1; off < G; off <<= 1) {
    const int y = __shfl_up(incl, off, G);
    if (l >= off) incl += y;
  }
  unsigned short* dst = lst + (incl - n);
  while (marks) {
    const int b = __builtin_ctz(marks);
    marks &= marks - 1u;
    *dst++ = (unsigned short)((nw.word(b >> 2) >> (8 * (b & 3))) & 255u);
  }
}

// Calls f(e) for each entry of lane l's share of a near list whose mark bit
// is set (bit 4q + b for entry 4(l + qG) + b), in bit order, with no list in
// LDS: the path of a particle with more candidates inside the support than
// its LDS list holds (the words must not have been consumed).
template <int G, int CAP, class F>
__device__ __forceinline__ void marked_visit(const NearWords<G, CAP>& nw, unsigned m, const OrdMap& map, F&& f) {
  while (m) {
    const int b = __builtin_ctz(m);
    m &= m - 1u;
    const unsigned w = nw.word(b >> 2);
    f(map((int)((w >> (8 * (b & 3))) & 255u)));
  }
}

// --------------------------------------------------------------------------
// particle sums
// --------------------------------------------------------------------------

// Fluid update of the previous step (if `integrate`), then
// rho_i = m sigma (sum_f shape + gamma1 sum_g shape), P and P/rho^2.
// Build (the first step after a rebuild): every candidate is walked, and
// each particle's near lists are written: the fluid candidates within RL of
// it and the ghosts within RG, at the positions of the rebuild (pos_sort).
// While every particle stays within skin/2 of those positions, every pair
// closer than the support is listed.  Otherwise a listed particle walks only
// its near lists.
// Eight waves per SIMD asked of the register allocator: the 4-lane variant
// then fits in 64 VGPRs without spilling (72 otherwise, seven waves).
template <int G, bool Build>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8))) sph_density(const float2* __restrict__ pos_in,
                                                      const float2* __restrict__ vel_in,
                                                      const float2* __restrict__ acc_in, int integrate,
                                                      const float2* __restrict__ pos_sort,
                                                      const int* __restrict__ pkey,
                                                      const int4* __restrict__ rng,
                                                      const float2* __restrict__ gpos,
                                                      const TileRef* __restrict__ tiles, int single_n,
                                                      const Tank* __restrict__ tanks,
                                                      const DevRigid* __restrict__ rigid,
                                                      float2* __restrict__ pos_out,
                                                      float2* __restrict__ vel_out,
                                                      float2* __restrict__ rp,
                                                      unsigned* __restrict__ status,
                                                      int* __restrict__ near_n,
                                                      unsigned* __restrict__ near_f,
                                                      unsigned* __restrict__ near_g,
                                                      unsigned* __restrict__ marks_out) {
  constexpr int TP = kBlock / G;
  constexpr int kStageF = stage_f<TP>();
  __shared__ float2 f_pos[kStageF];
  __shared__ float2 f_raw[Build ? kStageF : 1];
  __shared__ float2 g_pos[kStageG];
  __shared__ unsigned nb_f[Build ? TP : 1][kNearF / 4], nb_g[Build ? TP : 1][kNearG / 4];
  __shared__ TileLds<TP> tl;
  __shared__ Seg sg;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const TileRef tr = tile_ref<TP>(tiles, tile, single_n);
  const Tank& tk = tanks[tr.tank];
  const Consts& k = tk.k;
  const int pl = threadIdx.x / G, l = threadIdx.x % G;
  const int p = tr.p0 + pl;
  const bool mine = pl < tr.np;
  const Frame fr = load_frame(&rigid[tr.tank]);
  const float dt = k.dt;
  tile_load<TP>(tr.p0, tr.np, tk, pkey, rng, tl, Build ? nullptr : near_n);
  float2 s = make_float2(0.f, 0.f), w = make_float2(0.f, 0.f), s_raw = s;
  NearWords<G, kNearF> nwf;
  NearWords<G, kNearG> nwg;
  if (!Build && mine && near_n) {
    nwf.load(near_f + (size_t)p * (kNearF / 4), l);
    nwg.load(near_g + (size_t)p * (kNearG / 4), l);
  }
  if (mine) {
    s = pos_in[p];
    if (Build) s_raw = pos_sort[p];   // near lists use the positions of the rebuild
    w = vel_in[p];
    if (integrate) fluid_update(s, w, acc_in[p], fr, dt);
  }
  __syncthreads();
  float sf = 0.0f, sgs = 0.0f;
  const float inv_h = k.inv_h, R2 = k.R2, Rs2 = k.Rs2;
  unsigned marks = 0u;
  int nf_out = kNearNone, ng_out = kNearNone;
  int first = 0;
  while (first < TP && tl.cy[first] >= 0) {
    if (threadIdx.x < 64) make_segment<TP>(sg, tl, first, true, kStageF, kStageG);
    __syncthreads();
    const bool fst = sg.nf <= kStageF, gst = sg.ng <= kStageG;
    if (fst)
      for (int e = threadIdx.x; e < sg.nf; e += kBlock) {
        const int j = seg_src6(sg.lo, sg.off, e);
        float2 sj = pos_in[j];
        if (Build) f_raw[e] = pos_sort[j];
        if (integrate) {
          float2 wj = vel_in[j];
          fluid_update(sj, wj, acc_in[j], fr, dt);
        }
        f_pos[e] = sj;
      }
    if (gst)
      for (int e = threadIdx.x; e < sg.ng; e += kBlock) g_pos[e] = gpos[seg_src6(sg.glo, sg.goff, e)];
    __syncthreads();
    if (mine && pl >= sg.first && pl <= sg.last) {
      // this particle's segment's ranges in the stage
      const int sh = pl < sg.split ? 0 : 3;
      const int *lo = sg.lo + sh, *off = sg.off + sh, *glo = sg.glo + sh, *goff = sg.goff + sh;
      // its own updated position as staged (row 1 holds its own cell), so
      // that it is bit for bit the value its neighbours see: the marks of
      // the support test must equal the force kernel's test
      if (fst) s = f_pos[off[1] + p - lo[1]];
      auto fluid = [&](float2 sj) {
        const float d2 = dist2(s.x - sj.x, s.y - sj.y);
        sf += cubic_shape_clamped(fsqrt(d2) * inv_h, d2 < R2);
        return d2 < R2 && d2 > 0.0f;
      };
      int total;
      const OrdMap fm = ord_map<TP>(tl, pl, false, lo, off, &total);
      const int nlf = tl.near[pl] & 255;
      bool walked = false;
      if (Build && fst && total <= 255) {
        // list first, then the density over the list just written
        unsigned char* lb = reinterpret_cast<unsigned char*>(nb_f[pl]);
        const int cnt = near_build<G>(fm, total, l, lb, kNearF, [&](int e) {
          const float2 r = f_raw[e];
          return dist2(s_raw.x - r.x, s_raw.y - r.y) < k.RL2;
        });
        nf_out = cnt <= kNearF ? cnt : kNearNone;
        if (cnt <= kNearF) {
          wave_sync();
          marks = lds_list_marks<G, kNearF>(lb, cnt, l, fm, [&](int e) { return fluid(f_pos[e]); });
          walked = true;
        }
      } else if (!Build && fst && nlf <= kNearF) {
        marks = near_visit_marks<G, kNearF>(nwf, nlf, l, fm, [&](int e) { return fluid(f_pos[e]); });
        walked = true;
      }
      if (!walked) {
        if (fst) {
          visit<G, TP>(tl, pl, false, lo, off, l, [&](int, int e) { fluid(f_pos[e]); });
        } else {
          visit<G, TP>(tl, pl, false, lo, off, l, [&](int j, int) {
            float2 sj = pos_in[j];
            if (integrate) {
              float2 wj = vel_in[j];
              fluid_update(sj, wj, acc_in[j], fr, dt);
            }
            fluid(sj);
          });
        }
      }
      auto ghost = [&](float2 gj) {
        const float d2 = dist2(s.x - gj.x, s.y - gj.y);
        sgs += cubic_shape_clamped(fsqrt(d2) * inv_h, d2 < R2);
        return d2 < Rs2 && d2 > 0.0f;   // inside the spiky support of the wall terms
      };
      int gtotal;
      const OrdMap gm = ord_map<TP>(tl, pl, true, glo, goff, &gtotal);
      const int nlg = (tl.near[pl] >> 8) & 255;
      bool gwalked = false;
      if (Build && gst && gtotal <= 255) {
        unsigned char* lb = reinterpret_cast<unsigned char*>(nb_g[pl]);
        const int cnt = near_build<G>(gm, gtotal, l, lb, kNearG, [&](int e) {
          const float2 r = g_pos[e];
          return dist2(s_raw.x - r.x, s_raw.y - r.y) < k.RG2;
        });
        ng_out = cnt <= kNearG ? cnt : kNearNone;
        if (cnt <= kNearG) {
          wave_sync();
          marks |= lds_list_marks<G, kNearG>(lb, cnt, l, gm, [&](int e) { return ghost(g_pos[e]); })
                   << kMarkGhostShift;
          gwalked = true;
        }
      } else if (!Build && gst && nlg <= kNearG) {
        marks |= near_visit_marks<G, kNearG>(nwg, nlg, l, gm, [&](int e) { return ghost(g_pos[e]); })
                 << kMarkGhostShift;
        gwalked = true;
      }
      if (!gwalked) {
        if (gst)
          visit<G, TP>(tl, pl, true, glo, goff, l, [&](int, int e) { ghost(g_pos[e]); });
        else
          visit<G, TP>(tl, pl, true, glo, goff, l, [&](int j, int) { ghost(gpos[j]); });
      }
    }
    const int next = sg.last + 1;
    __syncthreads();
    first = next;
  }
  sf = group_sum<G>(sf);
  sgs = group_sum<G>(sgs);
  if (Build && mine) {
    // near lists out, as whole words (the group's lanes wrote the bytes)
    wave_sync();
    const int nwf = nf_out == kNearNone ? 0 : (nf_out + 3) / 4;
    const int nwg = ng_out == kNearNone ? 0 : (ng_out + 3) / 4;
    for (int q = l; q < nwf; q += G) near_f[(size_t)p * (kNearF / 4) + q] = nb_f[pl][q];
    for (int q = l; q < nwg; q += G) near_g[(size_t)p * (kNearG / 4) + q] = nb_g[pl][q];
    if (l == 0) near_n[p] = nf_out | ng_out << 8;
  }
  if (marks_out && mine) marks_out[(size_t)p * G + l] = marks;
  if (!mine || l != 0) return;
  const float2 s0 = pos_sort[p];
  float rho = k.mass * k.wc * (sf + k.gamma1 * sgs);
  float pr = eos_over_rho2(rho, k, nullptr);
  rp[p] = make_float2(rho, pr);
  pos_out[p] = s;
  vel_out[p] = w;
  unsigned bad = 0;
  if (!isfinite(s.x) || !isfinite(s.y) || !isfinite(w.x) || !isfinite(w.y)) {
    bad |= SPH_ST_NONFINITE;
  } else {
    const Box& box = tk.box;
    if (!((double)s.x >= box.lo_x && (double)s.x < box.hi_x && (double)s.y >= box.lo_y &&
          (double)s.y < box.hi_y))
      bad |= SPH_ST_ESCAPED;
    if (dist2(s.x - s0.x, s.y - s0.y) > k.half_skin2) bad |= SPH_ST_SORT;
    if (dist2(w.x, w.y) > k.cfl_w2) bad |= SPH_ST_CFL;
  }
  flag(status, bad);
}

// Inputs of a tank's rigid-body step that live in memory other than the
// wrench: the applied force/torque of the step and, at a controller sample,
// the attitude reference.  Separate so that they can be fetched early.
struct RigidIn {
  double u[3], ref;
  long long n, loc;
};

__device__ RigidIn rigid_inputs(const DevRigid* rb, const DevRollout* ro, int tank, int mode,
                                const RigidArgs& ra) {
  RigidIn in;
  in.n = rb->step;
  in.loc = in.n - rb->step0;
  in.u[0] = in.u[1] = in.u[2] = 0.0;
  in.ref = 0.0;
  if (mode == kStep && ro->u && in.loc >= 0 && in.loc < ro->n_steps) {
    const float* ut = ro->u + ((size_t)tank * ro->n_steps + in.loc) * 3;
    in.u[0] = ut[0];
    in.u[1] = ut[1];
    in.u[2] = ut[2];
  } else if (mode == kEval && ro->u) {
    const float* ut = ro->u + (size_t)tank * 3;
    in.u[0] = ut[0];
    in.u[1] = ut[1];
    in.u[2] = ut[2];
  }
  if (mode == kStep && ra.ctrl == SPH_CTRL_PD_ZOH && ra.ctrl_period > 0 && in.n % ra.ctrl_period == 0 &&
      ro->theta_ref && ro->n_ref > 0) {
    const long long kk = in.n / ra.ctrl_period;
    in.ref = ro->theta_ref[(size_t)tank * ro->n_ref + (kk < ro->n_ref ? kk : ro->n_ref - 1)];
  }
  return in;
}

// Rigid-body part of a step, run by one thread after the tank's wrench is
// reduced: zero-order-hold attitude law, eq. tankdynamics, logs, symplectic
// Euler.
__device__ void rigid_step(DevRigid* rb, const DevRollout* ro, int tank, const double F[3], int mode,
                           const RigidArgs& ra, const RigidIn& in) {
  const long long n = in.n;
  const long long loc = in.loc;
  const double* u = in.u;
  if (mode == kStep && ra.ctrl == SPH_CTRL_PD_ZOH && ra.ctrl_period > 0 && n % ra.ctrl_period == 0)
    rb->tau_ctrl = ra.kp * (in.ref - rb->theta) - ra.kd * rb->thetadot;
  double th, thd, acc[3];
  if (ra.motion == SPH_MOTION_SINE) {
    double w = 2.0 * M_PI * ra.sine_freq, t = (double)n * ra.dt;
    th = ra.sine_amp * sin(w * t);
    thd = ra.sine_amp * w * cos(w * t);
    acc[0] = acc[1] = 0.0;
    acc[2] = -ra.sine_amp * w * w * sin(w * t);
  } else {
    th = rb->theta;
    thd = rb->thetadot;
  }
  double s, c;
  sincos(th, &s, &c);
  if (ra.motion != SPH_MOTION_SINE) {
    acc[0] = (c * F[0] - s * F[1] + u[0]) / ra.body_mass;
    acc[1] = (s * F[0] + c * F[1] + u[1]) / ra.body_mass;
    acc[2] = (F[2] + u[2] + rb->tau_ctrl) / ra.body_inertia;
  }
  for (int d = 0; d < 3; ++d) {
    rb->wrench[d] = F[d];
    rb->acc[d] = acc[d];
  }
  rb->th_eval = th;
  rb->thd_eval = thd;
  rb->c = (float)c;
  rb->s = (float)s;
  rb->abx = (float)(c * acc[0] + s * acc[1]);    // R^T r''
  rb->aby = (float)(-s * acc[0] + c * acc[1]);
  rb->thd = (float)thd;
  rb->thdd = (float)acc[2];
  if (mode != kStep) return;

  if (ro->log_stride > 0 && loc >= 0 && loc < ro->n_steps) {
    const long long kk = loc / ro->log_stride;
    const size_t row = (size_t)tank * ro->n_log + kk;
    if (loc % ro->log_stride == 0) {
      if (ro->y_log) {
        float* y = ro->y_log + 6 * row;
        y[0] = (float)rb->r[0];
        y[1] = (float)rb->r[1];
        y[2] = (float)rb->theta;
        y[3] = (float)rb->rdot[0];
        y[4] = (float)rb->rdot[1];
        y[5] = (float)rb->thetadot;
      }
      if (ro->w_log)
        for (int d = 0; d < 3; ++d) ro->w_log[3 * row + d] = (float)F[d];
      if (ro->u_log) {
        ro->u_log[3 * row] = (float)u[0];
        ro->u_log[3 * row + 1] = (float)u[1];
        ro->u_log[3 * row + 2] = (float)(u[2] + rb->tau_ctrl);
      }
    }
    for (int d = 0; d < 3; ++d) rb->wsum[d] += F[d];
    rb->wcount += 1;
    if (loc % ro->log_stride == ro->log_stride - 1 || loc == ro->n_steps - 1) {
      if (ro->wm_log)
        for (int d = 0; d < 3; ++d) ro->wm_log[3 * row + d] = (float)(rb->wsum[d] / rb->wcount);
      rb->wsum[0] = rb->wsum[1] = rb->wsum[2] = 0.0;
      rb->wcount = 0;
    }
  }
  if (ra.motion == SPH_MOTION_SINE) {
    double w = 2.0 * M_PI * ra.sine_freq, t = (double)(n + 1) * ra.dt;
    rb->theta = ra.sine_amp * sin(w * t);
    rb->thetadot = ra.sine_amp * w * cos(w * t);
    rb->r[0] = rb->r[1] = rb->rdot[0] = rb->rdot[1] = 0.0;
  } else {
    rb->rdot[0] += ra.dt * acc[0];
    rb->rdot[1] += ra.dt * acc[1];
    rb->thetadot += ra.dt * acc[2];
    rb->r[0] += ra.dt * rb->rdot[0];
    rb->r[1] += ra.dt * rb->rdot[1];
    rb->theta += ra.dt * rb->thetadot;
  }
  rb->step = n + 1;
}

// Forces and the slosh wrench.  a_i = m sum_j [-(P_i/rho_i^2 + P_j/rho_j^2)
//   + 2 alpha h (w_ij . s_ij) / ((rho_i + rho_j)(r^2 + eps h^2))] grad_i W_ij
//   + sum_g m [-2 P_i/rho_i^2 + (2 beta / (2 rho_i)) min(w_i . s_ig, 0)/(r^2 + eps h^2)] grad_i W_s3
// The tank receives -m * (wall term) per pair, with torque arm g.
// Occupancy: the 4-lane variant's 23 KB of LDS (stages and the in-support
// lists, sized for the neighbour counts of h = 1.3 dx with room to spare)
// and 79 VGPRs give six workgroups per CU; a register budget of seven waves
// spills and was slower.
template <int G, bool Bin>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) sph_force(const float2* __restrict__ pos,
                                                    const float2* __restrict__ vel,
                                                    const float2* __restrict__ rp,
                                                    const int* __restrict__ pkey,
                                                    const int4* __restrict__ rng,
                                                    const float2* __restrict__ gpos,
                                                    const TileRef* __restrict__ tiles, int single_n,
                                                    const Tank* __restrict__ tanks,
                                                    float2* __restrict__ acc,
                                                    double* __restrict__ partials,
                                                    int* __restrict__ key, int* __restrict__ count,
                                                    const int* __restrict__ near_n,
                                                    const unsigned* __restrict__ near_f,
                                                    const unsigned* __restrict__ near_g,
                                                    const unsigned* __restrict__ marks_in) {
  constexpr int TP = kBlock / G;
  constexpr int kStageF = stage_f<TP>();
  __shared__ float2 f_pos[kStageF], f_vel[kStageF], f_rp[kStageF];
  __shared__ float2 g_pos[kStageG];
  constexpr int kLF = list_cap_f<G>(), kLG = list_cap_g<G>();
  __shared__ unsigned short f_list[TP][kLF], g_list[TP][kLG];
  __shared__ TileLds<TP> tl;
  __shared__ Seg sg;
  __shared__ double red[3][kBlock / 64];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const TileRef tr = tile_ref<TP>(tiles, tile, single_n);
  const Tank& tk = tanks[tr.tank];
  const Consts& k = tk.k;
  const int pl = threadIdx.x / G, l = threadIdx.x % G;
  const int p = tr.p0 + pl;
  const bool mine = pl < tr.np;
  tile_load<TP>(tr.p0, tr.np, tk, pkey, rng, tl, near_n);
  float2 s = make_float2(0.f, 0.f), w = make_float2(0.f, 0.f), me = make_float2(1.f, 0.f);
  NearWords<G, kNearF> nwf;
  NearWords<G, kNearG> nwg;
  unsigned marks = 0u;
  if (mine) {
    if (near_n) {
      nwf.load(near_f + (size_t)p * (kNearF / 4), l);
      nwg.load(near_g + (size_t)p * (kNearG / 4), l);
      marks = marks_in[(size_t)p * G + l];
    }
    s = pos[p];
    w = vel[p];
    me = rp[p];
  }
  const float rho_i = me.x, Pi = me.y;
  const float visc_g = k.beta2 / (2.0f * rho_i);   // wall viscosity with rho_g = rho_i
  __syncthreads();
  float axf = 0.0f, ayf = 0.0f, axg = 0.0f, ayg = 0.0f;
  float fx = 0.0f, fy = 0.0f, tq = 0.0f;
  int first = 0;
  while (first < TP && tl.cy[first] >= 0) {
    if (threadIdx.x < 64) make_segment<TP>(sg, tl, first, true, kStageF, kStageG);
    __syncthreads();
    const bool fst = sg.nf <= kStageF, gst = sg.ng <= kStageG;
    if (fst)
      for (int e = threadIdx.x; e < sg.nf; e += kBlock) {
        const int j = seg_src6(sg.lo, sg.off, e);
        f_pos[e] = pos[j];
        f_vel[e] = vel[j];
        f_rp[e] = rp[j];
      }
    if (gst)
      for (int e = threadIdx.x; e < sg.ng; e += kBlock) g_pos[e] = gpos[seg_src6(sg.glo, sg.goff, e)];
    __syncthreads();
    if (mine && pl >= sg.first && pl <= sg.last) {
      // this particle's segment's ranges in the stage
      const int sh = pl < sg.split ? 0 : 3;
      const int *lo = sg.lo + sh, *off = sg.off + sh, *glo = sg.glo + sh, *goff = sg.goff + sh;
      // pair terms of a neighbour inside the support (0 < r < 2h)
      auto fluid = [&](float2 sj, float2 wj, float2 o) {
        float dx = s.x - sj.x, dy = s.y - sj.y;
        float d2 = dist2(dx, dy);
        float q = fsqrt(d2) * k.inv_h;
        float gW = k.dwc * cubic_grad_f(q);
        float vr = (w.x - wj.x) * dx + (w.y - wj.y) * dy;
        float coef = (-(Pi + o.y) + k.a2h * vr * frcp((rho_i + o.x) * (d2 + k.eps_h2))) * gW;
        axf += coef * dx;
        ayf += coef * dy;
      };
      auto fluid_test = [&](float2 sj, float2 wj, float2 o) {
        float d2 = dist2(s.x - sj.x, s.y - sj.y);
        if (d2 < k.R2 && d2 > 0.0f) fluid(sj, wj, o);
      };
      if (fst) {
        // list the neighbours inside the support, then all G lanes work on the list
        unsigned short* lst = f_list[pl];
        int total;
        const OrdMap fm = ord_map<TP>(tl, pl, false, lo, off, &total);
        auto inside = [&](int e) {
          const float2 sj = f_pos[e];
          const float d2 = dist2(s.x - sj.x, s.y - sj.y);
          return d2 < k.R2 && d2 > 0.0f;
        };
        auto pairs = [&](int cnt) {
          wave_sync();
          for (int q = l; q < cnt; q += G) {
            const int e = lst[q];
            fluid(f_pos[e], f_vel[e], f_rp[e]);
          }
          wave_sync();
        };
        const int nlf = tl.near[pl] & 255;
        if (nlf <= kNearF) {
          // the density kernel marked the listed candidates inside the support
          const unsigned mf = marks & ((1u << kMarkGhostShift) - 1u);
          const int nin = (int)group_sum<G>((float)__popc(mf));   // the same on the G lanes
          if (nin <= kLF) {
            near_list_marked<G, kNearF>(nwf, mf, l, lst);
            wave_sync();
            for (int q = l; q < nin; q += G) {
              const int e = fm(lst[q]);
              fluid(f_pos[e], f_vel[e], f_rp[e]);
            }
            wave_sync();
          } else {
            marked_visit<G, kNearF>(nwf, mf, fm, [&](int e) { fluid(f_pos[e], f_vel[e], f_rp[e]); });
          }
        } else {
          int c = 0;
          while (c < total) pairs(list_pass<G, kLF>(fm, total, l, c, lst, inside));
        }
      } else {
        visit<G, TP>(tl, pl, false, lo, off, l, [&](int j, int) { fluid_test(pos[j], vel[j], rp[j]); });
      }
      // wall terms of a ghost inside the spiky support (0 < r < h_s)
      auto ghost = [&](float2 gj) {
        float dx = s.x - gj.x, dy = s.y - gj.y;
        float d2 = dist2(dx, dy);
        float r = fsqrt(d2);
        float tt = k.hs - r;
        float gW = k.dws * tt * tt * frcp(r);
        float vr = w.x * dx + w.y * dy;
        float coef = k.mass * (-2.0f * Pi + visc_g * fminf(vr, 0.0f) * frcp(d2 + k.eps_h2)) * gW;
        float ax = coef * dx, ay = coef * dy;   // wall force on the fluid / m
        axg += ax;
        ayg += ay;
        float Fx = k.mass * ax, Fy = k.mass * ay;
        fx -= Fx;
        fy -= Fy;
        tq -= gj.x * Fy - gj.y * Fx;
      };
      if (gst) {
        unsigned short* lst = g_list[pl];
        int total;
        const OrdMap gm = ord_map<TP>(tl, pl, true, glo, goff, &total);
        auto inside = [&](int e) {
          const float2 gj = g_pos[e];
          const float d2 = dist2(s.x - gj.x, s.y - gj.y);
          return d2 < k.Rs2 && d2 > 0.0f;
        };
        auto walls = [&](int cnt) {
          wave_sync();
          for (int q = l; q < cnt; q += G) ghost(g_pos[lst[q]]);
          wave_sync();
        };
        const int nlg = (tl.near[pl] >> 8) & 255;
        if (nlg <= kNearG) {
          const unsigned mg = marks >> kMarkGhostShift;
          const int nin = (int)group_sum<G>((float)__popc(mg));   // the same on the G lanes
          if (nin <= kLG) {
            near_list_marked<G, kNearG>(nwg, mg, l, lst);
            wave_sync();
            for (int q = l; q < nin; q += G) ghost(g_pos[gm(lst[q])]);
            wave_sync();
          } else {
            marked_visit<G, kNearG>(nwg, mg, gm, [&](int e) { ghost(g_pos[e]); });
          }
        } else {
          int c = 0;
          while (c < total) walls(list_pass<G, kLG>(gm, total, l, c, lst, inside));
        }
      } else {
        visit<G, TP>(tl, pl, true, glo, goff, l, [&](int j, int) {
          const float2 gj = gpos[j];
          const float d2 = dist2(s.x - gj.x, s.y - gj.y);
          if (d2 < k.Rs2 && d2 > 0.0f) ghost(gj);
        });
      }
    }
    const int next = sg.last + 1;
    __syncthreads();
    first = next;
  }
  axf = group_sum<G>(axf);
  ayf = group_sum<G>(ayf);
  axg = group_sum<G>(axg);
  ayg = group_sum<G>(ayg);
  if (mine && l == 0) acc[p] = make_float2(k.mass * axf + axg, k.mass * ayf + ayg);
  if (Bin) {
    // the binning pass of the rebuild that follows this step, on the
    // positions this step ends with
    int kc = -1;
    if (mine && l == 0) {
      int cx, cy;
      cell_of(s, tk.g, cx, cy);
      kc = tk.c0 + cy * tk.g.ncx + cx;
      key[p] = kc;
    }
    add_runs<G>(count, kc, mine && l == 0);
  }

  // workgroup reduction of the wrench, in double, fixed order; a wave
  // without any wall term (all its sums +0) contributes +0 without the sum
  double v[3] = {(double)fx, (double)fy, (double)tq};
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const bool walls = __ballot(fx != 0.0f || fy != 0.0f || tq != 0.0f) != 0ull;
  for (int d = 0; d < 3; ++d) {
    double t = walls ? wave_sum0(v[d]) : 0.0;
    if (lane == 0) red[d][wv] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int d = 0; d < 3; ++d) {
      double t = 0.0;
      for (int q = 0; q < kBlock / 64; ++q) t += red[d][q];
      partials[3 * tile + d] = t;
    }
  }
}

// One workgroup per tank: the tank's tile partials summed in a fixed order,
// then the rigid-body part of the step.
__global__ void __launch_bounds__(kWrenchThreads) sph_wrench(const double* __restrict__ partials,
                                                     const int* __restrict__ tank_tile0, int single_nt,
                                                     const Tank* __restrict__ tanks, DevRigid* rigid,
                                                     const DevRollout* __restrict__ ro, int mode) {
  __shared__ double red[3][kWrenchThreads / 64];
  const int tank = blockIdx.x;
  // thread 0's copies of the rigid state, parameters and rollout, loaded
  // while the partials are summed (reads of them after the barrier would
  // each wait a memory round trip)
  DevRigid rb;
  RigidArgs ra;
  DevRollout rl;
  RigidIn in;
  if (threadIdx.x == 0) {
    rb = rigid[tank];
    ra = tanks[tank].ra;
    rl = *ro;
    in = rigid_inputs(&rb, &rl, tank, mode, ra);
  }
  // a single tank's tiles are 0 .. single_nt - 1 (no table load)
  const int t0 = single_nt >= 0 ? 0 : tank_tile0[tank];
  const int nt = single_nt >= 0 ? single_nt : tank_tile0[tank + 1] - t0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double acc3[3] = {0.0, 0.0, 0.0};
#pragma unroll 4
  for (int b = threadIdx.x; b < nt; b += kWrenchThreads)
    for (int d = 0; d < 3; ++d) acc3[d] += partials[3 * (t0 + b) + d];
  for (int d = 0; d < 3; ++d) {
    double t = wave_sum0(acc3[d]);
    if (lane == 0) red[d][wv] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double F[3];
    for (int d = 0; d < 3; ++d) {
      double t = 0.0;
      for (int q = 0; q < kWrenchThreads / 64; ++q) t += red[d][q];
      F[d] = t;
    }
    rigid_step(&rb, &rl, tank, F, mode, ra, in);
    rigid[tank] = rb;
  }
}

// Final fluid update at the end of a rollout (the update sph_density defers).
__global__ void __launch_bounds__(kBlock) sph_integrate(float2* __restrict__ pos, float2* __restrict__ vel,
                                                        const float2* __restrict__ acc, int n,
                                                        const int* __restrict__ owner,
                                                        const Tank* __restrict__ tanks,
                                                        const DevRigid* __restrict__ rigid,
                                                        unsigned* __restrict__ status) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int t = owner[i];
  const Consts& k = tanks[t].k;
  float2 s = pos[i], w = vel[i];
  fluid_update(s, w, acc[i], load_frame(&rigid[t]), k.dt);
  pos[i] = s;
  vel[i] = w;
  if (!isfinite(s.x) || !isfinite(s.y) || !isfinite(w.x) || !isfinite(w.y))
    flag(status, SPH_ST_NONFINITE);
  else if (dist2(w.x, w.y) > k.cfl_w2)
    flag(status, SPH_ST_CFL);
}

// Outputs of sph_rhs in caller order.
__global__ void sph_rhs_out(const float2* __restrict__ pos, const float2* __restrict__ vel,
                            const float2* __restrict__ acc, const float2* __restrict__ rp,
                            const int* __restrict__ id, int n, const int* __restrict__ owner,
                            const Tank* __restrict__ tanks, const DevRigid* __restrict__ rigid,
                            float* rho_o, float* p_o, float2* a_o, float2* wd_o) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const int t = owner[q];
  int i = id[q];
  float rho = rp[q].x;
  float P;
  eos_over_rho2(rho, tanks[t].k, &P);
  if (rho_o) rho_o[i] = rho;
  if (p_o) p_o[i] = P;
  float2 a = acc[q], s = pos[q], w = vel[q];
  if (a_o) a_o[i] = a;
  if (wd_o) wd_o[i] = body_frame_accel(s, w, a, load_frame(&rigid[t]));
}

__global__ void sph_small_out(const DevRigid* __restrict__ rigid, int n_tanks, float* wrench, float* acc3,
                              int frame) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tanks) return;
  const DevRigid* rb = &rigid[t];
  double F0 = rb->wrench[0], F1 = rb->wrench[1];
  if (frame == SPH_FRAME_WORLD) {
    double c = cos(rb->th_eval), s = sin(rb->th_eval);
    double a = c * F0 - s * F1, b = s * F0 + c * F1;
    F0 = a;
    F1 = b;
  }
  if (wrench) {
    wrench[3 * t] = (float)F0;
    wrench[3 * t + 1] = (float)F1;
    wrench[3 * t + 2] = (float)rb->wrench[2];
  }
  if (acc3)
    for (int d = 0; d < 3; ++d) acc3[3 * t + d] = (float)rb->acc[d];
}

__global__ void sph_unpermute(const float2* __restrict__ src, const int* __restrict__ id, int n,
                              float2* __restrict__ dst) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  dst[id[q]] = src[q];
}

__global__ void sph_set_rollout(DevRollout* ro, DevRollout v, DevRigid* rigid, int n_tanks) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) *ro = v;
  if (t < n_tanks) rigid[t].step0 = rigid[t].step;
}

// Test hook: neighbour ids (caller order) of every particle, ascending, found
// by the same tile / row-segment / LDS-staged traversal the particle sums use.
template <int G>
__global__ void __launch_bounds__(kBlock) sph_nbr_list(const float2* __restrict__ pos,
                                                       const int* __restrict__ pkey,
                                                       const int4* __restrict__ rng,
                                                       const int* __restrict__ id,
                                                       const TileRef* __restrict__ tiles, int single_n,
                                                       const Tank* __restrict__ tanks, int max_nbr,
                                                       int* __restrict__ nbr, int* __restrict__ cnt) {
  constexpr int TP = kBlock / G;
  constexpr int kStageF = stage_f<TP>();
  __shared__ float2 f_pos[kStageF];
  __shared__ int f_id[kStageF];
  __shared__ TileLds<TP> tl;
  __shared__ Seg sg;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const TileRef tr = tile_ref<TP>(tiles, tile, single_n);
  const Tank& tk = tanks[tr.tank];
  const int pl = threadIdx.x / G, l = threadIdx.x % G;
  const int p = tr.p0 + pl;
  tile_load<TP>(tr.p0, tr.np, tk, pkey, rng, tl);
  __syncthreads();
  int first = 0;
  while (first < TP && tl.cy[first] >= 0) {
    if (threadIdx.x < 64) make_segment<TP>(sg, tl, first);
    __syncthreads();
    const bool fst = sg.nf <= kStageF;
    if (fst)
      for (int e = threadIdx.x; e < sg.nf; e += kBlock) {
        const int j = seg_src(sg.lo, sg.off, e);
        f_pos[e] = pos[j];
        f_id[e] = j;
      }
    __syncthreads();
    // one lane per particle collects, so that the count is exact
    if (pl < tr.np && l == 0 && pl >= sg.first && pl <= sg.last) {
      const float2 s = pos[p];
      const int i = id[p];
      int* row_out = nbr + (size_t)i * max_nbr;
      int c = 0;
      auto take = [&](int j, float2 sj) {
        if (j == p) return;
        if (dist2(s.x - sj.x, s.y - sj.y) < tk.k.R2) {
          if (c < max_nbr) row_out[c] = id[j];
          ++c;
        }
      };
      if (fst)
        visit<1, TP>(tl, pl, false, sg.lo, sg.off, 0, [&](int, int e) { take(f_id[e], f_pos[e]); });
      else
        visit<1, TP>(tl, pl, false, sg.lo, sg.off, 0, [&](int j, int) { take(j, pos[j]); });
      cnt[i] = c;
      const int m = c < max_nbr ? c : max_nbr;
      for (int a2 = 1; a2 < m; ++a2) {
        int v = row_out[a2], b2 = a2 - 1;
        while (b2 >= 0 && row_out[b2] > v) {
          row_out[b2 + 1] = row_out[b2];
          --b2;
        }
        row_out[b2 + 1] = v;
      }
    }
    const int next = sg.last + 1;
    __syncthreads();
    first = next;
  }
}

// --------------------------------------------------------------------------
// LDS-resident rollout for small tanks.  One workgroup per tank keeps the
// fluid state, the ghosts, the cell structure (cells of side 2h) and the
// rigid state in LDS and runs many steps per launch: a step is a few
// workgroup barriers instead of three launches with their global-memory
// round trips.  The particles are kept sorted by cell (a stable counting
// sort after every step, ties in the order of the previous step), so the
// candidates of a cell row are one contiguous run of LDS and the summation
// order, and the result, do not depend on timing.  The arithmetic of every
// term is the multi-kernel path's (density and EOS, pair and wall terms,
// wrench, rigid step, symplectic update); the wrench is summed per thread in
// double, then over the waves in a fixed order.
// --------------------------------------------------------------------------

constexpr int kResThreads = 1024;
constexpr int kResMaxF = 2048;     // fluid particles per tank
constexpr int kResMaxG = 1024;     // ghosts per tank
constexpr int kResMaxC = 2048;     // cells of side 2h per tank
constexpr int kResPer = kResMaxF / kResThreads;
constexpr int kResChunk = 4096;    // steps per launch

struct ResLds {
  float2 s[2][kResMaxF], w[2][kResMaxF];   // cell-sorted state; [par] is current
  float2 rp[kResMaxF];                     // rho, P / rho^2 of each sorted slot
  float2 g[kResMaxG];                      // ghosts in cell order
  unsigned short id[2][kResMaxF];          // slot in the handle's arrays
  unsigned short ckey[kResMaxF];           // cell of each sorted slot
  unsigned short key[kResMaxF];            // cell of each slot before sorting
  unsigned short tmp[kResMaxF];            // a cell's members in arrival order
  int start[kResMaxC + 1];
  int cnt[kResMaxC];
  int gstart[kResMaxC + 1];
  double red[3][kResThreads / 64];
  int wsum[kResThreads / 64];
  DevRigid rb;
  DevRollout ro;
  float frame[4];
  unsigned bad;
};

// Exclusive workgroup scan: thread t holds v; returns its exclusive prefix
// and the total.  Ends with a barrier after the totals are read.
__device__ int res_scan(int v, ResLds& L, int* total) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  int x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) L.wsum[wv] = x;
  __syncthreads();
  if (wv == 0) {
    int w = lane < kResThreads / 64 ? L.wsum[lane] : 0;
    for (int off = 1; off < kResThreads / 64; off <<= 1) {
      const int y = __shfl_up(w, off, 64);
      if (lane >= off) w += y;
    }
    if (lane < kResThreads / 64) L.wsum[lane] = w;
  }
  __syncthreads();
  const int ex = (wv > 0 ? L.wsum[wv - 1] : 0) + x - v;
  *total = L.wsum[kResThreads / 64 - 1];
  __syncthreads();
  return ex;
}

// Cell starts from the counts in cnt (thread t owns cells 2t, 2t + 1);
// leaves cnt zero.
__device__ void res_starts(ResLds& L, int nc) {
  const int t = threadIdx.x, c0 = 2 * t, c1 = 2 * t + 1;
  const int v0 = c0 < nc ? L.cnt[c0] : 0, v1 = c1 < nc ? L.cnt[c1] : 0;
  int total;
  const int ex = res_scan(v0 + v1, L, &total);
  if (c0 < nc) {
    L.start[c0] = ex;
    L.cnt[c0] = 0;
  }
  if (c1 < nc) {
    L.start[c1] = ex + v0;
    L.cnt[c1] = 0;
  }
  if (t == 0) L.start[nc] = total;
  __syncthreads();
}

// Position of slot i among its cell's members (ascending slot), after every
// member has been appended to tmp.
__device__ __forceinline__ int res_rank(const ResLds& L, int i, int c) {
  const int a = L.start[c], b = L.start[c + 1];
  int rank = 0;
  for (int q = a; q < b; ++q) rank += L.tmp[q] < i ? 1 : 0;
  return a + rank;
}

// Stable counting sort of the fluid from buffer par into buffer 1 - par by
// key (counts already in cnt); also writes ckey and the cell starts.
__device__ void res_sort(ResLds& L, int n, int nc, int par) {
  res_starts(L, nc);
  for (int i = threadIdx.x; i < n; i += kResThreads) {
    const int c = L.key[i];
    L.tmp[L.start[c] + atomicAdd(&L.cnt[c], 1)] = (unsigned short)i;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += kResThreads) {
    const int c = L.key[i];
    const int d = res_rank(L, i, c);
    L.s[1 - par][d] = L.s[par][i];
    L.w[1 - par][d] = L.w[par][i];
    L.id[1 - par][d] = L.id[par][i];
    L.ckey[d] = (unsigned short)c;
  }
  for (int c = threadIdx.x; c < nc; c += kResThreads) L.cnt[c] = 0;
  __syncthreads();
}

__device__ __forceinline__ int res_key(float2 p, const Grid& g) {
  int cx, cy;
  cell_of(p, g, cx, cy);
  return cy * g.ncx + cx;
}

// The rigid-body part, kept out of line: thread 0 runs it once per step and
// its FP64 code would otherwise take registers from the particle loops.
__device__ __noinline__ void res_rigid_step(DevRigid* rb, const DevRollout* ro, int tank, double F0, double F1,
                                            double F2, RigidArgs ra, RigidIn in) {
  const double F[3] = {F0, F1, F2};
  rigid_step(rb, ro, tank, F, kStep, ra, in);
}

__global__ void __launch_bounds__(kResThreads) sph_resident(float2* __restrict__ pos, float2* __restrict__ vel,
                                                            const float2* __restrict__ gpos,
                                                            const Tank* __restrict__ tanks, DevRigid* rigid,
                                                            const DevRollout* __restrict__ rollout, int n_steps,
                                                            unsigned* __restrict__ status) {
  __shared__ ResLds L;
  const int tank = blockIdx.x, t = threadIdx.x;
  const Tank& tk = tanks[tank];
  const Consts k = tk.k;
  const Grid g2 = tk.g2;
  const RigidArgs ra = tk.ra;
  const int n = tk.n, ng = tk.ng, nc = g2.ncx * g2.ncy;
  if (t == 0) {
    L.rb = rigid[tank];
    L.ro = *rollout;
    L.bad = 0u;
  }
  for (int c = t; c < nc; c += kResThreads) L.cnt[c] = 0;
  __syncthreads();
  // ghosts, once: counting sort into L.g (staged in s[1])
  for (int i = t; i < ng; i += kResThreads) {
    const float2 p = gpos[tk.q0 + i];
    L.s[1][i] = p;
    const int c = res_key(p, g2);
    L.key[i] = (unsigned short)c;
    atomicAdd(&L.cnt[c], 1);
  }
  __syncthreads();
  res_starts(L, nc);
  for (int i = t; i < ng; i += kResThreads) {
    const int c = L.key[i];
    L.tmp[L.start[c] + atomicAdd(&L.cnt[c], 1)] = (unsigned short)i;
  }
  __syncthreads();
  for (int i = t; i < ng; i += kResThreads) L.g[res_rank(L, i, L.key[i])] = L.s[1][i];
  for (int c = t; c <= nc; c += kResThreads) L.gstart[c] = L.start[c];
  for (int c = t; c < nc; c += kResThreads) L.cnt[c] = 0;
  __syncthreads();
  // fluid, sorted into buffer 1
  for (int i = t; i < n; i += kResThreads) {
    const float2 p = pos[tk.p0 + i];
    L.s[0][i] = p;
    L.w[0][i] = vel[tk.p0 + i];
    L.id[0][i] = (unsigned short)i;
    const int c = res_key(p, g2);
    L.key[i] = (unsigned short)c;
    atomicAdd(&L.cnt[c], 1);
  }
  __syncthreads();
  res_sort(L, n, nc, 0);
  int par = 1;

  const int ncx = g2.ncx, ncy = g2.ncy;
  for (int step = 0; step < n_steps; ++step) {
    RigidIn in;
    if (t == 0) in = rigid_inputs(&L.rb, &L.ro, tank, kStep, ra);   // loads in flight during the sums
    const float2* S = L.s[par];
    const float2* V = L.w[par];
    // density and EOS
#pragma unroll
    for (int e = 0; e < kResPer; ++e) {
      const int i = t + e * kResThreads;
      if (i < n) {
        const float2 si = S[i];
        const int c = L.ckey[i], cx = c % ncx, cy = c / ncx;
        const int xa = cx > 0 ? cx - 1 : 0, xb = cx < ncx - 1 ? cx + 1 : ncx - 1;
        float sf = 0.0f, sgs = 0.0f;
        for (int yy = cy - 1; yy <= cy + 1; ++yy) {
          if (yy < 0 || yy >= ncy) continue;
          const int row = yy * ncx;
#pragma unroll 4
          for (int q = L.start[row + xa], qe = L.start[row + xb + 1]; q < qe; ++q) {
            const float2 sj = S[q];
            const float d2 = dist2(si.x - sj.x, si.y - sj.y);
            if (d2 < k.R2) sf += cubic_shape(fsqrt(d2) * k.inv_h);
          }
#pragma unroll 4
          for (int q = L.gstart[row + xa], qe = L.gstart[row + xb + 1]; q < qe; ++q) {
            const float2 gj = L.g[q];
            const float d2 = dist2(si.x - gj.x, si.y - gj.y);
            if (d2 < k.R2) sgs += cubic_shape(fsqrt(d2) * k.inv_h);
          }
        }
        const float rho = k.mass * k.wc * (sf + k.gamma1 * sgs);
        L.rp[i] = make_float2(rho, eos_over_rho2(rho, k, nullptr));
      }
    }
    __syncthreads();
    // pair and wall terms, the tank's reactions
    float2 acc[kResPer];
    double F[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int e = 0; e < kResPer; ++e) {
      const int i = t + e * kResThreads;
      acc[e] = make_float2(0.0f, 0.0f);
      if (i < n) {
        const float2 s = S[i], w = V[i], me = L.rp[i];
        const float rho_i = me.x, Pi = me.y;
        const float visc_g = k.beta2 / (2.0f * rho_i);
        const int c = L.ckey[i], cx = c % ncx, cy = c / ncx;
        const int xa = cx > 0 ? cx - 1 : 0, xb = cx < ncx - 1 ? cx + 1 : ncx - 1;
        float axf = 0.0f, ayf = 0.0f, axg = 0.0f, ayg = 0.0f, fx = 0.0f, fy = 0.0f, tq = 0.0f;
        for (int yy = cy - 1; yy <= cy + 1; ++yy) {
          if (yy < 0 || yy >= ncy) continue;
          const int row = yy * ncx;
#pragma unroll 2
          for (int q = L.start[row + xa], qe = L.start[row + xb + 1]; q < qe; ++q) {
            const float2 sj = S[q];
            const float dx = s.x - sj.x, dy = s.y - sj.y;
            const float d2 = dist2(dx, dy);
            if (d2 < k.R2 && d2 > 0.0f) {
              const float2 wj = V[q], o = L.rp[q];
              const float qq = fsqrt(d2) * k.inv_h;
              const float gW = k.dwc * cubic_grad_f(qq);
              const float vr = (w.x - wj.x) * dx + (w.y - wj.y) * dy;
              const float coef = (-(Pi + o.y) + k.a2h * vr * frcp((rho_i + o.x) * (d2 + k.eps_h2))) * gW;
              axf += coef * dx;
              ayf += coef * dy;
            }
          }
#pragma unroll 2
          for (int q = L.gstart[row + xa], qe = L.gstart[row + xb + 1]; q < qe; ++q) {
            const float2 gj = L.g[q];
            const float dx = s.x - gj.x, dy = s.y - gj.y;
            const float d2 = dist2(dx, dy);
            if (d2 < k.Rs2 && d2 > 0.0f) {
              const float r = fsqrt(d2);
              const float tt = k.hs - r;
              const float gW = k.dws * tt * tt * frcp(r);
              const float vr = w.x * dx + w.y * dy;
              const float coef = k.mass * (-2.0f * Pi + visc_g * fminf(vr, 0.0f) * frcp(d2 + k.eps_h2)) * gW;
              const float ax = coef * dx, ay = coef * dy;
              axg += ax;
              ayg += ay;
              const float Fx = k.mass * ax, Fy = k.mass * ay;
              fx -= Fx;
              fy -= Fy;
              tq -= gj.x * Fy - gj.y * Fx;
            }
          }
        }
        acc[e] = make_float2(k.mass * axf + axg, k.mass * ayf + ayg);
        F[0] += (double)fx;
        F[1] += (double)fy;
        F[2] += (double)tq;
      }
    }
    const int lane = t & 63, wv = t >> 6;
    for (int d = 0; d < 3; ++d) {
      const double v = wave_sum0(F[d]);
      if (lane == 0) L.red[d][wv] = v;
    }
    __syncthreads();
    // the rigid-body part of the step (one thread), then the fluid update
    if (t == 0) {
      double Ft[3];
      for (int d = 0; d < 3; ++d) {
        double v = 0.0;
        for (int q = 0; q < kResThreads / 64; ++q) v += L.red[d][q];
        Ft[d] = v;
      }
      res_rigid_step(&L.rb, &L.ro, tank, Ft[0], Ft[1], Ft[2], ra, in);
      L.frame[0] = L.rb.abx;
      L.frame[1] = L.rb.aby;
      L.frame[2] = L.rb.thd;
      L.frame[3] = L.rb.thdd;
    }
    __syncthreads();
    const Frame fr{L.frame[0], L.frame[1], L.frame[2], L.frame[3]};
    unsigned bad = 0;
#pragma unroll
    for (int e = 0; e < kResPer; ++e) {
      const int i = t + e * kResThreads;
      if (i < n) {
        float2 s = L.s[par][i], w = L.w[par][i];
        fluid_update(s, w, acc[e], fr, k.dt);
        L.s[par][i] = s;
        L.w[par][i] = w;
        if (!isfinite(s.x) || !isfinite(s.y) || !isfinite(w.x) || !isfinite(w.y)) {
          bad |= SPH_ST_NONFINITE;
        } else {
          if (!((double)s.x >= tk.box.lo_x && (double)s.x < tk.box.hi_x && (double)s.y >= tk.box.lo_y &&
                (double)s.y < tk.box.hi_y))
            bad |= SPH_ST_ESCAPED;
          if (dist2(w.x, w.y) > k.cfl_w2) bad |= SPH_ST_CFL;
        }
        const int c = res_key(s, g2);
        L.key[i] = (unsigned short)c;
        atomicAdd(&L.cnt[c], 1);
      }
    }
    if (bad) atomicOr(&L.bad, bad);
    __syncthreads();
    res_sort(L, n, nc, par);
    par = 1 - par;
  }
  for (int i = t; i < n; i += kResThreads) {
    const int slot = L.id[par][i];
    pos[tk.p0 + slot] = L.s[par][i];
    vel[tk.p0 + slot] = L.w[par][i];
  }
  if (t == 0) {
    rigid[tank] = L.rb;
    if (L.bad) atomicOr(status, L.bad);
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

double support_of(const sph_params* p) { return 2.0 * p->h > p->h_spiky ? 2.0 * p->h : p->h_spiky; }

// Courant number of a step: dt (c + |w|) / h, with c the equation of state's
// sound speed at rest (c0 for the Tait law; sqrt(dP/drho) = sqrt(k) for the
// linear law of eq. EOS).  The workloads set dt for 0.2 at rest; a step is
// flagged above twice that.
constexpr double kCourantMax = 0.4;

double sound_speed(const sph_params* p) {
  return (p->eos == SPH_EOS_LINEAR || p->eos == SPH_EOS_LINEAR_CLAMPED) ? std::sqrt(p->k_lin) : p->c0;
}

// The largest particle speed within the limit (not positive: dt is over the
// limit at rest).
double cfl_speed(const sph_params* p) { return kCourantMax * p->h / p->dt - sound_speed(p); }

bool make_grid(const sph_params* p, Grid* g, double skin_over_h = kSkinOverH) {
  double cell = (support_of(p) + skin_over_h * p->h) * (1.0 + 1e-6);
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

int nblocks(long long threads) { return threads > 0 ? (int)((threads + kBlock - 1) / kBlock) : 1; }

bool params_ok(const sph_params* p) {
  if (!p) return false;
  if (!(p->h > 0 && p->h_spiky > 0 && p->mass > 0 && p->dt > 0 && p->rho0 > 0)) return false;
  if (p->eos != SPH_EOS_TAIT && p->eos != SPH_EOS_LINEAR && p->eos != SPH_EOS_LINEAR_CLAMPED &&
      p->eos != SPH_EOS_TAIT_CLAMPED)
    return false;
  if ((p->eos == SPH_EOS_TAIT || p->eos == SPH_EOS_TAIT_CLAMPED) && !(p->c0 > 0 && p->tait_gamma > 0)) return false;
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
  k.B = (float)(p->eos == SPH_EOS_TAIT || p->eos == SPH_EOS_TAIT_CLAMPED ? p->rho0 * p->c0 * p->c0 / p->tait_gamma
                                                                          : 0.0);
  k.k_lin = (float)p->k_lin;
  k.a2h = (float)(2.0 * p->visc_alpha * h);
  k.beta2 = (float)(2.0 * p->visc_beta);
  k.eps_h2 = (float)(p->eps * h * h);
  k.dt = (float)p->dt;
  // a slightly smaller bound than skin/2 absorbs the rounding of the check
  double hsk = 0.5 * kSkinOverH * h * (1.0 - 1e-5);
  k.half_skin2 = (float)(hsk * hsk);
  // near-list radii, slightly enlarged against rounding of the test
  const double skin = kSkinOverH * h;
  const double rl = (2.0 * h + skin) * (1.0 + 1e-5), rg = (support_of(p) + 0.5 * skin) * (1.0 + 1e-5);
  k.RL2 = (float)(rl * rl);
  k.RG2 = (float)(rg * rg);
  const double wmax = cfl_speed(p);
  k.cfl_w2 = wmax > 0.0 ? (float)(wmax * wmax) : 0.0f;
  k.eos = p->eos;
  double gi = std::round(p->tait_gamma);
  k.tgamma = (std::fabs(gi - p->tait_gamma) < 1e-12 && gi >= 1 && gi <= 64) ? (int)gi : 0;
  k.tgamma_f = (float)p->tait_gamma;
  return k;
}

// Sizes of a batch, known on the host.
struct Plan {
  int T = 0;
  long long N = 0, Gh = 0, C = 0;          // particles, ghosts, cells (totals)
  long long tiles[kNumVariants] = {0, 0, 0, 0};
  std::vector<Tank> tanks;
};

int make_plan(int T, const sph_params* params, const int32_t* n_fluid, const int32_t* n_ghost, Plan* pl) {
  if (T < 1 || !params || !n_fluid || !n_ghost) return SPH_E_INVAL;
  pl->T = T;
  pl->tanks.resize(T);
  long long p0 = 0, q0 = 0, c0 = 0;
  for (int t = 0; t < T; ++t) {
    const sph_params* p = &params[t];
    if (!params_ok(p) || n_fluid[t] < 0 || n_ghost[t] < 0) return SPH_E_INVAL;
    if (n_fluid[t] > 0 && !(cfl_speed(p) > 0.0)) {
      snprintf(g_err, sizeof g_err, "tank %d: dt (c / h) = %g is above the Courant limit %g", t,
               p->dt * sound_speed(p) / p->h, kCourantMax);
      return SPH_E_INVAL;
    }
    Tank& tk = pl->tanks[t];
    memset(&tk, 0, sizeof tk);
    if (!make_grid(p, &tk.g) || !make_grid(p, &tk.g2, 0.0)) return SPH_E_INVAL;
    tk.k = make_consts(p);
    tk.box = Box{p->domain_min[0], p->domain_min[1], p->domain_max[0], p->domain_max[1]};
    tk.ra = RigidArgs{p->dt, p->body_mass, p->body_inertia, p->kp, p->kd, p->sine_amp, p->sine_freq,
                      p->motion, p->ctrl, p->ctrl_period, 0};
    tk.p0 = (int)p0;
    tk.n = n_fluid[t];
    tk.q0 = (int)q0;
    tk.ng = n_ghost[t];
    tk.c0 = (int)c0;
    tk.nc = tk.g.ncx * tk.g.ncy;
    p0 += tk.n;
    q0 += tk.ng;
    c0 += tk.nc;
    for (int v = 0; v < kNumVariants; ++v) {
      const int tp = kBlock / kLanes[v];
      pl->tiles[v] += tk.n > 0 ? (tk.n + tp - 1) / tp : 1;   // an empty tank still reduces its wrench
    }
    if (p0 > (1LL << 30) || q0 > (1LL << 30) || c0 > (1LL << 30)) return SPH_E_INVAL;
  }
  pl->N = p0;
  pl->Gh = q0;
  pl->C = c0;
  return SPH_OK;
}

struct Layout {
  size_t pos[2], vel[2], acc[2], id[2], cstart[2], pos_sort, rng, pkey, rp, near_n, near_f, near_g, marks, key, slot,
      order, count, scanpart, gpos,
      graw, gstart, owner, gowner, cowner, tanks, tiles[kNumVariants], tile0[kNumVariants], partials,
      rigid, rollout, status, total;
};

Layout make_layout(const Plan& pl) {
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes > 0 ? bytes : 1);
    return at;
  };
  const size_t n = (size_t)pl.N, gg = (size_t)pl.Gh, nc = (size_t)pl.C, T = (size_t)pl.T;
  const size_t mx = n > gg ? n : gg;
  size_t max_tiles = 0;
  for (int v = 0; v < kNumVariants; ++v) max_tiles = max_tiles > (size_t)pl.tiles[v] ? max_tiles : (size_t)pl.tiles[v];
  for (int b = 0; b < 2; ++b) {
    L.pos[b] = take(n * 8);
    L.vel[b] = take(n * 8);
    L.acc[b] = take(n * 8);
    L.id[b] = take(n * 4);
    L.cstart[b] = take((nc + 1) * 4);
  }
  L.pos_sort = take(n * 8);
  L.scanpart = take((nc / kChunkCells + 2) * 4);
  L.rng = take(n * 48);
  L.pkey = take(n * 4);
  L.rp = take(n * 8);
  L.near_n = take(n * 4);
  L.near_f = take(n * kNearF);
  L.near_g = take(n * kNearG);
  L.marks = take(n * 4 * kLanes[kNumVariants - 1]);
  L.key = take(mx * 4);
  L.slot = take(mx * 4);
  L.order = take(mx * 4);
  L.count = take(nc * 4);
  L.gpos = take(gg * 8);
  L.graw = take(gg * 8);
  L.gstart = take((nc + 1) * 4);
  L.owner = take(n * 4);
  L.gowner = take(gg * 4);
  L.cowner = take(nc * 4);
  L.tanks = take(T * sizeof(Tank));
  for (int v = 0; v < kNumVariants; ++v) {
    L.tiles[v] = take((size_t)pl.tiles[v] * sizeof(TileRef));
    L.tile0[v] = take((T + 1) * 4);
  }
  L.partials = take(max_tiles * 3 * 8);
  L.rigid = take(T * sizeof(DevRigid));
  L.rollout = take(sizeof(DevRollout));
  L.status = take(4);
  L.total = o;
  return L;
}

// --------------------------------------------------------------------------
// tangent-linear rollout: the step's derivative along given directions
// --------------------------------------------------------------------------
//
// Forward-mode derivative of the whole coupled step (the linearization the
// paper obtains by automatic differentiation, Section 3.5), along n_dir
// directions, each a perturbation of the initial fluid state, the initial
// rigid state and the sequence of applied forces and torque.  Every
// quantity of the step carries one tangent per direction, differentiated by
// hand in the order of the step (product, quotient and chain rules), with
// the neighbour sets of the primal.  One thread per particle, particles in
// caller order; the cell list is rebuilt every step as an index (keys, scan,
// stable scatter), so tangents never move.  Density and force handle
// kJvpChunk directions per launch and recompute the primal for each chunk.

constexpr int kJvpChunk = 8;
constexpr int kJvpMaxDir = 64;

struct JvpRigid {     // rigid-body primal, FP64
  double r[2], th, rd[2], thd, tau;
  long long step, step0;
};
// tangents of the rigid state, per direction: r0, r1, th, rd0, rd1, thd, tau
constexpr int kJvpRigidT = 7;

// d shape / dq of the cubic spline (shape as in cubic_shape).
__device__ __forceinline__ float cubic_shape_d(float q) {
  float a = 2.0f - q;
  float d = -3.0f * a * a;
  if (q < 1.0f) {
    float b = 1.0f - q;
    d += 12.0f * b * b;
  }
  return d;
}

// d cubic_grad_f / dq.
__device__ __forceinline__ float cubic_grad_f_d(float q) {
  if (q < 1.0f) return 9.0f;
  float a = 2.0f - q;
  return 6.0f * a / q + 3.0f * a * a / (q * q);
}

// P/rho^2 and its derivative with respect to rho.
__device__ __forceinline__ float eos_over_rho2_d(float rho, const Consts& k, float* dpi) {
  float P, dP;
  if (k.eos == SPH_EOS_LINEAR || k.eos == SPH_EOS_LINEAR_CLAMPED) {
    P = k.k_lin * (rho - k.rho0);
    dP = k.k_lin;
    if (k.eos == SPH_EOS_LINEAR_CLAMPED && !(P > 0.0f)) {
      P = 0.0f;
      dP = 0.0f;
    }
  } else {
    const float x = rho * k.rho0_inv;
    float xp1;   // x^(gamma - 1)
    if (k.tgamma > 0) {
      xp1 = 1.0f;
      for (int e = 1; e < k.tgamma; ++e) xp1 *= x;
    } else {
      xp1 = powf(x, k.tgamma_f - 1.0f);
    }
    P = k.B * (xp1 * x - 1.0f);
    dP = k.B * k.tgamma_f * xp1 * k.rho0_inv;
    if (k.eos == SPH_EOS_TAIT_CLAMPED && !(P > 0.0f)) {
      P = 0.0f;
      dP = 0.0f;
    }
  }
  const float r2 = rho * rho;
  *dpi = dP / r2 - 2.0f * P / (r2 * rho);
  return P / r2;
}

// Index range [lo, hi) of row yy's cells cx-1 .. cx+1 in a start array.
__device__ __forceinline__ bool jvp_row(const Tank& tk, int cx, int yy, const int* __restrict__ start, int* lo,
                                        int* hi) {
  if (yy < 0 || yy >= tk.g.ncy) return false;
  const int ncx = tk.g.ncx;
  const int xa = cx > 0 ? cx - 1 : 0, xb = cx < ncx - 1 ? cx + 1 : ncx - 1;
  const int c = tk.c0 + yy * ncx;
  *lo = start[c + xa];
  *hi = start[c + xb + 1];
  return true;
}

template <int KC>
__global__ void __launch_bounds__(kBlock) jvp_density(const float2* __restrict__ s, const float2* __restrict__ ds,
                                                      int n, int n_dir, int k0, const int* __restrict__ order,
                                                      const int* __restrict__ cstart,
                                                      const float2* __restrict__ gpos,
                                                      const int* __restrict__ gstart,
                                                      const Tank* __restrict__ tanks, float2* __restrict__ rp,
                                                      float2* __restrict__ drp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Tank& tk = tanks[0];
  const Consts& k = tk.k;
  const float2 si = s[i];
  float2 dsi[KC];
  float tf[KC], tg[KC];
#pragma unroll
  for (int q = 0; q < KC; ++q) {
    dsi[q] = k0 + q < n_dir ? ds[(size_t)(k0 + q) * n + i] : make_float2(0.f, 0.f);
    tf[q] = tg[q] = 0.0f;
  }
  float sf = 0.0f, sg = 0.0f;
  int cx, cy;
  cell_of(si, tk.g, cx, cy);
  for (int yy = cy - 1; yy <= cy + 1; ++yy) {
    int lo, hi;
    if (jvp_row(tk, cx, yy, cstart, &lo, &hi))
      for (int e = lo; e < hi; ++e) {
        const int j = order[e];
        const float2 sj = s[j];
        const float dx = si.x - sj.x, dy = si.y - sj.y, d2 = dist2(dx, dy);
        if (!(d2 < k.R2)) continue;
        const float r = sqrtf(d2), q = r * k.inv_h;
        sf += cubic_shape(q);
        if (j == i || r == 0.0f) continue;
        const float fac = cubic_shape_d(q) * k.inv_h / r;
#pragma unroll
        for (int c = 0; c < KC; ++c) {
          if (k0 + c >= n_dir) break;
          const float2 dsj = ds[(size_t)(k0 + c) * n + j];
          tf[c] += fac * (dx * (dsi[c].x - dsj.x) + dy * (dsi[c].y - dsj.y));
        }
      }
    if (jvp_row(tk, cx, yy, gstart, &lo, &hi))
      for (int e = lo; e < hi; ++e) {
        const float2 gp = gpos[e];
        const float dx = si.x - gp.x, dy = si.y - gp.y, d2 = dist2(dx, dy);
        if (!(d2 < k.R2)) continue;
        const float r = sqrtf(d2), q = r * k.inv_h;
        sg += cubic_shape(q);
        if (r == 0.0f) continue;
        const float fac = cubic_shape_d(q) * k.inv_h / r;
#pragma unroll
        for (int c = 0; c < KC; ++c) tg[c] += fac * (dx * dsi[c].x + dy * dsi[c].y);
      }
  }
  const float rho = k.mass * k.wc * (sf + k.gamma1 * sg);
  float dpi;
  const float pi = eos_over_rho2_d(rho, k, &dpi);
  if (k0 == 0) rp[i] = make_float2(rho, pi);
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    if (k0 + c >= n_dir) break;
    const float drho = k.mass * k.wc * (tf[c] + k.gamma1 * tg[c]);
    drp[(size_t)(k0 + c) * n + i] = make_float2(drho, dpi * drho);
  }
}

template <int KC>
__global__ void __launch_bounds__(kBlock) jvp_force(const float2* __restrict__ s, const float2* __restrict__ w,
                                                    const float2* __restrict__ rp, const float2* __restrict__ ds,
                                                    const float2* __restrict__ dw, const float2* __restrict__ drp,
                                                    int n, int n_dir, int k0, const int* __restrict__ order,
                                                    const int* __restrict__ cstart,
                                                    const float2* __restrict__ gpos,
                                                    const int* __restrict__ gstart,
                                                    const Tank* __restrict__ tanks, float2* __restrict__ a,
                                                    float2* __restrict__ da, double* __restrict__ part,
                                                    double* __restrict__ dpart) {
  __shared__ double red[3 * (1 + KC)][kBlock / 64];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < n;
  const Tank& tk = tanks[0];
  const Consts& k = tk.k;
  float ax = 0.f, ay = 0.f, agx = 0.f, agy = 0.f, fx = 0.f, fy = 0.f, tq = 0.f;
  float tax[KC], tay[KC], tagx[KC], tagy[KC], tfx[KC], tfy[KC], ttq[KC];
#pragma unroll
  for (int c = 0; c < KC; ++c) tax[c] = tay[c] = tagx[c] = tagy[c] = tfx[c] = tfy[c] = ttq[c] = 0.0f;
  if (valid) {
    const float2 si = s[i], wi = w[i], mi = rp[i];
    const float rho_i = mi.x, pi_i = mi.y;
    float2 dsi[KC], dwi[KC], dmi[KC];
#pragma unroll
    for (int c = 0; c < KC; ++c) {
      const bool on = k0 + c < n_dir;
      dsi[c] = on ? ds[(size_t)(k0 + c) * n + i] : make_float2(0.f, 0.f);
      dwi[c] = on ? dw[(size_t)(k0 + c) * n + i] : make_float2(0.f, 0.f);
      dmi[c] = on ? drp[(size_t)(k0 + c) * n + i] : make_float2(0.f, 0.f);
    }
    int cx, cy;
    cell_of(si, tk.g, cx, cy);
    for (int yy = cy - 1; yy <= cy + 1; ++yy) {
      int lo, hi;
      if (jvp_row(tk, cx, yy, cstart, &lo, &hi))
        for (int e = lo; e < hi; ++e) {
          const int j = order[e];
          const float2 sj = s[j];
          const float dx = si.x - sj.x, dy = si.y - sj.y, d2 = dist2(dx, dy);
          if (!(d2 < k.R2 && d2 > 0.0f)) continue;
          const float2 wj = w[j], mj = rp[j];
          const float rn = sqrtf(d2), q = rn * k.inv_h;
          const float gW = k.dwc * cubic_grad_f(q), gWd = k.dwc * cubic_grad_f_d(q);
          const float vx = wi.x - wj.x, vy = wi.y - wj.y, vr = vx * dx + vy * dy;
          const float S = rho_i + mj.x, E = d2 + k.eps_h2, D = S * E;
          const float visc = k.a2h * vr / D;
          const float C0 = -(pi_i + mj.y) + visc, coef = C0 * gW;
          ax += coef * dx;
          ay += coef * dy;
#pragma unroll
          for (int c = 0; c < KC; ++c) {
            if (k0 + c >= n_dir) break;
            const size_t o = (size_t)(k0 + c) * n + j;
            const float2 dsj = ds[o], dwj = dw[o], dmj = drp[o];
            const float ddx = dsi[c].x - dsj.x, ddy = dsi[c].y - dsj.y;
            const float rdr = dx * ddx + dy * ddy;
            const float dgW = gWd * rdr * k.inv_h / rn;
            const float dvr = (dwi[c].x - dwj.x) * dx + (dwi[c].y - dwj.y) * dy + vx * ddx + vy * ddy;
            const float dD = (dmi[c].x + dmj.x) * E + S * 2.0f * rdr;
            const float dvisc = k.a2h * (dvr * D - vr * dD) / (D * D);
            const float dC0 = -(dmi[c].y + dmj.y) + dvisc;
            const float dcoef = dC0 * gW + C0 * dgW;
            tax[c] += dcoef * dx + coef * ddx;
            tay[c] += dcoef * dy + coef * ddy;
          }
        }
      if (jvp_row(tk, cx, yy, gstart, &lo, &hi))
        for (int e = lo; e < hi; ++e) {
          const float2 gp = gpos[e];
          const float dx = si.x - gp.x, dy = si.y - gp.y, d2 = dist2(dx, dy);
          if (!(d2 < k.Rs2 && d2 > 0.0f)) continue;
          const float rn = sqrtf(d2), tt = k.hs - rn;
          const float gWs = k.dws * tt * tt / rn;
          const float vr = wi.x * dx + wi.y * dy, mv = fminf(vr, 0.0f);
          const float vg = k.beta2 / (2.0f * rho_i), E = d2 + k.eps_h2, term = vg * mv / E;
          const float C0 = -2.0f * pi_i + term, coef = k.mass * C0 * gWs;
          const float awx = coef * dx, awy = coef * dy;
          agx += awx;
          agy += awy;
          const float Fx = k.mass * awx, Fy = k.mass * awy;
          fx -= Fx;
          fy -= Fy;
          tq -= gp.x * Fy - gp.y * Fx;
#pragma unroll
          for (int c = 0; c < KC; ++c) {
            const float ddx = dsi[c].x, ddy = dsi[c].y;
            const float rdr = dx * ddx + dy * ddy, drn = rdr / rn, dtt = -drn;
            const float dgWs = k.dws * (2.0f * tt * dtt / rn - tt * tt * drn / (rn * rn));
            const float dvr = dwi[c].x * dx + dwi[c].y * dy + wi.x * ddx + wi.y * ddy;
            const float dmv = vr < 0.0f ? dvr : 0.0f;
            const float dvg = -k.beta2 / (2.0f * rho_i * rho_i) * dmi[c].x;
            const float dterm = (dvg * mv + vg * dmv) / E - vg * mv * (2.0f * rdr) / (E * E);
            const float dcoef = k.mass * ((-2.0f * dmi[c].y + dterm) * gWs + C0 * dgWs);
            const float dawx = dcoef * dx + coef * ddx, dawy = dcoef * dy + coef * ddy;
            tagx[c] += dawx;
            tagy[c] += dawy;
            const float dFx = k.mass * dawx, dFy = k.mass * dawy;
            tfx[c] -= dFx;
            tfy[c] -= dFy;
            ttq[c] -= gp.x * dFy - gp.y * dFx;
          }
        }
    }
    if (k0 == 0) a[i] = make_float2(k.mass * ax + agx, k.mass * ay + agy);
#pragma unroll
    for (int c = 0; c < KC; ++c)
      if (k0 + c < n_dir)
        da[(size_t)(k0 + c) * n + i] = make_float2(k.mass * tax[c] + tagx[c], k.mass * tay[c] + tagy[c]);
  }
  // workgroup sums of the wall reactions and their tangents, in double
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  auto put = [&](int slot, float v) {
    const double t = wave_sum((double)v);
    if (lane == 0) red[slot][wv] = t;
  };
  put(0, fx);
  put(1, fy);
  put(2, tq);
#pragma unroll
  for (int c = 0; c < KC; ++c) {
    put(3 + 3 * c, tfx[c]);
    put(4 + 3 * c, tfy[c]);
    put(5 + 3 * c, ttq[c]);
  }
  __syncthreads();
  for (int slot = threadIdx.x; slot < 3 * (1 + KC); slot += blockDim.x) {
    double t = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) t += red[slot][q];
    if (slot < 3) {
      if (k0 == 0) part[3 * blockIdx.x + slot] = t;
    } else {
      const int c = (slot - 3) / 3, d = (slot - 3) % 3;
      if (k0 + c < n_dir) dpart[((size_t)blockIdx.x * n_dir + k0 + c) * 3 + d] = t;
    }
  }
}

// One workgroup: wrench sums in a fixed order, then the rigid-body step with
// its tangents (zero-order-hold law, eq. tankdynamics, symplectic Euler), and
// the coefficients of the fluid update.  frame: abx, aby, thetadot,
// thetaddot (binary32, as the step uses them); tframe the same per direction.
__global__ void __launch_bounds__(kBlock) jvp_rigid(const double* __restrict__ part,
                                                    const double* __restrict__ dpart, int nb, int n_dir,
                                                    const Tank* __restrict__ tanks, JvpRigid* st,
                                                    double* __restrict__ tst, const float* __restrict__ u,
                                                    const float* __restrict__ du, long long n_steps,
                                                    const double* __restrict__ theta_ref, int n_ref,
                                                    float4* __restrict__ frame, float4* __restrict__ tframe,
                                                    double* __restrict__ wout, double* __restrict__ twout) {
  __shared__ double F[3], dF[kJvpMaxDir][3];
  __shared__ double P[8];   // primal: th, thd, tau, c, s, acc x, acc y, theta''
  const RigidArgs& ra = tanks[0].ra;
  for (int slot = threadIdx.x; slot < 3 * (1 + n_dir); slot += blockDim.x) {
    double t = 0.0;
    if (slot < 3) {
      for (int b = 0; b < nb; ++b) t += part[3 * b + slot];
      F[slot] = t;
    } else {
      const int c = (slot - 3) / 3, d = (slot - 3) % 3;
      for (int b = 0; b < nb; ++b) t += dpart[((size_t)b * n_dir + c) * 3 + d];
      dF[c][d] = t;
    }
  }
  __syncthreads();
  const long long n = st->step, loc = n - st->step0;
  const bool have_u = u && loc >= 0 && loc < n_steps;
  const bool sample = ra.ctrl == SPH_CTRL_PD_ZOH && ra.ctrl_period > 0 && n % ra.ctrl_period == 0;
  const bool sine = ra.motion == SPH_MOTION_SINE;
  if (threadIdx.x == 0) {
    double uu[3] = {0.0, 0.0, 0.0};
    if (have_u)
      for (int d = 0; d < 3; ++d) uu[d] = u[loc * 3 + d];
    double tau = st->tau;
    if (sample) {
      double ref = 0.0;
      if (theta_ref && n_ref > 0) {
        const long long kk = n / ra.ctrl_period;
        ref = theta_ref[kk < n_ref ? kk : n_ref - 1];
      }
      tau = ra.kp * (ref - st->th) - ra.kd * st->thd;
    }
    double th, thd, acc[3];
    if (sine) {
      const double om = 2.0 * M_PI * ra.sine_freq, t = (double)n * ra.dt;
      th = ra.sine_amp * sin(om * t);
      thd = ra.sine_amp * om * cos(om * t);
      acc[0] = acc[1] = 0.0;
      acc[2] = -ra.sine_amp * om * om * sin(om * t);
    } else {
      th = st->th;
      thd = st->thd;
    }
    double sn, cs;
    sincos(th, &sn, &cs);
    if (!sine) {
      acc[0] = (cs * F[0] - sn * F[1] + uu[0]) / ra.body_mass;
      acc[1] = (sn * F[0] + cs * F[1] + uu[1]) / ra.body_mass;
      acc[2] = (F[2] + uu[2] + tau) / ra.body_inertia;
    }
    P[0] = th; P[1] = thd; P[2] = tau; P[3] = cs; P[4] = sn; P[5] = acc[0]; P[6] = acc[1]; P[7] = acc[2];
    frame[0] = make_float4((float)(cs * acc[0] + sn * acc[1]), (float)(-sn * acc[0] + cs * acc[1]), (float)thd,
                           (float)acc[2]);
    for (int d = 0; d < 3; ++d) wout[d] = F[d];
  }
  __syncthreads();
  const double cs = P[3], sn = P[4], ax = P[5], ay = P[6];
  for (int c = threadIdx.x; c < n_dir; c += blockDim.x) {
    double* t = tst + (size_t)c * kJvpRigidT;
    for (int d = 0; d < 3; ++d) twout[3 * c + d] = dF[c][d];
    if (sine) {
      tframe[c] = make_float4(0.f, 0.f, 0.f, 0.f);
      for (int q = 0; q < kJvpRigidT; ++q) t[q] = 0.0;
      continue;
    }
    double tu[3] = {0.0, 0.0, 0.0};
    if (have_u && du)
      for (int d = 0; d < 3; ++d) tu[d] = du[((size_t)c * n_steps + loc) * 3 + d];
    double tth = t[2], tthd = t[5], ttau = t[6];
    if (sample) ttau = -ra.kp * tth - ra.kd * tthd;
    const double Fx = F[0], Fy = F[1];
    const double tax = (-sn * tth * Fx + cs * dF[c][0] - cs * tth * Fy - sn * dF[c][1] + tu[0]) / ra.body_mass;
    const double tay = (cs * tth * Fx + sn * dF[c][0] - sn * tth * Fy + cs * dF[c][1] + tu[1]) / ra.body_mass;
    const double tal = (dF[c][2] + tu[2] + ttau) / ra.body_inertia;
    tframe[c] = make_float4((float)(-sn * tth * ax + cs * tax + cs * tth * ay + sn * tay),
                            (float)(-cs * tth * ax - sn * tax - sn * tth * ay + cs * tay), (float)tthd, (float)tal);
    // symplectic Euler, velocity first
    t[3] += ra.dt * tax;
    t[4] += ra.dt * tay;
    t[5] += ra.dt * tal;
    t[0] += ra.dt * t[3];
    t[1] += ra.dt * t[4];
    t[2] += ra.dt * t[5];
    t[6] = ttau;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (sine) {
      const double om = 2.0 * M_PI * ra.sine_freq, t = (double)(n + 1) * ra.dt;
      st->th = ra.sine_amp * sin(om * t);
      st->thd = ra.sine_amp * om * cos(om * t);
      st->r[0] = st->r[1] = st->rd[0] = st->rd[1] = 0.0;
    } else {
      st->rd[0] += ra.dt * P[5];
      st->rd[1] += ra.dt * P[6];
      st->thd += ra.dt * P[7];
      st->r[0] += ra.dt * st->rd[0];
      st->r[1] += ra.dt * st->rd[1];
      st->th += ra.dt * st->thd;
    }
    st->tau = P[2];
    st->step = n + 1;
  }
}

// Fluid update with the fictitious terms (as fluid_update) and its tangents.
__global__ void __launch_bounds__(kBlock) jvp_update(float2* __restrict__ s, float2* __restrict__ w,
                                                     const float2* __restrict__ a, float2* __restrict__ ds,
                                                     float2* __restrict__ dw, const float2* __restrict__ da,
                                                     int n, int n_dir, const float4* __restrict__ frame,
                                                     const float4* __restrict__ tframe, float dt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float4 f = frame[0];
  const float2 si = s[i], wi = w[i], ai = a[i];
  const float om2 = f.z * f.z;
  for (int c = 0; c < n_dir; ++c) {
    const float4 tf = tframe[c];
    const size_t o = (size_t)c * n + i;
    const float2 tsi = ds[o], twi = dw[o], tai = da[o];
    const float tdx = tai.x - tf.x + 2.0f * (tf.z * wi.y + f.z * twi.y) + (tf.w * si.y + f.w * tsi.y) +
                      2.0f * f.z * tf.z * si.x + om2 * tsi.x;
    const float tdy = tai.y - tf.y - 2.0f * (tf.z * wi.x + f.z * twi.x) - (tf.w * si.x + f.w * tsi.x) +
                      2.0f * f.z * tf.z * si.y + om2 * tsi.y;
    const float2 tw = make_float2(twi.x + dt * tdx, twi.y + dt * tdy);
    dw[o] = tw;
    ds[o] = make_float2(tsi.x + dt * tw.x, tsi.y + dt * tw.y);
  }
  float2 sn = si, wn = wi;
  fluid_update(sn, wn, ai, Frame{f.x, f.y, f.z, f.w}, dt);
  s[i] = sn;
  w[i] = wn;
}

// --------------------------------------------------------------------------
// adjoint rollout: reverse-mode derivatives of the step
// --------------------------------------------------------------------------
//
// The transpose of the tangent-linear step: given the adjoints of a step's
// outputs (fluid state, rigid state) and of the wrench it evaluated, the
// adjoints of its inputs and of its applied force/torque.  The primal of a
// step is recomputed from its stored input state with the kernels above
// (no directions), then the step is reversed in the opposite order: fluid
// update, rigid body (one thread), forces (a gather over each particle's
// neighbours: a pair term f_ij enters a_i with +m and a_j with -m, so its
// adjoint is m (abar_i - abar_j) and each particle accumulates the
// derivatives with respect to its own variables), equation of state and
// density (a gather with rhobar_i + rhobar_j).

// Reverse of the fluid update x' = (s + dt w', w + dt D).  sb, wb hold the
// adjoints of (s', w') on entry and those of (s, w) on exit; ab receives
// the adjoint of a_sph; fpart[block] the sums of the frame adjoints (abx,
// aby, thetadot, theta'').
__global__ void __launch_bounds__(kBlock) vjp_update(const float2* __restrict__ s, const float2* __restrict__ w,
                                                     float2* __restrict__ sb, float2* __restrict__ wb,
                                                     float2* __restrict__ ab, int n,
                                                     const float4* __restrict__ frame, float dt,
                                                     double* __restrict__ fpart) {
  __shared__ double red[4][kBlock / 64];
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  float g0 = 0.f, g1 = 0.f, g2 = 0.f, g3 = 0.f;
  if (i < n) {
    const float4 f = frame[0];
    const float2 si = s[i], wi = w[i], sbp = sb[i], wbp = wb[i];
    const float2 wt = make_float2(wbp.x + dt * sbp.x, wbp.y + dt * sbp.y);
    const float2 Db = make_float2(dt * wt.x, dt * wt.y);
    ab[i] = Db;
    const float om2 = f.z * f.z;
    wb[i] = make_float2(wt.x - 2.0f * f.z * Db.y, wt.y + 2.0f * f.z * Db.x);
    sb[i] = make_float2(sbp.x - f.w * Db.y + om2 * Db.x, sbp.y + f.w * Db.x + om2 * Db.y);
    g0 = -Db.x;
    g1 = -Db.y;
    g2 = 2.0f * (wi.y * Db.x - wi.x * Db.y) + 2.0f * f.z * (si.x * Db.x + si.y * Db.y);
    g3 = si.y * Db.x - si.x * Db.y;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const float g[4] = {g0, g1, g2, g3};
  for (int d = 0; d < 4; ++d) {
    const double t = wave_sum((double)g[d]);
    if (lane == 0) red[d][wv] = t;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double t = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) t += red[threadIdx.x][q];
    fpart[4 * blockIdx.x + threadIdx.x] = t;
  }
}

// Reverse of the rigid-body step, one thread.  st: the step's input rigid
// state; F: the wrench the step evaluated; rb [7] (r0, r1, th, rd0, rd1,
// thd, tau): adjoints of the output state on entry, of the input state on
// exit; fb [3]: adjoint of the wrench (plus wbar at the last step); ub: the
// adjoint of the step's applied force/torque.
__global__ void vjp_rigid(const double* __restrict__ fpart, int nb, const Tank* __restrict__ tanks,
                          const JvpRigid* __restrict__ st, const double* __restrict__ F,
                          const float* __restrict__ u, long long n_steps, const double* __restrict__ theta_ref,
                          int n_ref, double* __restrict__ rb, double* __restrict__ fb,
                          float* __restrict__ ub, const double* __restrict__ wbar, int last) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const RigidArgs& ra = tanks[0].ra;
  double fr[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = 0; b < nb; ++b)
    for (int d = 0; d < 4; ++d) fr[d] += fpart[4 * b + d];
  const long long n = st->step, loc = n - st->step0;
  double Fb[3] = {0.0, 0.0, 0.0};
  if (last)
    for (int d = 0; d < 3; ++d) Fb[d] = wbar[d];
  if (ra.motion == SPH_MOTION_SINE) {
    // prescribed motion: the rigid state and the frame depend on time only
    for (int q = 0; q < kJvpRigidT; ++q) rb[q] = 0.0;
    for (int d = 0; d < 3; ++d) fb[d] = Fb[d];
    if (ub && loc >= 0 && loc < n_steps)
      for (int d = 0; d < 3; ++d) ub[loc * 3 + d] = 0.0f;
    return;
  }
  double uu[3] = {0.0, 0.0, 0.0};
  if (u && loc >= 0 && loc < n_steps)
    for (int d = 0; d < 3; ++d) uu[d] = u[loc * 3 + d];
  // the held torque enters the step linearly, so its reverse needs only
  // whether this step samples the attitude law, not the torque's value
  const bool sample = ra.ctrl == SPH_CTRL_PD_ZOH && ra.ctrl_period > 0 && n % ra.ctrl_period == 0;
  (void)theta_ref;
  (void)n_ref;
  double sn, cs;
  sincos(st->th, &sn, &cs);
  const double M = ra.body_mass, J = ra.body_inertia, dt = ra.dt;
  const double ax = (cs * F[0] - sn * F[1] + uu[0]) / M;
  const double ay = (sn * F[0] + cs * F[1] + uu[1]) / M;
  // output state: r' = r + dt rd', th' = th + dt thd', rd' = rd + dt a, thd' = thd + dt alpha, tau' = tau
  const double thb = rb[2], thdp = rb[5] + dt * rb[2];
  const double rd0p = rb[3] + dt * rb[0], rd1p = rb[4] + dt * rb[1];
  const double alb = dt * thdp + fr[3];
  double axb = dt * rd0p, ayb = dt * rd1p;
  // frame: abx = c ax + s ay, aby = -s ax + c ay, thetadot, theta''
  axb += cs * fr[0] - sn * fr[1];
  ayb += sn * fr[0] + cs * fr[1];
  double cb = ax * fr[0] + ay * fr[1], sb = ay * fr[0] - ax * fr[1];
  // alpha = (F_tau + u_tau + tau) / J
  Fb[2] += alb / J;
  const double taub = alb / J + rb[6];
  // a = (R F + u) / M
  Fb[0] += (cs * axb + sn * ayb) / M;
  Fb[1] += (-sn * axb + cs * ayb) / M;
  cb += (F[0] * axb + F[1] * ayb) / M;
  sb += (-F[1] * axb + F[0] * ayb) / M;
  if (ub && loc >= 0 && loc < n_steps) {
    ub[loc * 3 + 0] = (float)(axb / M);
    ub[loc * 3 + 1] = (float)(ayb / M);
    ub[loc * 3 + 2] = (float)(alb / J);
  }
  double th_in = thb - sn * cb + cs * sb;
  double thd_in = thdp + fr[2];
  double tau_in = taub;
  if (sample) {
    th_in -= ra.kp * taub;
    thd_in -= ra.kd * taub;
    tau_in = 0.0;
  }
  rb[0] = rb[0];
  rb[1] = rb[1];
  rb[2] = th_in;
  rb[3] = rd0p;
  rb[4] = rd1p;
  rb[5] = thd_in;
  rb[6] = tau_in;
  for (int d = 0; d < 3; ++d) fb[d] = Fb[d];
}

// Reverse of the forces and wall reactions: accumulates into sb, wb the
// derivatives with respect to each particle's own position and velocity,
// and writes rhob = the adjoint of its density (through the pair terms, the
// wall terms and the equation of state).
__global__ void __launch_bounds__(kBlock) vjp_force(const float2* __restrict__ s, const float2* __restrict__ w,
                                                    const float2* __restrict__ rp, const float2* __restrict__ ab,
                                                    const double* __restrict__ fb, int n,
                                                    const int* __restrict__ order, const int* __restrict__ cstart,
                                                    const float2* __restrict__ gpos, const int* __restrict__ gstart,
                                                    const Tank* __restrict__ tanks, float2* __restrict__ sb,
                                                    float2* __restrict__ wb, float* __restrict__ rhob) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Tank& tk = tanks[0];
  const Consts& k = tk.k;
  const float2 si = s[i], wi = w[i], mi = rp[i], abi = ab[i];
  const float rho_i = mi.x, pi_i = mi.y;
  const float Fbx = (float)fb[0], Fby = (float)fb[1], Tb = (float)fb[2];
  float sbx = 0.f, sby = 0.f, wbx = 0.f, wby = 0.f, rhb = 0.f, pib = 0.f;
  int cx, cy;
  cell_of(si, tk.g, cx, cy);
  for (int yy = cy - 1; yy <= cy + 1; ++yy) {
    int lo, hi;
    if (jvp_row(tk, cx, yy, cstart, &lo, &hi))
      for (int e = lo; e < hi; ++e) {
        const int j = order[e];
        const float2 sj = s[j];
        const float dx = si.x - sj.x, dy = si.y - sj.y, d2 = dist2(dx, dy);
        if (!(d2 < k.R2 && d2 > 0.0f)) continue;
        const float2 wj = w[j], mj = rp[j], abj = ab[j];
        const float fbx = k.mass * (abi.x - abj.x), fby = k.mass * (abi.y - abj.y);
        const float rn = sqrtf(d2), q = rn * k.inv_h;
        const float g = cubic_grad_f(q), gW = k.dwc * g;
        const float vx = wi.x - wj.x, vy = wi.y - wj.y, vr = vx * dx + vy * dy;
        const float S = rho_i + mj.x, E = d2 + k.eps_h2, D = S * E;
        const float visc = k.a2h * vr / D, C0 = -(pi_i + mj.y) + visc, coef = C0 * gW;
        const float coefb = fbx * dx + fby * dy;
        float rbx = coef * fbx, rby = coef * fby;
        const float C0b = coefb * gW, gWb = coefb * C0;
        pib -= C0b;
        const float vrb = C0b * k.a2h / D, Db = -C0b * visc / D;
        rhb += Db * E;
        float d2b = Db * S;
        wbx += vrb * dx;
        wby += vrb * dy;
        rbx += vrb * vx;
        rby += vrb * vy;
        const float rnb = gWb * k.dwc * cubic_grad_f_d(q) * k.inv_h;
        d2b += rnb / (2.0f * rn);
        sbx += rbx + 2.0f * d2b * dx;
        sby += rby + 2.0f * d2b * dy;
      }
    if (jvp_row(tk, cx, yy, gstart, &lo, &hi))
      for (int e = lo; e < hi; ++e) {
        const float2 gp = gpos[e];
        const float dx = si.x - gp.x, dy = si.y - gp.y, d2 = dist2(dx, dy);
        if (!(d2 < k.Rs2 && d2 > 0.0f)) continue;
        // adjoint of the wall term h (acceleration of the fluid particle)
        const float hbx = abi.x - k.mass * Fbx + k.mass * Tb * gp.y;
        const float hby = abi.y - k.mass * Fby - k.mass * Tb * gp.x;
        const float rn = sqrtf(d2), tt = k.hs - rn, gWs = k.dws * tt * tt / rn;
        const float vr = wi.x * dx + wi.y * dy, mv = fminf(vr, 0.0f);
        const float vg = k.beta2 / (2.0f * rho_i), E = d2 + k.eps_h2, term = vg * mv / E;
        const float C0 = -2.0f * pi_i + term, coef = k.mass * C0 * gWs;
        const float coefb = hbx * dx + hby * dy;
        float rbx = coef * hbx, rby = coef * hby;
        const float C0b = coefb * k.mass * gWs, gWsb = coefb * k.mass * C0;
        pib -= 2.0f * C0b;
        const float vgb = C0b * mv / E, mvb = C0b * vg / E;
        float d2b = -C0b * term / E;
        rhb -= vgb * vg / rho_i;
        const float vrb = vr < 0.0f ? mvb : 0.0f;
        wbx += vrb * dx;
        wby += vrb * dy;
        rbx += vrb * wi.x;
        rby += vrb * wi.y;
        const float ttb = gWsb * k.dws * 2.0f * tt / rn;
        const float rnb = -gWsb * k.dws * tt * tt / (rn * rn) - ttb;
        d2b += rnb / (2.0f * rn);
        sbx += rbx + 2.0f * d2b * dx;
        sby += rby + 2.0f * d2b * dy;
      }
  }
  float dpi;
  eos_over_rho2_d(rho_i, k, &dpi);
  rhob[i] = rhb + dpi * pib;
  const float2 s0 = sb[i], w0 = wb[i];
  sb[i] = make_float2(s0.x + sbx, s0.y + sby);
  wb[i] = make_float2(w0.x + wbx, w0.y + wby);
}

// Reverse of the density sums: sb_i += m sigma sum_j (rhob_i + rhob_j) dW/dr r_ij / r
// (+ the ghost terms with rhob_i alone).
__global__ void __launch_bounds__(kBlock) vjp_density(const float2* __restrict__ s, const float* __restrict__ rhob,
                                                      int n, const int* __restrict__ order,
                                                      const int* __restrict__ cstart, const float2* __restrict__ gpos,
                                                      const int* __restrict__ gstart, const Tank* __restrict__ tanks,
                                                      float2* __restrict__ sb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Tank& tk = tanks[0];
  const Consts& k = tk.k;
  const float2 si = s[i];
  const float rbi = rhob[i], ms = k.mass * k.wc;
  float sbx = 0.f, sby = 0.f;
  int cx, cy;
  cell_of(si, tk.g, cx, cy);
  for (int yy = cy - 1; yy <= cy + 1; ++yy) {
    int lo, hi;
    if (jvp_row(tk, cx, yy, cstart, &lo, &hi))
      for (int e = lo; e < hi; ++e) {
        const int j = order[e];
        const float2 sj = s[j];
        const float dx = si.x - sj.x, dy = si.y - sj.y, d2 = dist2(dx, dy);
        if (!(d2 < k.R2 && d2 > 0.0f)) continue;
        const float r = sqrtf(d2);
        const float fac = ms * (rbi + rhob[j]) * cubic_shape_d(r * k.inv_h) * k.inv_h / r;
        sbx += fac * dx;
        sby += fac * dy;
      }
    if (jvp_row(tk, cx, yy, gstart, &lo, &hi))
      for (int e = lo; e < hi; ++e) {
        const float2 gp = gpos[e];
        const float dx = si.x - gp.x, dy = si.y - gp.y, d2 = dist2(dx, dy);
        if (!(d2 < k.R2 && d2 > 0.0f)) continue;
        const float r = sqrtf(d2);
        const float fac = ms * k.gamma1 * rbi * cubic_shape_d(r * k.inv_h) * k.inv_h / r;
        sbx += fac * dx;
        sby += fac * dy;
      }
  }
  const float2 s0 = sb[i];
  sb[i] = make_float2(s0.x + sbx, s0.y + sby);
}

}  // namespace

struct sph_handle {
  Plan plan;
  int T, N, Gh, C;
  hipStream_t stream;
  char* ws;
  Layout L;
  int cur;          // buffer of the current particle state (pos, vel, acc)
  int ord;          // buffer of the current ordering (id, cell starts)
  int since_sort;   // steps since the last cell-list rebuild
  int sort_every;   // steps between rebuilds, a divisor of kChunk
  bool binned;      // the last force launch computed the keys and counts of the next rebuild
  int variant;      // lanes per particle = kLanes[variant]
  bool near;        // walk near lists (else every candidate of the 3x3 block)
  bool near_valid;  // the near lists belong to the current cell order
  hipGraphExec_t graph[kNumVariants][2][2][2];   // [variant][near] kChunk steps from (cur, ord),
                                                 // for the current sort_every
  bool graph_ok[kNumVariants][2][2][2];

  template <class T_>
  T_* at(size_t off) { return reinterpret_cast<T_*>(ws + off); }
};

namespace {

// Exclusive scan of the cell counts into start: one workgroup per tank, or,
// for a single tank with more than four chunks of cells, the three-launch
// form (same result).
void enqueue_scan(sph_handle* h, int* start, int ghosts, unsigned* status) {
  const long long nc = h->plan.tanks[0].nc;
  if (h->T == 1 && nc > 4LL * kChunkCells) {
    const int parts = (int)((nc + kChunkCells - 1) / kChunkCells);
    int* part = h->at<int>(h->L.scanpart);
    hipLaunchKernelGGL(sph_scan_sums, dim3(parts), dim3(kScanThreads), 0, h->stream, h->at<int>(h->L.count),
                       h->at<Tank>(h->L.tanks), part);
    hipLaunchKernelGGL(sph_scan_tops, dim3(1), dim3(kScanThreads), 0, h->stream, part, parts);
    hipLaunchKernelGGL(sph_scan_chunks, dim3(parts), dim3(kScanThreads), 0, h->stream, h->at<int>(h->L.count),
                       h->at<Tank>(h->L.tanks), ghosts, (const int*)part, parts, start, status);
  } else {
    hipLaunchKernelGGL(sph_scan, dim3(h->T), dim3(kScanThreads), 0, h->stream, h->at<int>(h->L.count),
                       h->at<Tank>(h->L.tanks), h->T, ghosts, start, status);
  }
}

// Rebuilds the cell list from the current state: key + count, per-tank scan,
// stable placement into the other buffers.  ev, if given, holds 4 events.
void enqueue_sort(sph_handle* h, hipEvent_t* ev = nullptr) {
  const int c = h->cur, o = h->ord;
  auto mark = [&](int i) {
    if (ev) (void)hipEventRecord(ev[i], h->stream);
  };
  mark(0);
  if (!h->binned)   // else the force kernel of the last step binned the particles
    hipLaunchKernelGGL(sph_bin, dim3(nblocks(h->N)), dim3(kBlock), 0, h->stream, h->at<float2>(h->L.pos[c]),
                       h->N, h->at<int>(h->L.owner), h->at<Tank>(h->L.tanks), h->at<int>(h->L.key),
                       h->at<int>(h->L.count), (int*)nullptr);
  h->binned = false;
  h->near_valid = false;
  mark(1);
  enqueue_scan(h, h->at<int>(h->L.cstart[1 - o]), 0, h->at<unsigned>(h->L.status));
  mark(2);
  hipLaunchKernelGGL(sph_place, dim3(nblocks((long long)h->C * kPlaceGroup)), dim3(kBlock), 0, h->stream,
                     h->at<int>(h->L.key), h->at<int>(h->L.cowner), h->at<Tank>(h->L.tanks), h->C,
                     h->at<int>(h->L.cstart[o]), h->at<int>(h->L.cstart[1 - o]), h->at<int>(h->L.gstart),
                     h->at<int4>(h->L.rng), h->at<int>(h->L.pkey), h->at<float2>(h->L.pos[c]),
                     h->at<float2>(h->L.vel[c]), h->at<float2>(h->L.acc[c]), h->at<int>(h->L.id[o]),
                     h->at<float2>(h->L.pos[1 - c]), h->at<float2>(h->L.vel[1 - c]),
                     h->at<float2>(h->L.acc[1 - c]), h->at<int>(h->L.id[1 - o]),
                     h->at<float2>(h->L.pos_sort), h->at<unsigned>(h->L.status));
  mark(3);
  h->cur = 1 - c;
  h->ord = 1 - o;
  h->since_sort = 0;
}

// Particle count of a single-tank handle (its tiles are computed in the
// kernels), -1 for a batch.
int single_n(const sph_handle* h) { return h->T == 1 ? h->N : -1; }

template <int G>
void launch_pair(sph_handle* h, int v, bool integrate, int mode, hipEvent_t* ev) {
  const int c = h->cur;
  const int nt = (int)h->plan.tiles[v];
  auto mark = [&](int i) {
    if (ev) (void)hipEventRecord(ev[i], h->stream);
  };
  mark(0);
  // with near lists on, the first step after a rebuild walks every candidate
  // and writes them; without, every step walks every candidate
  const bool build = h->near && !h->near_valid;
  auto density = build ? sph_density<G, true> : sph_density<G, false>;
  int* near_n = h->near ? h->at<int>(h->L.near_n) : nullptr;
  hipLaunchKernelGGL(density, dim3(nt), dim3(kBlock), 0, h->stream, h->at<float2>(h->L.pos[c]),
                     h->at<float2>(h->L.vel[c]), h->at<float2>(h->L.acc[c]), integrate ? 1 : 0,
                     h->at<float2>(h->L.pos_sort), h->at<int>(h->L.pkey), h->at<int4>(h->L.rng),
                     h->at<float2>(h->L.gpos), h->at<TileRef>(h->L.tiles[v]), single_n(h),
                     h->at<Tank>(h->L.tanks), h->at<DevRigid>(h->L.rigid), h->at<float2>(h->L.pos[1 - c]),
                     h->at<float2>(h->L.vel[1 - c]), h->at<float2>(h->L.rp), h->at<unsigned>(h->L.status),
                     near_n, h->at<unsigned>(h->L.near_f), h->at<unsigned>(h->L.near_g),
                     near_n ? h->at<unsigned>(h->L.marks) : nullptr);
  if (build) h->near_valid = true;
  mark(1);
  // the step before a scheduled rebuild also bins the particles for it
  const bool bin = mode == kStep && h->since_sort + 1 >= h->sort_every;
  auto force = bin ? sph_force<G, true> : sph_force<G, false>;
  hipLaunchKernelGGL(force, dim3(nt), dim3(kBlock), 0, h->stream, h->at<float2>(h->L.pos[1 - c]),
                     h->at<float2>(h->L.vel[1 - c]), h->at<float2>(h->L.rp), h->at<int>(h->L.pkey),
                     h->at<int4>(h->L.rng), h->at<float2>(h->L.gpos), h->at<TileRef>(h->L.tiles[v]),
                     single_n(h), h->at<Tank>(h->L.tanks), h->at<float2>(h->L.acc[1 - c]),
                     h->at<double>(h->L.partials),
                     h->at<int>(h->L.key), h->at<int>(h->L.count), near_n,
                     h->at<unsigned>(h->L.near_f), h->at<unsigned>(h->L.near_g), h->at<unsigned>(h->L.marks));
  h->binned = bin;
  mark(2);
  hipLaunchKernelGGL(sph_wrench, dim3(h->T), dim3(kWrenchThreads), 0, h->stream, h->at<double>(h->L.partials),
                     h->at<int>(h->L.tile0[v]), h->T == 1 ? nt : -1, h->at<Tank>(h->L.tanks), h->at<DevRigid>(h->L.rigid),
                     h->at<DevRollout>(h->L.rollout), mode);
  mark(3);
}

// Enqueues the three kernels of one step.  integrate = 0 when the state is
// already integrated (first step of a rollout).  ev, if given, holds 4 events.
void enqueue_step(sph_handle* h, bool integrate, int mode, hipEvent_t* ev = nullptr) {
  switch (h->variant) {
    case 0: launch_pair<4>(h, 0, integrate, mode, ev); break;
    case 1: launch_pair<8>(h, 1, integrate, mode, ev); break;
    case 2: launch_pair<16>(h, 2, integrate, mode, ev); break;
    default: launch_pair<32>(h, 3, integrate, mode, ev); break;
  }
  h->cur = 1 - h->cur;
  h->since_sort += 1;
}

void enqueue_integrate(sph_handle* h) {
  hipLaunchKernelGGL(sph_integrate, dim3(nblocks(h->N)), dim3(kBlock), 0, h->stream,
                     h->at<float2>(h->L.pos[h->cur]), h->at<float2>(h->L.vel[h->cur]),
                     h->at<float2>(h->L.acc[h->cur]), h->N, h->at<int>(h->L.owner), h->at<Tank>(h->L.tanks),
                     h->at<DevRigid>(h->L.rigid), h->at<unsigned>(h->L.status));
}

// Steps of a rollout with the rebuild schedule; the state is integrated on
// entry and on exit.
void enqueue_steps(sph_handle* h, int n_steps) {
  if (h->since_sort >= h->sort_every) enqueue_sort(h);   // overdue after a shorter interval was set
  for (int s = 0; s < n_steps; ++s) {
    enqueue_step(h, s > 0, kStep);
    if (h->since_sort >= h->sort_every) enqueue_sort(h);
  }
  enqueue_integrate(h);
}

// Full stable sort of raw fluid arrays (caller order) into buffers (cur, ord) = (0, 0).
int sort_fluid(sph_handle* h, const float2* s, const float2* w) {
  const int nb = nblocks(h->N);
  if (h->N > 0) {
    if (s != h->at<float2>(h->L.pos[1]))
      HIPCHK(hipMemcpyAsync(h->at<float2>(h->L.pos[1]), s, (size_t)h->N * 8, hipMemcpyDeviceToDevice, h->stream));
    if (w != h->at<float2>(h->L.vel[1]))
      HIPCHK(hipMemcpyAsync(h->at<float2>(h->L.vel[1]), w, (size_t)h->N * 8, hipMemcpyDeviceToDevice, h->stream));
    HIPCHK(hipMemsetAsync(h->at<float2>(h->L.acc[0]), 0, (size_t)h->N * 8, h->stream));
  }
  HIPCHK(hipMemsetAsync(h->at<int>(h->L.count), 0, (size_t)h->C * 4, h->stream));
  hipLaunchKernelGGL(sph_check, dim3(nb), dim3(kBlock), 0, h->stream, h->at<float2>(h->L.pos[1]),
                     h->at<float2>(h->L.vel[1]), h->N, h->at<int>(h->L.owner), h->at<Tank>(h->L.tanks),
                     h->at<unsigned>(h->L.status));
  hipLaunchKernelGGL(sph_bin, dim3(nb), dim3(kBlock), 0, h->stream, h->at<float2>(h->L.pos[1]), h->N,
                     h->at<int>(h->L.owner), h->at<Tank>(h->L.tanks), h->at<int>(h->L.key),
                     h->at<int>(h->L.count), h->at<int>(h->L.slot));
  enqueue_scan(h, h->at<int>(h->L.cstart[0]), 0, h->at<unsigned>(h->L.status));
  if (h->N > 0) {
    hipLaunchKernelGGL(sph_scatter, dim3(nb), dim3(kBlock), 0, h->stream, h->at<int>(h->L.key),
                       h->at<int>(h->L.slot), h->N, h->at<int>(h->L.cstart[0]), h->at<int>(h->L.order));
    hipLaunchKernelGGL(sph_cell_order, dim3(nblocks(h->C)), dim3(kBlock), 0, h->stream,
                       h->at<int>(h->L.cstart[0]), h->C, h->at<int>(h->L.order));
    hipLaunchKernelGGL(sph_gather, dim3(nb), dim3(kBlock), 0, h->stream, h->at<int>(h->L.order), h->N,
                       h->at<float2>(h->L.pos[1]), h->at<float2>(h->L.vel[1]), h->at<float2>(h->L.pos[0]),
                       h->at<float2>(h->L.vel[0]), h->at<int>(h->L.id[0]), h->at<float2>(h->L.pos_sort));
    hipLaunchKernelGGL(sph_ranges, dim3(nb), dim3(kBlock), 0, h->stream, h->at<float2>(h->L.pos_sort), h->N,
                       h->at<int>(h->L.owner), h->at<Tank>(h->L.tanks), h->at<int>(h->L.cstart[0]),
                       h->at<int>(h->L.gstart), h->at<int4>(h->L.rng), h->at<int>(h->L.pkey));
  }
  HIPCHK(hipGetLastError());
  h->cur = 0;
  h->ord = 0;
  h->since_sort = 0;
  h->near_valid = false;
  return SPH_OK;
}

int sort_ghosts(sph_handle* h, const float2* graw) {
  const int nb = nblocks(h->Gh);
  HIPCHK(hipMemsetAsync(h->at<int>(h->L.count), 0, (size_t)h->C * 4, h->stream));
  hipLaunchKernelGGL(sph_bin, dim3(nb), dim3(kBlock), 0, h->stream, graw, h->Gh, h->at<int>(h->L.gowner),
                     h->at<Tank>(h->L.tanks), h->at<int>(h->L.key), h->at<int>(h->L.count),
                     h->at<int>(h->L.slot));
  enqueue_scan(h, h->at<int>(h->L.gstart), 1, (unsigned*)nullptr);
  if (h->Gh > 0) {
    hipLaunchKernelGGL(sph_scatter, dim3(nb), dim3(kBlock), 0, h->stream, h->at<int>(h->L.key),
                       h->at<int>(h->L.slot), h->Gh, h->at<int>(h->L.gstart), h->at<int>(h->L.order));
    hipLaunchKernelGGL(sph_cell_order, dim3(nblocks(h->C)), dim3(kBlock), 0, h->stream,
                       h->at<int>(h->L.gstart), h->C, h->at<int>(h->L.order));
    hipLaunchKernelGGL(sph_gather, dim3(nb), dim3(kBlock), 0, h->stream, h->at<int>(h->L.order), h->Gh,
                       graw, (const float2*)nullptr, h->at<float2>(h->L.gpos), (float2*)nullptr, (int*)nullptr,
                       (float2*)nullptr);
  }
  HIPCHK(hipGetLastError());
  return SPH_OK;
}

int set_rigid(sph_handle* h, const double* rigid, double tau_ctrl, long long step) {
  std::vector<DevRigid> rs(h->T);
  for (int t = 0; t < h->T; ++t) {
    DevRigid& r = rs[t];
    memset(&r, 0, sizeof r);
    const double* g = rigid + 6 * t;
    r.r[0] = g[0];
    r.r[1] = g[1];
    r.theta = g[2];
    r.rdot[0] = g[3];
    r.rdot[1] = g[4];
    r.thetadot = g[5];
    r.tau_ctrl = tau_ctrl;
    r.step = step;
    r.step0 = step;
  }
  HIPCHK(hipMemcpyAsync(h->at<DevRigid>(h->L.rigid), rs.data(), sizeof(DevRigid) * h->T,
                        hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return SPH_OK;
}

int set_rollout(sph_handle* h, const float* u, const double* ref, int n_ref, int stride, long long n_steps,
                float* y, float* wl, float* ul, float* wm) {
  DevRollout v;
  memset(&v, 0, sizeof v);
  v.u = u;
  v.theta_ref = ref;
  v.n_ref = n_ref;
  v.log_stride = stride;
  v.n_steps = n_steps;
  v.n_log = stride > 0 ? (int)((n_steps + stride - 1) / stride) : 0;
  v.y_log = y;
  v.w_log = wl;
  v.u_log = ul;
  v.wm_log = wm;
  hipLaunchKernelGGL(sph_set_rollout, dim3(nblocks(h->T)), dim3(kBlock), 0, h->stream,
                     h->at<DevRollout>(h->L.rollout), v, h->at<DevRigid>(h->L.rigid), h->T);
  HIPCHK(hipGetLastError());
  return SPH_OK;
}

// Every tank fits the LDS-resident rollout.
bool resident_ok(const sph_handle* h) {
  for (const Tank& tk : h->plan.tanks)
    if (tk.n > kResMaxF || tk.ng > kResMaxG || (long long)tk.g2.ncx * tk.g2.ncy > kResMaxC) return false;
  static_assert(kResMaxF <= 65536 && kResMaxC <= 65536 && 2 * kResThreads >= kResMaxC, "resident sizes");
  return true;
}

// Captures kChunk steps starting from (cur, ord) with since_sort == 0 (the
// first captured step rebuilds the near lists, whatever their host state).
int build_graph(sph_handle* h) {
  const int c = h->cur, o = h->ord, v = h->variant, n = h->near ? 1 : 0;
  if (h->graph_ok[v][n][c][o]) return SPH_OK;
  const bool valid = h->near_valid;
  h->near_valid = false;
  hipGraph_t gr;
  HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  enqueue_steps(h, kChunk);
  hipError_t e = hipStreamEndCapture(h->stream, &gr);
  h->cur = c;   // the capture only recorded the launches
  h->ord = o;
  h->since_sort = 0;
  h->binned = false;
  h->near_valid = valid;
  if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
  e = hipGraphInstantiate(&h->graph[v][n][c][o], gr, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gr);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  h->graph_ok[v][n][c][o] = true;
  return SPH_OK;
}

// Host tables: tank of every particle, ghost and cell; the tiles of each variant.
int upload_tables(sph_handle* h) {
  const Plan& pl = h->plan;
  std::vector<int> owner((size_t)pl.N), gowner((size_t)pl.Gh), cowner((size_t)pl.C);
  for (int t = 0; t < pl.T; ++t) {
    const Tank& tk = pl.tanks[t];
    for (int i = 0; i < tk.n; ++i) owner[(size_t)tk.p0 + i] = t;
    for (int i = 0; i < tk.ng; ++i) gowner[(size_t)tk.q0 + i] = t;
    for (int i = 0; i < tk.nc; ++i) cowner[(size_t)tk.c0 + i] = t;
  }
  HIPCHK(hipMemcpyAsync(h->at<Tank>(h->L.tanks), pl.tanks.data(), sizeof(Tank) * pl.T, hipMemcpyHostToDevice,
                        h->stream));
  if (pl.N) HIPCHK(hipMemcpyAsync(h->at<int>(h->L.owner), owner.data(), 4 * pl.N, hipMemcpyHostToDevice, h->stream));
  if (pl.Gh)
    HIPCHK(hipMemcpyAsync(h->at<int>(h->L.gowner), gowner.data(), 4 * pl.Gh, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(h->at<int>(h->L.cowner), cowner.data(), 4 * pl.C, hipMemcpyHostToDevice, h->stream));
  for (int v = 0; v < kNumVariants; ++v) {
    const int tp = kBlock / kLanes[v];
    std::vector<TileRef> tiles;
    std::vector<int> tile0(pl.T + 1);
    tiles.reserve((size_t)pl.tiles[v]);
    for (int t = 0; t < pl.T; ++t) {
      const Tank& tk = pl.tanks[t];
      tile0[t] = (int)tiles.size();
      if (tk.n == 0) tiles.push_back(TileRef{t, tk.p0, 0, 0});
      for (int a = 0; a < tk.n; a += tp) tiles.push_back(TileRef{t, tk.p0 + a, tk.n - a < tp ? tk.n - a : tp, 0});
    }
    tile0[pl.T] = (int)tiles.size();
    HIPCHK(hipMemcpyAsync(h->at<TileRef>(h->L.tiles[v]), tiles.data(), sizeof(TileRef) * tiles.size(),
                          hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipMemcpyAsync(h->at<int>(h->L.tile0[v]), tile0.data(), 4 * tile0.size(), hipMemcpyHostToDevice,
                          h->stream));
  }
  HIPCHK(hipStreamSynchronize(h->stream));   // the host vectors die here
  return SPH_OK;
}

int init_common(int T, const sph_params* params, const int32_t* n_fluid, const float* s0_dev,
                const float* w0_dev, const int32_t* n_ghost, const float* g_dev, const double* rigid0,
                void* ws_dev, size_t ws_bytes, void* stream, sph_handle** out) {
  if (!out || !rigid0 || !ws_dev) return SPH_E_INVAL;
  if (reinterpret_cast<uintptr_t>(ws_dev) & 255) return SPH_E_INVAL;
  Plan pl;
  int rc = make_plan(T, params, n_fluid, n_ghost, &pl);
  if (rc) return rc;
  if ((pl.N > 0 && (!s0_dev || !w0_dev)) || (pl.Gh > 0 && !g_dev)) return SPH_E_INVAL;
  Layout L = make_layout(pl);
  if (ws_bytes < L.total) return SPH_E_CAPACITY;
  sph_handle* h = new (std::nothrow) sph_handle();
  if (!h) return SPH_E_INVAL;
  h->plan = pl;
  h->T = T;
  h->N = (int)pl.N;
  h->Gh = (int)pl.Gh;
  h->C = (int)pl.C;
  h->stream = reinterpret_cast<hipStream_t>(stream);
  h->ws = reinterpret_cast<char*>(ws_dev);
  h->L = L;
  h->cur = h->ord = h->since_sort = 0;
  h->sort_every = kSortEvery;
  h->binned = false;
  h->variant = kDefaultVariant;
  h->near = false;
  h->near_valid = false;
  for (int v = 0; v < kNumVariants; ++v)
    for (int n = 0; n < 2; ++n)
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) h->graph_ok[v][n][a][b] = false;
  auto fail = [&](int code) {
    delete h;
    return code;
  };
  hipError_t e = hipMemsetAsync(h->ws, 0, L.total, h->stream);
  if (e != hipSuccess) return fail(hip_fail(e, "hipMemsetAsync"));
  // no particle has a near list until the first step after a rebuild writes one
  e = hipMemsetAsync(h->ws + L.near_n, 0xff, (size_t)pl.N * 4, h->stream);
  if (e != hipSuccess) return fail(hip_fail(e, "hipMemsetAsync"));
  if ((rc = upload_tables(h)) != SPH_OK) return fail(rc);
  if ((rc = set_rigid(h, rigid0, 0.0, 0)) != SPH_OK) return fail(rc);
  if (pl.Gh > 0) {
    e = hipMemcpyAsync(h->at<float2>(L.graw), g_dev, (size_t)pl.Gh * 8, hipMemcpyDeviceToDevice, h->stream);
    if (e != hipSuccess) return fail(hip_fail(e, "hipMemcpyAsync"));
  }
  if ((rc = sort_ghosts(h, h->at<float2>(L.graw))) != SPH_OK) return fail(rc);
  if ((rc = sort_fluid(h, reinterpret_cast<const float2*>(s0_dev), reinterpret_cast<const float2*>(w0_dev))) !=
      SPH_OK)
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

}  // namespace

extern "C" {

int sph_batch_workspace_bytes(int32_t n_tanks, const sph_params* params, const int32_t* n_fluid,
                              const int32_t* n_ghost, size_t* bytes) {
  if (!bytes) return SPH_E_INVAL;
  Plan pl;
  int rc = make_plan(n_tanks, params, n_fluid, n_ghost, &pl);
  if (rc) return rc;
  *bytes = make_layout(pl).total;
  return SPH_OK;
}

int sph_workspace_bytes(const sph_params* p, int32_t n_fluid, int32_t n_ghost, size_t* bytes) {
  return sph_batch_workspace_bytes(1, p, &n_fluid, &n_ghost, bytes);
}

int sph_batch_init(int32_t n_tanks, const sph_params* params, const int32_t* n_fluid, const float* s0_dev,
                   const float* w0_dev, const int32_t* n_ghost, const float* g_dev, const double* rigid0,
                   void* ws_dev, size_t ws_bytes, void* stream, sph_handle** out) {
  return init_common(n_tanks, params, n_fluid, s0_dev, w0_dev, n_ghost, g_dev, rigid0, ws_dev, ws_bytes,
                     stream, out);
}

int sph_init(const sph_params* p, int32_t n_fluid, const float* s0_dev, const float* w0_dev,
             int32_t n_ghost, const float* g_dev, const double* rigid0, void* ws_dev,
             size_t ws_bytes, void* stream, sph_handle** out) {
  return init_common(1, p, &n_fluid, s0_dev, w0_dev, &n_ghost, g_dev, rigid0, ws_dev, ws_bytes, stream, out);
}

// Destroys every captured graph of the handle.
void drop_graphs(sph_handle* h) {
  for (int v = 0; v < kNumVariants; ++v)
    for (int n = 0; n < 2; ++n)
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
          if (h->graph_ok[v][n][a][b]) {
            (void)hipGraphExecDestroy(h->graph[v][n][a][b]);
            h->graph_ok[v][n][a][b] = false;
          }
}

int sph_destroy(sph_handle* h) {
  if (!h) return SPH_E_INVAL;
  drop_graphs(h);
  delete h;
  return SPH_OK;
}

int sph_rollout(sph_handle* h, int32_t n_steps, const float* u_seq_dev, const double* theta_ref_dev,
                int32_t n_ref, int32_t log_stride, float* y_log_dev, float* wrench_log_dev,
                float* u_log_dev, float* wmean_log_dev) {
  if (!h || n_steps < 0 || log_stride < 0 || n_ref < 0) return SPH_E_INVAL;
  if (n_steps == 0) return SPH_OK;
  int rc = set_rollout(h, u_seq_dev, theta_ref_dev, n_ref, log_stride, n_steps, y_log_dev, wrench_log_dev,
                       u_log_dev, wmean_log_dev);
  if (rc) return rc;
  if (!h->stream || n_steps < kChunk) {
    // no capturable stream, or too short for a graph: direct launches
    enqueue_steps(h, n_steps);
    HIPCHK(hipGetLastError());
    return SPH_OK;
  }
  int left = n_steps;
  // align to the rebuild schedule so that every graph starts right after a rebuild
  if (h->since_sort >= h->sort_every) enqueue_sort(h);   // overdue after a shorter interval was set
  int lead = (h->sort_every - h->since_sort) % h->sort_every;
  if (lead > 0) {
    enqueue_steps(h, lead);
    left -= lead;
  }
  while (left >= kChunk) {
    if ((rc = build_graph(h)) != SPH_OK) return rc;
    HIPCHK(hipGraphLaunch(h->graph[h->variant][h->near ? 1 : 0][h->cur][h->ord], h->stream));
    h->near_valid = false;   // the chunk ends with a rebuild
    left -= kChunk;
  }
  if (left > 0) enqueue_steps(h, left);
  HIPCHK(hipGetLastError());
  return SPH_OK;
}

int sph_resident_fits(sph_handle* h, int32_t* fits) {
  if (!h || !fits) return SPH_E_INVAL;
  *fits = resident_ok(h) ? 1 : 0;
  return SPH_OK;
}

int sph_rollout_resident(sph_handle* h, int32_t n_steps, const float* u_seq_dev, const double* theta_ref_dev,
                         int32_t n_ref, int32_t log_stride, float* y_log_dev, float* wrench_log_dev,
                         float* u_log_dev, float* wmean_log_dev) {
  if (!h || n_steps < 0 || log_stride < 0 || n_ref < 0) return SPH_E_INVAL;
  if (!resident_ok(h)) return SPH_E_CAPACITY;
  if (n_steps == 0) return SPH_OK;
  int rc = set_rollout(h, u_seq_dev, theta_ref_dev, n_ref, log_stride, n_steps, y_log_dev, wrench_log_dev,
                       u_log_dev, wmean_log_dev);
  if (rc) return rc;
  // the state of buffer `cur` is integrated between rollouts; the kernel
  // keeps each particle in its slot
  for (int s0 = 0; s0 < n_steps; s0 += kResChunk) {
    const int steps = n_steps - s0 < kResChunk ? n_steps - s0 : kResChunk;
    hipLaunchKernelGGL(sph_resident, dim3(h->T), dim3(kResThreads), 0, h->stream, h->at<float2>(h->L.pos[h->cur]),
                       h->at<float2>(h->L.vel[h->cur]), h->at<float2>(h->L.gpos), h->at<Tank>(h->L.tanks),
                       h->at<DevRigid>(h->L.rigid), h->at<DevRollout>(h->L.rollout), steps,
                       h->at<unsigned>(h->L.status));
  }
  HIPCHK(hipGetLastError());
  // particles may have crossed many cells of the multi-kernel path's list:
  // back to caller order in the other buffer, then the general sort
  const int c = h->cur, other = 1 - c;
  if (h->N > 0) {
    hipLaunchKernelGGL(sph_unpermute, dim3(nblocks(h->N)), dim3(kBlock), 0, h->stream,
                       h->at<float2>(h->L.pos[c]), h->at<int>(h->L.id[h->ord]), h->N, h->at<float2>(h->L.pos[other]));
    hipLaunchKernelGGL(sph_unpermute, dim3(nblocks(h->N)), dim3(kBlock), 0, h->stream,
                       h->at<float2>(h->L.vel[c]), h->at<int>(h->L.id[h->ord]), h->N, h->at<float2>(h->L.vel[other]));
  }
  h->binned = false;
  return sort_fluid(h, h->at<float2>(h->L.pos[other]), h->at<float2>(h->L.vel[other]));
}

int sph_time_kernels(sph_handle* h, int32_t n_steps, const float* u_seq_dev, const double* theta_ref_dev,
                     int32_t n_ref, float* avg_us) {
  if (!h || n_steps < 1 || !avg_us || n_ref < 0) return SPH_E_INVAL;
  int rc = set_rollout(h, u_seq_dev, theta_ref_dev, n_ref, 0, n_steps, nullptr, nullptr, nullptr, nullptr);
  if (rc) return rc;
  hipEvent_t ev[4];
  for (int i = 0; i < 4; ++i) HIPCHK(hipEventCreate(&ev[i]));
  double sum[6] = {0, 0, 0, 0, 0, 0};
  int sorts = 0;
  for (int st = 0; st < n_steps; ++st) {
    enqueue_step(h, st > 0, kStep, ev);
    HIPCHK(hipEventSynchronize(ev[3]));
    for (int k = 0; k < 3; ++k) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
      sum[3 + k] += ms;
    }
    if (h->since_sort >= h->sort_every) {
      enqueue_sort(h, ev);
      HIPCHK(hipEventSynchronize(ev[3]));
      for (int k = 0; k < 3; ++k) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, ev[k], ev[k + 1]));
        sum[k] += ms;
      }
      ++sorts;
    }
  }
  enqueue_integrate(h);
  HIPCHK(hipStreamSynchronize(h->stream));
  for (int i = 0; i < 4; ++i) (void)hipEventDestroy(ev[i]);
  for (int k = 0; k < 3; ++k) avg_us[k] = sorts ? (float)(sum[k] * 1000.0 / sorts) : 0.0f;
  for (int k = 3; k < 6; ++k) avg_us[k] = (float)(sum[k] * 1000.0 / n_steps);
  return SPH_OK;
}

int sph_autotune(sph_handle* h, int32_t reps, int32_t* lanes) {
  if (!h || reps < 1) return SPH_E_INVAL;
  int rc = set_rollout(h, nullptr, nullptr, 0, 0, 0, nullptr, nullptr, nullptr, nullptr);
  if (rc) return rc;
  hipEvent_t ev[4];
  for (int i = 0; i < 4; ++i) HIPCHK(hipEventCreate(&ev[i]));
  enqueue_sort(h);
  int best = kDefaultVariant;
  bool best_near = false;
  double best_ms = 1e300;
  const int cur = h->cur, ord = h->ord;
  for (int v = 0; v < kNumVariants; ++v)
    for (int nr = 0; nr < 2; ++nr) {
      h->variant = v;
      h->near = nr != 0;
      double total = 0.0;
      for (int r = 0; r <= reps; ++r) {   // the first round warms up
        // one rebuild interval: with near lists, its first step builds them
        h->near_valid = false;
        float ms = 0.f;
        for (int k = 0; k < h->sort_every; ++k) {
          h->cur = cur;
          h->ord = ord;
          enqueue_step(h, false, kEval, ev);
          HIPCHK(hipEventSynchronize(ev[3]));
          float t = 0.f;
          HIPCHK(hipEventElapsedTime(&t, ev[0], ev[3]));
          ms += t;
        }
        if (r > 0) total += ms;
      }
      if (total < best_ms) {
        best_ms = total;
        best = v;
        best_near = nr != 0;
      }
    }
  for (int i = 0; i < 4; ++i) (void)hipEventDestroy(ev[i]);
  // evaluation only: the state is what it was after the rebuild
  h->cur = 1 - cur;
  h->ord = ord;
  h->since_sort = 0;
  h->variant = best;
  h->near = best_near;
  h->near_valid = false;
  if (lanes) *lanes = kLanes[best];
  return SPH_OK;
}

int sph_set_lanes(sph_handle* h, int32_t lanes) {
  if (!h) return SPH_E_INVAL;
  for (int v = 0; v < kNumVariants; ++v)
    if (kLanes[v] == lanes) {
      h->variant = v;
      return SPH_OK;
    }
  return SPH_E_INVAL;
}

int sph_set_near_lists(sph_handle* h, int32_t on) {
  if (!h || (on != 0 && on != 1)) return SPH_E_INVAL;
  if (h->near != (on != 0)) h->near_valid = false;
  h->near = on != 0;
  return SPH_OK;
}

int sph_set_rebuild_interval(sph_handle* h, int32_t steps) {
  if (!h || steps < 1 || steps > kChunk || kChunk % steps != 0) return SPH_E_INVAL;
  if (steps != h->sort_every) drop_graphs(h);   // the graphs hold the old schedule
  h->sort_every = steps;
  return SPH_OK;
}

int sph_get_rebuild_interval(sph_handle* h, int32_t* steps) {
  if (!h || !steps) return SPH_E_INVAL;
  *steps = h->sort_every;
  return SPH_OK;
}

int sph_get_tuning(sph_handle* h, int32_t* lanes, int32_t* near_lists) {
  if (!h) return SPH_E_INVAL;
  if (lanes) *lanes = kLanes[h->variant];
  if (near_lists) *near_lists = h->near ? 1 : 0;
  return SPH_OK;
}

int sph_step(sph_handle* h, const float* u_dev) {
  return sph_rollout(h, 1, u_dev, nullptr, 0, 0, nullptr, nullptr, nullptr, nullptr);
}

int sph_rhs(sph_handle* h, const float* u_dev, float* rho_dev, float* p_dev, float* a_sph_dev, float* wdot_dev,
            float* wrench_dev, float* acc_dev) {
  if (!h) return SPH_E_INVAL;
  int rc = set_rollout(h, u_dev, nullptr, 0, 0, 0, nullptr, nullptr, nullptr, nullptr);
  if (rc) return rc;
  // the cell list and near lists of the last rebuild stay valid until the
  // next scheduled one (the displacement check still runs)
  if (h->since_sort >= h->sort_every) enqueue_sort(h);
  const int since = h->since_sort;
  enqueue_step(h, false, kEval);
  h->since_sort = since;   // evaluation only: the positions did not move
  hipLaunchKernelGGL(sph_rhs_out, dim3(nblocks(h->N)), dim3(kBlock), 0, h->stream,
                     h->at<float2>(h->L.pos[h->cur]), h->at<float2>(h->L.vel[h->cur]),
                     h->at<float2>(h->L.acc[h->cur]), h->at<float2>(h->L.rp), h->at<int>(h->L.id[h->ord]), h->N,
                     h->at<int>(h->L.owner), h->at<Tank>(h->L.tanks), h->at<DevRigid>(h->L.rigid), rho_dev, p_dev,
                     reinterpret_cast<float2*>(a_sph_dev), reinterpret_cast<float2*>(wdot_dev));
  hipLaunchKernelGGL(sph_small_out, dim3(nblocks(h->T)), dim3(kBlock), 0, h->stream, h->at<DevRigid>(h->L.rigid),
                     h->T, wrench_dev, acc_dev, (int)SPH_FRAME_BODY);
  HIPCHK(hipGetLastError());
  return SPH_OK;
}

int sph_slosh_wrench(sph_handle* h, int32_t frame, float* out_dev) {
  if (!h || !out_dev || (frame != SPH_FRAME_BODY && frame != SPH_FRAME_WORLD)) return SPH_E_INVAL;
  hipLaunchKernelGGL(sph_small_out, dim3(nblocks(h->T)), dim3(kBlock), 0, h->stream, h->at<DevRigid>(h->L.rigid),
                     h->T, out_dev, (float*)nullptr, (int)frame);
  HIPCHK(hipGetLastError());
  return SPH_OK;
}

int sph_get_state(sph_handle* h, float* s_dev, float* w_dev, double* rigid, double* tau_ctrl, int64_t* step) {
  if (!h) return SPH_E_INVAL;
  const int nb = nblocks(h->N);
  if (s_dev && h->N > 0)
    hipLaunchKernelGGL(sph_unpermute, dim3(nb), dim3(kBlock), 0, h->stream, h->at<float2>(h->L.pos[h->cur]),
                       h->at<int>(h->L.id[h->ord]), h->N, reinterpret_cast<float2*>(s_dev));
  if (w_dev && h->N > 0)
    hipLaunchKernelGGL(sph_unpermute, dim3(nb), dim3(kBlock), 0, h->stream, h->at<float2>(h->L.vel[h->cur]),
                       h->at<int>(h->L.id[h->ord]), h->N, reinterpret_cast<float2*>(w_dev));
  HIPCHK(hipGetLastError());
  std::vector<DevRigid> rs(h->T);
  HIPCHK(hipMemcpyAsync(rs.data(), h->at<DevRigid>(h->L.rigid), sizeof(DevRigid) * h->T, hipMemcpyDeviceToHost,
                        h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  for (int t = 0; t < h->T; ++t) {
    const DevRigid& r = rs[t];
    if (rigid) {
      double* g = rigid + 6 * t;
      g[0] = r.r[0];
      g[1] = r.r[1];
      g[2] = r.theta;
      g[3] = r.rdot[0];
      g[4] = r.rdot[1];
      g[5] = r.thetadot;
    }
    if (tau_ctrl) tau_ctrl[t] = r.tau_ctrl;
    if (step) step[t] = r.step;
  }
  return SPH_OK;
}

int sph_set_state(sph_handle* h, const float* s_dev, const float* w_dev, const double* rigid, double tau_ctrl,
                  int64_t step) {
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
  enqueue_sort(h);
  const int v = h->variant;
  const int nt = (int)h->plan.tiles[v];
  auto args = [&](auto kern) {
    hipLaunchKernelGGL(kern, dim3(nt), dim3(kBlock), 0, h->stream, h->at<float2>(h->L.pos[h->cur]),
                       h->at<int>(h->L.pkey), h->at<int4>(h->L.rng), h->at<int>(h->L.id[h->ord]),
                       h->at<TileRef>(h->L.tiles[v]), single_n(h), h->at<Tank>(h->L.tanks), max_nbr, nbr_dev,
                       count_dev);
  };
  if (v == 0) args(sph_nbr_list<4>);
  else if (v == 1) args(sph_nbr_list<8>);
  else if (v == 2) args(sph_nbr_list<16>);
  else args(sph_nbr_list<32>);
  HIPCHK(hipGetLastError());
  return SPH_OK;
}

int sph_num_tanks(sph_handle* h, int32_t* n_tanks) {
  if (!h || !n_tanks) return SPH_E_INVAL;
  *n_tanks = h->T;
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

// ---- tangent-linear rollout: workspace layout and the C entry points ----

namespace {

struct JvpLayout {
  size_t s, w, ds, dw, rp, drp, a, da, key, slot, order, count, cstart, part, dpart, st, tst, frame, tframe, wout,
      twout, total;
  int nb;
};

JvpLayout jvp_layout(const sph_handle* h, int n_dir) {
  JvpLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes > 0 ? bytes : 1);
    return at;
  };
  const size_t n = (size_t)h->N, K = (size_t)n_dir, C = (size_t)h->C;
  L.nb = nblocks(h->N);
  L.s = take(n * 8);
  L.w = take(n * 8);
  L.ds = take(K * n * 8);
  L.dw = take(K * n * 8);
  L.rp = take(n * 8);
  L.drp = take(K * n * 8);
  L.a = take(n * 8);
  L.da = take(K * n * 8);
  L.key = take(n * 4);
  L.slot = take(n * 4);
  L.order = take(n * 4);
  L.count = take(C * 4);
  L.cstart = take((C + 1) * 4);
  L.part = take((size_t)L.nb * 3 * 8);
  L.dpart = take((size_t)L.nb * K * 3 * 8);
  L.st = take(sizeof(JvpRigid));
  L.tst = take(K * kJvpRigidT * 8);
  L.frame = take(16);
  L.tframe = take(K * 16);
  L.wout = take(3 * 8);
  L.twout = take(K * 3 * 8);
  L.total = o;
  return L;
}

template <int KC>
void jvp_chunks(sph_handle* h, const JvpLayout& L, char* ws, int n_dir) {
  auto at = [&](size_t off) { return reinterpret_cast<void*>(ws + off); };
  const int nb = L.nb;
  for (int k0 = 0; k0 < n_dir; k0 += KC)
    hipLaunchKernelGGL(jvp_density<KC>, dim3(nb), dim3(kBlock), 0, h->stream, (const float2*)at(L.s),
                       (const float2*)at(L.ds), h->N, n_dir, k0, (const int*)at(L.order), (const int*)at(L.cstart),
                       h->at<float2>(h->L.gpos), h->at<int>(h->L.gstart), h->at<Tank>(h->L.tanks),
                       (float2*)at(L.rp), (float2*)at(L.drp));
  for (int k0 = 0; k0 < n_dir; k0 += KC)
    hipLaunchKernelGGL(jvp_force<KC>, dim3(nb), dim3(kBlock), 0, h->stream, (const float2*)at(L.s),
                       (const float2*)at(L.w), (const float2*)at(L.rp), (const float2*)at(L.ds),
                       (const float2*)at(L.dw), (const float2*)at(L.drp), h->N, n_dir, k0, (const int*)at(L.order),
                       (const int*)at(L.cstart), h->at<float2>(h->L.gpos), h->at<int>(h->L.gstart),
                       h->at<Tank>(h->L.tanks), (float2*)at(L.a), (float2*)at(L.da), (double*)at(L.part),
                       (double*)at(L.dpart));
}

}  // namespace

extern "C" {

int sph_jvp_workspace_bytes(sph_handle* h, int32_t n_dir, size_t* bytes) {
  if (!h || !bytes || n_dir < 1 || n_dir > kJvpMaxDir) return SPH_E_INVAL;
  *bytes = jvp_layout(h, n_dir).total;
  return SPH_OK;
}

int sph_jvp_rollout(sph_handle* h, int32_t n_dir, int32_t n_steps, const float* u_seq_dev, const float* du_seq_dev,
                    const double* theta_ref_dev, int32_t n_ref, const double* drigid0, const float* ds0_dev,
                    const float* dw0_dev, void* ws_dev, size_t ws_bytes, double* wrench, double* dwrench,
                    double* rigid, double* drigid, float* ds_dev, float* dw_dev) {
  if (!h || h->T != 1 || n_dir < 1 || n_dir > kJvpMaxDir || n_steps < 1 || n_ref < 0 || !ws_dev) return SPH_E_INVAL;
  if ((ds0_dev == nullptr) != (dw0_dev == nullptr)) return SPH_E_INVAL;
  const JvpLayout L = jvp_layout(h, n_dir);
  if (ws_bytes < L.total || (reinterpret_cast<uintptr_t>(ws_dev) & 255)) return SPH_E_INVAL;
  char* ws = reinterpret_cast<char*>(ws_dev);
  auto at = [&](size_t off) { return reinterpret_cast<void*>(ws + off); };
  const int n = h->N, nb = L.nb;
  const size_t tb = (size_t)n_dir * n * 8;
  // the handle's state in caller order; rigid primal from the handle
  if (n > 0) {
    hipLaunchKernelGGL(sph_unpermute, dim3(nb), dim3(kBlock), 0, h->stream, h->at<float2>(h->L.pos[h->cur]),
                       h->at<int>(h->L.id[h->ord]), n, (float2*)at(L.s));
    hipLaunchKernelGGL(sph_unpermute, dim3(nb), dim3(kBlock), 0, h->stream, h->at<float2>(h->L.vel[h->cur]),
                       h->at<int>(h->L.id[h->ord]), n, (float2*)at(L.w));
    if (ds0_dev) {
      HIPCHK(hipMemcpyAsync(at(L.ds), ds0_dev, tb, hipMemcpyDeviceToDevice, h->stream));
      HIPCHK(hipMemcpyAsync(at(L.dw), dw0_dev, tb, hipMemcpyDeviceToDevice, h->stream));
    } else {
      HIPCHK(hipMemsetAsync(at(L.ds), 0, tb, h->stream));
      HIPCHK(hipMemsetAsync(at(L.dw), 0, tb, h->stream));
    }
  }
  DevRigid dr;
  HIPCHK(hipMemcpyAsync(&dr, h->at<DevRigid>(h->L.rigid), sizeof dr, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  JvpRigid js;
  js.r[0] = dr.r[0];
  js.r[1] = dr.r[1];
  js.th = dr.theta;
  js.rd[0] = dr.rdot[0];
  js.rd[1] = dr.rdot[1];
  js.thd = dr.thetadot;
  js.tau = dr.tau_ctrl;
  js.step = dr.step;
  js.step0 = dr.step;
  std::vector<double> tst((size_t)n_dir * kJvpRigidT, 0.0);
  if (drigid0)
    for (int c = 0; c < n_dir; ++c)
      for (int q = 0; q < 6; ++q) tst[(size_t)c * kJvpRigidT + q] = drigid0[6 * c + q];
  HIPCHK(hipMemcpyAsync(at(L.st), &js, sizeof js, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(at(L.tst), tst.data(), tst.size() * 8, hipMemcpyHostToDevice, h->stream));
  const float dt = (float)h->plan.tanks[0].ra.dt;
  for (int stp = 0; stp < n_steps; ++stp) {
    // cell index of the current positions: keys, counts, starts, stable order
    HIPCHK(hipMemsetAsync(at(L.count), 0, (size_t)h->C * 4, h->stream));
    if (n > 0) {
      hipLaunchKernelGGL(sph_bin, dim3(nb), dim3(kBlock), 0, h->stream, (const float2*)at(L.s), n,
                         h->at<int>(h->L.owner), h->at<Tank>(h->L.tanks), (int*)at(L.key), (int*)at(L.count),
                         (int*)at(L.slot));
    }
    hipLaunchKernelGGL(sph_scan, dim3(1), dim3(kScanThreads), 0, h->stream, (int*)at(L.count), h->at<Tank>(h->L.tanks),
                       1, 0, (int*)at(L.cstart), h->at<unsigned>(h->L.status));
    if (n > 0) {
      hipLaunchKernelGGL(sph_scatter, dim3(nb), dim3(kBlock), 0, h->stream, (const int*)at(L.key),
                         (const int*)at(L.slot), n, (const int*)at(L.cstart), (int*)at(L.order));
      hipLaunchKernelGGL(sph_cell_order, dim3(nblocks(h->C)), dim3(kBlock), 0, h->stream, (const int*)at(L.cstart),
                         h->C, (int*)at(L.order));
    }
    jvp_chunks<kJvpChunk>(h, L, ws, n_dir);
    hipLaunchKernelGGL(jvp_rigid, dim3(1), dim3(kBlock), 0, h->stream, (const double*)at(L.part),
                       (const double*)at(L.dpart), nb, n_dir, h->at<Tank>(h->L.tanks), (JvpRigid*)at(L.st),
                       (double*)at(L.tst), u_seq_dev, du_seq_dev, (long long)n_steps, theta_ref_dev, n_ref,
                       (float4*)at(L.frame), (float4*)at(L.tframe), (double*)at(L.wout), (double*)at(L.twout));
    if (n > 0)
      hipLaunchKernelGGL(jvp_update, dim3(nb), dim3(kBlock), 0, h->stream, (float2*)at(L.s), (float2*)at(L.w),
                         (const float2*)at(L.a), (float2*)at(L.ds), (float2*)at(L.dw), (const float2*)at(L.da), n,
                         n_dir, (const float4*)at(L.frame), (const float4*)at(L.tframe), dt);
    HIPCHK(hipGetLastError());
  }
  if (ds_dev && n > 0) HIPCHK(hipMemcpyAsync(ds_dev, at(L.ds), tb, hipMemcpyDeviceToDevice, h->stream));
  if (dw_dev && n > 0) HIPCHK(hipMemcpyAsync(dw_dev, at(L.dw), tb, hipMemcpyDeviceToDevice, h->stream));
  std::vector<double> wo(3), two((size_t)n_dir * 3);
  HIPCHK(hipMemcpyAsync(wo.data(), at(L.wout), 24, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(two.data(), at(L.twout), two.size() * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(&js, at(L.st), sizeof js, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(tst.data(), at(L.tst), tst.size() * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (wrench)
    for (int d = 0; d < 3; ++d) wrench[d] = wo[d];
  if (dwrench)
    for (size_t q = 0; q < two.size(); ++q) dwrench[q] = two[q];
  if (rigid) {
    rigid[0] = js.r[0];
    rigid[1] = js.r[1];
    rigid[2] = js.th;
    rigid[3] = js.rd[0];
    rigid[4] = js.rd[1];
    rigid[5] = js.thd;
  }
  if (drigid)
    for (int c = 0; c < n_dir; ++c)
      for (int q = 0; q < 6; ++q) drigid[6 * c + q] = tst[(size_t)c * kJvpRigidT + q];
  return SPH_OK;
}

}  // extern "C"

// ---- adjoint rollout: workspace layout and the C entry points ----

namespace {

struct VjpLayout {
  JvpLayout P;   // primal working arrays (no directions)
  size_t ck_s, ck_w, ck_st, seg_s, seg_w, seg_st, st_prev, sb, wb, ab, rhob, fpart, rb, fb, wbar, total;
  int n_ck, every;
};

VjpLayout vjp_layout(const sph_handle* h, int n_steps, int every) {
  VjpLayout V;
  V.P = jvp_layout(h, 0);
  size_t o = V.P.total;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes > 0 ? bytes : 1);
    return at;
  };
  const size_t n = (size_t)h->N;
  V.every = every;
  V.n_ck = (n_steps + every - 1) / every;
  V.ck_s = take((size_t)V.n_ck * n * 8);
  V.ck_w = take((size_t)V.n_ck * n * 8);
  V.ck_st = take((size_t)V.n_ck * sizeof(JvpRigid));
  V.seg_s = take((size_t)every * n * 8);
  V.seg_w = take((size_t)every * n * 8);
  V.seg_st = take((size_t)every * sizeof(JvpRigid));
  V.st_prev = take(sizeof(JvpRigid));
  V.sb = take(n * 8);
  V.wb = take(n * 8);
  V.ab = take(n * 8);
  V.rhob = take(n * 4);
  V.fpart = take((size_t)V.P.nb * 4 * 8);
  V.rb = take(kJvpRigidT * 8);
  V.fb = take(3 * 8);
  V.wbar = take(3 * 8);
  V.total = o;
  return V;
}

// One primal step of the derivative rollouts (caller order): cell index,
// density, forces, rigid body (advances the rigid state, writes the frame
// and the wrench), and, if `update`, the fluid update.
int derivative_primal_step(sph_handle* h, const JvpLayout& L, char* ws, const float* u, int n_steps,
                           const double* ref, int n_ref, bool update) {
  auto at = [&](size_t off) { return reinterpret_cast<void*>(ws + off); };
  const int n = h->N, nb = L.nb;
  HIPCHK(hipMemsetAsync(at(L.count), 0, (size_t)h->C * 4, h->stream));
  if (n > 0)
    hipLaunchKernelGGL(sph_bin, dim3(nb), dim3(kBlock), 0, h->stream, (const float2*)at(L.s), n, h->at<int>(h->L.owner),
                       h->at<Tank>(h->L.tanks), (int*)at(L.key), (int*)at(L.count), (int*)at(L.slot));
  hipLaunchKernelGGL(sph_scan, dim3(1), dim3(kScanThreads), 0, h->stream, (int*)at(L.count), h->at<Tank>(h->L.tanks), 1,
                     0, (int*)at(L.cstart), h->at<unsigned>(h->L.status));
  if (n > 0) {
    hipLaunchKernelGGL(sph_scatter, dim3(nb), dim3(kBlock), 0, h->stream, (const int*)at(L.key),
                       (const int*)at(L.slot), n, (const int*)at(L.cstart), (int*)at(L.order));
    hipLaunchKernelGGL(sph_cell_order, dim3(nblocks(h->C)), dim3(kBlock), 0, h->stream, (const int*)at(L.cstart), h->C,
                       (int*)at(L.order));
  }
  hipLaunchKernelGGL(jvp_density<1>, dim3(nb), dim3(kBlock), 0, h->stream, (const float2*)at(L.s), (const float2*)nullptr,
                     n, 0, 0, (const int*)at(L.order), (const int*)at(L.cstart), h->at<float2>(h->L.gpos),
                     h->at<int>(h->L.gstart), h->at<Tank>(h->L.tanks), (float2*)at(L.rp), (float2*)nullptr);
  hipLaunchKernelGGL(jvp_force<1>, dim3(nb), dim3(kBlock), 0, h->stream, (const float2*)at(L.s), (const float2*)at(L.w),
                     (const float2*)at(L.rp), (const float2*)nullptr, (const float2*)nullptr, (const float2*)nullptr,
                     n, 0, 0, (const int*)at(L.order), (const int*)at(L.cstart), h->at<float2>(h->L.gpos),
                     h->at<int>(h->L.gstart), h->at<Tank>(h->L.tanks), (float2*)at(L.a), (float2*)nullptr,
                     (double*)at(L.part), (double*)nullptr);
  hipLaunchKernelGGL(jvp_rigid, dim3(1), dim3(kBlock), 0, h->stream, (const double*)at(L.part), (const double*)nullptr,
                     nb, 0, h->at<Tank>(h->L.tanks), (JvpRigid*)at(L.st), (double*)nullptr, u, (const float*)nullptr,
                     (long long)n_steps, ref, n_ref, (float4*)at(L.frame), (float4*)nullptr, (double*)at(L.wout),
                     (double*)nullptr);
  if (update && n > 0)
    hipLaunchKernelGGL(jvp_update, dim3(nb), dim3(kBlock), 0, h->stream, (float2*)at(L.s), (float2*)at(L.w),
                       (const float2*)at(L.a), (float2*)nullptr, (float2*)nullptr, (const float2*)nullptr, n, 0,
                       (const float4*)at(L.frame), (const float4*)nullptr, (float)h->plan.tanks[0].ra.dt);
  HIPCHK(hipGetLastError());
  return SPH_OK;
}

// The handle's state into the derivative rollouts' primal arrays.
int derivative_start(sph_handle* h, const JvpLayout& L, char* ws) {
  auto at = [&](size_t off) { return reinterpret_cast<void*>(ws + off); };
  const int n = h->N, nb = L.nb;
  if (n > 0) {
    hipLaunchKernelGGL(sph_unpermute, dim3(nb), dim3(kBlock), 0, h->stream, h->at<float2>(h->L.pos[h->cur]),
                       h->at<int>(h->L.id[h->ord]), n, (float2*)at(L.s));
    hipLaunchKernelGGL(sph_unpermute, dim3(nb), dim3(kBlock), 0, h->stream, h->at<float2>(h->L.vel[h->cur]),
                       h->at<int>(h->L.id[h->ord]), n, (float2*)at(L.w));
  }
  DevRigid dr;
  HIPCHK(hipMemcpyAsync(&dr, h->at<DevRigid>(h->L.rigid), sizeof dr, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  JvpRigid js;
  js.r[0] = dr.r[0];
  js.r[1] = dr.r[1];
  js.th = dr.theta;
  js.rd[0] = dr.rdot[0];
  js.rd[1] = dr.rdot[1];
  js.thd = dr.thetadot;
  js.tau = dr.tau_ctrl;
  js.step = dr.step;
  js.step0 = dr.step;
  HIPCHK(hipMemcpyAsync(at(L.st), &js, sizeof js, hipMemcpyHostToDevice, h->stream));
  return SPH_OK;
}

}  // namespace

extern "C" {

int sph_vjp_workspace_bytes(sph_handle* h, int32_t n_steps, int32_t every, size_t* bytes) {
  if (!h || !bytes || n_steps < 1 || every < 1) return SPH_E_INVAL;
  *bytes = vjp_layout(h, n_steps, every).total;
  return SPH_OK;
}

int sph_vjp_rollout(sph_handle* h, int32_t n_steps, int32_t every, const float* u_seq_dev,
                    const double* theta_ref_dev, int32_t n_ref, const double* wbar, const double* rbar,
                    const float* sbar_dev, const float* wbar_dev, void* ws_dev, size_t ws_bytes, double* wrench,
                    double* grad_rigid0, float* grad_u_dev, float* grad_s0_dev, float* grad_w0_dev) {
  if (!h || h->T != 1 || n_steps < 1 || every < 1 || n_ref < 0 || !ws_dev || !wbar) return SPH_E_INVAL;
  if ((sbar_dev == nullptr) != (wbar_dev == nullptr)) return SPH_E_INVAL;
  const VjpLayout V = vjp_layout(h, n_steps, every);
  if (ws_bytes < V.total || (reinterpret_cast<uintptr_t>(ws_dev) & 255)) return SPH_E_INVAL;
  const JvpLayout& L = V.P;
  char* ws = reinterpret_cast<char*>(ws_dev);
  auto at = [&](size_t off) { return reinterpret_cast<void*>(ws + off); };
  const int n = h->N, nb = L.nb;
  const size_t fb_bytes = (size_t)n * 8;
  int rc = derivative_start(h, L, ws);
  if (rc) return rc;
  // forward sweep, keeping the state every `every` steps
  for (int k = 0; k < n_steps; ++k) {
    if (k % every == 0) {
      const int c = k / every;
      if (n > 0) {
        HIPCHK(hipMemcpyAsync(ws + V.ck_s + c * fb_bytes, at(L.s), fb_bytes, hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(ws + V.ck_w + c * fb_bytes, at(L.w), fb_bytes, hipMemcpyDeviceToDevice, h->stream));
      }
      HIPCHK(hipMemcpyAsync(ws + V.ck_st + c * sizeof(JvpRigid), at(L.st), sizeof(JvpRigid), hipMemcpyDeviceToDevice,
                            h->stream));
    }
    if ((rc = derivative_primal_step(h, L, ws, u_seq_dev, n_steps, theta_ref_dev, n_ref, true)) != SPH_OK) return rc;
  }
  std::vector<double> wo(3);
  HIPCHK(hipMemcpyAsync(wo.data(), at(L.wout), 24, hipMemcpyDeviceToHost, h->stream));
  // adjoints of the outputs
  double r7[kJvpRigidT] = {0, 0, 0, 0, 0, 0, 0};
  if (rbar)
    for (int q = 0; q < 6; ++q) r7[q] = rbar[q];
  HIPCHK(hipMemcpyAsync(at(V.rb), r7, sizeof r7, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(at(V.wbar), wbar, 24, hipMemcpyHostToDevice, h->stream));
  if (n > 0) {
    if (sbar_dev) {
      HIPCHK(hipMemcpyAsync(at(V.sb), sbar_dev, fb_bytes, hipMemcpyDeviceToDevice, h->stream));
      HIPCHK(hipMemcpyAsync(at(V.wb), wbar_dev, fb_bytes, hipMemcpyDeviceToDevice, h->stream));
    } else {
      HIPCHK(hipMemsetAsync(at(V.sb), 0, fb_bytes, h->stream));
      HIPCHK(hipMemsetAsync(at(V.wb), 0, fb_bytes, h->stream));
    }
  }
  // reverse sweep, one segment at a time: recompute its states, then reverse its steps
  for (int c = V.n_ck - 1; c >= 0; --c) {
    const int k0 = c * every, k1 = std::min(n_steps, k0 + every);
    if (n > 0) {
      HIPCHK(hipMemcpyAsync(at(L.s), ws + V.ck_s + c * fb_bytes, fb_bytes, hipMemcpyDeviceToDevice, h->stream));
      HIPCHK(hipMemcpyAsync(at(L.w), ws + V.ck_w + c * fb_bytes, fb_bytes, hipMemcpyDeviceToDevice, h->stream));
    }
    HIPCHK(hipMemcpyAsync(at(L.st), ws + V.ck_st + c * sizeof(JvpRigid), sizeof(JvpRigid), hipMemcpyDeviceToDevice,
                          h->stream));
    for (int k = k0; k < k1; ++k) {
      const int q = k - k0;
      if (n > 0) {
        HIPCHK(hipMemcpyAsync(ws + V.seg_s + q * fb_bytes, at(L.s), fb_bytes, hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(ws + V.seg_w + q * fb_bytes, at(L.w), fb_bytes, hipMemcpyDeviceToDevice, h->stream));
      }
      HIPCHK(hipMemcpyAsync(ws + V.seg_st + q * sizeof(JvpRigid), at(L.st), sizeof(JvpRigid), hipMemcpyDeviceToDevice,
                            h->stream));
      if (k + 1 < k1 &&
          (rc = derivative_primal_step(h, L, ws, u_seq_dev, n_steps, theta_ref_dev, n_ref, true)) != SPH_OK)
        return rc;
    }
    for (int k = k1 - 1; k >= k0; --k) {
      const int q = k - k0;
      if (n > 0) {
        HIPCHK(hipMemcpyAsync(at(L.s), ws + V.seg_s + q * fb_bytes, fb_bytes, hipMemcpyDeviceToDevice, h->stream));
        HIPCHK(hipMemcpyAsync(at(L.w), ws + V.seg_w + q * fb_bytes, fb_bytes, hipMemcpyDeviceToDevice, h->stream));
      }
      HIPCHK(hipMemcpyAsync(at(L.st), ws + V.seg_st + q * sizeof(JvpRigid), sizeof(JvpRigid),
                            hipMemcpyDeviceToDevice, h->stream));
      HIPCHK(hipMemcpyAsync(at(V.st_prev), at(L.st), sizeof(JvpRigid), hipMemcpyDeviceToDevice, h->stream));
      // the step's primal: index, density, forces, wrench, frame (no update)
      if ((rc = derivative_primal_step(h, L, ws, u_seq_dev, n_steps, theta_ref_dev, n_ref, false)) != SPH_OK)
        return rc;
      if (n > 0)
        hipLaunchKernelGGL(vjp_update, dim3(nb), dim3(kBlock), 0, h->stream, (const float2*)at(L.s),
                           (const float2*)at(L.w), (float2*)at(V.sb), (float2*)at(V.wb), (float2*)at(V.ab), n,
                           (const float4*)at(L.frame), (float)h->plan.tanks[0].ra.dt, (double*)at(V.fpart));
      else
        HIPCHK(hipMemsetAsync(at(V.fpart), 0, (size_t)nb * 4 * 8, h->stream));
      hipLaunchKernelGGL(vjp_rigid, dim3(1), dim3(64), 0, h->stream, (const double*)at(V.fpart), nb,
                         h->at<Tank>(h->L.tanks), (const JvpRigid*)at(V.st_prev), (const double*)at(L.wout),
                         u_seq_dev, (long long)n_steps, theta_ref_dev, n_ref, (double*)at(V.rb), (double*)at(V.fb),
                         grad_u_dev, (const double*)at(V.wbar), k == n_steps - 1 ? 1 : 0);
      if (n > 0) {
        hipLaunchKernelGGL(vjp_force, dim3(nb), dim3(kBlock), 0, h->stream, (const float2*)at(L.s),
                           (const float2*)at(L.w), (const float2*)at(L.rp), (const float2*)at(V.ab),
                           (const double*)at(V.fb), n, (const int*)at(L.order), (const int*)at(L.cstart),
                           h->at<float2>(h->L.gpos), h->at<int>(h->L.gstart), h->at<Tank>(h->L.tanks),
                           (float2*)at(V.sb), (float2*)at(V.wb), (float*)at(V.rhob));
        hipLaunchKernelGGL(vjp_density, dim3(nb), dim3(kBlock), 0, h->stream, (const float2*)at(L.s),
                           (const float*)at(V.rhob), n, (const int*)at(L.order), (const int*)at(L.cstart),
                           h->at<float2>(h->L.gpos), h->at<int>(h->L.gstart), h->at<Tank>(h->L.tanks),
                           (float2*)at(V.sb));
      }
      HIPCHK(hipGetLastError());
    }
  }
  if (grad_s0_dev && n > 0)
    HIPCHK(hipMemcpyAsync(grad_s0_dev, at(V.sb), fb_bytes, hipMemcpyDeviceToDevice, h->stream));
  if (grad_w0_dev && n > 0)
    HIPCHK(hipMemcpyAsync(grad_w0_dev, at(V.wb), fb_bytes, hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(hipMemcpyAsync(r7, at(V.rb), sizeof r7, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (wrench)
    for (int d = 0; d < 3; ++d) wrench[d] = wo[d];
  if (grad_rigid0)
    for (int q = 0; q < 6; ++q) grad_rigid0[q] = r7[q];
  return SPH_OK;
}

}  // extern "C"

// ---- analytic wall correction (eq. gamma1) --------------------------------

namespace {

// Cubic spline shape in FP64: (2-q)^3 - 4(1-q)^3 for q < 1, (2-q)^3 for q < 2.
__device__ __forceinline__ double cubic_shape_fp64(double q) {
  if (q >= 2.0) return 0.0;
  const double a = 2.0 - q;
  double w = a * a * a;
  if (q < 1.0) {
    const double b = 1.0 - q;
    w -= 4.0 * b * b * b;
  }
  return w;
}

// One thread per fluid particle: num_i = rho0/m - sum_f W_if (self term
// included, as in the density), den_i = sum_g W_ig, both in FP64 and in
// particle order.  A one-time set-up computation: plain loops.
__global__ __launch_bounds__(kBlock) void sph_gamma1_kernel(const float* __restrict__ fluid, int n,
                                                            const float* __restrict__ ghosts, int ng, double inv_h,
                                                            double c, double rho0_over_m, double* __restrict__ num,
                                                            double* __restrict__ den) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const double xi = fluid[2 * i], yi = fluid[2 * i + 1];
  double sf = 0.0, sg = 0.0;
  for (int j = 0; j < n; ++j)
    sf += cubic_shape_fp64(hypot(xi - (double)fluid[2 * j], yi - (double)fluid[2 * j + 1]) * inv_h);
  for (int k = 0; k < ng; ++k)
    sg += cubic_shape_fp64(hypot(xi - (double)ghosts[2 * k], yi - (double)ghosts[2 * k + 1]) * inv_h);
  num[i] = rho0_over_m - c * sf;
  den[i] = c * sg;
}

}  // namespace

extern "C" {

int sph_gamma1_terms(const sph_params* p, const float* fluid_dev, int32_t n_fluid, const float* ghost_dev,
                     int32_t n_ghost, double* num_dev, double* den_dev, void* stream) {
  if (!p || !(p->h > 0) || !(p->mass > 0) || !(p->rho0 > 0) || n_fluid <= 0 || n_ghost < 0 || !fluid_dev ||
      (n_ghost > 0 && !ghost_dev) || !num_dev || !den_dev)
    return SPH_E_INVAL;
  if (p->kernel_norm != SPH_KNORM_UNIT && p->kernel_norm != SPH_KNORM_PRINTED) return SPH_E_INVAL;
  const double c = (p->kernel_norm == SPH_KNORM_PRINTED ? 15.0 : 5.0) / (14.0 * M_PI * p->h * p->h);
  hipLaunchKernelGGL(sph_gamma1_kernel, dim3(nblocks(n_fluid)), dim3(kBlock), 0, (hipStream_t)stream, fluid_dev,
                     n_fluid, ghost_dev, n_ghost, 1.0 / p->h, c, p->rho0 / p->mass, num_dev, den_dev);
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? SPH_OK : hip_fail(e, "sph_gamma1_terms");
}

int sph_gamma1_estimate(const sph_params* p, const float* fluid_dev, int32_t n_fluid, const float* ghost_dev,
                        int32_t n_ghost, double top, double* num_dev, double* den_dev, double* gamma1) {
  if (!gamma1 || !(top > 0.0 && top <= 1.0)) return SPH_E_INVAL;
  int rc = sph_gamma1_terms(p, fluid_dev, n_fluid, ghost_dev, n_ghost, num_dev, den_dev, nullptr);
  if (rc != SPH_OK) return rc;
  std::vector<double> num(n_fluid), den(n_fluid);
  HIPCHK(hipMemcpy(num.data(), num_dev, sizeof(double) * n_fluid, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(den.data(), den_dev, sizeof(double) * n_fluid, hipMemcpyDeviceToHost));
  // the particles with the largest ghost sums (ties by index), as many as
  // the fraction `top` of those that see a ghost at all
  std::vector<int> idx;
  for (int i = 0; i < n_fluid; ++i)
    if (den[i] > 0.0) idx.push_back(i);
  if (idx.empty()) return SPH_E_INVAL;
  const long long k = std::max(1LL, std::llround(top * (double)idx.size()));
  std::sort(idx.begin(), idx.end(), [&](int a, int b) { return den[a] > den[b] || (den[a] == den[b] && a < b); });
  std::vector<double> ratio(k);
  for (long long q = 0; q < k; ++q) ratio[q] = num[idx[q]] / den[idx[q]];
  // median; of an even count the lower of the two middle values
  std::nth_element(ratio.begin(), ratio.begin() + (k - 1) / 2, ratio.end());
  *gamma1 = ratio[(k - 1) / 2];
  return SPH_OK;
}

}  // extern "C"
