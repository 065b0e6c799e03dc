// LPV state-space surrogate of the spacecraft velocities (Section 4, eqs.
// surrogate_form and LPVparametrization; identification set-up of Section
// 5.3): simulation, the loss of eqs. pem and regularization with its gradient
// by a hand-written reverse sweep, and the two optimizers the paper chains,
// Adam and L-BFGS, all on the device.
//
// The model is tiny (4 states, 4+4 hidden units) and its recurrence is
// serial in time, so the unit of parallelism is the model, not the sample:
// one quad of lanes per model, 16 models per wave, one wave per workgroup.
// Lane j of a quad owns state x_j, hidden units h1_j and h2_j, and the
// parameter rows that produce them, its "slice" (kSlots entries):
//   slot  0- 3  A0[j][:]      slot 22-28  W1[j][:] (4 state then 3 input columns)
//   slot  4- 7  A1[j][:]      slot 29     b1[j]
//   slot  8-10  B0[j][:]      slot 30-33  W2[j][:]
//   slot 11-13  B1[j][:]      slot 34     b2[j]
//   slot 14-17  C0[j][:]      slot 35     W3[0][j]
//   slot 18-21  C1[j][:]      slot 36     b3 (lane 3; zero elsewhere)
//                             slot 37     x0[j]
// (C rows exist for j < 3 only; the unused slots hold zero and get a zero
// gradient.)  A time step exchanges values inside the quad with DPP quad
// permutations: the state and the first hidden layer are broadcast, the
// scheduling variable p is a quad sum.  Everything is FP64.
//
// The reverse sweep stores, per step, x_j, h1_j, h2_j and p of every lane in
// the caller's workspace ([n][4][columns], coalesced across the wave) and
// walks back with the adjoint lambda_k = dL/dx_k:
//   lambda_k = A(p_k)^T lambda_{k+1} + C(p_k)^T ybar_k + (dp_k/dx_k)^T pbar_k,
//   pbar_k   = lambda_{k+1}.(A1 x_k + B1 u_k) + ybar_k.(C1 x_k),
// accumulating every parameter gradient in registers of the lane that owns
// the row.  x0's gradient is lambda_0.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>

#include "slosh.h"

namespace {

constexpr int kSlots = 38;
constexpr int kWave = 64;
constexpr int kModelsPerBlock = kWave / 4;
constexpr int kMemory = 10;                 // L-BFGS pairs kept

constexpr int sA0 = 0, sA1 = 4, sB0 = 8, sB1 = 11, sC0 = 14, sC1 = 18, sW1 = 22, sb1 = 29, sW2 = 30,
              sb2 = 34, sW3 = 35, sb3 = 36, sX0 = 37;
// offsets in the packed parameter vector (A0 B0 C0 A1 B1 C1 W1 b1 W2 b2 W3 b3 x0, row-major)
constexpr int pA0 = 0, pB0 = 16, pC0 = 28, pA1 = 40, pB1 = 56, pC1 = 68, pW1 = 80, pb1 = 108, pW2 = 112,
              pb2 = 128, pW3 = 132, pb3 = 136, pX0 = 137;
static_assert(pX0 == LPV_N_THETA && pX0 + 4 == LPV_N_PARAM, "packing");

// Packed index of slot s on lane j, or -1 for a structural zero.
__host__ __device__ inline int packed_index(int j, int s) {
  if (s < sA1) return pA0 + 4 * j + s;
  if (s < sB0) return pA1 + 4 * j + (s - sA1);
  if (s < sB1) return pB0 + 3 * j + (s - sB0);
  if (s < sC0) return pB1 + 3 * j + (s - sB1);
  if (s < sC1) return j < 3 ? pC0 + 4 * j + (s - sC0) : -1;
  if (s < sW1) return j < 3 ? pC1 + 4 * j + (s - sC1) : -1;
  if (s < sb1) return pW1 + 7 * j + (s - sW1);
  if (s == sb1) return pb1 + j;
  if (s < sb2) return pW2 + 4 * j + (s - sW2);
  if (s == sb2) return pb2 + j;
  if (s == sW3) return pW3 + j;
  if (s == sb3) return j == 3 ? pb3 : -1;
  return pX0 + j;
}

// 1 if slot s of lane j moves in a fit; an LTI fit moves A0, B0, C0 and x0 only.
__device__ inline bool trainable(int j, int s, int lti_only) {
  if (packed_index(j, s) < 0) return false;
  if (!lti_only) return true;
  return s < sA1 || (s >= sB0 && s < sB1) || (s >= sC0 && s < sC1) || s == sX0;
}

// ---- quad exchange --------------------------------------------------------

template <int L>
__device__ __forceinline__ double qb(double v) {   // value of quad lane L, on every lane of the quad
  constexpr int ctrl = L | (L << 2) | (L << 4) | (L << 6);
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), ctrl, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

template <int Ctrl>
__device__ __forceinline__ double qperm(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, Ctrl, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), Ctrl, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the quad, bit-identical on its four lanes: (v0 + v1) + (v2 + v3).
__device__ __forceinline__ double qsum(double v) {
  v += qperm<0xB1>(v);   // quad_perm [1,0,3,2]
  return v + qperm<0x4E>(v);   // quad_perm [2,3,0,1]
}

__device__ __forceinline__ double qmax(double v) {
  v = fmax(v, qperm<0xB1>(v));
  return fmax(v, qperm<0x4E>(v));
}

// ---- tanh in FP64 -----------------------------------------------------------
//
// tanh|z| = -t / (t + 2) with t = e^{-2|z|} - 1, which keeps full relative
// accuracy near zero.  e^x - 1 by Cody-Waite reduction x = n ln2 + r,
// |r| <= ln2/2 (ln2 split in a 32-bit head and a tail), the Taylor series
// of e^r - 1 to degree 13 (truncation below 1e-17 relative on that range)
// evaluated by Estrin's scheme to keep the dependent chain short, and
// e^x - 1 = 2^n (e^r - 1) + (2^n - 1).  The quotient uses the hardware
// reciprocal refined by two Newton steps and one residual correction.  Max
// relative error about 2 ulp; |z| >= 20 gives +-1; NaN propagates.

__device__ __forceinline__ double tanh_fp64(double z) {
  constexpr double kLog2e = 1.4426950408889634, kLn2Hi = 0x1.62e42fefa3800p-1, kLn2Lo = 0x1.ef35793c76730p-45;
  constexpr double c0 = 1.0 / 2, c1 = 1.0 / 6, c2 = 1.0 / 24, c3 = 1.0 / 120, c4 = 1.0 / 720, c5 = 1.0 / 5040,
                   c6 = 1.0 / 40320, c7 = 1.0 / 362880, c8 = 1.0 / 3628800, c9 = 1.0 / 39916800,
                   c10 = 1.0 / 479001600, c11 = 1.0 / 6227020800.0;
  const double x = -2.0 * fmin(fabs(z), 20.0);
  const double n = rint(x * kLog2e);
  const double r = fma(-n, kLn2Lo, fma(-n, kLn2Hi, x));
  const double r2 = r * r, r4 = r2 * r2, r8 = r4 * r4;
  const double q0 = fma(fma(c3, r, c2), r2, fma(c1, r, c0));
  const double q1 = fma(fma(c7, r, c6), r2, fma(c5, r, c4));
  const double q2 = fma(fma(c11, r, c10), r2, fma(c9, r, c8));
  const double em1 = fma(r2, fma(q2, r8, fma(q1, r4, q0)), r);
  const int ni = (int)n;
  const double t = ldexp(em1, ni) + (ldexp(1.0, ni) - 1.0);
  const double d = t + 2.0;                   // in [1, 2]
  double rc = __builtin_amdgcn_rcp(d);
  rc = fma(rc, fma(-d, rc, 1.0), rc);
  rc = fma(rc, fma(-d, rc, 1.0), rc);
  double q = -t * rc;
  q = fma(fma(-q, d, -t), rc, q);
  return z != z ? z : copysign(q, z);
}

// ---- one loss (and gradient) evaluation -----------------------------------

struct Data {
  const double* u;   // [n][3] (shared by all models) or [R][n][3]
  const double* y;   // [n][3] targets (may be null when no loss is wanted)
  int n;
  int u_per_model;
};

struct Scratch {
  double* traj;      // [n][4][cols]
  size_t cols;       // padded models * 4
};

// Loss of eqs. pem + regularization at the slice w, identical on the quad's
// lanes.  Grad: writes the gradient slice to g.  yout: if non-null, writes
// yhat [n][3] of this model (rows of the model's block).  col = model*4+j.
template <bool Grad>
__device__ double lpv_eval(const double (&w)[kSlots], double (&g)[kSlots], const Data& d, const Scratch& sc,
                           int model, int col, int j, double s2, double sx, double* yout, double* pout,
                           double (*lds)[kSlots]) {
  // columns of the transposed products, gathered through LDS (one wave per block)
  const int qbase = threadIdx.x & ~3;
#pragma unroll
  for (int s = 0; s < kSlots; ++s) lds[threadIdx.x][s] = w[s];
  __syncthreads();
  double cA0[4], cA1[4], cC0[3], cC1[3], cW1[4], cW2[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    cA0[i] = lds[qbase + i][sA0 + j];
    cA1[i] = lds[qbase + i][sA1 + j];
    cW1[i] = lds[qbase + i][sW1 + j];
    cW2[i] = lds[qbase + i][sW2 + j];
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    cC0[i] = lds[qbase + i][sC0 + j];
    cC1[i] = lds[qbase + i][sC1 + j];
  }
  const double b3 = lds[qbase + 3][sb3];
  __syncthreads();

  const int n = d.n;
  const double inv_n = 1.0 / (double)n;
  const double* u = d.u + (d.u_per_model ? (size_t)model * n * 3 : 0);
  const int jy = j < 3 ? j : 2;
  const bool has_y = d.y != nullptr;
  const double ymask = j < 3 ? 1.0 : 0.0;

  double xj = w[sX0];
  double acc = 0.0;
  double u0 = u[0], u1 = u[1], u2 = u[2];
  double yk = has_y ? d.y[jy] : 0.0;
  for (int k = 0; k < n; ++k) {
    const int kn = k + 1 < n ? k + 1 : k;
    const double nu0 = u[3 * kn], nu1 = u[3 * kn + 1], nu2 = u[3 * kn + 2];
    const double nyk = has_y ? d.y[3 * kn + jy] : 0.0;

    const double x0 = qb<0>(xj), x1 = qb<1>(xj), x2 = qb<2>(xj), x3 = qb<3>(xj);
    const double z1u = w[sb1] + w[sW1 + 4] * u0 + w[sW1 + 5] * u1 + w[sW1 + 6] * u2;
    const double z1 = z1u + ((w[sW1] * x0 + w[sW1 + 1] * x1) + (w[sW1 + 2] * x2 + w[sW1 + 3] * x3));
    const double h1 = tanh_fp64(z1);
    const double a_u = w[sB0] * u0 + w[sB0 + 1] * u1 + w[sB0 + 2] * u2;
    const double b_u = w[sB1] * u0 + w[sB1 + 1] * u1 + w[sB1 + 2] * u2;
    const double a = a_u + w[sA0] * x0 + w[sA0 + 1] * x1 + w[sA0 + 2] * x2 + w[sA0 + 3] * x3;
    const double b = b_u + w[sA1] * x0 + w[sA1 + 1] * x1 + w[sA1 + 2] * x2 + w[sA1 + 3] * x3;
    const double yc0 = w[sC0] * x0 + w[sC0 + 1] * x1 + w[sC0 + 2] * x2 + w[sC0 + 3] * x3;
    const double yc1 = w[sC1] * x0 + w[sC1 + 1] * x1 + w[sC1 + 2] * x2 + w[sC1 + 3] * x3;
    const double hb0 = qb<0>(h1), hb1 = qb<1>(h1), hb2 = qb<2>(h1), hb3 = qb<3>(h1);
    const double z2 = w[sb2] + ((w[sW2] * hb0 + w[sW2 + 1] * hb1) + (w[sW2 + 2] * hb2 + w[sW2 + 3] * hb3));
    const double h2 = tanh_fp64(z2);
    const double p = qsum(w[sW3] * h2) + b3;
    const double yh = yc0 + p * yc1;
    if (has_y) {
      const double r = (yh - yk) * ymask;
      acc += r * r;
    }
    if (Grad) {
      double* t = sc.traj + (size_t)k * 4 * sc.cols + col;
      t[0] = xj;
      t[sc.cols] = h1;
      t[2 * sc.cols] = h2;
      t[3 * sc.cols] = p;
    }
    if (yout && j < 3) yout[(size_t)k * 3 + j] = yh;
    if (pout && j == 0) pout[k] = p;
    xj = a + p * b;
    u0 = nu0;
    u1 = nu1;
    u2 = nu2;
    yk = nyk;
  }
  double reg = 0.0;
#pragma unroll
  for (int s = 0; s < sX0; ++s) reg += w[s] * w[s];
  reg = 0.5 * s2 * reg + 0.5 * sx * w[sX0] * w[sX0];
  const double loss = qsum(acc) * inv_n + qsum(reg);

  if (Grad) {
#pragma unroll
    for (int s = 0; s < kSlots; ++s) g[s] = 0.0;
    double lam = 0.0;
    const size_t cols = sc.cols;
    const int c0 = col - j;
    for (int k = n - 1; k >= 0; --k) {
      const double* t = sc.traj + (size_t)k * 4 * cols;
      const double xk0 = t[c0], xk1 = t[c0 + 1], xk2 = t[c0 + 2], xk3 = t[c0 + 3];
      const double hk0 = t[cols + c0], hk1 = t[cols + c0 + 1], hk2 = t[cols + c0 + 2], hk3 = t[cols + c0 + 3];
      const double h1 = t[cols + col];
      const double h2 = t[2 * cols + col];
      const double p = t[3 * cols + col];
      const double v0 = u[3 * k], v1 = u[3 * k + 1], v2 = u[3 * k + 2];
      const double yk = d.y[3 * k + jy];

      const double yc0 = w[sC0] * xk0 + w[sC0 + 1] * xk1 + w[sC0 + 2] * xk2 + w[sC0 + 3] * xk3;
      const double yc1 = w[sC1] * xk0 + w[sC1 + 1] * xk1 + w[sC1 + 2] * xk2 + w[sC1 + 3] * xk3;
      const double ybar = 2.0 * inv_n * (yc0 + p * yc1 - yk) * ymask;
      const double b = w[sB1] * v0 + w[sB1 + 1] * v1 + w[sB1 + 2] * v2 + w[sA1] * xk0 + w[sA1 + 1] * xk1 +
                       w[sA1 + 2] * xk2 + w[sA1 + 3] * xk3;
      const double pbar = qsum(lam * b + ybar * yc1);
      const double pl = p * lam, py = p * ybar;
      g[sA0] += lam * xk0; g[sA0 + 1] += lam * xk1; g[sA0 + 2] += lam * xk2; g[sA0 + 3] += lam * xk3;
      g[sA1] += pl * xk0;  g[sA1 + 1] += pl * xk1;  g[sA1 + 2] += pl * xk2;  g[sA1 + 3] += pl * xk3;
      g[sB0] += lam * v0;  g[sB0 + 1] += lam * v1;  g[sB0 + 2] += lam * v2;
      g[sB1] += pl * v0;   g[sB1 + 1] += pl * v1;   g[sB1 + 2] += pl * v2;
      g[sC0] += ybar * xk0; g[sC0 + 1] += ybar * xk1; g[sC0 + 2] += ybar * xk2; g[sC0 + 3] += ybar * xk3;
      g[sC1] += py * xk0;  g[sC1 + 1] += py * xk1;  g[sC1 + 2] += py * xk2;  g[sC1 + 3] += py * xk3;
      g[sW3] += pbar * h2;
      g[sb3] += pbar;
      const double h2bar = pbar * w[sW3] * (1.0 - h2 * h2);
      g[sW2] += h2bar * hk0; g[sW2 + 1] += h2bar * hk1; g[sW2 + 2] += h2bar * hk2; g[sW2 + 3] += h2bar * hk3;
      g[sb2] += h2bar;
      const double hb0 = qb<0>(h2bar), hb1 = qb<1>(h2bar), hb2 = qb<2>(h2bar), hb3 = qb<3>(h2bar);
      const double h1bar = (cW2[0] * hb0 + cW2[1] * hb1 + cW2[2] * hb2 + cW2[3] * hb3) * (1.0 - h1 * h1);
      g[sW1] += h1bar * xk0; g[sW1 + 1] += h1bar * xk1; g[sW1 + 2] += h1bar * xk2; g[sW1 + 3] += h1bar * xk3;
      g[sW1 + 4] += h1bar * v0; g[sW1 + 5] += h1bar * v1; g[sW1 + 6] += h1bar * v2;
      g[sb1] += h1bar;
      // A(p)^T lambda and C(p)^T ybar do not wait for the scheduling chain
      const double l0 = qb<0>(lam), l1 = qb<1>(lam), l2 = qb<2>(lam), l3 = qb<3>(lam);
      const double y0 = qb<0>(ybar), y1 = qb<1>(ybar), y2 = qb<2>(ybar);
      const double la = ((cA0[0] + p * cA1[0]) * l0 + (cA0[1] + p * cA1[1]) * l1) +
                        ((cA0[2] + p * cA1[2]) * l2 + (cA0[3] + p * cA1[3]) * l3);
      const double lc = (cC0[0] + p * cC1[0]) * y0 + (cC0[1] + p * cC1[1]) * y1 + (cC0[2] + p * cC1[2]) * y2;
      const double e0 = qb<0>(h1bar), e1 = qb<1>(h1bar), e2 = qb<2>(h1bar), e3 = qb<3>(h1bar);
      lam = (la + lc) + ((cW1[0] * e0 + cW1[1] * e1) + (cW1[2] * e2 + cW1[3] * e3));
    }
    g[sX0] = lam;
    if (j != 3) g[sb3] = 0.0;
#pragma unroll
    for (int s = 0; s < sX0; ++s) g[s] += s2 * w[s];
    g[sX0] += sx * w[sX0];
  }
  return loss;
}

// ---- kernels ---------------------------------------------------------------

struct FitArgs {
  Data d;
  Scratch sc;
  int R;                  // models
  double s2, sx;
  int lti_only;
  double* vec;            // [n_vec][kSlots][cols]
  double* scal;           // [kScal][cols]
};

// vectors of the fit state
enum { vX = 0, vG = 1, vD = 2, vM = 1, vV = 2, vS = 3, vY = 3 + kMemory, kVecs = 3 + 2 * kMemory };
// per-lane scalars of the L-BFGS state
enum { cF = 0, cAlpha, cGtd, cIter, cBack, cPhase, cStatus, cHead, cHist, cRho, cYY = cRho + kMemory,
       kScal = cYY + kMemory };

__device__ inline double* vslot(const FitArgs& a, int v, int s, int col) {
  return a.vec + ((size_t)v * kSlots + s) * a.sc.cols + col;
}
__device__ inline double* cslot(const FitArgs& a, int c, int col) { return a.scal + (size_t)c * a.sc.cols + col; }

// packed [R][141] -> slices of vector v (padded models: zero)
__global__ __launch_bounds__(kWave) void lpv_unpack(FitArgs a, const double* __restrict__ params, int v) {
  const int col = blockIdx.x * kWave + threadIdx.x;
  const int model = col >> 2, j = col & 3;
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    const int pi = packed_index(j, s);
    *vslot(a, v, s, col) = (model < a.R && pi >= 0) ? params[(size_t)model * LPV_N_PARAM + pi] : 0.0;
  }
}

__global__ __launch_bounds__(kWave) void lpv_pack(FitArgs a, double* __restrict__ params, int v) {
  const int col = blockIdx.x * kWave + threadIdx.x;
  const int model = col >> 2, j = col & 3;
  if (model >= a.R) return;
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    const int pi = packed_index(j, s);
    if (pi >= 0) params[(size_t)model * LPV_N_PARAM + pi] = *vslot(a, v, s, col);
  }
}

__global__ __launch_bounds__(kWave) void lpv_zero(FitArgs a, int v0, int v1) {
  const int col = blockIdx.x * kWave + threadIdx.x;
  for (int v = v0; v < v1; ++v)
#pragma unroll
    for (int s = 0; s < kSlots; ++s) *vslot(a, v, s, col) = 0.0;
}

// Simulation and loss/gradient straight from packed parameters.
__global__ __launch_bounds__(kWave) void lpv_forward_kernel(Data d, Scratch sc, int R, const double* __restrict__ params,
                                                            double s2, double sx, int lti_only, double* loss,
                                                            double* grad, double* yout, double* pout) {
  __shared__ double lds[kWave][kSlots];
  const int col = blockIdx.x * kWave + threadIdx.x;
  const int j = col & 3;
  const int model = col >> 2;
  const int m = model < R ? model : R - 1;
  double w[kSlots], g[kSlots];
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    const int pi = packed_index(j, s);
    w[s] = pi >= 0 ? params[(size_t)m * LPV_N_PARAM + pi] : 0.0;
  }
  double f;
  double* yo = (yout && model < R) ? yout + (size_t)model * d.n * 3 : nullptr;
  double* po = (pout && model < R) ? pout + (size_t)model * d.n : nullptr;
  if (grad) {
    f = lpv_eval<true>(w, g, d, sc, m, col, j, s2, sx, yo, po, lds);
  } else {
    f = lpv_eval<false>(w, g, d, sc, m, col, j, s2, sx, yo, po, lds);
  }
  if (model >= R) return;
  if (loss && j == 0) loss[model] = f;
  if (grad)
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      const int pi = packed_index(j, s);
      if (pi >= 0) grad[(size_t)model * LPV_N_PARAM + pi] = trainable(j, s, lti_only) ? g[s] : 0.0;
    }
}

// `iters` Adam steps (Kingma and Ba), step counter continuing from t0.
__global__ __launch_bounds__(kWave) void lpv_adam_kernel(FitArgs a, int iters, int t0, double lr, double beta1,
                                                         double beta2, double eps, double* loss) {
  __shared__ double lds[kWave][kSlots];
  const int col = blockIdx.x * kWave + threadIdx.x;
  const int j = col & 3;
  const int model = col >> 2;
  const int m = model < a.R ? model : a.R - 1;
  double w[kSlots], g[kSlots];
  double f = 0.0;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int s = 0; s < kSlots; ++s) w[s] = *vslot(a, vX, s, col);
    f = lpv_eval<true>(w, g, a.d, a.sc, m, col, j, a.s2, a.sx, nullptr, nullptr, lds);
    const int t = t0 + it + 1;
    const double bc1 = 1.0 - pow(beta1, (double)t), bc2 = 1.0 - pow(beta2, (double)t);
#pragma unroll
    for (int s = 0; s < kSlots; ++s) {
      const double gs = trainable(j, s, a.lti_only) ? g[s] : 0.0;
      double* pm = vslot(a, vM, s, col);
      double* pv = vslot(a, vV, s, col);
      const double mm = beta1 * *pm + (1.0 - beta1) * gs;
      const double vv = beta2 * *pv + (1.0 - beta2) * gs * gs;
      *pm = mm;
      *pv = vv;
      *vslot(a, vX, s, col) = w[s] - lr * (mm / bc1) / (sqrt(vv / bc2) + eps);
    }
  }
  if (loss && model < a.R && j == 0) loss[model] = f;
}

struct LbfgsOpts {
  double c1, gtol, ftol;
  int max_back, max_iter;
};

__device__ inline double masked(const FitArgs& a, int j, int s, double g) {
  return trainable(j, s, a.lti_only) ? g : 0.0;
}

__device__ inline void lbfgs_accept_checks(const FitArgs& a, int col, const LbfgsOpts& o, double f_old, double f,
                                           double gmax, double iter) {
  double st = 0.0;
  if (gmax <= o.gtol) st = 1.0;
  else if (f_old - f <= o.ftol * fmax(fabs(f_old), fabs(f))) st = 2.0;
  else if (iter >= o.max_iter) st = 4.0;
  *cslot(a, cStatus, col) = st;
}

// First evaluation of an L-BFGS run: f and g at X, memory cleared.
__global__ __launch_bounds__(kWave) void lpv_lbfgs_start(FitArgs a, LbfgsOpts o) {
  __shared__ double lds[kWave][kSlots];
  const int col = blockIdx.x * kWave + threadIdx.x;
  const int j = col & 3;
  const int model = col >> 2;
  const int m = model < a.R ? model : a.R - 1;
  double w[kSlots], g[kSlots];
#pragma unroll
  for (int s = 0; s < kSlots; ++s) w[s] = *vslot(a, vX, s, col);
  const double f = lpv_eval<true>(w, g, a.d, a.sc, m, col, j, a.s2, a.sx, nullptr, nullptr, lds);
  double gmax = 0.0;
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    const double gs = masked(a, j, s, g[s]);
    *vslot(a, vG, s, col) = gs;
    gmax = fmax(gmax, fabs(gs));
  }
  gmax = qmax(gmax);
  *cslot(a, cF, col) = f;
  *cslot(a, cIter, col) = 0.0;
  *cslot(a, cBack, col) = 0.0;
  *cslot(a, cPhase, col) = 0.0;
  *cslot(a, cHead, col) = 0.0;
  *cslot(a, cHist, col) = 0.0;
  *cslot(a, cStatus, col) = (model >= a.R) ? 5.0 : (gmax <= o.gtol ? 1.0 : (o.max_iter <= 0 ? 4.0 : 0.0));
}

// Up to `evals` loss/gradient evaluations of L-BFGS (two-loop recursion,
// backtracking Armijo line search with quadratic interpolation).  Each pass:
// every running model picks a trial point (a new direction, or the
// interpolated shorter step), all models evaluate
// (a finished model evaluates its own point and ignores the result), then
// each running model accepts or backtracks.  Status: 0 running, 1 gradient
// tolerance, 2 no further decrease, 3 line search failed, 4 iteration limit,
// 5 padding.
__global__ __launch_bounds__(kWave) void lpv_lbfgs_kernel(FitArgs a, LbfgsOpts o, int evals) {
  __shared__ double lds[kWave][kSlots];
  const int col = blockIdx.x * kWave + threadIdx.x;
  const int j = col & 3;
  const int model = col >> 2;
  const int m = model < a.R ? model : a.R - 1;
  double w[kSlots], g[kSlots];
  for (int e = 0; e < evals; ++e) {
    const bool done = *cslot(a, cStatus, col) != 0.0;
    if (__all(done)) break;
    double alpha = 0.0, gtd = 0.0;
    if (!done) {
      if (*cslot(a, cPhase, col) == 0.0) {
        // two-loop recursion: q = g; newest to oldest; r = gamma q; oldest to newest
        const int hist = (int)*cslot(a, cHist, col);
        const int head = (int)*cslot(a, cHead, col);
        double q[kSlots];
#pragma unroll
        for (int s = 0; s < kSlots; ++s) q[s] = *vslot(a, vG, s, col);
        double al[kMemory];
#pragma unroll
        for (int t = 0; t < kMemory; ++t) {
          al[t] = 0.0;
          if (t < hist) {
            const int idx = (head - 1 - t + kMemory) % kMemory;
            double dot = 0.0;
#pragma unroll
            for (int s = 0; s < kSlots; ++s) dot += *vslot(a, vS + idx, s, col) * q[s];
            al[t] = *cslot(a, cRho + idx, col) * qsum(dot);
#pragma unroll
            for (int s = 0; s < kSlots; ++s) q[s] -= al[t] * *vslot(a, vY + idx, s, col);
          }
        }
        double gamma = 1.0;
        if (hist > 0) {
          const int nw = (head - 1 + kMemory) % kMemory;
          gamma = (1.0 / *cslot(a, cRho + nw, col)) / *cslot(a, cYY + nw, col);
        }
#pragma unroll
        for (int s = 0; s < kSlots; ++s) q[s] *= gamma;
#pragma unroll
        for (int t = kMemory - 1; t >= 0; --t) {
          if (t < hist) {
            const int idx = (head - 1 - t + kMemory) % kMemory;
            double dot = 0.0;
#pragma unroll
            for (int s = 0; s < kSlots; ++s) dot += *vslot(a, vY + idx, s, col) * q[s];
            const double be = *cslot(a, cRho + idx, col) * qsum(dot);
#pragma unroll
            for (int s = 0; s < kSlots; ++s) q[s] += (al[t] - be) * *vslot(a, vS + idx, s, col);
          }
        }
        double dg = 0.0;
#pragma unroll
        for (int s = 0; s < kSlots; ++s) dg -= q[s] * *vslot(a, vG, s, col);
        gtd = qsum(dg);
        if (!(gtd < 0.0)) {
          *cslot(a, cHist, col) = 0.0;
          *cslot(a, cHead, col) = 0.0;
          double gg = 0.0;
#pragma unroll
          for (int s = 0; s < kSlots; ++s) {
            const double gs = *vslot(a, vG, s, col);
            q[s] = gs;
            gg += gs * gs;
          }
          gtd = -qsum(gg);
        }
#pragma unroll
        for (int s = 0; s < kSlots; ++s) *vslot(a, vD, s, col) = -q[s];
        if (*cslot(a, cIter, col) == 0.0) {
          double gg = 0.0;
#pragma unroll
          for (int s = 0; s < kSlots; ++s) {
            const double gs = *vslot(a, vG, s, col);
            gg += gs * gs;
          }
          alpha = 1.0 / fmax(1.0, sqrt(qsum(gg)));
        } else {
          alpha = 1.0;
        }
        *cslot(a, cGtd, col) = gtd;
        *cslot(a, cBack, col) = 0.0;
      } else {
        alpha = *cslot(a, cAlpha, col);
        gtd = *cslot(a, cGtd, col);
      }
      *cslot(a, cAlpha, col) = alpha;
    }
#pragma unroll
    for (int s = 0; s < kSlots; ++s) w[s] = *vslot(a, vX, s, col) + alpha * *vslot(a, vD, s, col);
    const double ft = lpv_eval<true>(w, g, a.d, a.sc, m, col, j, a.s2, a.sx, nullptr, nullptr, lds);
    if (done) continue;
    const double f = *cslot(a, cF, col);
    if (isfinite(ft) && ft <= f + o.c1 * alpha * gtd) {
      double sy = 0.0, ss = 0.0, yy = 0.0, gmax = 0.0;
#pragma unroll
      for (int s = 0; s < kSlots; ++s) {
        g[s] = masked(a, j, s, g[s]);
        const double sv = w[s] - *vslot(a, vX, s, col);
        const double yv = g[s] - *vslot(a, vG, s, col);
        sy += sv * yv;
        ss += sv * sv;
        yy += yv * yv;
        gmax = fmax(gmax, fabs(g[s]));
      }
      sy = qsum(sy);
      ss = qsum(ss);
      yy = qsum(yy);
      gmax = qmax(gmax);
      if (sy > 1e-10 * sqrt(ss) * sqrt(yy)) {
        const int head = (int)*cslot(a, cHead, col);
#pragma unroll
        for (int s = 0; s < kSlots; ++s) {
          *vslot(a, vS + head, s, col) = w[s] - *vslot(a, vX, s, col);
          *vslot(a, vY + head, s, col) = g[s] - *vslot(a, vG, s, col);
        }
        *cslot(a, cRho + head, col) = 1.0 / sy;
        *cslot(a, cYY + head, col) = yy;
        *cslot(a, cHead, col) = (double)((head + 1) % kMemory);
        *cslot(a, cHist, col) = fmin((double)kMemory, *cslot(a, cHist, col) + 1.0);
      }
#pragma unroll
      for (int s = 0; s < kSlots; ++s) {
        *vslot(a, vX, s, col) = w[s];
        *vslot(a, vG, s, col) = g[s];
      }
      const double iter = *cslot(a, cIter, col) + 1.0;
      *cslot(a, cIter, col) = iter;
      *cslot(a, cF, col) = ft;
      *cslot(a, cPhase, col) = 0.0;
      lbfgs_accept_checks(a, col, o, f, ft, gmax, iter);
    } else {
      // next trial: minimiser of the quadratic through f, g'd and ft
      // (Nocedal and Wright eq. 3.57) within [0.1, 0.5] alpha; 0.1 alpha
      // after a non-finite value
      double an = 0.1 * alpha;
      if (isfinite(ft)) {
        const double aq = -gtd * alpha * alpha / (2.0 * (ft - f - gtd * alpha));
        an = fmin(fmax(aq, 0.1 * alpha), 0.5 * alpha);
      }
      *cslot(a, cAlpha, col) = an;
      const double back = *cslot(a, cBack, col) + 1.0;
      *cslot(a, cBack, col) = back;
      *cslot(a, cPhase, col) = 1.0;
      if (back > o.max_back) *cslot(a, cStatus, col) = 3.0;
    }
  }
}

__global__ __launch_bounds__(kWave) void lpv_lbfgs_finish(FitArgs a, double* loss, int32_t* status, int32_t* iters) {
  const int col = blockIdx.x * kWave + threadIdx.x;
  const int model = col >> 2;
  if (model >= a.R || (col & 3) != 0) return;
  if (loss) loss[model] = *cslot(a, cF, col);
  if (status) status[model] = (int32_t)*cslot(a, cStatus, col);
  if (iters) iters[model] = (int32_t)*cslot(a, cIter, col);
}

// ---- closed-loop simulation of the augmented model -------------------------
//
// The velocity model augmented with position integrators (Section 5.3: the
// positions advance by Ts times the predicted velocities) in a loop with the
// attitude law of Section 5.1, tau_k = kp (ref_k - theta_k) - kd thetadot_k,
// held for one sample.  The model's output map C(p_k) depends on u_k through
// the scheduling map, so the law cannot read the output of sample k without
// an algebraic loop; it reads the output the model predicts while the
// previous input is still held, C(eta(x_k, u_{k-1})) x_k (u_{-1} = the first
// force with zero torque), as a sampled sensor would just before the hold
// switches.  The increment of the integrators uses C(p_k) x_k with the input
// actually applied.  Physical units at the boundary: the model sees inputs
// divided by u_scale and predicts outputs divided by y_scale.

struct Scales {
  double u[3], y[3];
};

// p = eta(x, u) for the quad (x broadcast as x0..x3, u the scaled input)
__device__ __forceinline__ double schedule(const double (&w)[kSlots], double b3, double x0, double x1, double x2,
                                           double x3, double u0, double u1, double u2) {
  double z1 = w[sb1] + w[sW1 + 4] * u0 + w[sW1 + 5] * u1 + w[sW1 + 6] * u2;
  z1 += w[sW1] * x0 + w[sW1 + 1] * x1 + w[sW1 + 2] * x2 + w[sW1 + 3] * x3;
  const double h1 = tanh_fp64(z1);
  const double hb0 = qb<0>(h1), hb1 = qb<1>(h1), hb2 = qb<2>(h1), hb3 = qb<3>(h1);
  const double z2 = w[sb2] + w[sW2] * hb0 + w[sW2 + 1] * hb1 + w[sW2 + 2] * hb2 + w[sW2 + 3] * hb3;
  return qsum(w[sW3] * tanh_fp64(z2)) + b3;
}

__global__ __launch_bounds__(kWave) void lpv_closed_loop_kernel(const double* __restrict__ params, int R,
                                                                const double* __restrict__ x0,
                                                                const double* __restrict__ force, int force_per_model,
                                                                const double* __restrict__ ref, int ref_per_model,
                                                                int n, double ts, double kp, double kd, Scales sc,
                                                                double* __restrict__ y6, double* __restrict__ tau) {
  __shared__ double lds[kWave][kSlots];
  const int col = blockIdx.x * kWave + threadIdx.x;
  const int j = col & 3;
  const int model = col >> 2;
  const int m = model < R ? model : R - 1;
  double w[kSlots];
#pragma unroll
  for (int s = 0; s < kSlots; ++s) {
    const int pi = packed_index(j, s);
    w[s] = pi >= 0 ? params[(size_t)m * LPV_N_PARAM + pi] : 0.0;
  }
#pragma unroll
  for (int s = 0; s < kSlots; ++s) lds[threadIdx.x][s] = w[s];
  __syncthreads();
  const double b3 = lds[(threadIdx.x & ~3) + 3][sb3];
  __syncthreads();
  const int jo = j < 3 ? j : 2;
  const double ysc = sc.y[jo];
  const double* F = force + (force_per_model ? (size_t)m * n * 2 : 0);
  const double* rf = ref + (ref_per_model ? (size_t)m * n : 0);
  double xj = x0 ? x0[(size_t)m * 4 + j] : 0.0;
  double pos = 0.0;                        // r_x, r_y, theta on lanes 0, 1, 2
  double up0 = F[0] / sc.u[0], up1 = F[1] / sc.u[1], up2 = 0.0;   // held input (scaled)
  const bool store = model < R;
  for (int k = 0; k < n; ++k) {
    const double x0b = qb<0>(xj), x1b = qb<1>(xj), x2b = qb<2>(xj), x3b = qb<3>(xj);
    const double yc0 = w[sC0] * x0b + w[sC0 + 1] * x1b + w[sC0 + 2] * x2b + w[sC0 + 3] * x3b;
    const double yc1 = w[sC1] * x0b + w[sC1 + 1] * x1b + w[sC1 + 2] * x2b + w[sC1 + 3] * x3b;
    const double pm = schedule(w, b3, x0b, x1b, x2b, x3b, up0, up1, up2);
    const double ymeas = (yc0 + pm * yc1) * ysc;                 // physical velocity j
    const double law = kp * (rf[k] - pos) - kd * ymeas;          // meaningful on lane 2
    const double t = qb<2>(law);
    const double u0 = F[2 * k] / sc.u[0], u1 = F[2 * k + 1] / sc.u[1], u2 = t / sc.u[2];
    const double p = schedule(w, b3, x0b, x1b, x2b, x3b, u0, u1, u2);
    if (store) {
      double* o = y6 + ((size_t)model * n + k) * 6;
      if (j < 3) {
        o[j] = pos;
        o[3 + j] = ymeas;
      }
      if (tau && j == 0) tau[(size_t)model * n + k] = t;
    }
    pos += ts * (yc0 + p * yc1) * ysc;
    const double a = w[sB0] * u0 + w[sB0 + 1] * u1 + w[sB0 + 2] * u2 + w[sA0] * x0b + w[sA0 + 1] * x1b +
                     w[sA0 + 2] * x2b + w[sA0 + 3] * x3b;
    const double b = w[sB1] * u0 + w[sB1 + 1] * u1 + w[sB1 + 2] * u2 + w[sA1] * x0b + w[sA1 + 1] * x1b +
                     w[sA1 + 2] * x2b + w[sA1 + 3] * x3b;
    xj = a + p * b;
    up0 = u0;
    up1 = u1;
    up2 = u2;
  }
}

}  // namespace

// ---- C ABI ------------------------------------------------------------------

namespace {

int hip_rc(hipError_t e) { return e == hipSuccess ? SPH_OK : SPH_E_HIP; }

size_t cols_for(int R) { return (size_t)((R + kModelsPerBlock - 1) / kModelsPerBlock) * kWave; }

struct WsLayout {
  size_t traj, vec, scal, total;
};

WsLayout ws_layout(int R, int n) {
  const size_t cols = cols_for(R);
  WsLayout L;
  size_t o = 0;
  auto take = [&](size_t doubles) {
    const size_t at = o;
    o += ((doubles * sizeof(double) + 255) / 256) * 256;
    return at;
  };
  L.traj = take((size_t)n * 4 * cols);
  L.vec = take((size_t)kVecs * kSlots * cols);
  L.scal = take((size_t)kScal * cols);
  L.total = o;
  return L;
}

bool valid_data(int R, int n, const void* u, const void* y) { return R > 0 && n > 0 && u && y; }

FitArgs fit_args(const lpv_opts* o, int R, const double* u, const double* y, int n, void* ws) {
  const WsLayout L = ws_layout(R, n);
  FitArgs a;
  a.d = Data{u, y, n, 0};
  a.sc = Scratch{(double*)((char*)ws + L.traj), cols_for(R)};
  a.R = R;
  a.s2 = o->sigma2;
  a.sx = o->sigmax;
  a.lti_only = o->lti_only;
  a.vec = (double*)((char*)ws + L.vec);
  a.scal = (double*)((char*)ws + L.scal);
  return a;
}

// evaluations per launch: about 2e5 model steps, so one launch stays near 0.1 s
int evals_per_launch(int n) { return n >= 200000 ? 1 : 200000 / n; }

// Reverse-sweep record of lpv_loss_grad_noalloc: a fixed array in device
// memory, one copy per GPU, held until the process ends.  Host code never
// passes `scratch` itself (on the host it names a stand-in, not a device
// address): it passes the device address that hipGetSymbolAddress returns
// for the current device, looked up once per device.
constexpr size_t kNoAllocScratchBytes = size_t(LPV_NOALLOC_SCRATCH_BYTES);
static_assert(kNoAllocScratchBytes % 256 == 0, "scratch size");
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call per device), or an error code.
int scratch_on_current_device(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SPH_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SPH_E_HIP;
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return SPH_OK;
}

}  // namespace

extern "C" {

int lpv_workspace_bytes(int32_t n_models, int32_t n_samples, size_t* bytes) {
  if (!bytes || n_models <= 0 || n_samples <= 0) return SPH_E_INVAL;
  *bytes = ws_layout(n_models, n_samples).total;
  return SPH_OK;
}

int lpv_simulate(const double* params_dev, int32_t n_models, const double* u_dev, int32_t u_per_model,
                 int32_t n_samples, double* y_dev, double* p_dev, void* stream) {
  if (!params_dev || !u_dev || !y_dev || n_models <= 0 || n_samples <= 0) return SPH_E_INVAL;
  const Data d{u_dev, nullptr, n_samples, u_per_model ? 1 : 0};
  const Scratch sc{nullptr, cols_for(n_models)};
  const int blocks = (int)(cols_for(n_models) / kWave);
  hipLaunchKernelGGL(lpv_forward_kernel, dim3(blocks), dim3(kWave), 0, (hipStream_t)stream, d, sc, n_models,
                     params_dev, 0.0, 0.0, 0, (double*)nullptr, (double*)nullptr, y_dev, p_dev);
  return hip_rc(hipGetLastError());
}

int lpv_loss_grad(const double* params_dev, int32_t n_models, const double* u_dev, const double* y_dev,
                  int32_t n_samples, const lpv_opts* opts, double* loss_dev, double* grad_dev, void* ws_dev,
                  size_t ws_bytes, void* stream) {
  if (!opts || !params_dev || !valid_data(n_models, n_samples, u_dev, y_dev)) return SPH_E_INVAL;
  if (grad_dev && (!ws_dev || ws_bytes < ws_layout(n_models, n_samples).total)) return SPH_E_CAPACITY;
  const FitArgs a = fit_args(opts, n_models, u_dev, y_dev, n_samples, ws_dev);
  const int blocks = (int)(a.sc.cols / kWave);
  hipLaunchKernelGGL(lpv_forward_kernel, dim3(blocks), dim3(kWave), 0, (hipStream_t)stream, a.d, a.sc, n_models,
                     params_dev, opts->sigma2, opts->sigmax, opts->lti_only, loss_dev, grad_dev, (double*)nullptr,
                     (double*)nullptr);
  return hip_rc(hipGetLastError());
}

int lpv_loss_grad_noalloc(const double* params_dev, int32_t n_models, const double* u_dev, const double* y_dev,
                          int32_t n_samples, const lpv_opts* opts, double* loss_dev, double* grad_dev,
                          void* stream) {
  if (!opts || !params_dev || !valid_data(n_models, n_samples, u_dev, y_dev)) return SPH_E_INVAL;
  // the record holds x, h1, h2 and p of every lane at every sample
  if ((size_t)n_samples * 4 * cols_for(n_models) * sizeof(double) > kNoAllocScratchBytes) return SPH_E_CAPACITY;
  double* traj = nullptr;
  const int rc = scratch_on_current_device(&traj);
  if (rc != SPH_OK) return rc;
  const Data d{u_dev, y_dev, n_samples, 0};
  const Scratch sc{traj, cols_for(n_models)};
  const int blocks = (int)(sc.cols / kWave);
  hipLaunchKernelGGL(lpv_forward_kernel, dim3(blocks), dim3(kWave), 0, (hipStream_t)stream, d, sc, n_models,
                     params_dev, opts->sigma2, opts->sigmax, opts->lti_only, loss_dev, grad_dev, (double*)nullptr,
                     (double*)nullptr);
  return hip_rc(hipGetLastError());
}

int lpv_adam(double* params_dev, int32_t n_models, const double* u_dev, const double* y_dev, int32_t n_samples,
             const lpv_opts* opts, int32_t iters, double* loss_dev, void* ws_dev, size_t ws_bytes, void* stream) {
  if (!opts || !params_dev || iters < 0 || !valid_data(n_models, n_samples, u_dev, y_dev)) return SPH_E_INVAL;
  if (!ws_dev || ws_bytes < ws_layout(n_models, n_samples).total) return SPH_E_CAPACITY;
  const FitArgs a = fit_args(opts, n_models, u_dev, y_dev, n_samples, ws_dev);
  const int blocks = (int)(a.sc.cols / kWave);
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(lpv_unpack, dim3(blocks), dim3(kWave), 0, st, a, (const double*)params_dev, (int)vX);
  hipLaunchKernelGGL(lpv_zero, dim3(blocks), dim3(kWave), 0, st, a, (int)vM, (int)vV + 1);
  const int chunk = evals_per_launch(n_samples);
  for (int t0 = 0; t0 < iters; t0 += chunk) {
    const int it = iters - t0 < chunk ? iters - t0 : chunk;
    hipLaunchKernelGGL(lpv_adam_kernel, dim3(blocks), dim3(kWave), 0, st, a, it, t0, opts->lr, opts->beta1,
                       opts->beta2, opts->eps, loss_dev);
  }
  hipLaunchKernelGGL(lpv_pack, dim3(blocks), dim3(kWave), 0, st, a, params_dev, (int)vX);
  return hip_rc(hipGetLastError());
}

int lpv_lbfgs(double* params_dev, int32_t n_models, const double* u_dev, const double* y_dev, int32_t n_samples,
              const lpv_opts* opts, int32_t max_iter, double* loss_dev, int32_t* status_dev, int32_t* iters_dev,
              void* ws_dev, size_t ws_bytes, void* stream) {
  if (!opts || !params_dev || max_iter < 0 || !valid_data(n_models, n_samples, u_dev, y_dev)) return SPH_E_INVAL;
  if (!ws_dev || ws_bytes < ws_layout(n_models, n_samples).total) return SPH_E_CAPACITY;
  const FitArgs a = fit_args(opts, n_models, u_dev, y_dev, n_samples, ws_dev);
  const int blocks = (int)(a.sc.cols / kWave);
  hipStream_t st = (hipStream_t)stream;
  const LbfgsOpts o{opts->c1, opts->gtol, opts->ftol, opts->max_backtracks, max_iter};
  hipLaunchKernelGGL(lpv_unpack, dim3(blocks), dim3(kWave), 0, st, a, (const double*)params_dev, (int)vX);
  hipLaunchKernelGGL(lpv_lbfgs_start, dim3(blocks), dim3(kWave), 0, st, a, o);
  const int chunk = evals_per_launch(n_samples);
  // every accepted step costs at most max_backtracks + 1 evaluations
  const long long max_evals = (long long)max_iter * (opts->max_backtracks + 1);
  const int R = n_models;
  const size_t cols = a.sc.cols;
  double* st_host = (double*)malloc(sizeof(double) * cols);
  if (!st_host) return SPH_E_INVAL;
  int rc = hip_rc(hipGetLastError());
  for (long long e = 0; rc == SPH_OK && e < max_evals; e += chunk) {
    hipLaunchKernelGGL(lpv_lbfgs_kernel, dim3(blocks), dim3(kWave), 0, st, a, o, chunk);
    rc = hip_rc(hipGetLastError());
    if (rc != SPH_OK) break;
    rc = hip_rc(hipMemcpyAsync(st_host, a.scal + (size_t)cStatus * cols, sizeof(double) * cols,
                               hipMemcpyDeviceToHost, st));
    if (rc == SPH_OK) rc = hip_rc(hipStreamSynchronize(st));
    if (rc != SPH_OK) break;
    bool all = true;
    for (int mm = 0; mm < R && all; ++mm) all = st_host[(size_t)mm * 4] != 0.0;
    if (all) break;
  }
  free(st_host);
  if (rc != SPH_OK) return rc;
  hipLaunchKernelGGL(lpv_pack, dim3(blocks), dim3(kWave), 0, st, a, params_dev, (int)vX);
  hipLaunchKernelGGL(lpv_lbfgs_finish, dim3(blocks), dim3(kWave), 0, st, a, loss_dev, status_dev, iters_dev);
  return hip_rc(hipGetLastError());
}

int lpv_closed_loop(const double* params_dev, int32_t n_models, const double* x0_dev, const double* force_dev,
                    int32_t force_per_model, const double* ref_dev, int32_t ref_per_model, int32_t n_samples,
                    double ts, double kp, double kd, const double* scales, double* y_dev, double* tau_dev,
                    void* stream) {
  if (!params_dev || !force_dev || !ref_dev || !scales || !y_dev || n_models <= 0 || n_samples <= 0 || !(ts > 0.0))
    return SPH_E_INVAL;
  Scales sc;
  for (int i = 0; i < 3; ++i) {
    sc.u[i] = scales[i];
    sc.y[i] = scales[3 + i];
    if (!(sc.u[i] > 0.0) || !(sc.y[i] > 0.0)) return SPH_E_INVAL;
  }
  const int blocks = (int)(cols_for(n_models) / kWave);
  hipLaunchKernelGGL(lpv_closed_loop_kernel, dim3(blocks), dim3(kWave), 0, (hipStream_t)stream, params_dev,
                     n_models, x0_dev, force_dev, force_per_model ? 1 : 0, ref_dev, ref_per_model ? 1 : 0, n_samples,
                     ts, kp, kd, sc, y_dev, tau_dev);
  return hip_rc(hipGetLastError());
}

}  // extern "C"
