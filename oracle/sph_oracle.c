/*
 * FP64 reference implementation ("oracle") of the sloshing simulator's step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the HIP kernels.
 *
 * What it computes, in the order of the paper's state-transition function
 * (Section 3.4, Algorithm "state transition function"), everything in double
 * precision and written for a reader to check against the equations by eye:
 *
 *   kernels        cubic spline W_cb (eq. cubicspline, support 2h) and spiky
 *                  W_s3 (eq. spiky3, support h_spiky), and dW/dr of both;
 *   neighbours     j is a neighbour of i iff |s_i - s_j|^2 < (2h)^2 (ghosts:
 *                  < (2h)^2 for density, < h_spiky^2 for wall forces); brute
 *                  force O(N^2) or a plain bucket grid, giving equal sets;
 *   density        rho_i = m (sum_f W_cb + gamma1 sum_g W_cb)  (eq. density_update,
 *                  self term included);
 *   pressure       Tait  P = B((rho/rho0)^gamma - 1), B = rho0 c0^2 / gamma,
 *                  or the paper's linear  P = k (rho - rho0)  (eq. EOS), each
 *                  also in a variant clamped at P >= 0 (no tension);
 *   fluid forces   symmetric pressure (eq. momentum) and artificial viscosity
 *                  (eq. viscous) with grad_i W = W'(r) r_ij / r  (Section 3.1);
 *   wall forces    ghost-to-fluid pressure (eq. pressure_b2f) and Akinci
 *                  viscosity (eq. viscous_b2f) with the spiky kernel; the tank
 *                  takes the equal and opposite reactions (eqs. pressure_f2b,
 *                  viscous_f2b), summed into the slosh wrench of eq. tankdynamics;
 *   rigid body     Newton-Euler in the plane (eq. tankdynamics), with the PD
 *                  attitude law and zero-order hold of Section 5.1, or a
 *                  prescribed rotation theta = A sin(2 pi f t);
 *   integrator     first-order symplectic Euler (Section 3.4): velocity first,
 *                  then position with the new velocity.
 *
 * Readings where the paper is silent, garbled or inconsistent:
 *   - the printed cubic-spline constant 15/(14 pi h^2) integrates to 3; the
 *     normalised constant 5/(14 pi h^2) is the default (kernel_norm = 0), the
 *     printed one is selectable (kernel_norm = 1);
 *   - the ghost-to-fluid pressure force acts on the fluid with the same sign
 *     as the fluid-fluid pressure force, -2 m^2 (P_i / rho_i^2) grad W_s3, so a
 *     positive pressure pushes the fluid away from the wall;
 *   - ghost density is the fluid particle's own (rho_g = rho_i) and ghost mass
 *     is the fluid mass;
 *   - the self term is in the density sum; no pair with r = 0 contributes a
 *     force (the gradient is taken as 0 there);
 *   - the fluid is integrated in the body frame of the tank, where the ghosts
 *     are fixed: the fluid acceleration gains the fictitious terms
 *       dw/dt = a_sph - R^T r'' - 2 theta' J w - theta'' J s + theta'^2 s,
 *     J v = (-v_y, v_x), obtained by differentiating x = r + R(theta) s twice;
 *     a world-frame mode (ora_rollout_world) follows eq. kinematicghost
 *     literally and converges to the body-frame mode as dt -> 0;
 *   - external force is given in the world frame (eq. tankdynamics).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
  int32_t eos;          /* 0 Tait, 1 linear, 2 linear and 3 Tait clamped at zero pressure */
  int32_t motion;       /* 0 free (Newton-Euler), 1 prescribed sine rotation */
  int32_t ctrl;         /* 0 none, 1 PD with zero-order hold */
  int32_t kernel_norm;  /* 0 normalised 5/(14 pi h^2), 1 as printed 15/(14 pi h^2) */
  double h, h_spiky, rho0, mass, c0, tait_gamma, k_lin;
  double visc_alpha, visc_beta, eps, gamma1, dt;
  double body_mass, body_inertia, kp, kd;
  int32_t ctrl_period;
  int32_t use_cells;    /* 1: bucket grid neighbour search, 0: brute force */
  double sine_amp, sine_freq;
  double domain_min[2], domain_max[2];
} ora_params;

/* rigid-body state carried between steps */
typedef struct {
  double r[2], theta, rdot[2], thetadot;
  double tau_ctrl;      /* torque held by the zero-order hold */
  int64_t step;         /* global step counter n; time t_n = n dt */
} ora_rigid;

enum { ORA_ESCAPED = 1, ORA_NONFINITE = 2, ORA_CFL = 4 };

/* Largest Courant number dt (c + |w|) / h a step may reach: twice the 0.2 the
 * time step is set from (the CFL condition of explicit weakly compressible
 * SPH; c is the equation of state's sound speed at rest). */
#define ORA_COURANT_MAX 0.4

/* When set (ora_set_round_f32), ora_rollout rounds the fluid state to
 * binary32 after every step: a reference for how far rounding at the
 * precision the GPU stores its state moves a long rollout and its finite
 * differences.  Off by default. */
static int g_round_f32 = 0;

void ora_set_round_f32(int on) { g_round_f32 = on ? 1 : 0; }

/* Sound speed at rest: c0 for the Tait law, sqrt(dP/drho) = sqrt(k) for the
 * linear law (eq. EOS). */
static double sound_speed(const ora_params* p) {
  return (p->eos == 1 || p->eos == 2) ? sqrt(p->k_lin) : p->c0;
}

/* ------------------------------------------------------------------------- */
/* kernels (eqs. cubicspline, spiky3)                                        */
/* ------------------------------------------------------------------------- */

static double cubic_const(double h, int printed) {
  return (printed ? 15.0 : 5.0) / (14.0 * M_PI * h * h);
}

double ora_w_cubic(double r, double h, int printed) {
  double q = r / h, c = cubic_const(h, printed);
  if (q < 1.0) return c * (pow(2.0 - q, 3) - 4.0 * pow(1.0 - q, 3));
  if (q < 2.0) return c * pow(2.0 - q, 3);
  return 0.0;
}

/* dW_cb / dr */
double ora_dw_cubic(double r, double h, int printed) {
  double q = r / h, c = cubic_const(h, printed);
  if (q < 1.0) return c / h * (-3.0 * pow(2.0 - q, 2) + 12.0 * pow(1.0 - q, 2));
  if (q < 2.0) return c / h * (-3.0 * pow(2.0 - q, 2));
  return 0.0;
}

double ora_w_spiky(double r, double hs) {
  if (r < hs) return 10.0 / (M_PI * pow(hs, 5)) * pow(hs - r, 3);
  return 0.0;
}

/* dW_s3 / dr */
double ora_dw_spiky(double r, double hs) {
  if (r < hs) return -30.0 / (M_PI * pow(hs, 5)) * pow(hs - r, 2);
  return 0.0;
}

/* equation of state (eq. EOS; Tait form for the stiffened variant) */
double ora_eos(const ora_params* p, double rho) {
  if (p->eos == 1) return p->k_lin * (rho - p->rho0);
  if (p->eos == 2) {              /* the linear law without tension */
    const double P = p->k_lin * (rho - p->rho0);
    return P > 0.0 ? P : 0.0;
  }
  double B = p->rho0 * p->c0 * p->c0 / p->tait_gamma;
  double P = B * (pow(rho / p->rho0, p->tait_gamma) - 1.0);
  if (p->eos == 3 && !(P > 0.0)) P = 0.0;   /* Tait without tension */
  return P;
}

/* ------------------------------------------------------------------------- */
/* neighbour search                                                          */
/* ------------------------------------------------------------------------- */

/* A plain bucket grid over [lo, lo + n*cell): cell >= the search radius, so
 * every neighbour of a point lies in its own or one of the 8 adjacent cells. */
typedef struct {
  double lo[2], cell;
  int n[2];
  int* start;   /* [ncells + 1] */
  int* items;   /* point indices, ascending within each cell */
} grid_t;

static void grid_cell(const grid_t* g, double x, double y, int* cx, int* cy) {
  double fx = floor((x - g->lo[0]) / g->cell), fy = floor((y - g->lo[1]) / g->cell);
  if (!(fx == fx)) fx = 0; /* NaN */
  if (!(fy == fy)) fy = 0;
  if (fx < 0) fx = 0;
  if (fy < 0) fy = 0;
  if (fx > g->n[0] - 1) fx = g->n[0] - 1;
  if (fy > g->n[1] - 1) fy = g->n[1] - 1;
  *cx = (int)fx;
  *cy = (int)fy;
}

static void grid_build(grid_t* g, const double* lo, const double* hi, double radius,
                       int np, const double* x, const double* y) {
  g->cell = radius * (1.0 + 1e-6);
  for (int d = 0; d < 2; ++d) {
    g->lo[d] = lo[d];
    g->n[d] = (int)ceil((hi[d] - lo[d]) / g->cell);
    if (g->n[d] < 1) g->n[d] = 1;
  }
  int nc = g->n[0] * g->n[1];
  g->start = (int*)calloc((size_t)nc + 1, sizeof(int));
  g->items = (int*)malloc(sizeof(int) * (size_t)(np > 0 ? np : 1));
  int* key = (int*)malloc(sizeof(int) * (size_t)(np > 0 ? np : 1));
  for (int i = 0; i < np; ++i) {
    int cx, cy;
    grid_cell(g, x[i], y[i], &cx, &cy);
    key[i] = cy * g->n[0] + cx;
    g->start[key[i] + 1]++;
  }
  for (int c = 0; c < nc; ++c) g->start[c + 1] += g->start[c];
  int* fillp = (int*)malloc(sizeof(int) * (size_t)nc);
  memcpy(fillp, g->start, sizeof(int) * (size_t)nc);
  for (int i = 0; i < np; ++i) g->items[fillp[key[i]]++] = i;
  free(fillp);
  free(key);
}

static void grid_free(grid_t* g) {
  free(g->start);
  free(g->items);
}

/* Collects, for point (xi, yi), the indices j of set (x, y) with squared
 * distance < radius^2 (self included if present), in ascending j order. */
typedef struct { int* j; int n, cap; } list_t;

static void list_push(list_t* l, int j) {
  if (l->n == l->cap) {
    l->cap = l->cap ? 2 * l->cap : 64;
    l->j = (int*)realloc(l->j, sizeof(int) * (size_t)l->cap);
  }
  l->j[l->n++] = j;
}

static int cmp_int(const void* a, const void* b) {
  int x = *(const int*)a, y = *(const int*)b;
  return (x > y) - (x < y);
}

static void find_within(const grid_t* g, int use_cells, double xi, double yi, double radius,
                        int np, const double* x, const double* y, list_t* out) {
  double r2 = radius * radius;
  out->n = 0;
  if (!use_cells) {
    for (int j = 0; j < np; ++j) {
      double dx = xi - x[j], dy = yi - y[j];
      if (dx * dx + dy * dy < r2) list_push(out, j);
    }
    return;
  }
  int cx, cy;
  grid_cell(g, xi, yi, &cx, &cy);
  for (int oy = -1; oy <= 1; ++oy) {
    int yy = cy + oy;
    if (yy < 0 || yy >= g->n[1]) continue;
    for (int ox = -1; ox <= 1; ++ox) {
      int xx = cx + ox;
      if (xx < 0 || xx >= g->n[0]) continue;
      int c = yy * g->n[0] + xx;
      for (int t = g->start[c]; t < g->start[c + 1]; ++t) {
        int j = g->items[t];
        double dx = xi - x[j], dy = yi - y[j];
        if (dx * dx + dy * dy < r2) list_push(out, j);
      }
    }
  }
  qsort(out->j, (size_t)out->n, sizeof(int), cmp_int);
}

/* Ordered pairs (i, j), i != j, of one point set within `radius`, sorted by
 * (i, j).  Returns the pair count (or -1 if it exceeds max_pairs). */
int ora_pairs(int np, const double* x, const double* y, double radius, int use_cells,
              const double* lo, const double* hi, int max_pairs, int* pi, int* pj) {
  grid_t g;
  memset(&g, 0, sizeof g);
  if (use_cells) grid_build(&g, lo, hi, radius, np, x, y);
  list_t l = {0, 0, 0};
  int count = 0;
  for (int i = 0; i < np; ++i) {
    find_within(&g, use_cells, x[i], y[i], radius, np, x, y, &l);
    for (int t = 0; t < l.n; ++t) {
      if (l.j[t] == i) continue;
      if (count < max_pairs) {
        pi[count] = i;
        pj[count] = l.j[t];
      }
      ++count;
    }
  }
  free(l.j);
  if (use_cells) grid_free(&g);
  return count <= max_pairs ? count : -1;
}

/* Same, in single precision with the distance formed as fmaf(dy, dy, dx*dx):
 * the predicate a single-precision implementation evaluates. */
int ora_pairs_f32(int np, const float* x, const float* y, float radius, int max_pairs,
                  int* pi, int* pj) {
  float r2 = radius * radius;
  int count = 0;
  for (int i = 0; i < np; ++i)
    for (int j = 0; j < np; ++j) {
      if (j == i) continue;
      float dx = x[i] - x[j];
      float dy = y[i] - y[j];
      float dxx = dx * dx;
      float d2 = fmaf(dy, dy, dxx);
      if (d2 < r2) {
        if (count < max_pairs) {
          pi[count] = i;
          pj[count] = j;
        }
        ++count;
      }
    }
  return count <= max_pairs ? count : -1;
}

/* ------------------------------------------------------------------------- */
/* SPH particle sums (Algorithm: density, EOS, forces, wall forces)          */
/* ------------------------------------------------------------------------- */

typedef struct {
  double* rho;       /* [n] */
  double* P;         /* [n] */
  double* ax;        /* [n] a_sph, the SPH acceleration (body-frame components) */
  double* ay;
  double wrench[3];  /* force of the fluid on the tank (frame of the inputs) and torque */
  double* fwall;     /* [n][3] or NULL: each particle's reaction on the tank (F_x, F_y, torque) */
  double* fwall_abs; /* [n][3] or NULL: per particle, the sums over its wall pairs of |F_x|, |F_y|
                        and |g_x F_y| + |g_y F_x| (the scale of the rounding of the wrench sums) */
} sums_t;

/* The particle sums.  Positions and velocities are in one frame (the body
 * frame in the body-frame mode); ghost velocities gvx/gvy may be NULL (zero).
 * Torque arms are measured from `arm_origin`.  */
static void particle_sums(const ora_params* p, int n, const double* sx, const double* sy,
                          const double* wx, const double* wy, int ng, const double* gx,
                          const double* gy, const double* gvx, const double* gvy,
                          const double* arm_origin, int use_cells, sums_t* out) {
  const double h = p->h, hs = p->h_spiky, m = p->mass;
  const int pr = p->kernel_norm;
  grid_t gf, gg;
  memset(&gf, 0, sizeof gf);
  memset(&gg, 0, sizeof gg);
  double lo[2] = {p->domain_min[0], p->domain_min[1]};
  double hi[2] = {p->domain_max[0], p->domain_max[1]};
  double rg = 2.0 * h > hs ? 2.0 * h : hs;
  if (use_cells) {
    grid_build(&gf, lo, hi, 2.0 * h, n, sx, sy);
    grid_build(&gg, lo, hi, rg, ng, gx, gy);
  }

  /* density and pressure */
#pragma omp parallel
  {
    list_t l = {0, 0, 0};
#pragma omp for schedule(static)
    for (int i = 0; i < n; ++i) {
      double sf = 0.0, sg = 0.0;
      find_within(&gf, use_cells, sx[i], sy[i], 2.0 * h, n, sx, sy, &l);
      for (int t = 0; t < l.n; ++t) {
        int j = l.j[t];
        sf += ora_w_cubic(hypot(sx[i] - sx[j], sy[i] - sy[j]), h, pr);
      }
      find_within(&gg, use_cells, sx[i], sy[i], 2.0 * h, ng, gx, gy, &l);
      for (int t = 0; t < l.n; ++t) {
        int k = l.j[t];
        sg += ora_w_cubic(hypot(sx[i] - gx[k], sy[i] - gy[k]), h, pr);
      }
      out->rho[i] = m * (sf + p->gamma1 * sg);
      out->P[i] = ora_eos(p, out->rho[i]);
    }
    free(l.j);
  }

  /* forces; wall forces per particle are kept to sum the wrench serially */
  double* fwx = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double* fwy = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double* fwt = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
  double* fwa = (double*)calloc((size_t)(n > 0 ? n : 1) * 3, sizeof(double));
#pragma omp parallel
  {
    list_t l = {0, 0, 0};
#pragma omp for schedule(static)
    for (int i = 0; i < n; ++i) {
      double ax = 0.0, ay = 0.0;
      double Pi = out->P[i] / (out->rho[i] * out->rho[i]);
      /* fluid-fluid: a_i = sum_j (-m (P_i/rho_i^2 + P_j/rho_j^2)
       *                          + m 2 alpha h/(rho_i+rho_j) (w_ij.s_ij)/(r^2+eps h^2)) grad_i W */
      find_within(&gf, use_cells, sx[i], sy[i], 2.0 * h, n, sx, sy, &l);
      for (int t = 0; t < l.n; ++t) {
        int j = l.j[t];
        if (j == i) continue;
        double rx = sx[i] - sx[j], ry = sy[i] - sy[j];
        double r = hypot(rx, ry);
        if (r == 0.0) continue;
        double gW = ora_dw_cubic(r, h, pr) / r;   /* grad_i W = gW * r_ij */
        double Pj = out->P[j] / (out->rho[j] * out->rho[j]);
        double press = m * (Pi + Pj);
        double vr = (wx[i] - wx[j]) * rx + (wy[i] - wy[j]) * ry;
        double visc = m * 2.0 * p->visc_alpha * h / (out->rho[i] + out->rho[j]) * vr /
                      (r * r + p->eps * h * h);
        ax += (-press + visc) * gW * rx;
        ay += (-press + visc) * gW * ry;
      }
      /* ghost-to-fluid: F_ik = m^2 (-2 P_i/rho_i^2 + 2 beta/(rho_i+rho_g) min(v.r,0)/(r^2+eps h^2)) grad W_s3 */
      double fx = 0.0, fy = 0.0, tq = 0.0, fxa = 0.0, fya = 0.0, tqa = 0.0;
      find_within(&gg, use_cells, sx[i], sy[i], hs, ng, gx, gy, &l);
      for (int t = 0; t < l.n; ++t) {
        int k = l.j[t];
        double rx = sx[i] - gx[k], ry = sy[i] - gy[k];
        double r = hypot(rx, ry);
        if (r == 0.0) continue;
        double gW = ora_dw_spiky(r, hs) / r;
        double vx = wx[i] - (gvx ? gvx[k] : 0.0), vy = wy[i] - (gvy ? gvy[k] : 0.0);
        double vr = vx * rx + vy * ry;
        double rho_g = out->rho[i];
        double coef = m * m * (-2.0 * Pi + 2.0 * p->visc_beta / (out->rho[i] + rho_g) *
                                              fmin(vr, 0.0) / (r * r + p->eps * h * h));
        double Fx = coef * gW * rx, Fy = coef * gW * ry;
        ax += Fx / m;
        ay += Fy / m;
        /* reaction on the tank at the ghost: -F_ik, torque arm g_k - origin */
        fx -= Fx;
        fy -= Fy;
        tq -= (gx[k] - arm_origin[0]) * Fy - (gy[k] - arm_origin[1]) * Fx;
        fxa += fabs(Fx);
        fya += fabs(Fy);
        tqa += fabs((gx[k] - arm_origin[0]) * Fy) + fabs((gy[k] - arm_origin[1]) * Fx);
      }
      out->ax[i] = ax;
      out->ay[i] = ay;
      fwx[i] = fx;
      fwy[i] = fy;
      fwt[i] = tq;
      fwa[3 * i] = fxa;
      fwa[3 * i + 1] = fya;
      fwa[3 * i + 2] = tqa;
    }
    free(l.j);
  }
  if (out->fwall)
    for (int i = 0; i < n; ++i) {
      out->fwall[3 * i] = fwx[i];
      out->fwall[3 * i + 1] = fwy[i];
      out->fwall[3 * i + 2] = fwt[i];
    }
  if (out->fwall_abs)
    for (int i = 0; i < 3 * n; ++i) out->fwall_abs[i] = fwa[i];
  free(fwa);
  out->wrench[0] = out->wrench[1] = out->wrench[2] = 0.0;
  for (int i = 0; i < n; ++i) {
    out->wrench[0] += fwx[i];
    out->wrench[1] += fwy[i];
    out->wrench[2] += fwt[i];
  }
  free(fwx);
  free(fwy);
  free(fwt);
  if (use_cells) {
    grid_free(&gf);
    grid_free(&gg);
  }
}

/* ------------------------------------------------------------------------- */
/* rigid body (eq. tankdynamics), controller, fictitious accelerations       */
/* ------------------------------------------------------------------------- */

static void prescribed(const ora_params* p, double t, double* th, double* thd, double* thdd) {
  double w = 2.0 * M_PI * p->sine_freq;
  *th = p->sine_amp * sin(w * t);
  *thd = p->sine_amp * w * cos(w * t);
  *thdd = -p->sine_amp * w * w * sin(w * t);
}

/* Controller update at step n (zero-order hold: a new torque only at
 * multiples of ctrl_period, from the sampled angle and rate). */
static void control(const ora_params* p, ora_rigid* b, const double* theta_ref, int n_ref) {
  if (p->ctrl != 1 || p->ctrl_period <= 0) return;
  if (b->step % p->ctrl_period != 0) return;
  int64_t k = b->step / p->ctrl_period;
  double ref = (theta_ref && n_ref > 0) ? theta_ref[k < n_ref ? k : n_ref - 1] : 0.0;
  b->tau_ctrl = p->kp * (ref - b->theta) - p->kd * b->thetadot;
}

/* Rigid-body accelerations at step n from the body-frame wrench. */
static void rigid_accel(const ora_params* p, const ora_rigid* b, const double wrench_body[3],
                        const double u[3], double acc[3], double* th, double* thd) {
  if (p->motion == 1) {
    double tt, td, tdd;
    prescribed(p, (double)b->step * p->dt, &tt, &td, &tdd);
    acc[0] = acc[1] = 0.0;
    acc[2] = tdd;
    *th = tt;
    *thd = td;
    return;
  }
  double c = cos(b->theta), s = sin(b->theta);
  double Fx = c * wrench_body[0] - s * wrench_body[1];
  double Fy = s * wrench_body[0] + c * wrench_body[1];
  acc[0] = (Fx + u[0]) / p->body_mass;
  acc[1] = (Fy + u[1]) / p->body_mass;
  acc[2] = (wrench_body[2] + u[2] + b->tau_ctrl) / p->body_inertia;
  *th = b->theta;
  *thd = b->thetadot;
}

/* ------------------------------------------------------------------------- */
/* state-transition function in the body frame                               */
/* ------------------------------------------------------------------------- */

/* Evaluates xdot = f(x, u) at the given state (Algorithm "state transition
 * function") without advancing it.  Outputs: rho, P, a_sph and the body-frame
 * fluid acceleration dw/dt [n]; the body-frame slosh wrench [3]; the rigid
 * accelerations (r''_x, r''_y, theta'') [3]; optionally (fwall non-NULL) the
 * per-particle terms of the wrench sum [n][3], and (fwall_abs non-NULL) per
 * particle the sums of the magnitudes of its pair terms [n][3].  `rigid` = r_x, r_y, theta,
 * rdot_x, rdot_y, thetadot; tau_ctrl the held controller torque; step n. */
int ora_rhs(const ora_params* p, int n, const double* sx, const double* sy, const double* wx,
            const double* wy, int ng, const double* gx, const double* gy, const double* rigid,
            double tau_ctrl, int64_t step, const double* u, double* rho, double* P, double* ax,
            double* ay, double* dwx, double* dwy, double* wrench, double* acc, double* fwall,
            double* fwall_abs) {
  sums_t s = {rho, P, ax, ay, {0, 0, 0}, fwall, fwall_abs};
  double origin[2] = {0.0, 0.0};
  particle_sums(p, n, sx, sy, wx, wy, ng, gx, gy, NULL, NULL, origin, p->use_cells, &s);
  ora_rigid b = {{rigid[0], rigid[1]}, rigid[2], {rigid[3], rigid[4]}, rigid[5], tau_ctrl, step};
  double th, thd;
  rigid_accel(p, &b, s.wrench, u, acc, &th, &thd);
  double c = cos(th), sn = sin(th);
  /* R^T r'' */
  double ab_x = c * acc[0] + sn * acc[1], ab_y = -sn * acc[0] + c * acc[1];
  for (int i = 0; i < n; ++i) {
    /* dw/dt = a_sph - R^T r'' - 2 thd J w - thdd J s + thd^2 s, J v = (-v_y, v_x) */
    dwx[i] = ax[i] - ab_x - 2.0 * thd * (-wy[i]) - acc[2] * (-sy[i]) + thd * thd * sx[i];
    dwy[i] = ay[i] - ab_y - 2.0 * thd * (wx[i]) - acc[2] * (sx[i]) + thd * thd * sy[i];
  }
  wrench[0] = s.wrench[0];
  wrench[1] = s.wrench[1];
  wrench[2] = s.wrench[2];
  return 0;
}

/* Advances the body-frame state by n_steps symplectic-Euler steps.
 *   state:   sx, sy, wx, wy [n] (in/out); rigid[6] (in/out); tau_ctrl (in/out);
 *            step (in/out), the global step counter.
 *   inputs:  u_seq [n_steps][3] (F_x, F_y in the world frame, torque), may be NULL;
 *            theta_ref [n_ref], the reference at control instants k = n / ctrl_period.
 *   logs:    entry k holds the state at local step k*log_stride and the wrench
 *            evaluated there: y_log [n_log][6] (r, theta, rdot, thetadot),
 *            wrench_log [n_log][3] (body frame), u_log [n_log][3] (applied
 *            F_x, F_y, total torque), wrench_mean_log [n_log][3] (mean body-frame
 *            wrench over the steps of the log interval); any may be NULL.
 *   returns: status bits (1 = a particle left the domain, 2 = non-finite value,
 *            4 = a particle's Courant number dt (c + |w|) / h exceeded
 *            ORA_COURANT_MAX after an update). */
int ora_rollout(const ora_params* p, int n, double* sx, double* sy, double* wx, double* wy,
                int ng, const double* gx, const double* gy, double* rigid, double* tau_ctrl,
                int64_t* step, int n_steps, const float* u_seq, const double* theta_ref,
                int n_ref, int log_stride, double* y_log, double* wrench_log, double* u_log,
                double* wrench_mean_log) {
  int status = 0;
  size_t nn = (size_t)(n > 0 ? n : 1);
  double* rho = (double*)malloc(nn * sizeof(double));
  double* P = (double*)malloc(nn * sizeof(double));
  double* ax = (double*)malloc(nn * sizeof(double));
  double* ay = (double*)malloc(nn * sizeof(double));
  double* dwx = (double*)malloc(nn * sizeof(double));
  double* dwy = (double*)malloc(nn * sizeof(double));
  ora_rigid b = {{rigid[0], rigid[1]}, rigid[2], {rigid[3], rigid[4]}, rigid[5], *tau_ctrl, *step};
  double mean_acc[3] = {0, 0, 0};
  int mean_cnt = 0;
  const double c_snd = sound_speed(p);
  for (int it = 0; it < n_steps; ++it) {
    double u[3] = {0, 0, 0};
    if (u_seq) {
      u[0] = u_seq[3 * it];
      u[1] = u_seq[3 * it + 1];
      u[2] = u_seq[3 * it + 2];
    }
    control(p, &b, theta_ref, n_ref);
    double rg[6] = {b.r[0], b.r[1], b.theta, b.rdot[0], b.rdot[1], b.thetadot};
    double wrench[3], acc[3];
    ora_rhs(p, n, sx, sy, wx, wy, ng, gx, gy, rg, b.tau_ctrl, b.step, u, rho, P, ax, ay, dwx, dwy,
            wrench, acc, NULL, NULL);
    if (log_stride > 0 && it % log_stride == 0) {
      int k = it / log_stride;
      if (y_log) {
        double* y = y_log + 6 * k;
        y[0] = b.r[0]; y[1] = b.r[1]; y[2] = b.theta;
        y[3] = b.rdot[0]; y[4] = b.rdot[1]; y[5] = b.thetadot;
      }
      if (wrench_log) {
        wrench_log[3 * k] = wrench[0];
        wrench_log[3 * k + 1] = wrench[1];
        wrench_log[3 * k + 2] = wrench[2];
      }
      if (u_log) {
        u_log[3 * k] = u[0];
        u_log[3 * k + 1] = u[1];
        u_log[3 * k + 2] = u[2] + b.tau_ctrl;
      }
    }
    for (int d = 0; d < 3; ++d) mean_acc[d] += wrench[d];
    ++mean_cnt;
    if (log_stride > 0 && (it % log_stride == log_stride - 1 || it == n_steps - 1)) {
      if (wrench_mean_log) {
        int k = it / log_stride;
        for (int d = 0; d < 3; ++d) wrench_mean_log[3 * k + d] = mean_acc[d] / mean_cnt;
      }
      mean_acc[0] = mean_acc[1] = mean_acc[2] = 0.0;
      mean_cnt = 0;
    }
    /* symplectic Euler: velocity, then position with the new velocity */
    for (int i = 0; i < n; ++i) {
      wx[i] += p->dt * dwx[i];
      wy[i] += p->dt * dwy[i];
      sx[i] += p->dt * wx[i];
      sy[i] += p->dt * wy[i];
      if (g_round_f32) {
        wx[i] = (double)(float)wx[i];
        wy[i] = (double)(float)wy[i];
        sx[i] = (double)(float)sx[i];
        sy[i] = (double)(float)sy[i];
      }
      if (!isfinite(sx[i]) || !isfinite(sy[i]) || !isfinite(wx[i]) || !isfinite(wy[i])) {
        status |= ORA_NONFINITE;
      } else {
        if (sx[i] < p->domain_min[0] || sx[i] >= p->domain_max[0] ||
            sy[i] < p->domain_min[1] || sy[i] >= p->domain_max[1])
          status |= ORA_ESCAPED;
        if (p->dt * (c_snd + sqrt(wx[i] * wx[i] + wy[i] * wy[i])) > ORA_COURANT_MAX * p->h)
          status |= ORA_CFL;
      }
    }
    if (p->motion == 1) {
      double th, thd, thdd;
      prescribed(p, (double)(b.step + 1) * p->dt, &th, &thd, &thdd);
      b.theta = th;
      b.thetadot = thd;
      b.r[0] = b.r[1] = b.rdot[0] = b.rdot[1] = 0.0;
    } else {
      b.rdot[0] += p->dt * acc[0];
      b.rdot[1] += p->dt * acc[1];
      b.thetadot += p->dt * acc[2];
      b.r[0] += p->dt * b.rdot[0];
      b.r[1] += p->dt * b.rdot[1];
      b.theta += p->dt * b.thetadot;
    }
    b.step += 1;
  }
  rigid[0] = b.r[0]; rigid[1] = b.r[1]; rigid[2] = b.theta;
  rigid[3] = b.rdot[0]; rigid[4] = b.rdot[1]; rigid[5] = b.thetadot;
  *tau_ctrl = b.tau_ctrl;
  *step = b.step;
  free(rho); free(P); free(ax); free(ay); free(dwx); free(dwy);
  return status;
}

/* ------------------------------------------------------------------------- */
/* world-frame mode: Algorithm "state transition function" read literally    */
/* ------------------------------------------------------------------------- */

/* Fluid positions xx, xy and velocities vx, vy are world-frame.  Each step
 * moves the ghosts with eq. kinematicghost (x_g = R g^B + r, v_g = rdot +
 * thetadot x (x_g - r)), evaluates the same particle sums on world-frame
 * quantities, and advances fluid and rigid body by symplectic Euler.  Brute-
 * force neighbours only (the grid is fixed in the body frame).  Optional
 * outputs: wrench_log [n_steps][3] (world force, torque) per step. */
int ora_rollout_world(const ora_params* p, int n, double* xx, double* xy, double* vx, double* vy,
                      int ng, const double* gbx, const double* gby, double* rigid,
                      double* tau_ctrl, int64_t* step, int n_steps, const float* u_seq,
                      const double* theta_ref, int n_ref, double* wrench_log) {
  size_t nn = (size_t)(n > 0 ? n : 1), gg = (size_t)(ng > 0 ? ng : 1);
  double* rho = (double*)malloc(nn * sizeof(double));
  double* P = (double*)malloc(nn * sizeof(double));
  double* ax = (double*)malloc(nn * sizeof(double));
  double* ay = (double*)malloc(nn * sizeof(double));
  double* gx = (double*)malloc(gg * sizeof(double));
  double* gy = (double*)malloc(gg * sizeof(double));
  double* gvx = (double*)malloc(gg * sizeof(double));
  double* gvy = (double*)malloc(gg * sizeof(double));
  ora_rigid b = {{rigid[0], rigid[1]}, rigid[2], {rigid[3], rigid[4]}, rigid[5], *tau_ctrl, *step};
  for (int it = 0; it < n_steps; ++it) {
    double u[3] = {0, 0, 0};
    if (u_seq) {
      u[0] = u_seq[3 * it];
      u[1] = u_seq[3 * it + 1];
      u[2] = u_seq[3 * it + 2];
    }
    control(p, &b, theta_ref, n_ref);
    double th = b.theta, thd = b.thetadot, thdd_pres = 0.0;
    if (p->motion == 1) prescribed(p, (double)b.step * p->dt, &th, &thd, &thdd_pres);
    double c = cos(th), s = sin(th);
    for (int k = 0; k < ng; ++k) {
      gx[k] = c * gbx[k] - s * gby[k] + b.r[0];
      gy[k] = s * gbx[k] + c * gby[k] + b.r[1];
      /* thetadot x (x_g - r) in the plane: thetadot * J (x_g - r) */
      gvx[k] = b.rdot[0] - thd * (gy[k] - b.r[1]);
      gvy[k] = b.rdot[1] + thd * (gx[k] - b.r[0]);
    }
    sums_t sm = {rho, P, ax, ay, {0, 0, 0}, NULL, NULL};
    ora_params q = *p;
    q.use_cells = 0;
    particle_sums(&q, n, xx, xy, vx, vy, ng, gx, gy, gvx, gvy, b.r, 0, &sm);
    double acc[3];
    if (p->motion == 1) {
      acc[0] = acc[1] = 0.0;
      acc[2] = thdd_pres;
    } else {
      acc[0] = (sm.wrench[0] + u[0]) / p->body_mass;
      acc[1] = (sm.wrench[1] + u[1]) / p->body_mass;
      acc[2] = (sm.wrench[2] + u[2] + b.tau_ctrl) / p->body_inertia;
    }
    if (wrench_log) {
      wrench_log[3 * it] = sm.wrench[0];
      wrench_log[3 * it + 1] = sm.wrench[1];
      wrench_log[3 * it + 2] = sm.wrench[2];
    }
    for (int i = 0; i < n; ++i) {
      vx[i] += p->dt * ax[i];
      vy[i] += p->dt * ay[i];
      xx[i] += p->dt * vx[i];
      xy[i] += p->dt * vy[i];
    }
    if (p->motion == 1) {
      double a, ad, add;
      prescribed(p, (double)(b.step + 1) * p->dt, &a, &ad, &add);
      b.theta = a;
      b.thetadot = ad;
      b.r[0] = b.r[1] = b.rdot[0] = b.rdot[1] = 0.0;
    } else {
      b.rdot[0] += p->dt * acc[0];
      b.rdot[1] += p->dt * acc[1];
      b.thetadot += p->dt * acc[2];
      b.r[0] += p->dt * b.rdot[0];
      b.r[1] += p->dt * b.rdot[1];
      b.theta += p->dt * b.thetadot;
    }
    b.step += 1;
  }
  rigid[0] = b.r[0]; rigid[1] = b.r[1]; rigid[2] = b.theta;
  rigid[3] = b.rdot[0]; rigid[4] = b.rdot[1]; rigid[5] = b.thetadot;
  *tau_ctrl = b.tau_ctrl;
  *step = b.step;
  free(rho); free(P); free(ax); free(ay); free(gx); free(gy); free(gvx); free(gvy);
  return 0;
}

int ora_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the parallel loops from now on (timing the oracle on one core
 * and on all of them). */
void ora_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* Terms of the analytic wall correction (eq. gamma1, after Koschier et al.):
 * for every fluid particle i, num_i = rho0 / m - sum_f W(r_if) (the fluid
 * sum of the density, self term included) and den_i = sum_g W(r_ig) (the
 * printed denominator index is read as a sum over the ghosts), so that
 * gamma1 = num_i / den_i makes particle i sit at rest density.  Positions
 * are separate x and y arrays; O(n (n + ng)), plain loops. */
void ora_gamma1_terms(const ora_params* p, int n, const double* sx, const double* sy, int ng, const double* gx,
                      const double* gy, double* num, double* den) {
  const int pr = p->kernel_norm;
  for (int i = 0; i < n; ++i) {
    double sf = 0.0, sg = 0.0;
    for (int j = 0; j < n; ++j) sf += ora_w_cubic(hypot(sx[i] - sx[j], sy[i] - sy[j]), p->h, pr);
    for (int k = 0; k < ng; ++k) sg += ora_w_cubic(hypot(sx[i] - gx[k], sy[i] - gy[k]), p->h, pr);
    num[i] = p->rho0 / p->mass - sf;
    den[i] = sg;
  }
}
