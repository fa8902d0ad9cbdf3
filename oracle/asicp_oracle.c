/*
 * asicp_oracle.c -- plain FP64 CPU oracle of the Annealed Stein ICP grasp
 * iteration (arXiv 2412.08346, Sec. III-IV and Algorithm 1).
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the CPU
 * baseline leg of the benchmark, never by the product path.  It is written to
 * be read against the paper, not to be fast: brute-force nearest neighbours,
 * sequential sums in a fixed order, a full sort for the median.  OpenMP runs
 * independent particles on separate threads; every per-particle quantity is
 * still summed in one fixed order, so results do not depend on thread count.
 *
 * Where the paper is silent or ambiguous the reading taken is stated at the
 * function that implements it (see also the readings table of the design
 * notes).
 */
#include "asicp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int32_t or_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads used by the parallel loops from now on (at least 1); results do not
 * depend on it. */
void or_set_threads(int32_t n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? (int)n : 1);
#else
  (void)n;
#endif
}

/* Rotation matrix of the unit quaternion q = (w, x, y, z) (Sec. III-A: R is
 * parametrised by theta^{4:7}); row-major. */
void or_quat_to_rot(const double q[4], double Rm[9]) {
  const double w = q[0], x = q[1], y = q[2], z = q[3];
  Rm[0] = 1.0 - 2.0 * (y * y + z * z);
  Rm[1] = 2.0 * (x * y - w * z);
  Rm[2] = 2.0 * (x * z + w * y);
  Rm[3] = 2.0 * (x * y + w * z);
  Rm[4] = 1.0 - 2.0 * (x * x + z * z);
  Rm[5] = 2.0 * (y * z - w * x);
  Rm[6] = 2.0 * (x * z - w * y);
  Rm[7] = 2.0 * (y * z + w * x);
  Rm[8] = 1.0 - 2.0 * (x * x + y * y);
}

/* Hamilton product a (x) b, scalar first. */
void or_quat_mul(const double a[4], const double b[4], double out[4]) {
  double r[4];
  r[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
  r[1] = a[0] * b[1] + b[0] * a[1] + (a[2] * b[3] - a[3] * b[2]);
  r[2] = a[0] * b[2] + b[0] * a[2] + (a[3] * b[1] - a[1] * b[3]);
  r[3] = a[0] * b[3] + b[0] * a[3] + (a[1] * b[2] - a[2] * b[1]);
  memcpy(out, r, sizeof r);
}

/* Unit quaternion of the rotation vector v (angle |v| about v/|v|). */
void or_quat_exp(const double v[3], double out[4]) {
  const double th = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  if (th == 0.0) {
    out[0] = 1.0; out[1] = out[2] = out[3] = 0.0;
    return;
  }
  const double s = sin(0.5 * th) / th;
  out[0] = cos(0.5 * th);
  out[1] = s * v[0]; out[2] = s * v[1]; out[3] = s * v[2];
}

static void mat_vec(const double Rm[9], const double v[3], double out[3]) {
  out[0] = Rm[0] * v[0] + Rm[1] * v[1] + Rm[2] * v[2];
  out[1] = Rm[3] * v[0] + Rm[4] * v[1] + Rm[5] * v[2];
  out[2] = Rm[6] * v[0] + Rm[7] * v[1] + Rm[8] * v[2];
}

static void mat_t_vec(const double Rm[9], const double v[3], double out[3]) {
  out[0] = Rm[0] * v[0] + Rm[3] * v[1] + Rm[6] * v[2];
  out[1] = Rm[1] * v[0] + Rm[4] * v[1] + Rm[7] * v[2];
  out[2] = Rm[2] * v[0] + Rm[5] * v[1] + Rm[8] * v[2];
}

static void cross(const double a[3], const double b[3], double out[3]) {
  out[0] = a[1] * b[2] - a[2] * b[1];
  out[1] = a[2] * b[0] - a[0] * b[2];
  out[2] = a[0] * b[1] - a[1] * b[0];
}

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the published mixing
 * function, used as a counter-based generator. */
uint64_t or_splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Mini-batch size of Table I at iteration k: the whole cloud scaled by
 * min(k, 2 k_max / 3) / (2 k_max / 3), at least one point (the table's "N" is
 * read as the object cloud size). */
int64_t or_batch_size(const or_config* cfg, int32_t k, int64_t M) {
  if (!cfg->minibatch) return M;
  const double full = 2.0 * (double)cfg->k_max / 3.0;
  const double frac = ((double)k < full ? (double)k : full) / full;
  int64_t m = (int64_t)ceil((double)M * frac);
  if (m < 1) m = 1;
  if (m > M) m = M;
  return m;
}

/* Key of the mini-batch of object o at iteration k. */
uint64_t or_batch_key(const or_config* cfg, int32_t k, int32_t o) {
  return or_splitmix64(or_splitmix64(cfg->seed) ^ ((uint64_t)(uint32_t)k << 20) ^ (uint64_t)(uint32_t)o);
}

/* A permutation of [0, M) keyed by `key`: a 4-round balanced Feistel network
 * on 2h bits (2^(2h) >= M) with SplitMix64 round functions, cycle-walked back
 * into [0, M).  The mini-batch of an iteration is {perm(j) : j < m_k}. */
int64_t or_batch_perm(int64_t j, int64_t M, uint64_t key) {
  int bits = 2;
  while (((int64_t)1 << bits) < M) ++bits;
  if (bits & 1) ++bits;
  const int hb = bits / 2;
  const uint64_t mask = ((uint64_t)1 << hb) - 1;
  uint64_t x = (uint64_t)j;
  do {
    uint64_t L = x >> hb, R = x & mask;
    for (uint64_t r = 0; r < 4; ++r) {
      const uint64_t F = or_splitmix64(key ^ (r << 56) ^ R) & mask;
      const uint64_t nL = R, nR = L ^ F;
      L = nL;
      R = nR;
    }
    x = (L << hb) | R;
  } while (x >= (uint64_t)M);
  return (int64_t)x;
}

/* Nearest neighbour of x among n points (eq. 1, point-to-point metric):
 * argmin of the squared distance; the lowest index wins an exact tie. */
int32_t or_nn_brute(const double* pts, int32_t n, const double x[3], double* d2) {
  int32_t best = -1;
  double bd = INFINITY;
  for (int32_t m = 0; m < n; ++m) {
    const double dx = x[0] - pts[3 * m + 0];
    const double dy = x[1] - pts[3 * m + 1];
    const double dz = x[2] - pts[3 * m + 2];
    const double d = dx * dx + dy * dy + dz * dz;
    if (d < bd) { bd = d; best = m; }
  }
  if (d2) *d2 = bd;
  return best;
}

/* As or_nn_brute over the points with mask[m] != 0. */
static int32_t or_nn_masked(const double* pts, int32_t n, const uint8_t* mask, const double x[3]) {
  int32_t best = -1;
  double bd = INFINITY;
  for (int32_t m = 0; m < n; ++m) {
    if (!mask[m]) continue;
    const double dx = x[0] - pts[3 * m + 0];
    const double dy = x[1] - pts[3 * m + 1];
    const double dz = x[2] - pts[3 * m + 2];
    const double d = dx * dx + dy * dy + dz * dz;
    if (d < bd) { bd = d; best = m; }
  }
  return best;
}

/* Trilinear interpolation of a signed distance grid (Sec. IV-C: the object
 * points are moved into the gripper frame and looked up in the gripper SDF).
 * Node (i, j, k) sits at origin + cell * (i, j, k); values are x fastest.
 * A point outside the node box is reported with *inside = 0 (it can never
 * collide).  The cell index is clamped so a point on the upper face uses the
 * last cell with weight 1.  Interpolation runs along x, then y, then z. */
double or_sdf_trilinear(const double* grid, const int32_t n[3], const double origin[3],
                        double cell, const double p[3], int32_t* inside) {
  int32_t i0[3];
  double f[3];
  for (int d = 0; d < 3; ++d) {
    const double u = (p[d] - origin[d]) / cell;
    if (!(u >= 0.0 && u <= (double)(n[d] - 1))) {
      *inside = 0;
      return NAN;
    }
    int32_t fl = (int32_t)floor(u);
    if (fl > n[d] - 2) fl = n[d] - 2;
    i0[d] = fl;
    f[d] = u - (double)fl;
  }
  *inside = 1;
  const int64_t nx = n[0], ny = n[1];
#define V(a, b, c) grid[((int64_t)(i0[2] + (c)) * ny + (i0[1] + (b))) * nx + (i0[0] + (a))]
  const double c00 = (1.0 - f[0]) * V(0, 0, 0) + f[0] * V(1, 0, 0);
  const double c10 = (1.0 - f[0]) * V(0, 1, 0) + f[0] * V(1, 1, 0);
  const double c01 = (1.0 - f[0]) * V(0, 0, 1) + f[0] * V(1, 0, 1);
  const double c11 = (1.0 - f[0]) * V(0, 1, 1) + f[0] * V(1, 1, 1);
#undef V
  const double c0 = (1.0 - f[1]) * c00 + f[1] * c10;
  const double c1 = (1.0 - f[1]) * c01 + f[1] * c11;
  return (1.0 - f[2]) * c0 + f[2] * c1;
}

/* Gradient of the trilinear interpolant with respect to the point (the
 * derivative of each lerp along its own axis, the other two weights held),
 * inside the node box; value as or_sdf_trilinear. */
double or_sdf_trilinear_grad(const double* grid, const int32_t n[3], const double origin[3],
                             double cell, const double p[3], int32_t* inside, double grad[3]) {
  const double phi = or_sdf_trilinear(grid, n, origin, cell, p, inside);
  grad[0] = grad[1] = grad[2] = 0.0;
  if (!*inside) return phi;
  int32_t i0[3];
  double f[3];
  for (int d = 0; d < 3; ++d) {
    const double u = (p[d] - origin[d]) / cell;
    int32_t fl = (int32_t)floor(u);
    if (fl > n[d] - 2) fl = n[d] - 2;
    i0[d] = fl;
    f[d] = u - (double)fl;
  }
  const int64_t nx = n[0], ny = n[1];
#define V(a, b, c) grid[((int64_t)(i0[2] + (c)) * ny + (i0[1] + (b))) * nx + (i0[0] + (a))]
  double g[3] = {0, 0, 0};
  for (int b = 0; b < 2; ++b)
    for (int c2 = 0; c2 < 2; ++c2) {
      const double wy = b ? f[1] : 1.0 - f[1], wz = c2 ? f[2] : 1.0 - f[2];
      g[0] += wy * wz * (V(1, b, c2) - V(0, b, c2));
    }
  for (int a = 0; a < 2; ++a)
    for (int c2 = 0; c2 < 2; ++c2) {
      const double wx = a ? f[0] : 1.0 - f[0], wz = c2 ? f[2] : 1.0 - f[2];
      g[1] += wx * wz * (V(a, 1, c2) - V(a, 0, c2));
    }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      const double wx = a ? f[0] : 1.0 - f[0], wy = b ? f[1] : 1.0 - f[1];
      g[2] += wx * wy * (V(a, b, 1) - V(a, b, 0));
    }
#undef V
  for (int d = 0; d < 3; ++d) grad[d] = g[d] / cell;
  return phi;
}

/* Per-object centre of mass (Algorithm 1 preprocessing; the centroid of the
 * object cloud, every point weighted equally), per-preshape tool centre point
 * (Sec. IV-B: the centre of the contact cloud), mean squared radius of the
 * contact cloud, and the diagonal preconditioner A of eq. (3).
 * Reading for A (the paper states it is 6x6 but gives no values): the
 * Gauss-Newton diagonal of the cost, 1/(1+lambda) on translation and
 * 3 / (2 (rho^2 + lambda |TCP|^2)) on the rotation vector; identity if asked. */
void or_setup(const or_problem* pb, const or_config* cfg, double* com, double* tcp,
              double* rho2, double* a_t, double* a_w) {
  for (int32_t o = 0; o < pb->n_obj; ++o) {
    double s[3] = {0, 0, 0};
    const int32_t m0 = pb->r_off[o], m1 = pb->r_off[o + 1];
    for (int32_t m = m0; m < m1; ++m)
      for (int d = 0; d < 3; ++d) s[d] += pb->R[3 * m + d];
    for (int d = 0; d < 3; ++d) com[3 * o + d] = (m1 > m0) ? s[d] / (double)(m1 - m0) : 0.0;
  }
  for (int32_t p = 0; p < pb->n_pre; ++p) {
    double s[3] = {0, 0, 0}, r2 = 0.0;
    const int32_t n0 = pb->s_off[p], n1 = pb->s_off[p + 1];
    for (int32_t n = n0; n < n1; ++n) {
      const double* sp = pb->S + 3 * n;
      for (int d = 0; d < 3; ++d) s[d] += sp[d];
      r2 += sp[0] * sp[0] + sp[1] * sp[1] + sp[2] * sp[2];
    }
    const double inv = 1.0 / (double)(n1 - n0);
    for (int d = 0; d < 3; ++d) tcp[3 * p + d] = s[d] * inv;
    rho2[p] = r2 * inv;
    const double* T = tcp + 3 * p;
    const double tcp2 = T[0] * T[0] + T[1] * T[1] + T[2] * T[2];
    if (cfg->precond == OR_PRECOND_IDENTITY) {
      a_t[p] = 1.0;
      a_w[p] = 1.0;
    } else {
      a_t[p] = 1.0 / (1.0 + cfg->lambda);
      a_w[p] = 3.0 / (2.0 * (rho2[p] + cfg->lambda * tcp2));
    }
  }
}

/* Annealing of iteration k.  Cyclic schedule of eq. (11) / Table I:
 * gamma = (mod(k, T/C) / (T/C))^p with T = k_max, repulsion weight tau = 1.
 * Geometric schedule: gamma = 1 and the repulsion is tempered by
 * tau_k = T0 (T1/T0)^(k/(k_max-1)). */
void or_schedule(const or_config* cfg, int32_t k, double* gamma, double* tau) {
  if (cfg->schedule == OR_SCHED_PAPER_CYCLIC) {
    const double period = (double)cfg->k_max / cfg->cyc_C;
    *gamma = pow(fmod((double)k, period) / period, cfg->cyc_p);
    *tau = 1.0;
  } else {
    *gamma = 1.0;
    const double frac = (cfg->k_max > 1) ? (double)k / (double)(cfg->k_max - 1) : 0.0;
    *tau = cfg->T0 * pow(cfg->T1 / cfg->T0, frac);
  }
}

static void locate(const or_problem* pb, int32_t i, int32_t* o, int32_t* p) {
  const int32_t g = i / pb->K;
  *o = g / pb->n_pre;
  *p = g % pb->n_pre;
}

static int32_t max_pre_points(const or_problem* pb) {
  int32_t mx = 0;
  for (int32_t p = 0; p < pb->n_pre; ++p) {
    const int32_t n = pb->s_off[p + 1] - pb->s_off[p];
    if (n > mx) mx = n;
  }
  return mx;
}

static int32_t max_col_points(const or_problem* pb) {
  int32_t mx = 0;
  for (int32_t o = 0; o < pb->n_obj; ++o) {
    const int32_t n = pb->c_off[o + 1] - pb->c_off[o];
    if (n > mx) mx = n;
  }
  return mx;
}

/* One evaluation of every particle at poses theta (Algorithm 1 loop body up
 * to the gradient replacement):
 *   1. transform the contact cloud, s' = R s + t;
 *   2. pair every s' with its nearest object point (eq. 1, full batch);
 *   3. cost C = 1/2 (L_ct + lambda L_com) (eqs. 13-15) and its gradient in
 *      translation g_t (eq. 16) and in a world-frame rotation vector g_w about
 *      the gripper origin; the quaternion gradient of eq. (17) is also
 *      returned;
 *   4. move every collision point into the gripper frame, c' = R^T (c - t),
 *      and look it up in the gripper SDF (Sec. IV-C).  Reading of the sign:
 *      the stored SDF is negative inside the gripper and a point collides when
 *      it is strictly inside, phi < 0 (the paper's "positive distance" uses
 *      the opposite sign convention);
 *   5. if any point collides, pair each colliding point with its nearest
 *      transformed contact point (eq. 18, the reverse direction of eq. 1) and
 *      replace the gradient by the gradient of 1/2 L_col taken as in eqs.
 *      (4)-(5); the TCP-CoM term is left out there. */
void or_eval(const or_problem* pb, const or_config* cfg, int32_t k, const double* theta,
             or_eval_out* out) {
  const int32_t Ktot = pb->n_obj * pb->n_pre * pb->K;
  const int32_t Nmax = max_pre_points(pb);
  const int32_t Mcmax = max_col_points(pb);
  double* com = (double*)malloc(sizeof(double) * 3 * (size_t)pb->n_obj);
  double* tcp = (double*)malloc(sizeof(double) * 3 * (size_t)pb->n_pre);
  double* rho2 = (double*)malloc(sizeof(double) * (size_t)pb->n_pre);
  double* a_t = (double*)malloc(sizeof(double) * (size_t)pb->n_pre);
  double* a_w = (double*)malloc(sizeof(double) * (size_t)pb->n_pre);
  or_setup(pb, cfg, com, tcp, rho2, a_t, a_w);
  const double lam = cfg->lambda;
  /* mini-batch of each object cloud (Algorithm 1 "select a mini-batch from R",
   * Table I size schedule; one batch per object and iteration, shared by its
   * particles): in_batch[m] over the concatenated clouds */
  const int32_t Mtot = pb->r_off[pb->n_obj];
  uint8_t* in_batch = (uint8_t*)malloc((size_t)Mtot + 1);
  for (int32_t o = 0; o < pb->n_obj; ++o) {
    const int32_t m0 = pb->r_off[o], M = pb->r_off[o + 1] - m0;
    const int64_t mb = or_batch_size(cfg, k, M);
    memset(in_batch + m0, mb == M ? 1 : 0, (size_t)M);
    if (mb < M) {
      const uint64_t key = or_batch_key(cfg, k, o);
      for (int64_t j = 0; j < mb; ++j) in_batch[m0 + or_batch_perm(j, M, key)] = 1;
    }
  }

#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t i = 0; i < Ktot; ++i) {
    int32_t o, p;
    locate(pb, i, &o, &p);
    const double* th = theta + 7 * (size_t)i;
    const double* tv = th;
    const double* q = th + 3;
    double Rm[9];
    or_quat_to_rot(q, Rm);
    const int32_t n0 = pb->s_off[p], N = pb->s_off[p + 1] - n0;
    const double* S = pb->S + 3 * (size_t)n0;
    const int32_t m0 = pb->r_off[o], M = pb->r_off[o + 1] - m0;
    const double* Rc = pb->R + 3 * (size_t)m0;
    const int32_t c0 = pb->c_off[o], Mc = pb->c_off[o + 1] - c0;
    const double* Cc = pb->C + 3 * (size_t)c0;
    double* sw = (double*)malloc(sizeof(double) * 3 * (size_t)N); /* s' */

    /* partial derivatives of R with respect to (w, x, y, z), row-major */
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    const double dR[4][9] = {
        {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0},
        {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x},
        {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y},
        {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0}};

    double sum_e2 = 0.0, sum_e[3] = {0, 0, 0}, sum_m[3] = {0, 0, 0}, sum_q[4] = {0, 0, 0, 0};
    for (int32_t n = 0; n < N; ++n) {
      double u[3], sp[3];
      mat_vec(Rm, S + 3 * n, u);
      for (int d = 0; d < 3; ++d) sp[d] = u[d] + tv[d];
      memcpy(sw + 3 * n, sp, sizeof sp);
      const int32_t j = or_nn_masked(Rc, M, in_batch + m0, sp);
      if (out->nn_idx) out->nn_idx[(size_t)i * Nmax + n] = j;
      double e[3], mxe[3];
      for (int d = 0; d < 3; ++d) e[d] = sp[d] - Rc[3 * j + d];
      sum_e2 += e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
      for (int d = 0; d < 3; ++d) sum_e[d] += e[d];
      cross(u, e, mxe);
      for (int d = 0; d < 3; ++d) sum_m[d] += mxe[d];
      for (int a = 0; a < 4; ++a) {
        double v[3];
        mat_vec(dR[a], S + 3 * n, v);
        sum_q[a] += e[0] * v[0] + e[1] * v[1] + e[2] * v[2];
      }
    }
    /* TCP-CoM term, eq. (15) */
    const double* T = tcp + 3 * p;
    double uT[3], eT[3], mT[3];
    mat_vec(Rm, T, uT);
    for (int d = 0; d < 3; ++d) eT[d] = uT[d] + tv[d] - com[3 * o + d];
    cross(uT, eT, mT);
    const double invN = 1.0 / (double)N;
    const double cost = 0.5 * (sum_e2 * invN + lam * (eT[0] * eT[0] + eT[1] * eT[1] + eT[2] * eT[2]));
    double gct[6];
    for (int d = 0; d < 3; ++d) {
      gct[d] = sum_e[d] * invN + lam * eT[d];
      gct[3 + d] = sum_m[d] * invN + lam * mT[d];
    }
    if (out->cost) out->cost[i] = cost;
    if (out->g_ct) memcpy(out->g_ct + 6 * (size_t)i, gct, sizeof gct);
    double* costp = out->cost ? out->cost + i : NULL;
    double* gctp = out->g_ct ? out->g_ct + 6 * (size_t)i : NULL;
    if (out->g_q) {
      for (int a = 0; a < 4; ++a) {
        double v[3];
        mat_vec(dR[a], T, v);
        out->g_q[4 * (size_t)i + a] = sum_q[a] * invN + lam * (eT[0] * v[0] + eT[1] * v[1] + eT[2] * v[2]);
      }
    }

    /* collision gate and reverse pairing */
    const double* grid = pb->sdf + pb->sdf_off[p];
    const int32_t* gn = pb->sdf_n + 3 * p;
    const double* gorg = pb->sdf_origin + 3 * p;
    const double gcell = pb->sdf_cell[p];
    int32_t ncol = 0;
    double col_e2 = 0.0, col_e[3] = {0, 0, 0}, col_m[3] = {0, 0, 0};
    double pen = 0.0, pen_t[3] = {0, 0, 0}, pen_w[3] = {0, 0, 0};
    for (int32_t m = 0; m < Mc; ++m) {
      const double* c = Cc + 3 * m;
      double dc[3], cp[3];
      for (int d = 0; d < 3; ++d) dc[d] = c[d] - tv[d];
      mat_t_vec(Rm, dc, cp);
      int32_t inside = 0;
      double gphi[3];
      const double phi = or_sdf_trilinear_grad(grid, gn, gorg, gcell, cp, &inside, gphi);
      const int collides = inside && (phi < 0.0);
      if (collides && cfg->w_pen > 0.0) {
        /* penetration phi^2 and its gradient: c' = R^T (c - t), so
         * d/dt = -R grad(phi) and d/dw = (R grad(phi)) x (c - t) */
        double rg[3], xg[3];
        mat_vec(Rm, gphi, rg);
        cross(rg, dc, xg);
        pen += phi * phi;
        for (int d = 0; d < 3; ++d) {
          pen_t[d] += 2.0 * phi * (-rg[d]);
          pen_w[d] += 2.0 * phi * xg[d];
        }
      }
      if (out->gate) out->gate[(size_t)i * Mcmax + m] = (uint8_t)collides;
      if (out->phi_c) out->phi_c[(size_t)i * Mcmax + m] = inside ? phi : NAN;
      int32_t jn = -1;
      if (collides) {
        ++ncol;
        jn = or_nn_brute(sw, N, c, NULL);
        double e[3], u[3], mxe[3];
        for (int d = 0; d < 3; ++d) e[d] = sw[3 * jn + d] - c[d];
        mat_vec(Rm, S + 3 * jn, u);
        cross(u, e, mxe);
        col_e2 += e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
        for (int d = 0; d < 3; ++d) { col_e[d] += e[d]; col_m[d] += mxe[d]; }
      }
      if (out->rev_idx) out->rev_idx[(size_t)i * Mcmax + m] = jn;
    }
    /* optional penetration term (w_pen (1/M_c) sum of phi^2 over colliding
     * points), added to the cost and to its gradient */
    double gpen[6] = {0, 0, 0, 0, 0, 0}, pcost = 0.0;
    if (cfg->w_pen > 0.0 && Mc > 0) {
      const double s = cfg->w_pen / (double)Mc;
      pcost = s * pen;
      for (int d = 0; d < 3; ++d) { gpen[d] = s * pen_t[d]; gpen[3 + d] = s * pen_w[d]; }
    }
    for (int d = 0; d < 6; ++d) gct[d] += gpen[d];
    if (costp) *costp = cost + pcost;
    if (gctp) memcpy(gctp, gct, sizeof gct);
    if (out->pen) out->pen[i] = pcost;
    double gcol[6] = {0, 0, 0, 0, 0, 0}, ccost = 0.0;
    if (ncol > 0) {
      const double inv = 1.0 / (double)ncol;
      ccost = 0.5 * col_e2 * inv;
      for (int d = 0; d < 3; ++d) { gcol[d] = col_e[d] * inv; gcol[3 + d] = col_m[d] * inv; }
    }
    if (out->ncol) out->ncol[i] = ncol;
    if (out->col_cost) out->col_cost[i] = ccost;
    if (out->g_col) memcpy(out->g_col + 6 * (size_t)i, gcol, sizeof gcol);
    if (out->g_fin) memcpy(out->g_fin + 6 * (size_t)i, ncol > 0 ? gcol : gct, sizeof gct);
    free(sw);
  }
  free(com); free(tcp); free(rho2); free(a_t); free(a_w);
  free(in_batch);
}

static int cmp_double(const void* a, const void* b) {
  const double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

/* RBF bandwidth h of eq. (9).  Reading: the median heuristic on squared
 * translation distances, h = lower-median_{i<j} |t_i - t_j|^2 / ln K, floored
 * at h_min; h = 1 for a single particle.  theta holds the group's K poses. */
double or_bandwidth(const double* theta, int32_t K, const or_config* cfg) {
  if (cfg->bw_mode == OR_BW_FIXED) return cfg->h_fixed;
  if (K < 2) return 1.0;
  const size_t P = (size_t)K * (size_t)(K - 1) / 2;
  double* d2 = (double*)malloc(sizeof(double) * P);
  size_t c = 0;
  for (int32_t i = 0; i < K; ++i)
    for (int32_t j = i + 1; j < K; ++j) {
      const double* a = theta + 7 * (size_t)i;
      const double* b = theta + 7 * (size_t)j;
      const double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
      d2[c++] = dx * dx + dy * dy + dz * dz;
    }
  qsort(d2, P, sizeof(double), cmp_double);
  const double med = d2[(P - 1) / 2];
  free(d2);
  const double h = med / log((double)K);
  return h > cfg->h_min ? h : cfg->h_min;
}

/* Stein ICP direction of eq. (8) for one group, in the 6-D tangent
 * (translation, world rotation vector).  Readings:
 *   - expectation form (1/K) sum_j, as in eq. (6);
 *   - the driving term is the preconditioned mean gradient, -gamma A g_j;
 *     no prior term (the paper gives no prior parameters);
 *   - kernel = RBF(translation, eq. 9) x |q_i . q_j| (rotation, eq. 10)
 *     in product mode; block mode uses the RBF for the translation rows and
 *     |q_i . q_j| for the rotation rows;
 *   - the repulsion is tau times the kernel gradient with respect to particle
 *     j, the translation part scaled by h/2: tau k_ij (t_i - t_j) and
 *     tau kt_ij s_ij 1/2 vec(q_i (x) conj(q_j)) with s_ij the sign of q_i . q_j.
 * kmat (optional) receives k_ij = kt_ij |q_i . q_j|; phi receives K x 6. */
void or_svgd_direction(const double* theta, const double* g, int32_t K, double h, double gamma,
                       double tau, double a_t, double a_w, int32_t kernel_mode, double* kmat,
                       double* phi) {
  for (int32_t i = 0; i < K; ++i) {
    const double* ti = theta + 7 * (size_t)i;
    const double* qi = ti + 3;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int32_t j = 0; j < K; ++j) {
      const double* tj = theta + 7 * (size_t)j;
      const double* qj = tj + 3;
      const double* gj = g + 6 * (size_t)j;
      const double dx = ti[0] - tj[0], dy = ti[1] - tj[1], dz = ti[2] - tj[2];
      const double kt = exp(-(dx * dx + dy * dy + dz * dz) / h);
      const double dot = qi[0] * qj[0] + qi[1] * qj[1] + qi[2] * qj[2] + qi[3] * qj[3];
      const double kr = fabs(dot);
      const double sgn = (dot >= 0.0) ? 1.0 : -1.0;
      if (kmat) kmat[(size_t)i * K + j] = kt * kr;
      double wdt, wrt, wdw, wrw; /* driving/repulsion weights, translation/rotation */
      if (kernel_mode == OR_KERNEL_BLOCK) {
        wdt = kt; wrt = kt; wdw = kr; wrw = sgn;
      } else {
        wdt = kt * kr; wrt = kt * kr; wdw = kt * kr; wrw = kt * sgn;
      }
      const double qjc[4] = {qj[0], -qj[1], -qj[2], -qj[3]};
      double qq[4];
      or_quat_mul(qi, qjc, qq);
      const double d[3] = {dx, dy, dz};
      for (int a = 0; a < 3; ++a) {
        acc[a] += wdt * (-gamma * a_t * gj[a]) + tau * wrt * d[a];
        acc[3 + a] += wdw * (-gamma * a_w * gj[3 + a]) + tau * wrw * 0.5 * qq[1 + a];
      }
    }
    for (int a = 0; a < 6; ++a) phi[6 * (size_t)i + a] = acc[a] / (double)K;
  }
}

/* Apply a tangent step to one pose: t += dt, q <- canon(normalize(Exp(dw) (x) q)),
 * canon choosing the sign with qw >= 0.  This is the update of eqs. (3) and (7)
 * carried out in the 6-D tangent that A in R^{6x6} acts on. */
void or_retract(double* th, const double dt[3], const double dw[3]) {
  for (int d = 0; d < 3; ++d) th[d] += dt[d];
  double e[4], qn[4];
  or_quat_exp(dw, e);
  or_quat_mul(e, th + 3, qn);
  const double nrm = sqrt(qn[0] * qn[0] + qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]);
  const double sg = (qn[0] < 0.0) ? -1.0 : 1.0;
  for (int a = 0; a < 4; ++a) th[3 + a] = sg * qn[a] / nrm;
}

/* One iteration k of Algorithm 1 for every group: evaluate, replace the
 * gradient on collision, then the SVGD update (k < k_stein, eqs. 7-8) computed
 * for all particles from the same poses before any pose moves, or the SGD-ICP
 * update (eq. 3).  Convergence (SGD phase only): relative cost change below
 * conv_tol against the previous iteration, and no collision; a converged
 * particle is frozen; a collision clears the flag.  h_out (per group) and
 * phi_out (per particle, 6) are optional.  Returns 0. */
int32_t or_step(const or_problem* pb, const or_config* cfg, int32_t k, double* theta,
                double* prev_cost, int32_t* converged, or_eval_out* ev, double* h_out,
                double* phi_out) {
  const int32_t G = pb->n_obj * pb->n_pre, K = pb->K, Ktot = G * K;
  or_eval_out local;
  memset(&local, 0, sizeof local);
  if (ev) local = *ev;
  double* cost = local.cost ? local.cost : (double*)malloc(sizeof(double) * Ktot);
  int32_t* ncol = local.ncol ? local.ncol : (int32_t*)malloc(sizeof(int32_t) * Ktot);
  double* g = local.g_fin ? local.g_fin : (double*)malloc(sizeof(double) * 6 * (size_t)Ktot);
  local.cost = cost; local.ncol = ncol; local.g_fin = g;
  or_eval(pb, cfg, k, theta, &local);

  double* com = (double*)malloc(sizeof(double) * 3 * (size_t)pb->n_obj);
  double* tcp = (double*)malloc(sizeof(double) * 3 * (size_t)pb->n_pre);
  double* rho2 = (double*)malloc(sizeof(double) * (size_t)pb->n_pre);
  double* a_t = (double*)malloc(sizeof(double) * (size_t)pb->n_pre);
  double* a_w = (double*)malloc(sizeof(double) * (size_t)pb->n_pre);
  or_setup(pb, cfg, com, tcp, rho2, a_t, a_w);
  double gamma, tau;
  or_schedule(cfg, k, &gamma, &tau);

  for (int32_t i = 0; i < Ktot; ++i)
    if (ncol[i] > 0) converged[i] = 0;

  if (k < cfg->k_stein) {
    double* phi = (double*)malloc(sizeof(double) * 6 * (size_t)Ktot);
    /* eq. (8): the driving term is the gradient of the log posterior, i.e.
     * minus the cost gradient plus the gradient of the log prior */
    double* gd = g;
    if (pb->prior) {
      gd = (double*)malloc(sizeof(double) * 6 * (size_t)Ktot);
      for (int32_t i = 0; i < Ktot; ++i) {
        double gp[6];
        or_log_prior(pb->prior + 9 * (size_t)(i / K), theta + 7 * (size_t)i, gp);
        for (int a = 0; a < 6; ++a) gd[6 * (size_t)i + a] = g[6 * (size_t)i + a] - gp[a];
      }
    }
    for (int32_t gi = 0; gi < G; ++gi) {
      const int32_t p = gi % pb->n_pre;
      const double* thg = theta + 7 * (size_t)gi * K;
      const double h = or_bandwidth(thg, K, cfg);
      if (h_out) h_out[gi] = h;
      or_svgd_direction(thg, gd + 6 * (size_t)gi * K, K, h, gamma, tau, a_t[p], a_w[p],
                        cfg->kernel_mode, NULL, phi + 6 * (size_t)gi * K);
    }
    if (gd != g) free(gd);
    for (int32_t i = 0; i < Ktot; ++i) {
      const double* ph = phi + 6 * (size_t)i;
      const double dt[3] = {cfg->eta * ph[0], cfg->eta * ph[1], cfg->eta * ph[2]};
      const double dw[3] = {cfg->eta * ph[3], cfg->eta * ph[4], cfg->eta * ph[5]};
      or_retract(theta + 7 * (size_t)i, dt, dw);
    }
    if (phi_out) memcpy(phi_out, phi, sizeof(double) * 6 * (size_t)Ktot);
    free(phi);
  } else {
    for (int32_t i = 0; i < Ktot; ++i) {
      const int32_t p = (i / K) % pb->n_pre;
      if (!converged[i] && ncol[i] == 0 && prev_cost[i] > 0.0 &&
          fabs(cost[i] - prev_cost[i]) < cfg->conv_tol * prev_cost[i])
        converged[i] = 1;
      const double* gi = g + 6 * (size_t)i;
      double* ph = phi_out ? phi_out + 6 * (size_t)i : NULL;
      const double dt[3] = {-a_t[p] * gi[0], -a_t[p] * gi[1], -a_t[p] * gi[2]};
      const double dw[3] = {-a_w[p] * gi[3], -a_w[p] * gi[4], -a_w[p] * gi[5]};
      if (ph) for (int a = 0; a < 3; ++a) { ph[a] = dt[a]; ph[3 + a] = dw[a]; }
      if (converged[i]) {
        if (ph) for (int a = 0; a < 6; ++a) ph[a] = 0.0;
        continue;
      }
      const double sdt[3] = {cfg->eta * dt[0], cfg->eta * dt[1], cfg->eta * dt[2]};
      const double sdw[3] = {cfg->eta * dw[0], cfg->eta * dw[1], cfg->eta * dw[2]};
      or_retract(theta + 7 * (size_t)i, sdt, sdw);
    }
    if (h_out) for (int32_t gi = 0; gi < G; ++gi) h_out[gi] = 0.0;
  }
  for (int32_t i = 0; i < Ktot; ++i) prev_cost[i] = cost[i];

  if (!ev || !ev->cost) free(cost);
  if (!ev || !ev->ncol) free(ncol);
  if (!ev || !ev->g_fin) free(g);
  free(com); free(tcp); free(rho2); free(a_t); free(a_w);
  return 0;
}

/* Log prior of a pose (Sec. III-C: Gaussian in translation, von Mises in
 * rotation), up to a constant, and its gradient in the 6-D tangent (t, world
 * rotation vector).  Translation: -w_t/2 |t - mu_t|^2.  Rotation: the matrix
 * von Mises-Fisher density on SO(3), kappa tr(R(mu_q)^T R(q)); its rotation
 * gradient is kappa times the axial vector of A - A^T with A = R(q) R(mu_q)^T,
 * the derivative of tr(M^T Exp(w) R) at w = 0. */
double or_log_prior(const double pr[9], const double theta[7], double grad[6]) {
  const double* mu = pr;
  const double w = pr[3], kappa = pr[8];
  double Rq[9], Rm[9], A[9];
  or_quat_to_rot(theta + 3, Rq);
  or_quat_to_rot(pr + 4, Rm);
  double lp = 0.0, tr = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double e = theta[a] - mu[a];
    lp -= 0.5 * w * e * e;
    grad[a] = -w * e;
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double v = 0.0;
      for (int m = 0; m < 3; ++m) v += Rq[3 * r + m] * Rm[3 * c + m];
      A[3 * r + c] = v;
    }
  tr = A[0] + A[4] + A[8];
  lp += kappa * tr;
  grad[3] = kappa * (A[5] - A[7]);
  grad[4] = kappa * (A[6] - A[2]);
  grad[5] = kappa * (A[1] - A[3]);
  return lp;
}

/* Returned grasp (Algorithm 1 return; Sec. VI-A): per object, the particle
 * with the lowest cost among those whose final pose does not collide, lowest
 * index on ties.  If every particle collides the lowest-cost particle overall
 * is returned with best_free = 0. */
void or_select(const or_problem* pb, const double* cost, const int32_t* ncol, int32_t* best_idx,
               int32_t* best_free) {
  const int32_t per_obj = pb->n_pre * pb->K;
  for (int32_t o = 0; o < pb->n_obj; ++o) {
    int32_t b = -1;
    double bc = INFINITY;
    for (int32_t i = o * per_obj; i < (o + 1) * per_obj; ++i)
      if (ncol[i] == 0 && cost[i] < bc) { bc = cost[i]; b = i; }
    best_free[o] = (b >= 0);
    if (b < 0) {
      for (int32_t i = o * per_obj; i < (o + 1) * per_obj; ++i)
        if (cost[i] < bc) { bc = cost[i]; b = i; }
    }
    best_idx[o] = b;
  }
}

/* Iterations k_start .. k_end-1, then (if k_end == k_max) the final
 * evaluation at theta_{k_max} and the selection.  Returns the iterations run. */
int32_t or_solve(const or_problem* pb, const or_config* cfg, int32_t k_start, int32_t k_end,
                 double* theta, double* prev_cost, int32_t* converged, or_eval_out* final_ev,
                 int32_t* best_idx, int32_t* best_free) {
  int32_t it = 0;
  for (int32_t k = k_start; k < k_end; ++k, ++it)
    or_step(pb, cfg, k, theta, prev_cost, converged, NULL, NULL, NULL);
  if (k_end == cfg->k_max) {
    const int32_t Ktot = pb->n_obj * pb->n_pre * pb->K;
    or_eval_out local;
    memset(&local, 0, sizeof local);
    if (final_ev) local = *final_ev;
    double* cost = local.cost ? local.cost : (double*)malloc(sizeof(double) * Ktot);
    int32_t* ncol = local.ncol ? local.ncol : (int32_t*)malloc(sizeof(int32_t) * Ktot);
    local.cost = cost; local.ncol = ncol;
    or_eval(pb, cfg, cfg->k_max, theta, &local);
    if (best_idx && best_free) or_select(pb, cost, ncol, best_idx, best_free);
    if (!final_ev || !final_ev->cost) free(cost);
    if (!final_ev || !final_ev->ncol) free(ncol);
  }
  return it;
}
