/*
 * asicp_oracle.h -- plain FP64 CPU oracle of the Annealed Stein ICP (AS-ICP)
 * grasp iteration of "Grasping by Parallel Shape Matching" (arXiv 2412.08346).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that the tests, the smoke
 * check and the CPU baseline of the benchmark can compare the HIP path with a
 * slow, obviously correct implementation written straight from the paper.  It
 * shares no code, header, table or helper with the HIP library and must never
 * be linked into, imported by or called from the product path.
 *
 * Conventions
 *   - every floating-point value is double; the caller converts the FP32 inputs
 *     (exactly) before calling;
 *   - point clouds are AoS, point i at [3*i + 0..2];
 *   - a pose theta is 7 doubles: translation (tx, ty, tz) then the unit
 *     quaternion (qw, qx, qy, qz), scalar first (Sec. III-A, Standard ICP);
 *   - particles are numbered i = ((o * n_pre) + p) * K + j for object o,
 *     preshape p, particle j; a "group" (o, p) holds K particles and is one
 *     SVGD population.
 */
#ifndef ASICP_ORACLE_H
#define ASICP_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n_obj;               /* objects                                        */
  int32_t n_pre;               /* preshapes (gripper finger configurations)      */
  int32_t K;                   /* particles per (object, preshape) group         */
  const double* R;             /* object clouds, concatenated, [3*Mtot]          */
  const int32_t* r_off;        /* [n_obj+1] point offsets into R                 */
  const double* C;             /* collision clouds, concatenated, [3*Mctot]      */
  const int32_t* c_off;        /* [n_obj+1]                                      */
  const double* S;             /* gripper contact clouds, concatenated [3*Ntot]  */
  const int32_t* s_off;        /* [n_pre+1]                                      */
  const double* sdf;           /* SDF grids, concatenated, x fastest             */
  const int64_t* sdf_off;      /* [n_pre] value offsets into sdf                 */
  const int32_t* sdf_n;        /* [3*n_pre] (nx, ny, nz)                         */
  const double* sdf_origin;    /* [3*n_pre] position of node (0,0,0)             */
  const double* sdf_cell;      /* [n_pre] node spacing                           */
  const double* prior;         /* optional [n_obj*n_pre*9] per group: mean
                                  translation mu_t[3], its precision w_t
                                  (1/sigma^2), mean rotation mu_q[4] (unit),
                                  concentration kappa; NULL: no prior          */
} or_problem;

enum { OR_PRECOND_GN_DIAG = 0, OR_PRECOND_IDENTITY = 1 };
enum { OR_SCHED_GEOMETRIC = 0, OR_SCHED_PAPER_CYCLIC = 1 };
enum { OR_KERNEL_PRODUCT = 0, OR_KERNEL_BLOCK = 1 };
enum { OR_BW_MEDIAN = 0, OR_BW_FIXED = 1 };

typedef struct {
  int32_t k_max;        /* total iterations                                    */
  int32_t k_stein;      /* iterations with the SVGD update; SGD-ICP after      */
  double eta;           /* learning rate                                       */
  double lambda;        /* weight of the TCP-CoM loss                          */
  int32_t precond;      /* OR_PRECOND_*                                        */
  int32_t schedule;     /* OR_SCHED_*                                          */
  double T0, T1;        /* geometric temperature, first and last iteration     */
  double cyc_C, cyc_p;  /* cyclic annealing: cycles C and exponent p           */
  int32_t kernel_mode;  /* OR_KERNEL_*                                         */
  int32_t bw_mode;      /* OR_BW_*                                             */
  double h_fixed;       /* bandwidth for OR_BW_FIXED                           */
  double h_min;         /* floor of the median-heuristic bandwidth             */
  double conv_tol;      /* relative cost change that counts as converged       */
  double w_pen;         /* weight of the SDF penetration term (0: paper's cost) */
  int32_t minibatch;    /* 0: whole object cloud; 1: Table I mini-batch schedule */
  uint64_t seed;        /* mini-batch sampling seed                             */
} or_config;

/* Per-particle results of one evaluation (steps 1-4 of an iteration).  Every
 * pointer may be NULL; sizes use Ktot = n_obj*n_pre*K, Nmax = max preshape
 * size, Mcmax = max collision-cloud size.                                     */
typedef struct {
  double* cost;       /* [Ktot]   C = 1/2 (L_ct + lambda L_com)                */
  double* g_ct;       /* [Ktot*6] (g_t, g_w) of C                              */
  double* g_q;        /* [Ktot*4] quaternion gradient of C, eq. (17) layout    */
  int32_t* ncol;      /* [Ktot]   colliding points of the collision cloud      */
  double* col_cost;   /* [Ktot]   1/2 L_col (0 when ncol == 0)                 */
  double* g_col;      /* [Ktot*6] gradient of 1/2 L_col (0 when ncol == 0)     */
  double* g_fin;      /* [Ktot*6] gradient the update uses                     */
  int32_t* nn_idx;    /* [Ktot*Nmax] forward NN index per gripper point        */
  uint8_t* gate;      /* [Ktot*Mcmax] 1 if the collision point collides        */
  double* phi_c;      /* [Ktot*Mcmax] SDF value at the point (NaN outside)     */
  int32_t* rev_idx;   /* [Ktot*Mcmax] reverse NN index (-1 if not colliding)   */
  double* pen;        /* [Ktot] penetration term included in cost              */
} or_eval_out;

/* --- geometry helpers ---------------------------------------------------- */
void or_quat_to_rot(const double q[4], double Rm[9]);
void or_quat_mul(const double a[4], const double b[4], double out[4]);
void or_quat_exp(const double v[3], double out[4]);
int32_t or_nn_brute(const double* pts, int32_t n, const double x[3], double* d2);
double or_sdf_trilinear(const double* grid, const int32_t n[3], const double origin[3],
                        double cell, const double p[3], int32_t* inside);
double or_sdf_trilinear_grad(const double* grid, const int32_t n[3], const double origin[3],
                             double cell, const double p[3], int32_t* inside, double grad[3]);

/* --- the method ---------------------------------------------------------- */
double or_log_prior(const double pr[9], const double theta[7], double grad[6]);
void or_setup(const or_problem* pb, const or_config* cfg, double* com, double* tcp,
              double* rho2, double* a_t, double* a_w);
void or_schedule(const or_config* cfg, int32_t k, double* gamma, double* tau);
void or_eval(const or_problem* pb, const or_config* cfg, int32_t k, const double* theta,
             or_eval_out* out);
uint64_t or_splitmix64(uint64_t x);
int64_t or_batch_size(const or_config* cfg, int32_t k, int64_t M);
int64_t or_batch_perm(int64_t j, int64_t M, uint64_t key);
uint64_t or_batch_key(const or_config* cfg, int32_t k, int32_t o);
double or_bandwidth(const double* theta, int32_t K, const or_config* cfg);
void or_svgd_direction(const double* theta, const double* g, int32_t K, double h, double gamma,
                       double tau, double a_t, double a_w, int32_t kernel_mode,
                       double* kmat, double* phi);
void or_retract(double* theta_i, const double dt[3], const double dw[3]);
int32_t or_step(const or_problem* pb, const or_config* cfg, int32_t k, double* theta,
                double* prev_cost, int32_t* converged, or_eval_out* ev, double* h_out,
                double* phi_out);
int32_t or_solve(const or_problem* pb, const or_config* cfg, int32_t k_start, int32_t k_end,
                 double* theta, double* prev_cost, int32_t* converged, or_eval_out* final_ev,
                 int32_t* best_idx, int32_t* best_free);
void or_select(const or_problem* pb, const double* cost, const int32_t* ncol, int32_t* best_idx,
               int32_t* best_free);
int32_t or_threads(void);
void or_set_threads(int32_t n);

#ifdef __cplusplus
}
#endif
#endif
