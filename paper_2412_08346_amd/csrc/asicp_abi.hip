// asicp_abi.hip -- host side of the C ABI declared in include/asicp.h:
// validation, workspace layout, the iteration schedule and the kernel
// sequence of Algorithm 1.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "asicp_internal.h"
#include "nn_core.h"

using namespace asicp;

namespace {

thread_local std::string g_err;

asicp_status fail(asicp_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

// Runs the body of an entry point so that no C++ exception crosses the C ABI:
// host memory exhaustion in a container or a message string becomes
// ASICP_E_HOST.
template <class F>
asicp_status guarded(F&& body) noexcept {
  try {
    return body();
  } catch (...) {
    g_err.clear();
    try {
      g_err = "host-side failure (out of host memory)";
    } catch (...) {
    }
    return ASICP_E_HOST;
  }
}

constexpr int kMaxPoints = 1 << 22;   // per object / collision cloud / preshape
// In a captured graph, forward launches of at most this many wavefronts (well
// below the 7168 the GPU holds at once) run the gate on a branch of its own.
constexpr long long kConcurrentGateWaves = 2048;
constexpr int kMaxGroups = 1 << 16;

struct Layout {
  size_t groups, objs, pres, obj_prep, pre_prep, obj_pts, pre_pts, obj_perm, pre_perm, obj_box, obj_box1, obj_blk, obj_blk1, kd_box, pre_box,
      col_box, col_leaf_box, sdf_bits, sdf_sum, sdf_flag;
  size_t gate_wg, sort_keys, wave_pairs, obj_com, pre_const, col_pts, col_perm, obj_prep_mb, batch_mark, prior;
  size_t theta, cost, col_cost, prev_cost, ncol, converged, grad, grad_ct, grad_col, phi, h, bw_hist, bw_state;
  size_t nn_part, col_part, pen_part, best, best_theta, flags, dbg_nn, dbg_rev;
  size_t total;
};

struct Shape {
  int n_obj, n_pre, K, G, Ktot;
  int obj_tg, pre_tg, max_waves_pp, max_gate_chunks, n_max, mc_max;
  long long gate_chunks;  // over all objects
  long long sort_keys;  // total power-of-two padded cloud sizes
  long long sdf_words, sdf_bricks, sdf_flags;  // SDF cull tables over all preshapes (32-bit words)
  int sdf_blocks;       // set-up workgroups per preshape building them
  long long c_total;    // collision points over all objects
  long long r_total;    // object points over all objects
  int max_m, max_m_pad;
  bool minibatch;
  bool prior;
  long long total_waves[kNumQ], total_gate_wgs;  // forward waves per query-block count
  bool debug;
  bool timing;
};

size_t bump(size_t& cur, size_t bytes) {
  const size_t off = cur;
  cur += (bytes + 255) & ~(size_t)255;
  return off;
}

Layout layout_of(const Shape& s) {
  Layout L;
  size_t c = 0;
  const size_t K = (size_t)s.Ktot;
  L.groups = bump(c, sizeof(GroupInfo) * s.G);
  L.objs = bump(c, sizeof(ObjInfo) * s.n_obj);
  L.pres = bump(c, sizeof(PreInfo) * s.n_pre);
  L.obj_prep = bump(c, (size_t)s.obj_tg * 64 * 16);
  L.pre_prep = bump(c, (size_t)s.pre_tg * 64 * 16);
  L.obj_pts = bump(c, (size_t)s.obj_tg * 64 * 16);
  L.pre_pts = bump(c, (size_t)s.pre_tg * 64 * 16);
  L.obj_perm = bump(c, (size_t)s.obj_tg * 64 * 4);
  L.pre_perm = bump(c, (size_t)s.pre_tg * 64 * 4);
  L.obj_box = bump(c, (size_t)s.obj_tg / 2 * 32);
  L.obj_box1 = bump(c, (size_t)s.obj_tg * 32);
  L.obj_blk = bump(c, (size_t)s.obj_tg / 4 * 32);  // ceil(chunks / 64) <= tile groups / 4 per object
  L.obj_blk1 = bump(c, (size_t)s.obj_tg / 4 * 32);
  L.kd_box = bump(c, 64 * ((size_t)s.obj_tg + 4 * (size_t)s.pre_tg + (size_t)(kGateChunk / 64) * (size_t)s.gate_chunks));
  L.pre_box = bump(c, (size_t)s.pre_tg / kChunkTG * 32);
  L.col_box = bump(c, 32 * (size_t)(s.gate_chunks > 0 ? s.gate_chunks : 1));
  L.col_leaf_box = bump(c, 32 * (size_t)(kGateChunk / 64) * (size_t)(s.gate_chunks > 0 ? s.gate_chunks : 1));
  L.sort_keys = bump(c, (size_t)s.sort_keys * 8);
  L.gate_wg = bump(c, sizeof(GateWG) * (size_t)(s.total_gate_wgs > 0 ? s.total_gate_wgs : 1));
  L.sdf_bits = bump(c, 4 * (size_t)s.sdf_words);
  L.sdf_sum = bump(c, 4 * (size_t)s.sdf_bricks);
  L.sdf_flag = bump(c, 4 * (size_t)s.sdf_flags);
  L.col_pts = bump(c, (size_t)(s.c_total > 0 ? s.c_total : 1) * 16);
  L.obj_prep_mb = s.minibatch ? bump(c, (size_t)s.obj_tg * 64 * 16) : 0;
  L.batch_mark = s.minibatch ? bump(c, (size_t)s.r_total) : 0;
  L.prior = s.prior ? bump(c, 48 * (size_t)s.G) : 0;
  L.col_perm = bump(c, (size_t)(s.c_total > 0 ? s.c_total : 1) * 4);
  L.wave_pairs = s.timing ? bump(c, 8 * (size_t)s.total_waves[0]) : 0;
  L.obj_com = bump(c, 16 * (size_t)s.n_obj);
  L.pre_const = bump(c, 32 * (size_t)s.n_pre);
  L.theta = bump(c, 2 * 4 * 7 * K);  // two pose buffers (Stein update: read one, write the other)
  L.cost = bump(c, 4 * K);
  L.col_cost = bump(c, 4 * K);
  L.prev_cost = bump(c, 4 * K);
  L.ncol = bump(c, 4 * K);
  L.converged = bump(c, 4 * K);
  L.grad = bump(c, 4 * 6 * K);
  L.grad_ct = bump(c, 4 * 6 * K);
  L.grad_col = bump(c, 4 * 6 * K);
  L.phi = bump(c, 4 * 6 * K);
  L.h = bump(c, 4 * (size_t)s.G);
  L.bw_hist = bump(c, 4 * 256 * (size_t)s.G);
  L.bw_state = bump(c, 16 * (size_t)s.G);
  L.nn_part = bump(c, 4 * kPartStride * K * (size_t)s.max_waves_pp);
  L.col_part = bump(c, 4 * kPartStride * K * (size_t)(s.max_gate_chunks > 0 ? s.max_gate_chunks : 1));
  L.pen_part = bump(c, 4 * kPartStride * K * (size_t)(s.max_gate_chunks > 0 ? s.max_gate_chunks : 1));
  L.best = bump(c, 8 * (size_t)s.n_obj);
  L.best_theta = bump(c, 32 * (size_t)s.n_obj);
  L.flags = bump(c, 16);
  L.dbg_nn = s.debug ? bump(c, 4 * K * (size_t)s.n_max) : 0;
  L.dbg_rev = s.debug ? bump(c, 4 * K * (size_t)(s.mc_max > 0 ? s.mc_max : 1)) : 0;
  L.total = c;
  return L;
}

bool finite_pos(float v) { return std::isfinite(v) && v > 0.f; }

long long pow2_at_least(long long n) {
  long long p = 2;
  while (p < n) p <<= 1;
  return p;
}

// Host-only validation of every argument; fills `s`.
asicp_status validate(const asicp_problem* pb, const asicp_config* cfg, Shape& s) {
  if (!pb || !cfg) return fail(ASICP_E_INVALID, "problem and config must not be NULL");
  if (pb->n_objects < 1) return fail(ASICP_E_INVALID, "n_objects must be >= 1");
  if (pb->n_preshapes < 1) return fail(ASICP_E_INVALID, "n_preshapes must be >= 1");
  if (pb->particles_per_group < 1 || pb->particles_per_group > 1024)
    return fail(ASICP_E_INVALID, "particles_per_group must be in 1..1024");
  if ((long long)pb->n_objects * pb->n_preshapes > kMaxGroups)
    return fail(ASICP_E_INVALID, "too many (object, preshape) groups");
  const long long ktot = (long long)pb->n_objects * pb->n_preshapes * pb->particles_per_group;
  if (ktot > (1ll << 24)) return fail(ASICP_E_INVALID, "too many particles");
  if (!pb->rx || !pb->ry || !pb->rz || !pb->sx || !pb->sy || !pb->sz || !pb->theta0)
    return fail(ASICP_E_INVALID, "object cloud, contact cloud and theta0 device pointers are required");
  if (!pb->r_off || !pb->c_off || !pb->s_off || !pb->sdf)
    return fail(ASICP_E_INVALID, "offset arrays and the SDF array are required");
  if (pb->r_off[0] != 0 || pb->c_off[0] != 0 || pb->s_off[0] != 0)
    return fail(ASICP_E_INVALID, "offset arrays must start at 0");
  s.n_obj = pb->n_objects;
  s.n_pre = pb->n_preshapes;
  s.K = pb->particles_per_group;
  s.G = s.n_obj * s.n_pre;
  s.Ktot = (int)ktot;
  s.obj_tg = s.pre_tg = 0;
  s.sort_keys = 0;
  s.sdf_words = s.sdf_bricks = s.sdf_flags = 0;
  long long max_cells = 0;
  s.n_max = s.mc_max = 0;
  s.max_waves_pp = 0;
  s.max_gate_chunks = 0;
  s.gate_chunks = 0;
  bool any_c = false;
  for (int o = 0; o < s.n_obj; ++o) {
    const long long m = (long long)pb->r_off[o + 1] - pb->r_off[o];
    const long long mc = (long long)pb->c_off[o + 1] - pb->c_off[o];
    if (m < 1 || m > kMaxPoints) return fail(ASICP_E_INVALID, "object " + std::to_string(o) + " must have 1..4194304 points");
    if (mc < 0 || mc > kMaxPoints) return fail(ASICP_E_INVALID, "collision cloud " + std::to_string(o) + " must have 0..4194304 points");
    s.obj_tg += (int)((m + kPadPoints - 1) / kPadPoints) * (kPadPoints / 64);
    s.sort_keys += pow2_at_least((long long)m);
    if (mc > 0) s.sort_keys += pow2_at_least((long long)mc);
    s.mc_max = std::max(s.mc_max, (int)mc);
    s.max_gate_chunks = std::max(s.max_gate_chunks, (int)((mc + kGateChunk - 1) / kGateChunk));
    s.gate_chunks += (mc + kGateChunk - 1) / kGateChunk;
    any_c = any_c || mc > 0;
  }
  if (any_c && (!pb->cx || !pb->cy || !pb->cz))
    return fail(ASICP_E_INVALID, "collision cloud device pointers are required");
  s.c_total = pb->c_off[s.n_obj];
  s.r_total = pb->r_off[s.n_obj];
  s.max_m = 0;
  s.max_m_pad = 0;
  for (int o = 0; o < s.n_obj; ++o) {
    const int m = pb->r_off[o + 1] - pb->r_off[o];
    s.max_m = std::max(s.max_m, m);
    s.max_m_pad = std::max(s.max_m_pad, ((m + kPadPoints - 1) / kPadPoints) * kPadPoints);
  }
  if ((long long)pb->r_off[s.n_obj] > (1ll << 30) || (long long)pb->c_off[s.n_obj] > (1ll << 30))
    return fail(ASICP_E_INVALID, "clouds too large");
  for (int p = 0; p < s.n_pre; ++p) {
    const long long n = (long long)pb->s_off[p + 1] - pb->s_off[p];
    if (n < 1 || n > kMaxPoints) return fail(ASICP_E_INVALID, "preshape " + std::to_string(p) + " must have 1..4194304 points");
    s.pre_tg += (int)((n + kPadPoints - 1) / kPadPoints) * (kPadPoints / 64);
    s.sort_keys += pow2_at_least((long long)n);
    s.n_max = std::max(s.n_max, (int)n);
    s.max_waves_pp = std::max(s.max_waves_pp, (int)((n + 15) / 16));  // 1 block of 16 queries per wave
    const asicp_sdf& g = pb->sdf[p];
    if (!g.values) return fail(ASICP_E_INVALID, "SDF values of preshape " + std::to_string(p) + " are NULL");
    if (g.nx < 2 || g.ny < 2 || g.nz < 2 || (long long)g.nx * g.ny * g.nz > (1ll << 30))
      return fail(ASICP_E_INVALID, "SDF grid of preshape " + std::to_string(p) + " needs 2..1024^3 nodes per axis product");
    if (!finite_pos(g.cell)) return fail(ASICP_E_INVALID, "SDF cell must be finite and > 0");
    if (!std::isfinite(g.origin[0]) || !std::isfinite(g.origin[1]) || !std::isfinite(g.origin[2]))
      return fail(ASICP_E_INVALID, "SDF origin must be finite");
    s.sdf_words += (long long)(g.nz - 1) * (g.ny - 1) * ((g.nx - 1 + 31) / 32);
    s.sdf_bricks += (long long)((g.nx - 1 + kBrick - 1) / kBrick + 1) * ((g.ny - 1 + kBrick - 1) / kBrick + 1) *
                    ((g.nz - 1 + kBrick - 1) / kBrick + 1);
    s.sdf_flags += (long long)((g.nx - 1 + kBrick - 1) / kBrick) * ((g.ny - 1 + kBrick - 1) / kBrick) *
                   ((g.nz - 1 + kBrick - 1) / kBrick);
    max_cells = std::max(max_cells, (long long)(g.nz - 1) * (g.ny - 1) * (g.nx - 1));
  }
  // one set-up workgroup (1024 threads) per 16 cells per thread, at most 64
  // per preshape (each takes a CU beside the sorts)
  s.sdf_blocks = (int)std::min<long long>(64, std::max<long long>(1, (max_cells + 16383) / 16384));
  if ((long long)pb->s_off[s.n_pre] > (1ll << 30)) return fail(ASICP_E_INVALID, "contact clouds too large");
  for (int qi = 0; qi < kNumQ; ++qi) s.total_waves[qi] = 0;
  s.total_gate_wgs = 0;
  for (int o = 0; o < s.n_obj; ++o)
    for (int p = 0; p < s.n_pre; ++p) {
      const long long n = (long long)pb->s_off[p + 1] - pb->s_off[p];
      const long long mc = (long long)pb->c_off[o + 1] - pb->c_off[o];
      for (int qi = 0; qi < kNumQ; ++qi)
        s.total_waves[qi] += (long long)s.K * ((n + 16 * q_blocks(qi) - 1) / (16 * q_blocks(qi)));
      s.total_gate_wgs += (long long)s.K * ((mc + kGateChunk - 1) / kGateChunk);
    }
  if (s.total_waves[0] > (1ll << 30) || s.total_gate_wgs > (1ll << 30))
    return fail(ASICP_E_INVALID, "problem too large for one launch");
  if (cfg->k_max < 1) return fail(ASICP_E_INVALID, "k_max must be >= 1");
  if (cfg->k_stein < 0 || cfg->k_stein > cfg->k_max) return fail(ASICP_E_INVALID, "k_stein must be in 0..k_max");
  if (pb->k_start < 0 || pb->k_start > cfg->k_max) return fail(ASICP_E_INVALID, "k_start must be in 0..k_max");
  if (!finite_pos(cfg->eta)) return fail(ASICP_E_INVALID, "eta must be finite and > 0");
  if (!std::isfinite(cfg->lambda) || cfg->lambda < 0.f) return fail(ASICP_E_INVALID, "lambda must be finite and >= 0");
  if (cfg->precond != ASICP_PRECOND_GN_DIAG && cfg->precond != ASICP_PRECOND_IDENTITY)
    return fail(ASICP_E_INVALID, "unknown preconditioner");
  if (cfg->schedule == ASICP_SCHED_GEOMETRIC) {
    if (!finite_pos(cfg->T0) || !finite_pos(cfg->T1)) return fail(ASICP_E_INVALID, "T0 and T1 must be finite and > 0");
  } else if (cfg->schedule == ASICP_SCHED_PAPER_CYCLIC) {
    if (!finite_pos(cfg->cyc_C) || !finite_pos(cfg->cyc_p)) return fail(ASICP_E_INVALID, "cyc_C and cyc_p must be finite and > 0");
  } else {
    return fail(ASICP_E_INVALID, "unknown schedule");
  }
  if (cfg->kernel_mode != ASICP_KERNEL_PRODUCT && cfg->kernel_mode != ASICP_KERNEL_BLOCK)
    return fail(ASICP_E_INVALID, "unknown kernel mode");
  if (cfg->bw_mode == ASICP_BW_FIXED) {
    if (!finite_pos(cfg->h_fixed)) return fail(ASICP_E_INVALID, "h_fixed must be finite and > 0");
  } else if (cfg->bw_mode != ASICP_BW_MEDIAN) {
    return fail(ASICP_E_INVALID, "unknown bandwidth mode");
  }
  if (!finite_pos(cfg->h_min)) return fail(ASICP_E_INVALID, "h_min must be finite and > 0");
  if (!std::isfinite(cfg->conv_tol) || cfg->conv_tol < 0.f) return fail(ASICP_E_INVALID, "conv_tol must be finite and >= 0");
  if (!std::isfinite(cfg->w_pen) || cfg->w_pen < 0.f) return fail(ASICP_E_INVALID, "w_pen must be finite and >= 0");
  if (cfg->flags & ~(ASICP_FLAG_DEBUG | ASICP_FLAG_TIMING | ASICP_FLAG_NO_PRUNE))
    return fail(ASICP_E_INVALID, "unknown flag bits");
  if (s.sort_keys > (1ll << 30)) return fail(ASICP_E_INVALID, "clouds too large to sort");
  if (cfg->minibatch != 0 && cfg->minibatch != 1) return fail(ASICP_E_INVALID, "minibatch must be 0 or 1");
  s.minibatch = cfg->minibatch == 1;
  s.prior = pb->prior != nullptr;
  if (s.prior) {
    for (int g = 0; g < s.G; ++g) {
      const float* pr = pb->prior + 9 * (size_t)g;
      bool finite = true;
      for (int a = 0; a < 9; ++a) finite = finite && std::isfinite(pr[a]);
      const double n2 = (double)pr[4] * pr[4] + (double)pr[5] * pr[5] + (double)pr[6] * pr[6] + (double)pr[7] * pr[7];
      if (!finite || pr[3] < 0.f || pr[8] < 0.f || std::fabs(std::sqrt(n2) - 1.0) > 1e-3)
        return fail(ASICP_E_INVALID, "prior of group " + std::to_string(g) +
                                         ": values must be finite, w_t and kappa >= 0, mu_q a unit quaternion");
    }
  }
  s.debug = (cfg->flags & ASICP_FLAG_DEBUG) != 0;
  s.timing = (cfg->flags & ASICP_FLAG_TIMING) != 0;
  return ASICP_OK;
}

asicp_status check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ASICP_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return ASICP_OK;
}

}  // namespace

__global__ void k_set_theta(float* dst, const float* src, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

// Cost and gradient of asicp_cost_grad.  ASICP_GRAD_POSE maps the rotation
// part g_w (world rotation vector) to the unit quaternion's parameters by
// eq. (17)'s tangent map: d/dq = 2 M(q) g_w, M(q) = [-q_v^T ; q_w I - [q_v]x].
__global__ void k_get_cost_grad(const float* theta, const float* cost, const float* grad_ct, float* cost_out,
                                float* grad_out, int form, int K) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= K) return;
  if (cost_out) cost_out[i] = cost[i];
  if (!grad_out) return;
  for (int a = 0; a < 3; ++a) grad_out[a * K + i] = grad_ct[a * K + i];
  const float gx = grad_ct[3 * K + i], gy = grad_ct[4 * K + i], gz = grad_ct[5 * K + i];
  if (form == ASICP_GRAD_TANGENT) {
    grad_out[3 * K + i] = gx;
    grad_out[4 * K + i] = gy;
    grad_out[5 * K + i] = gz;
    return;
  }
  const float w = theta[3 * K + i], x = theta[4 * K + i], y = theta[5 * K + i], z = theta[6 * K + i];
  grad_out[3 * K + i] = -2.f * (x * gx + y * gy + z * gz);
  grad_out[4 * K + i] = 2.f * (w * gx + z * gy - y * gz);
  grad_out[5 * K + i] = 2.f * (-z * gx + w * gy + x * gz);
  grad_out[6 * K + i] = 2.f * (y * gx - x * gy + w * gz);
}

__global__ void k_pose_vjp(const float* grad, const float* gout, float* dtheta, int K) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= K) return;
  const float s = gout[i];
  for (int a = 0; a < 7; ++a) dtheta[a * K + i] = s * grad[a * K + i];
}

struct asicp_ctx_s {
  Dev d;
  asicp_config cfg;
  int k;               // next iteration
  int k_start;
  bool final_done;
  float inv_log_k;
  std::vector<hipEvent_t> ev;  // start/stop pairs around forward-NN launches
  int n_timed;
  const float* theta0;          // borrowed set-up inputs, for asicp_replay
  const float* prev_cost0;
  const int32_t* converged0;
  hipGraphExec_t graph;         // whole-solve graph of asicp_replay
  float* graph_theta[2];        // the pose buffers (current, next) the graph ends with
  hipStream_t cap_stream;       // private stream the graph is captured on
  bool capturing;               // no timing events inside a captured graph
  // Side stream of an evaluation: the bandwidth select and the collision
  // gate depend only on the poses, so they run beside the forward NN launch
  // (fork after the caller's preceding work, join before the finaliser).
  hipStream_t side;
  hipStream_t side2;            // the gate's branch in a captured graph of a small problem
                                //   (created with the capture stream and kept with the graph:
                                //   releasing it after the capture slowed replays, 1.53 against
                                //   1.21 ms per small solve)
  hipEvent_t fork_ev, join_ev, join2_ev;
};

extern "C" {

const char* asicp_last_error(void) { return g_err.c_str(); }

asicp_status asicp_workspace_bytes(const asicp_problem* pb, const asicp_config* cfg, size_t* bytes) {
  return guarded([&]() -> asicp_status {
    g_err.clear();
    if (!bytes) return fail(ASICP_E_INVALID, "bytes must not be NULL");
    Shape s;
    const asicp_status st = validate(pb, cfg, s);
    if (st != ASICP_OK) return st;
    *bytes = layout_of(s).total;
    return ASICP_OK;
  });
}

asicp_status asicp_create(const asicp_problem* pb, const asicp_config* cfg, void* workspace,
                          size_t workspace_bytes, void* stream, asicp_ctx* out) {
  return guarded([&]() -> asicp_status {
    g_err.clear();
    if (!out) return fail(ASICP_E_INVALID, "out must not be NULL");
    *out = nullptr;
    Shape s;
    asicp_status st = validate(pb, cfg, s);
    if (st != ASICP_OK) return st;
    const Layout L = layout_of(s);
    if (!workspace) return fail(ASICP_E_INVALID, "workspace must not be NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(ASICP_E_INVALID, "workspace must be 256-byte aligned");
    if (workspace_bytes < L.total)
      return fail(ASICP_E_INVALID, "workspace too small: need " + std::to_string(L.total) + " bytes");

    // host tables
    std::vector<GroupInfo> groups(s.G);
    std::vector<ObjInfo> objs(s.n_obj);
    std::vector<PreInfo> pres(s.n_pre);
    int tg = 0;
    long long key_off = 0;
    int gbox = 0;
    for (int o = 0; o < s.n_obj; ++o) {
      ObjInfo& oi = objs[o];
      std::memset(&oi, 0, sizeof oi);
      oi.r_begin = pb->r_off[o];
      oi.m = pb->r_off[o + 1] - pb->r_off[o];
      oi.c_begin = pb->c_off[o];
      oi.mc = pb->c_off[o + 1] - pb->c_off[o];
      oi.prep_tg_begin = tg;
      oi.ntg = ((oi.m + kPadPoints - 1) / kPadPoints) * (kPadPoints / 64);
      oi.gate_chunks = (oi.mc + kGateChunk - 1) / kGateChunk;
      oi.gbox_begin = gbox;
      gbox += oi.gate_chunks;
      oi.key_off = (int32_t)key_off;
      key_off += pow2_at_least(oi.m);
      oi.c_key_off = (int32_t)key_off;
      if (oi.mc > 0) key_off += pow2_at_least(oi.mc);
      tg += oi.ntg;
    }
    tg = 0;
    std::vector<long long> bits_off(s.n_pre), sum_off(s.n_pre), flag_off(s.n_pre);
    long long bits_at = 0, sum_at = 0, flag_at = 0;
    for (int p = 0; p < s.n_pre; ++p) {
      PreInfo& pi = pres[p];
      std::memset(&pi, 0, sizeof pi);
      pi.s_begin = pb->s_off[p];
      pi.n = pb->s_off[p + 1] - pb->s_off[p];
      pi.prep_tg_begin = tg;
      pi.ntg = ((pi.n + kPadPoints - 1) / kPadPoints) * (kPadPoints / 64);
      for (int qi = 0; qi < kNumQ; ++qi) pi.waves[qi] = (pi.n + 16 * q_blocks(qi) - 1) / (16 * q_blocks(qi));
      pi.key_off = (int32_t)key_off;
      key_off += pow2_at_least(pi.n);
      tg += pi.ntg;
      const asicp_sdf& g = pb->sdf[p];
      pi.nx = g.nx; pi.ny = g.ny; pi.nz = g.nz;
      pi.sdf = g.values;
      pi.ox = g.origin[0]; pi.oy = g.origin[1]; pi.oz = g.origin[2];
      pi.cell = g.cell;
      pi.inv_cell = (float)(1.0 / (double)g.cell);
      for (int ax = 0; ax < 3; ++ax) {
        pi.neg_lo[ax] = 0x7fffffff;  // reduced on the device by the set-up
        pi.neg_hi[ax] = -1;
      }
      pi.cbw = (g.nx - 1 + 31) / 32;
      pi.bnx = (g.nx - 1 + kBrick - 1) / kBrick;
      pi.bny = (g.ny - 1 + kBrick - 1) / kBrick;
      pi.bnz = (g.nz - 1 + kBrick - 1) / kBrick;
      bits_off[p] = bits_at;
      sum_off[p] = sum_at;
      bits_at += (long long)(g.nz - 1) * (g.ny - 1) * pi.cbw;
      sum_at += (long long)(pi.bnx + 1) * (pi.bny + 1) * (pi.bnz + 1);
      flag_off[p] = flag_at;
      flag_at += (long long)pi.bnx * pi.bny * pi.bnz;
    }
    int wave_off[kNumQ] = {0, 0, 0}, gate_off = 0;
    for (int o = 0; o < s.n_obj; ++o)
      for (int p = 0; p < s.n_pre; ++p) {
        GroupInfo& gi = groups[o * s.n_pre + p];
        gi.obj = o;
        gi.pre = p;
        for (int qi = 0; qi < kNumQ; ++qi) gi.wave_off[qi] = wave_off[qi];
        gi.gate_off = gate_off;
        for (int qi = 0; qi < kNumQ; ++qi) wave_off[qi] += s.K * pres[p].waves[qi];
        gate_off += s.K * objs[o].gate_chunks;
      }

    char* ws = static_cast<char*>(workspace);
    Dev d;
    std::memset(&d, 0, sizeof d);
    d.rx = pb->rx; d.ry = pb->ry; d.rz = pb->rz;
    d.cx = pb->cx; d.cy = pb->cy; d.cz = pb->cz;
    d.sx = pb->sx; d.sy = pb->sy; d.sz = pb->sz;
    d.groups = reinterpret_cast<const GroupInfo*>(ws + L.groups);
    d.objs = reinterpret_cast<const ObjInfo*>(ws + L.objs);
    d.pres = reinterpret_cast<const PreInfo*>(ws + L.pres);
    d.n_obj = s.n_obj; d.n_pre = s.n_pre; d.K = s.K; d.G = s.G; d.Ktot = s.Ktot;
    for (int qi = 0; qi < kNumQ; ++qi) d.total_waves[qi] = (int)s.total_waves[qi];
    d.total_gate_wgs = (int)s.total_gate_wgs;
    d.max_waves_pp = s.max_waves_pp;
    d.max_gate_chunks = s.max_gate_chunks > 0 ? s.max_gate_chunks : 1;
    d.n_max = s.n_max;
    d.mc_max = s.mc_max > 0 ? s.mc_max : 1;
    d.obj_prep = reinterpret_cast<float4*>(ws + L.obj_prep);
    d.pre_prep = reinterpret_cast<float4*>(ws + L.pre_prep);
    d.obj_pts = reinterpret_cast<float4*>(ws + L.obj_pts);
    d.pre_pts = reinterpret_cast<float4*>(ws + L.pre_pts);
    d.obj_perm = reinterpret_cast<int32_t*>(ws + L.obj_perm);
    d.pre_perm = reinterpret_cast<int32_t*>(ws + L.pre_perm);
    d.obj_box = reinterpret_cast<float*>(ws + L.obj_box);
    d.obj_box1 = reinterpret_cast<float*>(ws + L.obj_box1);
    d.obj_blk = reinterpret_cast<float*>(ws + L.obj_blk);
    d.obj_blk1 = reinterpret_cast<float*>(ws + L.obj_blk1);
    d.kd_box = reinterpret_cast<float*>(ws + L.kd_box);
    d.kd_pre_off = s.obj_tg;
    d.kd_col_off = s.obj_tg + 4 * s.pre_tg;
    d.pre_box = reinterpret_cast<float*>(ws + L.pre_box);
    d.col_box = reinterpret_cast<float*>(ws + L.col_box);
    d.col_leaf_box = reinterpret_cast<float*>(ws + L.col_leaf_box);
    d.sdf_blocks = s.sdf_blocks;
    d.gate_wg = reinterpret_cast<GateWG*>(ws + L.gate_wg);
    for (int p = 0; p < s.n_pre; ++p) {
      pres[p].cell_bits = reinterpret_cast<const uint32_t*>(ws + L.sdf_bits) + bits_off[p];
      pres[p].brick_sum = reinterpret_cast<const int32_t*>(ws + L.sdf_sum) + sum_off[p];
      pres[p].brick_flag = reinterpret_cast<int32_t*>(ws + L.sdf_flag) + flag_off[p];
    }
    d.sort_keys = reinterpret_cast<unsigned long long*>(ws + L.sort_keys);
    d.col_pts = reinterpret_cast<float4*>(ws + L.col_pts);
    d.col_perm = reinterpret_cast<int32_t*>(ws + L.col_perm);
    d.wave_pairs = s.timing ? reinterpret_cast<unsigned long long*>(ws + L.wave_pairs) : nullptr;
    d.prune = (cfg->flags & ASICP_FLAG_NO_PRUNE) ? 0 : 1;
    d.obj_com = reinterpret_cast<float*>(ws + L.obj_com);
    d.pre_const = reinterpret_cast<float*>(ws + L.pre_const);
    d.theta = reinterpret_cast<float*>(ws + L.theta);
    d.theta_next = d.theta + 7 * (size_t)s.Ktot;
    d.cost = reinterpret_cast<float*>(ws + L.cost);
    d.col_cost = reinterpret_cast<float*>(ws + L.col_cost);
    d.prev_cost = reinterpret_cast<float*>(ws + L.prev_cost);
    d.ncol = reinterpret_cast<int32_t*>(ws + L.ncol);
    d.converged = reinterpret_cast<int32_t*>(ws + L.converged);
    d.grad = reinterpret_cast<float*>(ws + L.grad);
    d.grad_ct = reinterpret_cast<float*>(ws + L.grad_ct);
    d.grad_col = reinterpret_cast<float*>(ws + L.grad_col);
    d.phi = reinterpret_cast<float*>(ws + L.phi);
    d.h = reinterpret_cast<float*>(ws + L.h);
    d.bw_hist = reinterpret_cast<unsigned int*>(ws + L.bw_hist);
    d.bw_state = reinterpret_cast<unsigned int*>(ws + L.bw_state);
    d.nn_part = reinterpret_cast<float*>(ws + L.nn_part);
    d.col_part = reinterpret_cast<float*>(ws + L.col_part);
    d.pen_part = reinterpret_cast<float*>(ws + L.pen_part);
    d.best = reinterpret_cast<int32_t*>(ws + L.best);
    d.best_theta = reinterpret_cast<float*>(ws + L.best_theta);
    d.flags = reinterpret_cast<int32_t*>(ws + L.flags);
    d.dbg_nn = s.debug ? reinterpret_cast<int32_t*>(ws + L.dbg_nn) : nullptr;
    d.dbg_rev = s.debug ? reinterpret_cast<int32_t*>(ws + L.dbg_rev) : nullptr;
    d.eta = cfg->eta;
    d.lambda = cfg->lambda;
    d.k_stein = cfg->k_stein;
    d.kernel_mode = cfg->kernel_mode;
    d.bw_mode = cfg->bw_mode;
    d.precond = cfg->precond;
    d.h_fixed = cfg->h_fixed;
    d.h_min = cfg->h_min;
    d.conv_tol = cfg->conv_tol;
    d.w_pen = cfg->w_pen;
    d.minibatch = s.minibatch ? 1 : 0;
    d.seed = cfg->seed;
    d.obj_prep_mb = s.minibatch ? reinterpret_cast<float4*>(ws + L.obj_prep_mb) : nullptr;
    d.batch_mark = s.minibatch ? reinterpret_cast<unsigned char*>(ws + L.batch_mark) : nullptr;
    d.max_m = s.max_m;
    d.max_m_pad = s.max_m_pad;
    d.prior = s.prior ? reinterpret_cast<const float*>(ws + L.prior) : nullptr;
    d.xcd_map = 1;  // launch defaults (asicp_set_launch / asicp_autotune change them)
    d.fine = 1;
    d.nn_qi = 2;    // 4 blocks of 16 queries per forward wave
    d.nn_ch = 2;    // 128-point pruning chunks
    std::vector<float> prior_words;
    if (s.prior) {
      prior_words.assign(12 * (size_t)s.G, 0.f);
      for (int g = 0; g < s.G; ++g) {
        const float* pr = pb->prior + 9 * (size_t)g;
        float* w = prior_words.data() + 12 * (size_t)g;
        const double n = std::sqrt((double)pr[4] * pr[4] + (double)pr[5] * pr[5] + (double)pr[6] * pr[6] +
                                   (double)pr[7] * pr[7]);
        for (int a = 0; a < 4; ++a) w[a] = pr[a];
        for (int a = 0; a < 4; ++a) w[4 + a] = (float)(pr[4 + a] / n);
        w[8] = pr[8];
      }
    }

    hipStream_t hs = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();  // start from a clean error state
    upload_words(ws + L.groups, groups.data(), sizeof(GroupInfo) * groups.size(), hs);
    upload_words(ws + L.objs, objs.data(), sizeof(ObjInfo) * objs.size(), hs);
    upload_words(ws + L.pres, pres.data(), sizeof(PreInfo) * pres.size(), hs);
    if (s.prior) upload_words(ws + L.prior, prior_words.data(), 4 * prior_words.size(), hs);
    if ((st = check_launch("table upload")) != ASICP_OK) return st;
    zero_words(ws + L.sdf_flag, s.sdf_flags, hs);  // the brick flags start at zero; each set-up leaves them so
    if ((st = check_launch("flag clear")) != ASICP_OK) return st;
    launch_setup(d, pb->theta0, pb->prev_cost, pb->converged, hs);
    if ((st = check_launch("setup")) != ASICP_OK) return st;
    if (s.debug) {
      if (hipMemsetAsync(d.dbg_nn, 0xff, 4 * (size_t)s.Ktot * s.n_max, hs) != hipSuccess ||
          hipMemsetAsync(d.dbg_rev, 0xff, 4 * (size_t)s.Ktot * d.mc_max, hs) != hipSuccess)
        return fail(ASICP_E_HIP, "debug buffer clear failed");
    }

    asicp_ctx_s* c = new (std::nothrow) asicp_ctx_s();  // no exception crosses the C ABI
    if (!c) return fail(ASICP_E_HOST, "out of host memory for the context");
    c->d = d;
    c->cfg = *cfg;
    c->k = pb->k_start;
    c->k_start = pb->k_start;
    c->theta0 = pb->theta0;
    c->prev_cost0 = pb->prev_cost;
    c->converged0 = pb->converged;
    c->graph = nullptr;
    c->cap_stream = nullptr;
    c->capturing = false;
    c->final_done = false;
    c->inv_log_k = s.K >= 2 ? (float)(1.0 / std::log((double)s.K)) : 1.0f;
    c->n_timed = 0;
    c->side = c->side2 = nullptr;
    c->fork_ev = c->join_ev = c->join2_ev = nullptr;
    // default priority, like every stream here
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->join_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->join2_ev, hipEventDisableTiming) != hipSuccess) {
      asicp_destroy(c);
      return fail(ASICP_E_HIP, "creating the side stream or its events failed");
    }
    *out = c;
    return ASICP_OK;
  });
}

static void schedule_of(const asicp_config& cfg, int k, float* gamma, float* tau) {
  if (cfg.schedule == ASICP_SCHED_PAPER_CYCLIC) {
    const double period = (double)cfg.k_max / (double)cfg.cyc_C;
    *gamma = (float)std::pow(std::fmod((double)k, period) / period, (double)cfg.cyc_p);
    *tau = 1.0f;
  } else {
    *gamma = 1.0f;
    const double frac = cfg.k_max > 1 ? (double)k / (double)(cfg.k_max - 1) : 0.0;
    *tau = (float)((double)cfg.T0 * std::pow((double)cfg.T1 / (double)cfg.T0, frac));
  }
}

// One evaluation at the current poses (and, with bandwidth, the kernel
// bandwidth of the Stein update that follows): the forward NN on the caller's
// stream, the bandwidth select and the collision gate on the side stream,
// joined before the finaliser.
static asicp_status evaluate(asicp_ctx c, int k, int final_eval, bool bandwidth, hipStream_t hs) {
  asicp_status st;
  if (c->d.minibatch) {  // Table I: batch size grows linearly to the whole cloud at 2 k_max / 3
    const double full = 2.0 * (double)c->cfg.k_max / 3.0;
    const double frac = ((double)k < full ? (double)k : full) / full;
    launch_minibatch(c->d, k, frac, hs);
    if ((st = check_launch("minibatch")) != ASICP_OK) return st;
  }
  // With timing on (never inside a captured graph), the event that starts the
  // forward NN's timed interval is also the fork signal, so the caller's
  // stream records one event before the launch instead of two.
  const bool timing = (c->cfg.flags & ASICP_FLAG_TIMING) != 0 && !c->capturing;
  hipEvent_t e0 = c->fork_ev, e1 = nullptr;
  if (timing) {
    if ((size_t)(2 * c->n_timed + 2) > c->ev.size()) {
      hipEvent_t x, y;
      if (hipEventCreate(&x) != hipSuccess) return fail(ASICP_E_HIP, "hipEventCreate failed");
      if (hipEventCreate(&y) != hipSuccess) {
        (void)hipEventDestroy(x);
        return fail(ASICP_E_HIP, "hipEventCreate failed");
      }
      c->ev.push_back(x);
      c->ev.push_back(y);
    }
    e0 = c->ev[2 * c->n_timed];
    e1 = c->ev[2 * c->n_timed + 1];
  }
  if (hipEventRecord(e0, hs) != hipSuccess) return fail(ASICP_E_HIP, "hipEventRecord failed");
#ifndef ASICP_NN_FIRST
#define ASICP_NN_FIRST 1
#endif
  // The forward NN is enqueued before the side stream's work (the side
  // stream still waits only for e0): a captured graph then runs the two
  // branches concurrently.  The gate follows the bandwidth select: started
  // first, its workgroups take issue slots from the forward NN (which is
  // bound by instruction issue) and the solve runs 3-10 % slower; after the
  // select they mostly fill the forward launch's tail.
  auto forward = [&]() -> asicp_status {
    launch_nn_forward(c->d, hs);
    asicp_status s2 = check_launch("nn_forward");
    if (s2 != ASICP_OK) return s2;
    if (timing) {
      if (hipEventRecord(e1, hs) != hipSuccess) return fail(ASICP_E_HIP, "hipEventRecord failed");
      ++c->n_timed;
    }
    return ASICP_OK;
  };
  if (ASICP_NN_FIRST && (st = forward()) != ASICP_OK) return st;
  if (hipStreamWaitEvent(c->side, e0, 0) != hipSuccess) return fail(ASICP_E_HIP, "fork to the side stream failed");
  // In a captured graph, a forward launch too small to fill the GPU leaves
  // room for the gate beside the bandwidth select: then the gate gets a
  // branch of its own (a second side stream; on a small problem the
  // select-then-gate chain was the replayed iteration's critical path).  A
  // large forward launch is slowed by gate workgroups started early, so there
  // the gate follows the select; enqueued kernel by kernel, a third stream's
  // dependencies cost more than they save (small workload: 2.50 against
  // 1.50 ms per solve; replayed: 1.22 against 1.38 ms).
  const bool split = c->capturing && c->side2 && (long long)c->d.total_waves[c->d.nn_qi] <= kConcurrentGateWaves;
  if (split && hipStreamWaitEvent(c->side2, e0, 0) != hipSuccess)
    return fail(ASICP_E_HIP, "fork to the second side stream failed");
  hipStream_t gate_stream = split ? c->side2 : c->side;
#ifndef ASICP_GATE_FIRST
#define ASICP_GATE_FIRST 0
#endif
  if (ASICP_GATE_FIRST || split) {
    launch_gate_reverse(c->d, gate_stream);
    if ((st = check_launch("gate_reverse")) != ASICP_OK) return st;
  }
  if (bandwidth) {
    launch_bandwidth(c->d, c->inv_log_k, c->side);
    if ((st = check_launch("bandwidth")) != ASICP_OK) return st;
  }
  if (!ASICP_GATE_FIRST && !split) {
    launch_gate_reverse(c->d, gate_stream);
    if ((st = check_launch("gate_reverse")) != ASICP_OK) return st;
  }
  if (!ASICP_NN_FIRST && (st = forward()) != ASICP_OK) return st;
  if (hipEventRecord(c->join_ev, c->side) != hipSuccess || hipStreamWaitEvent(hs, c->join_ev, 0) != hipSuccess)
    return fail(ASICP_E_HIP, "join of the side stream failed");
  if (split && (hipEventRecord(c->join2_ev, c->side2) != hipSuccess || hipStreamWaitEvent(hs, c->join2_ev, 0) != hipSuccess))
    return fail(ASICP_E_HIP, "join of the second side stream failed");
  launch_finalize(c->d, k, final_eval, hs);
  return check_launch("finalize");
}

// Iteration k: evaluation, then (in the Stein phase) the Stein update.
static asicp_status iterate(asicp_ctx c, int k, hipStream_t hs) {
  const bool stein = k < c->cfg.k_stein;
  asicp_status st = evaluate(c, k, 0, stein, hs);
  if (st != ASICP_OK || !stein) return st;
  float gamma, tau;
  schedule_of(c->cfg, k, &gamma, &tau);
  // the update reads every pose of a group from one buffer and writes the
  // next poses to the other, which becomes the current one
  Dev& d = c->d;
  float* next = d.theta_next;
  launch_stein(d, gamma, tau, hs);
  d.theta_next = d.theta;
  d.theta = next;
  return check_launch("svgd");
}

asicp_status asicp_reset(asicp_ctx c, void* stream) {
  return guarded([&]() -> asicp_status {
    g_err.clear();
    if (!c) return fail(ASICP_E_INVALID, "ctx is NULL");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    Dev ds = c->d;
    ds.wave_pairs = nullptr;  // the pair counts of the timing records are kept
    launch_setup(ds, c->theta0, c->prev_cost0, c->converged0, hs);
    asicp_status st = check_launch("setup");
    if (st != ASICP_OK) return st;
    if (c->d.dbg_nn) {
      if (hipMemsetAsync(c->d.dbg_nn, 0xff, 4 * (size_t)c->d.Ktot * c->d.n_max, hs) != hipSuccess ||
          hipMemsetAsync(c->d.dbg_rev, 0xff, 4 * (size_t)c->d.Ktot * c->d.mc_max, hs) != hipSuccess)
        return fail(ASICP_E_HIP, "debug buffer clear failed");
    }
    c->k = c->k_start;
    c->final_done = false;
    return ASICP_OK;
  });
}

asicp_status asicp_step(asicp_ctx c, int32_t n_iters, void* stream) {
  return guarded([&]() -> asicp_status {
    g_err.clear();
    if (!c) return fail(ASICP_E_INVALID, "ctx is NULL");
    if (n_iters < 0) return fail(ASICP_E_INVALID, "n_iters must be >= 0");
    if (c->final_done) return fail(ASICP_E_STATE, "the solve has already run its final evaluation");
    if (c->k + n_iters > c->cfg.k_max)
      return fail(ASICP_E_STATE, "stepping past k_max (" + std::to_string(c->cfg.k_max) + ")");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    for (int it = 0; it < n_iters; ++it) {
      const asicp_status st = iterate(c, c->k, hs);
      if (st != ASICP_OK) return st;
      ++c->k;
    }
    return ASICP_OK;
  });
}

asicp_status asicp_solve(asicp_ctx c, void* stream) {
  return guarded([&]() -> asicp_status {
    g_err.clear();
    if (!c) return fail(ASICP_E_INVALID, "ctx is NULL");
    if (c->final_done) return fail(ASICP_E_STATE, "the solve has already run its final evaluation");
    asicp_status st = asicp_step(c, c->cfg.k_max - c->k, stream);
    if (st != ASICP_OK) return st;
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if ((st = evaluate(c, c->k, 1, false, hs)) != ASICP_OK) return st;
    launch_select(c->d, hs);
    if ((st = check_launch("select")) != ASICP_OK) return st;
    c->final_done = true;
    return ASICP_OK;
  });
}

// Enqueue iterations k0 .. k_max-1, the final evaluation and the selection.
static asicp_status enqueue_rest(asicp_ctx c, int k0, hipStream_t hs) {
  asicp_status st;
  for (int k = k0; k < c->cfg.k_max; ++k)
    if ((st = iterate(c, k, hs)) != ASICP_OK) return st;
  if ((st = evaluate(c, c->cfg.k_max, 1, false, hs)) != ASICP_OK) return st;
  launch_select(c->d, hs);
  return check_launch("select");
}

asicp_status asicp_cost_grad(asicp_ctx c, const float* theta, float* cost_out, float* grad_out, int32_t grad_form,
                             void* stream) {
  return guarded([&]() -> asicp_status {
    g_err.clear();
    if (!c || !theta) return fail(ASICP_E_INVALID, "ctx and theta must not be NULL");
    if (grad_form != ASICP_GRAD_TANGENT && grad_form != ASICP_GRAD_POSE)
      return fail(ASICP_E_INVALID, "grad_form must be ASICP_GRAD_TANGENT or ASICP_GRAD_POSE");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const int K = c->d.Ktot;
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_set_theta, dim3((7 * K + 255) / 256), dim3(256), 0, hs, c->d.theta, theta, 7 * K);
    asicp_status st = check_launch("set theta");
    if (st != ASICP_OK) return st;
    if ((st = evaluate(c, c->cfg.k_max, 1, false, hs)) != ASICP_OK) return st;
    hipLaunchKernelGGL(k_get_cost_grad, dim3((K + 255) / 256), dim3(256), 0, hs, c->d.theta, c->d.cost,
                       c->d.grad_ct, cost_out, grad_out, (int)grad_form, K);
    return check_launch("cost/grad copy");
  });
}

asicp_status asicp_pose_vjp(const float* grad, const float* gout, float* dtheta, int32_t ktot, void* stream) {
  return guarded([&]() -> asicp_status {
    g_err.clear();
    if (ktot < 0) return fail(ASICP_E_INVALID, "ktot must be >= 0");
    if (ktot == 0) return ASICP_OK;
    if (!grad || !gout || !dtheta) return fail(ASICP_E_INVALID, "grad, gout and dtheta must not be NULL");
    (void)hipGetLastError();
    hipLaunchKernelGGL(k_pose_vjp, dim3((unsigned)((ktot + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), grad, gout, dtheta, (int)ktot);
    return check_launch("pose vjp");
  });
}

asicp_status asicp_replay(asicp_ctx c, void* stream) {
  return guarded([&]() -> asicp_status {
    g_err.clear();
    if (!c) return fail(ASICP_E_INVALID, "ctx is NULL");
    if (c->d.dbg_nn) return fail(ASICP_E_STATE, "asicp_replay is not available with ASICP_FLAG_DEBUG");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    if (!c->graph) {
      // Capture on a private stream (the caller's may be the null stream,
      // which cannot be captured); capturing enqueues nothing.  Default
      // priority.
      if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        c->cap_stream = nullptr;
        return fail(ASICP_E_HIP, "hipStreamCreateWithFlags failed");
      }
      if (!c->side2 && hipStreamCreateWithFlags(&c->side2, hipStreamNonBlocking) != hipSuccess) {
        c->side2 = nullptr;
        return fail(ASICP_E_HIP, "hipStreamCreateWithFlags failed");
      }
      hipStream_t cs = c->cap_stream;
      (void)hipGetLastError();
      if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return fail(ASICP_E_HIP, "hipStreamBeginCapture failed");
      c->capturing = true;
      launch_setup(c->d, c->theta0, c->prev_cost0, c->converged0, cs);
      asicp_status st = check_launch("setup");
      if (st == ASICP_OK) st = enqueue_rest(c, c->k_start, cs);
      c->capturing = false;
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(cs, &g);
      if (st != ASICP_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess || !g) return fail(ASICP_E_HIP, "hipStreamEndCapture failed");
      c->graph_theta[0] = c->d.theta;
      c->graph_theta[1] = c->d.theta_next;
      const hipError_t ei = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) {
        c->graph = nullptr;
        return fail(ASICP_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
      }
    }
    if (hipGraphLaunch(c->graph, hs) != hipSuccess) return fail(ASICP_E_HIP, "hipGraphLaunch failed");
    // the double-buffered poses: an eager solve since the capture (after
    // asicp_reset) may have left the other buffer current
    c->d.theta = c->graph_theta[0];
    c->d.theta_next = c->graph_theta[1];
    c->k = c->cfg.k_max;
    c->final_done = true;
    return ASICP_OK;
  });
}

asicp_status asicp_result(asicp_ctx c, asicp_result_t* out, void* stream) {
  return guarded([&]() -> asicp_status {
    g_err.clear();
    if (!c || !out) return fail(ASICP_E_INVALID, "ctx and out must not be NULL");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    const Dev& d = c->d;
    const size_t K = (size_t)d.Ktot;
    struct Cp { void* dst; const void* src; size_t bytes; };
    const Cp dev[] = {
        {out->theta, d.theta, 4 * 7 * K},        {out->cost, d.cost, 4 * K},
        {out->col_cost, d.col_cost, 4 * K},      {out->ncol, d.ncol, 4 * K},
        {out->converged, d.converged, 4 * K},    {out->prev_cost, d.prev_cost, 4 * K},
        {out->grad, d.grad, 4 * 6 * K},          {out->grad_ct, d.grad_ct, 4 * 6 * K},
        {out->grad_col, d.grad_col, 4 * 6 * K},  {out->phi, d.phi, 4 * 6 * K},
        {out->h, d.h, 4 * (size_t)d.G},
    };
    for (const Cp& x : dev)
      if (x.dst && hipMemcpyAsync(x.dst, x.src, x.bytes, hipMemcpyDeviceToDevice, hs) != hipSuccess)
        return fail(ASICP_E_HIP, "device-to-device copy of a result failed");
    if (out->nn_idx) {
      if (!d.dbg_nn) return fail(ASICP_E_STATE, "nn_idx needs ASICP_FLAG_DEBUG");
      if (hipMemcpyAsync(out->nn_idx, d.dbg_nn, 4 * K * d.n_max, hipMemcpyDeviceToDevice, hs) != hipSuccess)
        return fail(ASICP_E_HIP, "copy of nn_idx failed");
    }
    if (out->rev_idx) {
      if (!d.dbg_rev) return fail(ASICP_E_STATE, "rev_idx needs ASICP_FLAG_DEBUG");
      if (hipMemcpyAsync(out->rev_idx, d.dbg_rev, 4 * K * d.mc_max, hipMemcpyDeviceToDevice, hs) != hipSuccess)
        return fail(ASICP_E_HIP, "copy of rev_idx failed");
    }
    std::vector<int32_t> best(2 * (size_t)d.n_obj);
    std::vector<float> bt(8 * (size_t)d.n_obj);
    int32_t flags[4] = {0, 0, 0, 0};
    if (hipMemcpyAsync(flags, d.flags, sizeof flags, hipMemcpyDeviceToHost, hs) != hipSuccess)
      return fail(ASICP_E_HIP, "copy of the device flags failed");
    if (c->final_done) {
      if (hipMemcpyAsync(best.data(), d.best, 4 * best.size(), hipMemcpyDeviceToHost, hs) != hipSuccess ||
          hipMemcpyAsync(bt.data(), d.best_theta, 4 * bt.size(), hipMemcpyDeviceToHost, hs) != hipSuccess)
        return fail(ASICP_E_HIP, "copy of the selected grasps failed");
    }
    const hipError_t e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return fail(ASICP_E_HIP, std::string("stream synchronisation: ") + hipGetErrorString(e));
    out->iterations_done = c->k;
    out->final_evaluated = c->final_done ? 1 : 0;
    for (int o = 0; o < d.n_obj; ++o) {
      if (out->best_particle) out->best_particle[o] = c->final_done ? best[2 * o] : -1;
      if (out->best_free) out->best_free[o] = c->final_done ? best[2 * o + 1] : 0;
      if (out->best_cost) out->best_cost[o] = c->final_done ? bt[8 * o + 7] : NAN;
      if (out->best_theta)
        for (int a = 0; a < 7; ++a) out->best_theta[7 * o + a] = c->final_done ? bt[8 * o + a] : NAN;
    }
    if (flags[1] != 0) return fail(ASICP_E_NUMERIC, "nearest-neighbour re-scan missed (non-finite distances)");
    if (flags[0] != 0) return fail(ASICP_E_NUMERIC, "a pose, cost or gradient became non-finite");
    return ASICP_OK;
  });
}

asicp_status asicp_kernel_time(asicp_ctx c, double* total_ms, int32_t* launches, double* nn_pairs) {
  return guarded([&]() -> asicp_status {
    g_err.clear();
    if (!c || !total_ms || !launches) return fail(ASICP_E_INVALID, "NULL argument");
    if (!(c->cfg.flags & ASICP_FLAG_TIMING)) return fail(ASICP_E_STATE, "context was created without ASICP_FLAG_TIMING");
    double tot = 0.0;
    for (int j = 0; j < c->n_timed; ++j) {
      if (hipEventSynchronize(c->ev[2 * j + 1]) != hipSuccess) return fail(ASICP_E_HIP, "hipEventSynchronize failed");
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, c->ev[2 * j], c->ev[2 * j + 1]) != hipSuccess)
        return fail(ASICP_E_HIP, "hipEventElapsedTime failed");
      tot += ms;
    }
    if (nn_pairs) {  // one slot per forward wave (no shared counter to contend for)
      std::vector<unsigned long long> per((size_t)c->d.total_waves[0], 0ull);
      if (c->n_timed > 0 && hipMemcpy(per.data(), c->d.wave_pairs, 8 * per.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(ASICP_E_HIP, "reading the pair counts failed");
      double cnt = 0.0;
      for (unsigned long long v : per) cnt += (double)v;
      *nn_pairs = cnt;
    }
    *total_ms = tot;
    *launches = c->n_timed;
    return ASICP_OK;
  });
}

static void launch_of(const Dev& d, asicp_launch_t* out) {
  out->xcd_map = d.xcd_map;
  out->fine = d.fine;
  out->query_blocks = q_blocks(d.nn_qi);
  out->chunk_points = 64 * d.nn_ch;
}

// The launch choice with index v (the order of asicp_autotune's ms_out).
static void choice_of(int v, Dev& d) {
  d.fine = v & 1;
  d.xcd_map = (v >> 1) & 1;
  d.nn_ch = ((v >> 2) & 1) ? 2 : 1;
  d.nn_qi = v >> 3;
}

asicp_status asicp_get_launch(asicp_ctx c, asicp_launch_t* out) {
  return guarded([&]() -> asicp_status {
    g_err.clear();
    if (!c || !out) return fail(ASICP_E_INVALID, "NULL argument");
    launch_of(c->d, out);
    return ASICP_OK;
  });
}

static void drop_graph(asicp_ctx c) {  // a captured solve holds the old launch choices
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  c->graph = nullptr;
}

asicp_status asicp_set_launch(asicp_ctx c, const asicp_launch_t* in) {
  return guarded([&]() -> asicp_status {
    g_err.clear();
    if (!c || !in) return fail(ASICP_E_INVALID, "NULL argument");
    if ((in->xcd_map != 0 && in->xcd_map != 1) || (in->fine != 0 && in->fine != 1))
      return fail(ASICP_E_INVALID, "xcd_map and fine must be 0 or 1");
    if (in->query_blocks != 1 && in->query_blocks != 2 && in->query_blocks != 4)
      return fail(ASICP_E_INVALID, "query_blocks must be 1, 2 or 4");
    if (in->chunk_points != 64 && in->chunk_points != 128)
      return fail(ASICP_E_INVALID, "chunk_points must be 64 or 128");
    c->d.xcd_map = in->xcd_map;
    c->d.fine = in->fine;
    c->d.nn_qi = in->query_blocks == 1 ? 0 : (in->query_blocks == 2 ? 1 : 2);
    c->d.nn_ch = in->chunk_points / 64;
    drop_graph(c);
    return ASICP_OK;
  });
}

asicp_status asicp_autotune(asicp_ctx c, int32_t reps, void* stream, asicp_launch_t* chosen, float* ms_out) {
  return guarded([&]() -> asicp_status {
    g_err.clear();
    if (!c) return fail(ASICP_E_INVALID, "ctx is NULL");
    if (reps < 1 || reps > 1000) return fail(ASICP_E_INVALID, "reps must be in 1..1000");
    hipStream_t hs = static_cast<hipStream_t>(stream);
    (void)hipGetLastError();
    if (c->d.minibatch) {  // the forward kernel reads the current mini-batch operand
      const int k = std::min(c->k, c->cfg.k_max);
      const double full = 2.0 * (double)c->cfg.k_max / 3.0;
      launch_minibatch(c->d, k, ((double)k < full ? (double)k : full) / full, hs);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      if (e0) (void)hipEventDestroy(e0);
      return fail(ASICP_E_HIP, "hipEventCreate failed");
    }
    auto timed = [&](auto&& launch, float* ms) -> bool {
      launch();  // warm-up
      if (hipEventRecord(e0, hs) != hipSuccess) return false;
      for (int r = 0; r < reps; ++r) launch();
      if (hipEventRecord(e1, hs) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return false;
      return hipEventElapsedTime(ms, e0, e1) == hipSuccess;
    };
    // Each choice is timed on one evaluation as an iteration runs it: the
    // side stream forks from `stream`, runs the bandwidth select (in the Stein
    // phase) and the collision kernel while the forward NN runs on `stream`,
    // and joins; how the three share the GPU depends on the choice.
    const bool bandwidth = c->k < c->cfg.k_stein;
    float ev_ms[ASICP_LAUNCH_CHOICES] = {};
    bool ok = true, streams_ok = true;
    for (int v = 0; v < ASICP_LAUNCH_CHOICES && ok; ++v) {
      Dev dv = c->d;
      dv.wave_pairs = nullptr;  // tuning launches are not counted
      choice_of(v, dv);
      ok = timed([&] {
        streams_ok = streams_ok && hipEventRecord(c->fork_ev, hs) == hipSuccess &&
                     hipStreamWaitEvent(c->side, c->fork_ev, 0) == hipSuccess;
        if (bandwidth) launch_bandwidth(dv, c->inv_log_k, c->side);
        launch_gate_reverse(dv, c->side);
        launch_nn_forward(dv, hs);
        streams_ok = streams_ok && hipEventRecord(c->join_ev, c->side) == hipSuccess &&
                     hipStreamWaitEvent(hs, c->join_ev, 0) == hipSuccess;
      }, &ev_ms[v]);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!ok || !streams_ok) return fail(ASICP_E_HIP, "timing a launch variant failed");
    const asicp_status st = check_launch("autotune");
    if (st != ASICP_OK) return st;
    // keep the current choice unless another is faster
    int bestv = ((c->d.nn_qi * 2 + (c->d.nn_ch == 2)) * 2 + c->d.xcd_map) * 2 + c->d.fine;
    for (int v = 0; v < ASICP_LAUNCH_CHOICES; ++v) {
      if (ev_ms[v] < ev_ms[bestv]) bestv = v;
      if (ms_out) ms_out[v] = ev_ms[v] / (float)reps;
    }
    choice_of(bestv, c->d);
    drop_graph(c);
    if (chosen) launch_of(c->d, chosen);
    return ASICP_OK;
  });
}

void asicp_destroy(asicp_ctx c) {
  if (!c) return;
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->side) (void)hipStreamDestroy(c->side);
  if (c->side2) (void)hipStreamDestroy(c->side2);
  if (c->fork_ev) (void)hipEventDestroy(c->fork_ev);
  if (c->join_ev) (void)hipEventDestroy(c->join_ev);
  if (c->join2_ev) (void)hipEventDestroy(c->join2_ev);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  delete c;
}

}  // extern "C"
