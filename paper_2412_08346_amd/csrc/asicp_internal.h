// asicp_internal.h -- device-side data layout and helpers shared by the HIP
// translation units of libasicp (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/asicp.h"

namespace asicp {

constexpr int kWave = 64;          // CDNA wavefront
constexpr int kTileGroup = 64;     // points per MFMA-ready tile group (4 tiles of 16)
constexpr int kQueriesPerWave = 64;
constexpr int kGateChunk = 256;    // collision points per gate workgroup
constexpr int kPartStride = 8;     // floats per partial-sum record
constexpr float kDummyNorm = 1.0e30f;  // |r|^2 of padding points: never a nearest neighbour

// Per-group descriptor (group = (object, preshape)).
struct GroupInfo {
  int32_t obj, pre;
  int32_t wave_off;   // first forward-NN wave of this group
  int32_t gate_off;   // first gate workgroup of this group
};

// Per-object descriptor.
struct ObjInfo {
  int32_t r_begin, m;      // offset into R inputs, point count
  int32_t c_begin, mc;     // offset into C inputs, point count
  int32_t prep_tg_begin;   // first tile group in the prepared object clouds
  int32_t ntg;             // tile groups (ceil(m / 64))
  int32_t gate_chunks;     // ceil(mc / 256)
  int32_t pad;
};

// Per-preshape descriptor.
struct PreInfo {
  int32_t s_begin, n;      // offset into S inputs, point count
  int32_t prep_tg_begin, ntg;
  int32_t waves;           // forward-NN waves per particle: ceil(n / 64)
  int32_t nx, ny, nz;
  const float* sdf;
  float ox, oy, oz, cell, inv_cell;
  float pad[3];
};

// Everything a kernel needs, passed by value.
struct Dev {
  // inputs (borrowed)
  const float *rx, *ry, *rz, *cx, *cy, *cz, *sx, *sy, *sz;
  // tables (workspace)
  const GroupInfo* groups;
  const ObjInfo* objs;
  const PreInfo* pres;
  int32_t n_obj, n_pre, K, G, Ktot;
  int32_t total_waves, total_gate_wgs;
  int32_t max_waves_pp, max_gate_chunks;  // partial-record strides
  int32_t n_max, mc_max;
  // prepared clouds: float4 per point in MFMA A-operand order
  float4* obj_prep;
  float4* pre_prep;
  float* obj_com;   // [n_obj][4]
  float* pre_const; // [n_pre][8]: tcp xyz, rho2, a_t, a_w, -, -
  // state
  float* theta;     // [7][Ktot]
  float* cost;
  float* col_cost;
  float* prev_cost;
  int32_t* ncol;
  int32_t* converged;
  float* grad;      // [6][Ktot]
  float* grad_ct;
  float* grad_col;
  float* phi;       // [6][Ktot]
  float* h;         // [G]
  float* nn_part;   // [Ktot][max_waves_pp][8]
  float* col_part;  // [Ktot][max_gate_chunks][8]
  int32_t* best;    // [n_obj][2]: particle, free flag
  float* best_theta;  // [n_obj][8]: theta(7), cost
  int32_t* flags;   // [0] non-finite, [1] NN re-scan miss
  int32_t* dbg_nn;  // [Ktot][n_max] or null
  int32_t* dbg_rev; // [Ktot][mc_max] or null
  // settings
  float eta, lambda;
  int32_t k_stein, kernel_mode, bw_mode, precond;
  float h_fixed, h_min, conv_tol;
};

typedef float f4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void quat_to_rot(float w, float x, float y, float z, float R[9]) {
  R[0] = 1.0f - 2.0f * (y * y + z * z);
  R[1] = 2.0f * (x * y - w * z);
  R[2] = 2.0f * (x * z + w * y);
  R[3] = 2.0f * (x * y + w * z);
  R[4] = 1.0f - 2.0f * (x * x + z * z);
  R[5] = 2.0f * (y * z - w * x);
  R[6] = 2.0f * (x * z - w * y);
  R[7] = 2.0f * (y * z + w * x);
  R[8] = 1.0f - 2.0f * (x * x + y * y);
}

__device__ __forceinline__ void load_pose(const float* theta, int Ktot, int i, float t[3], float q[4]) {
  t[0] = theta[0 * Ktot + i];
  t[1] = theta[1 * Ktot + i];
  t[2] = theta[2 * Ktot + i];
  q[0] = theta[3 * Ktot + i];
  q[1] = theta[4 * Ktot + i];
  q[2] = theta[5 * Ktot + i];
  q[3] = theta[6 * Ktot + i];
}

// Sum over the 64 lanes of a wave in a fixed butterfly order; every lane gets the total.
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Launchers (host side), one per kernel family.
void launch_setup(const Dev& d, const float* theta0, const float* prev_cost0,
                  const int32_t* converged0, hipStream_t s);
void launch_nn_forward(const Dev& d, hipStream_t s);
void launch_gate_reverse(const Dev& d, hipStream_t s);
void launch_finalize(const Dev& d, int k, int final_eval, hipStream_t s);
void launch_svgd(const Dev& d, float gamma, float tau, float inv_log_k, hipStream_t s);
void launch_select(const Dev& d, hipStream_t s);
void upload_words(void* dst, const void* src, size_t bytes, hipStream_t s);

}  // namespace asicp
