// asicp_internal.h -- device-side data layout and helpers shared by the HIP
// translation units of libasicp (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/asicp.h"

namespace asicp {

constexpr int kWave = 64;          // CDNA wavefront
constexpr int kTileGroup = 64;     // points per MFMA-ready tile group (4 tiles of 16)
// Forward-NN launch shapes, chosen per context at run time (asicp_set_launch,
// asicp_autotune): 1, 2 or 4 blocks of 16 queries per wavefront (index qi =
// 0, 1, 2: 1 << qi blocks) and pruning chunks of 1 or 2 tile groups.  A
// waves-per-SIMD occupancy request for the pruned kernels (0: compiler's).
constexpr int kNumQ = 3;
__host__ __device__ constexpr int q_blocks(int qi) { return 1 << qi; }
#ifndef ASICP_NN_WPE
#define ASICP_NN_WPE 7
#endif
// Candidate chunks compared between refreshes of the pruning bound.
#ifndef ASICP_NN_REFRESH
#define ASICP_NN_REFRESH 4
#endif
constexpr int kGateChunk = 2048;   // collision points per gate workgroup (8 per thread)
constexpr int kPartStride = 8;     // floats per partial-sum record
constexpr int kBrick = 4;          // cells per brick edge of the SDF cull table
constexpr int kBwSlices = 32;      // workgroups per group in each bandwidth pass
constexpr float kDummyNorm = 1.0e30f;  // |r|^2 of padding points: never a nearest neighbour

// Per gate workgroup: its group, particle, chunk of the collision cloud and
// that chunk's box (written at set-up, so a workgroup finds its work with
// one read).
struct GateWG {
  int32_t g, i, cc, box;
};

// Per-group descriptor (group = (object, preshape)).
struct GroupInfo {
  int32_t obj, pre;
  int32_t gate_off;            // first gate workgroup of this group
  int32_t wave_off[kNumQ];     // first forward-NN wave of this group, per query-block count
};

// Per-object descriptor.
struct ObjInfo {
  int32_t r_begin, m;      // offset into R inputs, point count
  int32_t c_begin, mc;     // offset into C inputs, point count
  int32_t prep_tg_begin;   // first tile group in the prepared object clouds
  int32_t ntg;             // tile groups (ceil(m / 64))
  int32_t gate_chunks;     // ceil(mc / kGateChunk)
  int32_t key_off;         // offset of this cloud's sort keys (uint64) in the scratch
  int32_t c_key_off;       // sort keys of the collision cloud
  int32_t gbox_begin;      // first of this cloud's gate-chunk boxes
};

// Per-preshape descriptor.
struct PreInfo {
  int32_t s_begin, n;      // offset into S inputs, point count
  int32_t prep_tg_begin, ntg;
  int32_t waves[kNumQ];    // forward-NN waves per particle: ceil(n / (16 q_blocks(qi)))
  int32_t nx, ny, nz;
  const float* sdf;
  float ox, oy, oz, cell, inv_cell;
  int32_t neg_lo[3];       // per axis: lowest / highest node index with a
  int32_t neg_hi[3];       //   negative value (set on the device at set-up)
  int32_t key_off;         // offset of this cloud's sort keys (uint64) in the scratch
  // Cull tables of the grid (written on the device at set-up):
  // cell_bits: bit (x % 32) of word ((z (ny - 1) + y) cbw + x / 32) is set when
  //   cell (x, y, z) (nodes x..x+1, y..y+1, z..z+1) has a negative node;
  // brick_sum: over bricks of kBrick^3 cells, entry (z (bny + 1) + y) (bnx + 1) + x
  //   counts the bricks (bx < x, by < y, bz < z) holding such a cell;
  // brick_flag: per brick (z bny + y) bnx + x, set-up scratch, zero between set-ups.
  const uint32_t* cell_bits;
  const int32_t* brick_sum;
  int32_t* brick_flag;
  int32_t cbw, bnx, bny, bnz;
  int32_t sdf_done;        // set-up workgroups finished on the tables (0 between set-ups)
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
  int32_t total_waves[kNumQ], total_gate_wgs;  // forward waves per query-block count
  int32_t max_waves_pp, max_gate_chunks;  // partial-record strides (max_waves_pp at 1 block per wave)
  int32_t n_max, mc_max;
  int32_t max_m, max_m_pad;  // largest object cloud, and padded to whole tile groups
  // clouds in k-d leaf order (index = prep_tg_begin*64 + k): MFMA-ready float4
  // (A-operand order), plain float4 (x, y, z, 0), original index (-1 for
  // padding), and one bounding box per pruning chunk of kChunkTG tile groups
  // (lo xyz, -, hi xyz, -).  Object and collision clouds are stored relative
  // to their object's centroid, contact clouds in the gripper frame.
  float4* obj_prep;
  float4* pre_prep;
  float4* obj_pts;
  float4* pre_pts;
  int32_t* obj_perm;
  int32_t* pre_perm;
  float* obj_box;   // per chunk of 2 tile groups (128 points)
  float* obj_box1;  // per tile group (64 points): the forward NN's 64-point chunks
  float* obj_blk;   // per block of 64 chunks of obj_box (a k-d subtree), at prep_tg_begin / 4 + b
  float* obj_blk1;  // the same for the 64-point chunks of obj_box1
  float* pre_box;
  float* col_box;  // [gate chunks][8]: box of each kGateChunk points of the sorted collision clouds
  float* col_leaf_box;  // [gate chunks][kGateChunk / 64][8]: box of each 64-point leaf of them
  float4* col_pts;    // collision clouds in k-d leaf order (offsets as the input's)
  int32_t* col_perm;
  unsigned long long* sort_keys;
  float* kd_box;      // the set-up's k-d build scratch, 16 floats per leaf: object clouds
                     //   per tile group, then contact clouds from kd_pre_off (4 per tile
                     //   group), then collision clouds from kd_col_off (32 per gate chunk)
  int32_t kd_pre_off, kd_col_off;
  int32_t sdf_blocks;  // set-up workgroups per preshape building the SDF cull tables
  GateWG* gate_wg;     // [total_gate_wgs]
  unsigned long long* wave_pairs;  // [total_waves[0]] distances evaluated per forward wave,
                                   //   summed over launches (ASICP_FLAG_TIMING only, else NULL)
  int32_t prune;                 // skip object chunks that cannot hold a nearest neighbour
  float* obj_com;   // [n_obj][4]: centroid xyz, largest |r - centroid|^2
  float* pre_const; // [n_pre][8]: tcp xyz, rho2, a_t, a_w, largest |s|^2, -
  // state
  float* theta;     // [7][Ktot] current poses: one of two buffers (the Stein
                    //   update writes the other, which then becomes current)
  float* theta_next;  // the Stein update's output buffer (set per launch)
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
  unsigned int* bw_hist;   // [G][256] radix histogram (zero between passes)
  unsigned int* bw_state;  // [G][4] prefix, mask, rank, finished workgroups
  float* nn_part;   // [Ktot][max_waves_pp][8]
  float* col_part;  // [Ktot][max_gate_chunks][8]
  float* pen_part;  // [Ktot][max_gate_chunks][8] penetration sums (w_pen > 0)
  int32_t* best;    // [n_obj][2]: particle, free flag
  float* best_theta;  // [n_obj][8]: theta(7), cost
  int32_t* flags;   // [0] non-finite, [1] NN re-scan miss
  int32_t* dbg_nn;  // [Ktot][n_max] or null
  int32_t* dbg_rev; // [Ktot][mc_max] or null
  // settings
  float eta, lambda;
  int32_t k_stein, kernel_mode, bw_mode, precond;
  float h_fixed, h_min, conv_tol;
  float w_pen;      // weight of the optional SDF penetration term
  int32_t minibatch;        // Table I mini-batch schedule of the object clouds
  unsigned long long seed;  // its sampling seed
  float4* obj_prep_mb;      // MFMA-ready object clouds with points outside the
                            //   iteration's mini-batch at |r|^2 = 1e30
  unsigned char* batch_mark;  // [sum M] 1 if the point is in the mini-batch
  const float* prior;       // [G][12] mu_t[3], w_t, mu_q[4] (unit), kappa, pad; NULL: none
  // launch choices that change no result (ASICP launch options)
  int32_t xcd_map;          // 0: contiguous work per XCD, 1: dispatch order
  int32_t fine;             // forward NN: per-query chunk test
  int32_t nn_qi;            // forward NN: 1 << nn_qi blocks of 16 queries per wave
  int32_t nn_ch;            // forward NN: tile groups per pruning chunk (1 or 2)
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

// A wave-uniform float computed on the vector unit, moved to a scalar
// register (gfx9 has no scalar float arithmetic).
__device__ __forceinline__ float uniform_f(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// The lane's index in its wavefront, from the execution mask (two VALU
// instructions that the compiler can repeat instead of keeping a register).
__device__ __forceinline__ int lane_id() {
  return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Cross-lane helpers built from VALU lane permutes only (no LDS crossbar):
// DPP within a row of 16 lanes, and gfx950's permlane16/32 swaps across rows.
template <int CTRL>
__device__ __forceinline__ float dppf(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ int dppi(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
constexpr int kDppXor1 = 0xB1;         // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141;  // lane l <-> 7-l within each 8
constexpr int kDppMirror = 0x140;      // lane l <-> 15-l within each row

// Value of the same position j in row 2k and row 2k+1 (k = lane's row pair),
// and of rows (0,2) / (1,3) after the 32-lane swap.
struct RowPair {
  float even, odd;
};
__device__ __forceinline__ RowPair swap16(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return {__uint_as_float(r[0]), __uint_as_float(r[1])};
}
__device__ __forceinline__ RowPair swap32(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
  return {__uint_as_float(r[0]), __uint_as_float(r[1])};
}
__device__ __forceinline__ int2 swap16i(int v) {
  const auto r = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
  return make_int2((int)r[0], (int)r[1]);
}
__device__ __forceinline__ int2 swap32i(int v) {
  const auto r = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
  return make_int2((int)r[0], (int)r[1]);
}

// Reductions over the four rows (lanes j, j+16, j+32, j+48); every lane gets the result.
__device__ __forceinline__ float rows_min(float v) {
  const RowPair a = swap16(v);
  v = fminf(a.even, a.odd);
  const RowPair b = swap32(v);
  return fminf(b.even, b.odd);
}
__device__ __forceinline__ int rows_min_i(int v) {
  const int2 a = swap16i(v);
  v = min(a.x, a.y);
  const int2 b = swap32i(v);
  return min(b.x, b.y);
}
__device__ __forceinline__ int rows_sum_i(int v) {
  const int2 a = swap16i(v);
  v = a.x + a.y;
  const int2 b = swap32i(v);
  return b.x + b.y;
}
// Reductions within each row of 16 lanes.
__device__ __forceinline__ float row_max(float v) {
  v = fmaxf(v, dppf<kDppXor1>(v));
  v = fmaxf(v, dppf<kDppXor2>(v));
  v = fmaxf(v, dppf<kDppHalfMirror>(v));
  return fmaxf(v, dppf<kDppMirror>(v));
}
__device__ __forceinline__ float row_min(float v) {
  v = fminf(v, dppf<kDppXor1>(v));
  v = fminf(v, dppf<kDppXor2>(v));
  v = fminf(v, dppf<kDppHalfMirror>(v));
  return fminf(v, dppf<kDppMirror>(v));
}

// Minimum over the 64 lanes of a wave (unsigned); every lane gets it.
__device__ __forceinline__ unsigned wave_min_u(unsigned v) {
  v = min(v, (unsigned)dppi<kDppXor1>((int)v));
  v = min(v, (unsigned)dppi<kDppXor2>((int)v));
  v = min(v, (unsigned)dppi<kDppHalfMirror>((int)v));
  v = min(v, (unsigned)dppi<kDppMirror>((int)v));
  const auto a = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  v = min(a[0], a[1]);
  const auto b = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  return min(b[0], b[1]);
}

// Eight sums over the 64 lanes of a wave at once, in a fixed order: register
// pairs are folded through the 32-lane swap (a[k] keeps the low half's sums of
// a[k], the high half's of a[k+4]), then the 16-lane swap, then within rows.
// Afterwards lane 8k (k = 0..7) holds the total of a[k].
__device__ __forceinline__ float wave_sum8(const float a[8]) {
  float b[4], c[2];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a[k]), __float_as_uint(a[k + 4]), false, false);
    b[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(b[k]), __float_as_uint(b[k + 2]), false, false);
    c[k] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  // row r: c[0] holds a[2r]'s partial sums, c[1] a[2r+1]'s; fold each row's
  // halves so lanes 0-7 carry c[0] and lanes 8-15 carry c[1]
  const float t0 = c[0] + dppf<kDppMirror>(c[0]);
  const float t1 = c[1] + dppf<kDppMirror>(c[1]);
  float v = (lane_id() & 8) ? t1 : t0;
  v += dppf<kDppHalfMirror>(v);
  v += dppf<kDppXor2>(v);
  v += dppf<kDppXor1>(v);
  return v;
}

// Eight sums over each row of 16 lanes at once, in a fixed order (the same
// for every row, whatever the other rows hold): values k and k + 4 are folded
// across the row's halves (lane l with 15 - l), then across quarter rows
// (l with 7 - l), then lane pairs (l with l ^ 1) and (l with l ^ 2).
// Afterwards lane 4m + j (j = 0, 1) of each row holds the row's total of
// value 2m + j.
__device__ __forceinline__ float row_sum8(const float a[8]) {
  const int l = lane_id() & 15;
  float b[4], c[2];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float keep = l < 8 ? a[k] : a[k + 4], send = l < 8 ? a[k + 4] : a[k];
    b[k] = keep + dppf<kDppMirror>(send);
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float keep = (l & 7) < 4 ? b[k] : b[k + 2], send = (l & 7) < 4 ? b[k + 2] : b[k];
    c[k] = keep + dppf<kDppHalfMirror>(send);
  }
  const float keep = (l & 1) ? c[1] : c[0], send = (l & 1) ? c[0] : c[1];
  const float d = keep + dppf<kDppXor1>(send);
  return d + dppf<kDppXor2>(d);
}

// Sum over the 64 lanes of a wave in a fixed order; every lane gets the total.
__device__ __forceinline__ float wave_sum(float v) {
  v += dppf<kDppXor1>(v);
  v += dppf<kDppXor2>(v);
  v += dppf<kDppHalfMirror>(v);
  v += dppf<kDppMirror>(v);
  const RowPair a = swap16(v);
  v = a.even + a.odd;
  const RowPair b = swap32(v);
  return b.even + b.odd;
}

// Launchers (host side), one per kernel family.
void zero_words(void* dst, long long n, hipStream_t s);  // n 32-bit words, a fill kernel
void launch_setup(const Dev& d, const float* theta0, const float* prev_cost0,
                  const int32_t* converged0, hipStream_t s);
void launch_nn_forward(const Dev& d, hipStream_t s);
void launch_gate_reverse(const Dev& d, hipStream_t s);
void launch_finalize(const Dev& d, int k, int final_eval, hipStream_t s);
void launch_bandwidth(const Dev& d, float inv_log_k, hipStream_t s);  // h of eq. (9), from the poses only
void launch_stein(const Dev& d, float gamma, float tau, hipStream_t s);  // phi and the pose update
void launch_select(const Dev& d, hipStream_t s);
void launch_minibatch(const Dev& d, int k, double frac, hipStream_t s);
void upload_words(void* dst, const void* src, size_t bytes, hipStream_t s);

}  // namespace asicp
