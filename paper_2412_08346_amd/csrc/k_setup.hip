// k_setup.hip -- per-object and per-preshape set-up (Algorithm 1
// preprocessing): centre of mass of each object cloud (its centroid), tool
// centre point of each contact cloud (its centroid, Sec. IV-B), the
// Gauss-Newton diagonal preconditioner of eq. (3), spatially sorted MFMA-ready
// copies of the clouds with per-chunk bounding boxes, the SDF cull tables (box
// of negative nodes, cell bits, brick counts), the table of gate workgroups,
// and the initial particle state.  Sums run in FP64 over a fixed order
// (strided per thread, then a fixed tree).
#include "nn_core.h"

namespace asicp {

__device__ void block_sum4(double v[4], double (*sh)[4]) {
  const int tid = threadIdx.x;
  for (int a = 0; a < 4; ++a) sh[tid][a] = v[a];
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (tid < off)
      for (int a = 0; a < 4; ++a) sh[tid][a] += sh[tid + off][a];
    __syncthreads();
  }
  for (int a = 0; a < 4; ++a) v[a] = sh[0][a];
  __syncthreads();
}

__device__ float block_max(float v, float* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 128; off >= 1; off >>= 1) {
    if (tid < off) sh[tid] = fmaxf(sh[tid], sh[tid + off]);
    __syncthreads();
  }
  v = sh[0];
  __syncthreads();
  return v;
}

// One workgroup per object: the centroid (the CoM of Sec. IV-B), and the
// largest squared distance of a point from it.  Every kernel works on the
// object's clouds and the poses relative to this centroid, so FP32 rounding
// scales with the object's size rather than its distance from the origin.
__global__ __launch_bounds__(256) void k_setup_obj(Dev d) {
  __shared__ double sh[256][4];
  __shared__ float shm[256];
  const int o = blockIdx.x, tid = threadIdx.x;
  const ObjInfo oi = d.objs[o];
  double v[4] = {0, 0, 0, 0};
  for (int m = tid; m < oi.m; m += 256) {
    v[0] += d.rx[oi.r_begin + m];
    v[1] += d.ry[oi.r_begin + m];
    v[2] += d.rz[oi.r_begin + m];
  }
  block_sum4(v, sh);
  float com[3];
  for (int a = 0; a < 3; ++a) com[a] = (float)(v[a] / (double)oi.m);
  float r2 = 0.f;
  for (int m = tid; m < oi.m; m += 256) {
    const float x = d.rx[oi.r_begin + m] - com[0], y = d.ry[oi.r_begin + m] - com[1],
                z = d.rz[oi.r_begin + m] - com[2];
    r2 = fmaxf(r2, __builtin_fmaf(z, z, __builtin_fmaf(y, y, x * x)));
  }
  r2 = block_max(r2, shm);
  if (tid == 0) {
    for (int a = 0; a < 3; ++a) d.obj_com[4 * o + a] = com[a];
    d.obj_com[4 * o + 3] = r2;
  }
}

// one workgroup per preshape
__global__ __launch_bounds__(256) void k_setup_pre(Dev d) {
  __shared__ double sh[256][4];
  __shared__ float shm[256];
  const int p = blockIdx.x, tid = threadIdx.x;
  const PreInfo pi = d.pres[p];
  double v[4] = {0, 0, 0, 0};
  float s2 = 0.f;  // largest |s|^2 (gripper frame)
  for (int n = tid; n < pi.n; n += 256) {
    const float fx = d.sx[pi.s_begin + n], fy = d.sy[pi.s_begin + n], fz = d.sz[pi.s_begin + n];
    const double x = fx, y = fy, z = fz;
    v[0] += x; v[1] += y; v[2] += z;
    v[3] += x * x + y * y + z * z;
    s2 = fmaxf(s2, __builtin_fmaf(fz, fz, __builtin_fmaf(fy, fy, fx * fx)));
  }
  block_sum4(v, sh);
  s2 = block_max(s2, shm);
  if (tid == 0) {
    const double inv = 1.0 / (double)pi.n;
    const double tx = v[0] * inv, ty = v[1] * inv, tz = v[2] * inv, rho2 = v[3] * inv;
    const double lam = (double)d.lambda;
    double at = 1.0, aw = 1.0;
    if (d.precond == ASICP_PRECOND_GN_DIAG) {
      at = 1.0 / (1.0 + lam);
      aw = 3.0 / (2.0 * (rho2 + lam * (tx * tx + ty * ty + tz * tz)));
    }
    float* pc = d.pre_const + 8 * p;
    pc[0] = (float)tx; pc[1] = (float)ty; pc[2] = (float)tz; pc[3] = (float)rho2;
    pc[4] = (float)at; pc[5] = (float)aw; pc[6] = s2; pc[7] = 0.f;
  }
}

// Clouds of up to this many (power-of-two padded) points, and of up to
// kLdsLeaves k-d leaves, are ordered in LDS.
constexpr int kLdsKeys = 8192;
constexpr int kLdsLeaves = 512;
// A sort key ends in the point's original index (clouds hold < 2^22 points).
constexpr unsigned long long kOrigMask = (1ull << 22) - 1;

// Ascending bitonic sort of npow2 (a power of two) keys, in LDS or global
// memory, by one workgroup of 1024 threads (inlined, so that LDS arrays are
// addressed as LDS).  With seg < npow2 (a power of two) each aligned block of
// seg keys is sorted on its own (fewer stages: the blocks need no merging).
template <typename K>
__device__ __forceinline__ void bitonic_sort(K* keys, int npow2, int tid, int seg) {
  for (int size = 2; size <= seg; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = tid; t < (npow2 >> 1); t += 1024) {
        const int i = ((t & ~(stride - 1)) << 1) | (t & (stride - 1));  // stride is a power of two
        const int j = i + stride;
        const bool asc = size == seg || (i & size) == 0;
        const K a = keys[i], c = keys[j];
        if ((a > c) == asc) {
          keys[i] = c;
          keys[j] = a;
        }
      }
      __syncthreads();
    }
  }
}

// The same sort for keys in LDS with the keys held in registers: thread t
// keeps the E = max(1, npow2 / 1024) consecutive keys
// E t .. E t + E - 1.  A compare-exchange at stride s pairs key positions p
// and p ^ s: for s < E both lie in one thread, for s < 64 E in two lanes of
// one wavefront (a lane exchange, no barrier), and only larger strides go
// through LDS with a workgroup barrier.  Keys are unique, so the result is
// the one bitonic_sort gives.
template <typename K, int E>
__device__ __forceinline__ void bitonic_sort_lds(K* keys, int npow2, int tid, int seg) {
  const bool act = tid * E < npow2;
  K k[E];
  auto load = [&]() {
#pragma unroll
    for (int e = 0; e < E; ++e) k[e] = act ? keys[tid * E + e] : (K)~0ull;
  };
  auto store = [&]() {
    if (act)
#pragma unroll
      for (int e = 0; e < E; ++e) keys[tid * E + e] = k[e];
  };
  load();
  for (int size = 2; size <= seg; size <<= 1) {
    int stride = size >> 1;
    if (stride >= 64 * E) {
      store();
      __syncthreads();
      for (; stride >= 64 * E; stride >>= 1) {
        for (int t = tid; t < (npow2 >> 1); t += 1024) {
          const int i = ((t & ~(stride - 1)) << 1) | (t & (stride - 1));
          const int j = i + stride;
          const bool asc = size == seg || (i & size) == 0;
          const K a = keys[i], c = keys[j];
          if ((a > c) == asc) {
            keys[i] = c;
            keys[j] = a;
          }
        }
        __syncthreads();
      }
      load();
    }
    for (; stride >= E; stride >>= 1) {  // partner lane tid ^ (stride / E)
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const K o = __shfl_xor(k[e], stride / E, 64);
        const int pos = tid * E + e;
        const bool lower = (pos & stride) == 0, asc = size == seg || (pos & size) == 0;
        k[e] = (lower == asc) ? (o < k[e] ? o : k[e]) : (o > k[e] ? o : k[e]);
      }
    }
    for (; stride >= 1; stride >>= 1) {  // within the thread
#pragma unroll
      for (int e = 0; e < E; ++e) {
        if (e & stride) continue;
        const int e2 = e | stride;
        const bool asc = size == seg || ((tid * E + e) & size) == 0;
        const K a = k[e], c = k[e2];
        if ((a > c) == asc) {
          k[e] = c;
          k[e2] = a;
        }
      }
    }
  }
  store();
  __syncthreads();
}

// Lane exchanges pay off while each thread holds one key: there a
// workgroup barrier per stage costs more than the exchange.  With several
// keys per thread both partners of a pair compute it, and the LDS stages
// were faster (8192 keys: 0.64 against 0.48 ms per paper-scale set-up).
template <typename K>
__device__ __forceinline__ void sort_keys(K* keys, int npow2, int tid, int seg, bool lds) {
  if (lds && npow2 <= 1024) bitonic_sort_lds<K, 1>(keys, npow2, tid, seg);
  else bitonic_sort(keys, npow2, tid, seg);
}

// The k-d layout of a cloud: leaves of `unit` points; a part of L >= 2
// leaves splits after A max(1, round(L / 2A)) leaves, A the largest power of
// two below L capped at `cap`, so every aligned block of cap leaves (and of
// every power of two below it) is one subtree.  One split: [a, b), the
// leaves of the part holding leaf lf, becomes the half holding lf.
__device__ __forceinline__ void kd_split(int cap, int lf, int& a, int& b) {
  const int L = b - a;
  if (L <= 1) return;
  int sh = 0;  // A = 2^sh
  while ((2 << sh) < L && (1 << sh) < cap) ++sh;
  const int m = a + (max(1, (L + (1 << sh)) >> (sh + 1)) << sh);
  if (lf < m) b = m; else a = m;
}

// Orders a cloud's n points as the leaves of a k-d tree: each part is sorted
// along the longest axis of its bounding box and split at the leaf boundary
// above (the halves of a median split, rounded to whole aligned leaves).
// Consecutive runs of points (pruning chunks, query blocks, gate workgroups)
// then have tight boxes, which the exact pruning of the scans depends on
// (space-filling-curve orders leave some runs spanning a jump of the curve).
// One level per pass: every point's key becomes (first leaf of its part,
// 16-bit position along the part's axis, original index), and one sort
// orders all parts at once; ties fall to the original index, so the order is
// deterministic.  unit: points per leaf (16 or 64); kb: 16 floats of scratch
// per leaf (its box, the part's axis and quantisation in the part's first
// leaf, and the bounds [a, b) of the leaf's current part, updated by one
// split per level).  Inlined, so that LDS arrays passed in are addressed as
// LDS.
template <typename K>
__device__ __forceinline__ void kd_leaf_order(K* keys, int n, int npow2, int unit, int cap, const float* sx,
                                              const float* sy, const float* sz, float* kb, int* s_split, int tid,
                                              bool lds) {
  // 64-bit keys: (first leaf of the part, 16-bit position, original index);
  // 32-bit keys, when every part is an aligned block sorted on its own (the
  // part is implied by the position): (10-bit position, original index)
  constexpr bool k32 = sizeof(K) == 4;
  constexpr float kQ = k32 ? 1023.0f : 65535.0f;
  const int ush = unit == 16 ? 4 : 6;  // unit is 16 or 64
  const int nleaf = (n + unit - 1) >> ush;
  const int w = tid >> 6, lane = tid & 63;
  // the part of leaf l: [kb[16 l + 12], kb[16 l + 13]) (integers)
  auto part_of = [&](int l, int& a, int& b) {
    a = __float_as_int(kb[(size_t)l * 16 + 12]);
    b = __float_as_int(kb[(size_t)l * 16 + 13]);
  };
  for (int k = tid; k < npow2; k += 1024) keys[k] = k < n ? (K)k : (K)~0ull;
  for (int l = tid; l < nleaf; l += 1024) {
    kb[(size_t)l * 16 + 12] = __int_as_float(0);
    kb[(size_t)l * 16 + 13] = __int_as_float(nleaf);
  }
  __syncthreads();
  for (int level = 0;; ++level) {
    // the box of every leaf in the current order: a wavefront covers 64
    // consecutive points, 64 / unit leaves, kBoxBatch runs of them with their
    // point reads in flight together
    constexpr int kBoxBatch = 4;
    for (int base0 = w * 64; base0 < nleaf * unit; base0 += kBoxBatch * 16 * 64) {
      float p[kBoxBatch][3];
#pragma unroll
      for (int u = 0; u < kBoxBatch; ++u) {
        const int pos = base0 + u * 16 * 64 + lane;
        p[u][0] = p[u][1] = p[u][2] = 0.f;
        if (pos < n) {
          const int o = (int)(keys[pos] & kOrigMask);
          p[u][0] = sx[o];
          p[u][1] = sy[o];
          p[u][2] = sz[o];
        }
      }
#pragma unroll
      for (int u = 0; u < kBoxBatch; ++u) {
        if (base0 + u * 16 * 64 >= nleaf * unit) break;  // uniform over the wavefront
        const int pos = base0 + u * 16 * 64 + lane;
        const bool in = pos < n;
        float v[6] = {in ? p[u][0] : __builtin_inff(), in ? p[u][1] : __builtin_inff(), in ? p[u][2] : __builtin_inff(),
                      in ? p[u][0] : -__builtin_inff(), in ? p[u][1] : -__builtin_inff(), in ? p[u][2] : -__builtin_inff()};
        for (int off = unit >> 1; off >= 1; off >>= 1) {
          for (int a = 0; a < 3; ++a) v[a] = fminf(v[a], __shfl_xor(v[a], off, 64));
          for (int a = 3; a < 6; ++a) v[a] = fmaxf(v[a], __shfl_xor(v[a], off, 64));
        }
        if ((lane & (unit - 1)) == 0 && (pos >> ush) < nleaf)
          for (int a = 0; a < 6; ++a) kb[(size_t)(pos >> ush) * 16 + a] = v[a];
      }
    }
    if (tid == 0) *s_split = 0;
    __syncthreads();
    // every part that still splits: its box from its leaves (one wavefront
    // per part), the longest axis and the quantisation along it, kept in the
    // part's first leaf
    for (int lf = w; lf < nleaf; lf += 16) {
      int a, b;
      part_of(lf, a, b);
      if (lf != a || b - a < 2) continue;  // uniform over the wavefront
      float v[6] = {__builtin_inff(), __builtin_inff(), __builtin_inff(),
                    -__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
      for (int l = a + lane; l < b; l += 64) {
        for (int c = 0; c < 3; ++c) v[c] = fminf(v[c], kb[(size_t)l * 16 + c]);
        for (int c = 3; c < 6; ++c) v[c] = fmaxf(v[c], kb[(size_t)l * 16 + c]);
      }
      for (int off = 32; off >= 1; off >>= 1) {
        for (int c = 0; c < 3; ++c) v[c] = fminf(v[c], __shfl_xor(v[c], off, 64));
        for (int c = 3; c < 6; ++c) v[c] = fmaxf(v[c], __shfl_xor(v[c], off, 64));
      }
      if (lane == 0) {
        int ax = 0;
        for (int c = 1; c < 3; ++c)
          if (v[3 + c] - v[c] > v[3 + ax] - v[ax]) ax = c;
        const float ext = v[3 + ax] - v[ax];
        kb[(size_t)a * 16 + 8] = __int_as_float(ax);
        kb[(size_t)a * 16 + 9] = v[ax];
        kb[(size_t)a * 16 + 10] = ext > 0.f ? kQ / ext : 0.f;
        *s_split = 1;
      }
    }
    __syncthreads();
    if (*s_split == 0) break;  // every part is one leaf
    // new keys, kKeyBatch points per thread with their coordinate reads in
    // flight together
    constexpr int kKeyBatch = 4;
    for (int pos0 = tid; pos0 < n; pos0 += kKeyBatch * 1024) {
      int o[kKeyBatch], a[kKeyBatch], b[kKeyBatch];
      float x[kKeyBatch];
#pragma unroll
      for (int u = 0; u < kKeyBatch; ++u) {
        const int pos = pos0 + u * 1024;
        o[u] = 0;
        a[u] = b[u] = 0;
        x[u] = 0.f;
        if (pos < n) {
          o[u] = (int)(keys[pos] & kOrigMask);
          part_of(pos >> ush, a[u], b[u]);
          if (b[u] - a[u] >= 2) {
            const int ax = __float_as_int(kb[(size_t)a[u] * 16 + 8]);
            x[u] = (ax == 0 ? sx : (ax == 1 ? sy : sz))[o[u]];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < kKeyBatch; ++u) {
        const int pos = pos0 + u * 1024;
        if (pos >= n) continue;
        unsigned int q = 0;
        if (b[u] - a[u] >= 2)
          q = (unsigned int)fminf(fmaxf((x[u] - kb[(size_t)a[u] * 16 + 9]) * kb[(size_t)a[u] * 16 + 10], 0.f), kQ);
        if (k32)  // position (10 bits) | original index (< 2^22)
          keys[pos] = (K)((q << 22) | (unsigned int)o[u]);
        else      // part (< 2^18 leaves) | position (16 bits) | original index (< 2^22)
          keys[pos] = (K)(((unsigned long long)a[u] << 38) | ((unsigned long long)q << 22) | (unsigned int)o[u]);
      }
    }
    __syncthreads();
    // each leaf's part for the next level: the half of the current one
    // holding it (read above only, so no barrier is needed before the sort)
    for (int l = tid; l < nleaf; l += 1024) {
      int a, b;
      part_of(l, a, b);
      kd_split(cap, l, a, b);
      kb[(size_t)l * 16 + 12] = __int_as_float(a);
      kb[(size_t)l * 16 + 13] = __int_as_float(b);
    }
    // a cloud of a power-of-two number of whole leaves splits into aligned
    // halves, so at this level every part is an aligned block of n >> level
    // points and sorts on its own
    const bool halves = n == npow2 && (nleaf & (nleaf - 1)) == 0;
    sort_keys(keys, npow2, tid, halves ? (npow2 >> level) : npow2, lds);
  }
}

// SDF cull tables of preshape p, built by workgroup j of d.sdf_blocks (1024
// threads each) beside the cloud sorts, in one pass over the cells (each
// node is a corner of some cell): one bit per cell telling whether any of its
// 8 nodes is negative (a trilinear value is a convex combination of the
// cell's node values, so only such a cell can give a negative value), the
// box of the negative nodes, and a flag per brick of kBrick^3 cells holding
// such a cell.  The last workgroup to finish turns the flags into 3-D prefix
// counts (the number of such bricks in any box of bricks from 8 entries)
// and clears them for the next set-up.
__device__ void sdf_tables(const Dev& d, int p, int j) {
  __shared__ int s_last;
  PreInfo* pi = const_cast<PreInfo*>(d.pres) + p;
  const int nx = pi->nx, ny = pi->ny, nz = pi->nz;
  const float* v = pi->sdf;
  const int tid = threadIdx.x, lane = tid & 63;
  const long long stride = (long long)d.sdf_blocks * 1024;
  const int cbw = pi->cbw, bnx = pi->bnx, bny = pi->bny, bnz = pi->bnz;
  uint32_t* bits = const_cast<uint32_t*>(pi->cell_bits);
  int* F = pi->brick_flag;
  const long long nwords = (long long)(nz - 1) * (ny - 1) * cbw;
  const long long sy = nx, sz = (long long)nx * ny;
  int lo[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, hi[3] = {-1, -1, -1};
  // slot s is bit s % 32 of word s / 32; the 64 slots of a wave are two
  // whole words (the loop bound is uniform over the wave)
  for (long long s0 = (long long)j * 1024 + (tid & ~63); s0 < 32 * nwords; s0 += stride) {
    const long long w = (s0 + lane) >> 5;
    bool neg = false;
    if (w < nwords) {
      const int x = (int)(w % cbw) * 32 + (lane & 31);
      const long long row = w / cbw;
      const int y = (int)(row % (ny - 1)), z = (int)(row / (ny - 1));
      if (x < nx - 1) {
        const float* g = v + (long long)z * sz + (long long)y * sy + x;
        // n[4 dz + 2 dy + dx]: node (x + dx, y + dy, z + dz) is negative
        const bool n0 = g[0] < 0.f, n1 = g[1] < 0.f, n2 = g[sy] < 0.f, n3 = g[sy + 1] < 0.f;
        const bool n4 = g[sz] < 0.f, n5 = g[sz + 1] < 0.f, n6 = g[sz + sy] < 0.f, n7 = g[sz + sy + 1] < 0.f;
        neg = n0 || n1 || n2 || n3 || n4 || n5 || n6 || n7;
        if (neg) {
          // the cell's negative corners: per axis the lower coordinate if
          // one of them lies on the lower face, the upper one likewise
          lo[0] = min(lo[0], (n0 || n2 || n4 || n6) ? x : x + 1);
          hi[0] = max(hi[0], (n1 || n3 || n5 || n7) ? x + 1 : x);
          lo[1] = min(lo[1], (n0 || n1 || n4 || n5) ? y : y + 1);
          hi[1] = max(hi[1], (n2 || n3 || n6 || n7) ? y + 1 : y);
          lo[2] = min(lo[2], (n0 || n1 || n2 || n3) ? z : z + 1);
          hi[2] = max(hi[2], (n4 || n5 || n6 || n7) ? z + 1 : z);
          // every writer stores the same value
          F[((long long)(z / kBrick) * bny + y / kBrick) * bnx + x / kBrick] = 1;
        }
      }
    }
    const unsigned long long b = __ballot(neg);
    if ((lane & 31) == 0 && w < nwords) bits[w] = (uint32_t)(b >> (lane & 32));
  }
  for (int a = 0; a < 3; ++a) {
    for (int off = 32; off >= 1; off >>= 1) {
      lo[a] = min(lo[a], __shfl_xor(lo[a], off, 64));
      hi[a] = max(hi[a], __shfl_xor(hi[a], off, 64));
    }
  }
  if (lane == 0) {
    for (int a = 0; a < 3; ++a) {
      if (lo[a] != 0x7fffffff) atomicMin(&pi->neg_lo[a], lo[a]);
      if (hi[a] != -1) atomicMax(&pi->neg_hi[a], hi[a]);
    }
  }
  // the last workgroup to finish: prefix counts from the flags (written by
  // other workgroups, so read, and the table written and re-read, with
  // device-scope atomics, 8 entries of a line in flight at a time)
  __threadfence();
  __syncthreads();
  if (tid == 0) s_last = atomicAdd(&pi->sdf_done, 1) == d.sdf_blocks - 1;
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  const int ex = bnx + 1, ey = bny + 1;
  const long long plane = (long long)ex * ey;
  int* S = const_cast<int*>(pi->brick_sum);
  // src (null: zeros) holds len - 1 values; dst gets 0 and their running sums
  auto scan_line = [&](int* src, long long sstep, int* dst, long long dstep, int len, bool clear) {
    int acc = 0;
    __hip_atomic_store(dst, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int x0 = 0; x0 < len - 1; x0 += 8) {
      int val[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        val[u] = (src && x0 + u < len - 1)
                     ? __hip_atomic_load(src + (x0 + u) * sstep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                     : 0;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        acc += val[u];
        if (x0 + u < len - 1) {
          __hip_atomic_store(dst + (x0 + u + 1) * dstep, acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (clear) __hip_atomic_store(src + (x0 + u) * sstep, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
  };
  // along x: S line (y', z') from flag line (y' - 1, z' - 1); lines with
  // y' = 0 or z' = 0 are zero
  for (long long l = tid; l < (long long)ey * (bnz + 1); l += 1024) {
    const int yy = (int)(l % ey), zz = (int)(l / ey);
    int* src = (yy > 0 && zz > 0) ? F + ((long long)(zz - 1) * bny + (yy - 1)) * bnx : nullptr;
    scan_line(src, 1, S + l * ex, 1, ex, src != nullptr);
  }
  __syncthreads();
  // along y and z, in place (entry 0 of each line is already 0)
  for (long long l = tid; l < (long long)ex * (bnz + 1); l += 1024) {
    int* r = S + (l / ex) * plane + (l % ex);
    scan_line(r + ex, ex, r, ex, ey, false);
  }
  __syncthreads();
  for (long long l = tid; l < plane; l += 1024) scan_line(S + l + plane, plane, S + l, plane, bnz + 1, false);
  if (tid == 0) pi->sdf_done = 0;  // ready for the next set-up
}

// One workgroup (1024 threads) per cloud: blocks [0, n_obj) sort object
// clouds, blocks [n_obj, n_obj + n_pre) contact clouds, the last n_obj blocks
// collision clouds (object and collision clouds relative to the object's
// centroid).  Points are put in k-d leaf order (kd_leaf_order; ties by
// original index, so the order is deterministic), then written as
// MFMA-ready float4, plain
// float4, the original index, and one bounding box per pruning chunk; a
// collision cloud gets a plain copy, the original index and one box per
// kGateChunk points (one gate workgroup's share).  Padding points carry
// |r|^2 = 1e30.
__global__ __launch_bounds__(1024) void k_sort_cloud(Dev d) {
  const int tid = threadIdx.x;
  if ((int)blockIdx.x >= 2 * d.n_obj + d.n_pre) {  // uniform: an SDF table workgroup
    const int b = (int)blockIdx.x - 2 * d.n_obj - d.n_pre;
    sdf_tables(d, b / d.sdf_blocks, b % d.sdf_blocks);
    return;
  }
  // kind 0: object cloud, 1: contact cloud, 2: collision cloud (no MFMA copy)
  const int kind = blockIdx.x < d.n_obj ? 0 : (blockIdx.x < d.n_obj + d.n_pre ? 1 : 2);
  const float *sx, *sy, *sz;
  int n, tg0 = 0, ntg = 0, key_off;
  float4 *prep = nullptr, *pts;
  int32_t* perm;
  float* box = nullptr;
  size_t base;  // first output index
  // object and collision clouds are stored relative to the object's centroid
  // (written by k_setup_obj earlier on the stream); contact clouds stay in
  // the gripper frame
  float c0 = 0.f, c1 = 0.f, c2 = 0.f;
  if (kind != 1) {
    const float* com = d.obj_com + 4 * (kind == 0 ? blockIdx.x : blockIdx.x - d.n_obj - d.n_pre);
    c0 = com[0]; c1 = com[1]; c2 = com[2];
  }
  if (kind == 0) {
    const ObjInfo& oi = d.objs[blockIdx.x];
    sx = d.rx + oi.r_begin; sy = d.ry + oi.r_begin; sz = d.rz + oi.r_begin;
    n = oi.m; tg0 = oi.prep_tg_begin; ntg = oi.ntg; key_off = oi.key_off;
    prep = d.obj_prep; pts = d.obj_pts; perm = d.obj_perm; box = d.obj_box;
    base = (size_t)tg0 * 64;
  } else if (kind == 1) {
    const PreInfo& pi = d.pres[blockIdx.x - d.n_obj];
    sx = d.sx + pi.s_begin; sy = d.sy + pi.s_begin; sz = d.sz + pi.s_begin;
    n = pi.n; tg0 = pi.prep_tg_begin; ntg = pi.ntg; key_off = pi.key_off;
    prep = d.pre_prep; pts = d.pre_pts; perm = d.pre_perm; box = d.pre_box;
    base = (size_t)tg0 * 64;
  } else {
    const ObjInfo& oi = d.objs[blockIdx.x - d.n_obj - d.n_pre];
    sx = d.cx + oi.c_begin; sy = d.cy + oi.c_begin; sz = d.cz + oi.c_begin;
    n = oi.mc; key_off = oi.c_key_off;
    pts = d.col_pts; perm = d.col_perm;
    base = (size_t)oi.c_begin;
  }
  if (n == 0) return;  // uniform: an empty collision cloud
  // keys, padded to a power of two with the largest key, and the k-d
  // scratch: in LDS when they fit, else in the workspace
  int npow2 = 2;
  while (npow2 < n) npow2 <<= 1;
  __shared__ unsigned long long lkeys[kLdsKeys];
  __shared__ float lkb[kLdsLeaves * 16];
  __shared__ int s_split;
  // k-d leaf order: object clouds in 64-point leaves (pruning chunks of 64
  // and 128 points are subtrees), contact clouds in 16-point leaves (query
  // blocks of 16 to 64 points and the reverse scan's 128-point chunks are
  // subtrees), collision clouds in 64-point leaves within aligned blocks of
  // kGateChunk points (one gate workgroup's share)
  const int unit = kind == 1 ? 16 : 64;
  const int cap = kind == 2 ? kGateChunk / 64 : 128 / unit;
  const bool lds = npow2 <= kLdsKeys && (n + unit - 1) / unit <= kLdsLeaves;  // uniform
  unsigned long long* keys = lds ? lkeys : d.sort_keys + key_off;
  const bool halves = n == npow2 && (((n + unit - 1) / unit) & ((n + unit - 1) / unit - 1)) == 0;
  if (lds && halves) {
    // 32-bit keys in the first half of lkeys, widened to the 64-bit keys the
    // code below reads
    unsigned int* k32 = reinterpret_cast<unsigned int*>(lkeys);
    kd_leaf_order(k32, n, npow2, unit, cap, sx, sy, sz, lkb, &s_split, tid, true);
    unsigned int v[kLdsKeys / 1024];
    for (int r = 0; r < kLdsKeys / 1024; ++r) v[r] = tid + r * 1024 < npow2 ? k32[tid + r * 1024] : 0u;
    __syncthreads();
    for (int r = 0; r < kLdsKeys / 1024; ++r)
      if (tid + r * 1024 < npow2) lkeys[tid + r * 1024] = v[r] == ~0u ? ~0ull : (unsigned long long)(v[r] & kOrigMask);
    __syncthreads();
  } else if (lds) {
    kd_leaf_order(lkeys, n, npow2, unit, cap, sx, sy, sz, lkb, &s_split, tid, true);
  } else {
    float* kb = d.kd_box + 16 * (kind == 0 ? (size_t)tg0
                                 : kind == 1 ? (size_t)d.kd_pre_off + (size_t)tg0 * 4
                                             : (size_t)d.kd_col_off + (size_t)d.objs[blockIdx.x - d.n_obj - d.n_pre].gbox_begin * (kGateChunk / 64));
    kd_leaf_order(d.sort_keys + key_off, n, npow2, unit, cap, sx, sy, sz, kb, &s_split, tid, false);
  }
  // emit the sorted copies
  if (kind == 2) {
    for (int k = tid; k < n; k += 1024) {
      const int orig = (int)(keys[k] & kOrigMask);
      pts[base + k] = make_float4(sx[orig] - c0, sy[orig] - c1, sz[orig] - c2, 0.f);
      perm[base + k] = orig;
    }
    // the box of every kGateChunk consecutive sorted points (one gate
    // workgroup's share), read back from the unsorted inputs
    const ObjInfo& oi = d.objs[blockIdx.x - d.n_obj - d.n_pre];
    __syncthreads();  // the sorted points are read back below
    // the box of every 64-point leaf (one wavefront per leaf, a lane per
    // point), then of every kGateChunk points (one gate workgroup's share,
    // 32 leaves: one wavefront per chunk, a lane per leaf)
    const int w = tid >> 6, lane = tid & 63, nleaf = (n + 63) >> 6;
    float* leaf = d.col_leaf_box + (size_t)oi.gbox_begin * (kGateChunk / 64) * 8;
    for (int lf = w; lf < oi.gate_chunks * (kGateChunk / 64); lf += 16) {
      float e[6] = {__builtin_inff(), __builtin_inff(), __builtin_inff(),
                    -__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
      const int k = lf * 64 + lane;
      if (lf < nleaf && k < n) {
        const float4 p = pts[base + k];
        e[0] = e[3] = p.x;
        e[1] = e[4] = p.y;
        e[2] = e[5] = p.z;
      }
      for (int off = 32; off >= 1; off >>= 1) {
        for (int a = 0; a < 3; ++a) e[a] = fminf(e[a], __shfl_xor(e[a], off, 64));
        for (int a = 3; a < 6; ++a) e[a] = fmaxf(e[a], __shfl_xor(e[a], off, 64));
      }
      if (lane < 8) leaf[(size_t)lf * 8 + lane] = lane == 3 || lane == 7 ? 0.f : e[lane < 3 ? lane : lane - 1];
    }
    __syncthreads();
    for (int c = w; c < oi.gate_chunks; c += 16) {
      float e[6] = {__builtin_inff(), __builtin_inff(), __builtin_inff(),
                    -__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
      if (lane < kGateChunk / 64) {
        const float* lb = leaf + ((size_t)c * (kGateChunk / 64) + lane) * 8;
        for (int a = 0; a < 3; ++a) {
          e[a] = lb[a];
          e[3 + a] = lb[4 + a];
        }
      }
      for (int off = 32; off >= 1; off >>= 1) {
        for (int a = 0; a < 3; ++a) e[a] = fminf(e[a], __shfl_xor(e[a], off, 64));
        for (int a = 3; a < 6; ++a) e[a] = fmaxf(e[a], __shfl_xor(e[a], off, 64));
      }
      if (lane < 8) d.col_box[(size_t)(oi.gbox_begin + c) * 8 + lane] = lane == 3 || lane == 7 ? 0.f : e[lane < 3 ? lane : lane - 1];
    }
    return;
  }
  float* pf = reinterpret_cast<float*>(prep + (size_t)tg0 * 64);
  for (int k = tid; k < ntg * 64; k += 1024) {
    const size_t g = base + k;
    if (k < n) {
      const int orig = (int)(keys[k] & kOrigMask);
      const float x = sx[orig] - c0, y = sy[orig] - c1, z = sz[orig] - c2;
      prep_store(pf, k, -2.f * x, -2.f * y, -2.f * z, __builtin_fmaf(z, z, __builtin_fmaf(y, y, x * x)));
      pts[g] = make_float4(x, y, z, 0.f);
      perm[g] = orig;
    } else {
      prep_store(pf, k, 0.f, 0.f, 0.f, kDummyNorm);
      pts[g] = make_float4(0.f, 0.f, 0.f, 0.f);
      perm[g] = -1;
    }
  }
  __syncthreads();
  // chunk boxes (an all-padding chunk gets an empty box): every 128 points
  // (2 tile groups), and for an object cloud also every 64 points (the
  // forward NN's pruning chunk is a launch choice)
  auto chunk_boxes = [&](int tgs, float* out) {
    // one wavefront per chunk, a lane per point
    const int pts_per = 64 * tgs, nch = ntg / tgs, w = tid >> 6, lane = tid & 63;
    for (int c = w; c < nch; c += 16) {
      float bb[6] = {__builtin_inff(), __builtin_inff(), __builtin_inff(),
                     -__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
      const int k1 = min(n, (c + 1) * pts_per);
      for (int k = c * pts_per + lane; k < k1; k += 64) {
        const float4 p = pts[base + k];
        bb[0] = fminf(bb[0], p.x); bb[1] = fminf(bb[1], p.y); bb[2] = fminf(bb[2], p.z);
        bb[3] = fmaxf(bb[3], p.x); bb[4] = fmaxf(bb[4], p.y); bb[5] = fmaxf(bb[5], p.z);
      }
      for (int off = 32; off >= 1; off >>= 1) {
        for (int a = 0; a < 3; ++a) bb[a] = fminf(bb[a], __shfl_xor(bb[a], off, 64));
        for (int a = 3; a < 6; ++a) bb[a] = fmaxf(bb[a], __shfl_xor(bb[a], off, 64));
      }
      float* o = out + ((size_t)tg0 / tgs + c) * 8;
      if (lane < 8) o[lane] = lane == 3 || lane == 7 ? 0.f : bb[lane < 3 ? lane : lane - 1];
    }
  };
  chunk_boxes(kChunkTG, box);
  if (kind == 0) {
    chunk_boxes(1, d.obj_box1);
    __syncthreads();  // the chunk boxes are read back below
    // the box of every block of 64 chunks (a k-d subtree): one wavefront per
    // block, a lane per chunk; lets a scan skip a whole block with one test
    auto block_boxes = [&](const float* cb, int nch, float* out) {
      const int w = tid >> 6, lane = tid & 63;
      for (int b = w; b * 64 < nch; b += 16) {
        const int c = b * 64 + lane;
        float v[6] = {__builtin_inff(), __builtin_inff(), __builtin_inff(),
                      -__builtin_inff(), -__builtin_inff(), -__builtin_inff()};
        if (c < nch) {
          for (int a = 0; a < 3; ++a) {
            v[a] = cb[(size_t)c * 8 + a];
            v[3 + a] = cb[(size_t)c * 8 + 4 + a];
          }
        }
        for (int off = 32; off >= 1; off >>= 1) {
          for (int a = 0; a < 3; ++a) v[a] = fminf(v[a], __shfl_xor(v[a], off, 64));
          for (int a = 3; a < 6; ++a) v[a] = fmaxf(v[a], __shfl_xor(v[a], off, 64));
        }
        if (lane < 8) out[(size_t)b * 8 + lane] = lane == 3 || lane == 7 ? 0.f : v[lane < 3 ? lane : lane - 1];
      }
    };
    block_boxes(box + (size_t)tg0 / kChunkTG * 8, ntg / kChunkTG, d.obj_blk + (size_t)tg0 / 4 * 8);
    block_boxes(d.obj_box1 + (size_t)tg0 * 8, ntg, d.obj_blk1 + (size_t)tg0 / 4 * 8);
  }
}

__global__ __launch_bounds__(256) void k_setup_state(Dev d, const float* theta0, const float* prev0,
                                                     const int32_t* conv0) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < d.G) {
    d.h[i] = 0.f;
    for (int a = 0; a < 4; ++a) d.bw_state[4 * i + a] = 0u;
  }
  for (int w = i; w < d.G * 256; w += gridDim.x * 256) d.bw_hist[w] = 0u;
  // the work of every gate workgroup (its group by a search over the groups'
  // first workgroups)
  for (int w = i; w < d.total_gate_wgs; w += gridDim.x * 256) {
    int lo = 0, hi = d.G - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (d.groups[mid].gate_off <= w) lo = mid; else hi = mid - 1;
    }
    const ObjInfo& oi = d.objs[d.groups[lo].obj];
    const int local = w - d.groups[lo].gate_off;
    const int pj = local / oi.gate_chunks, cc = local - pj * oi.gate_chunks;
    d.gate_wg[w] = GateWG{lo, lo * d.K + pj, cc, oi.gbox_begin + cc};
  }
  if (i < 4) d.flags[i] = 0;
  if (d.wave_pairs)
    for (int w = i; w < d.total_waves[0]; w += gridDim.x * 256) d.wave_pairs[w] = 0ull;
  if (i >= d.Ktot) return;
  const int K = d.Ktot;
  for (int a = 0; a < 7; ++a) d.theta[a * K + i] = theta0[a * K + i];
  d.prev_cost[i] = prev0 ? prev0[i] : -1.f;
  d.converged[i] = conv0 ? conv0[i] : 0;
  d.cost[i] = 0.f;
  d.col_cost[i] = 0.f;
  d.ncol[i] = 0;
  for (int a = 0; a < 6; ++a) {
    d.grad[a * K + i] = 0.f;
    d.grad_ct[a * K + i] = 0.f;
    d.grad_col[a * K + i] = 0.f;
    d.phi[a * K + i] = 0.f;
  }
}

// Small host tables travel as kernel arguments (copied at launch), so the
// host copy need not outlive the call.
struct UploadChunk {
  int32_t nwords;
  uint32_t words[960];
};

__global__ void k_upload(uint32_t* dst, UploadChunk c) {
  for (int w = threadIdx.x; w < c.nwords; w += blockDim.x) dst[w] = c.words[w];
}

__global__ void k_zero_words(uint32_t* dst, long long n) {
  for (long long w = (long long)blockIdx.x * 256 + threadIdx.x; w < n; w += (long long)gridDim.x * 256) dst[w] = 0u;
}

// A fill kernel rather than a memset node, so that a captured stream gets
// an ordinary kernel.
void zero_words(void* dst, long long n, hipStream_t s) {
  if (n <= 0) return;
  const long long blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)(blocks < 1024 ? blocks : 1024)), dim3(256), 0, s,
                     static_cast<uint32_t*>(dst), n);
}

void upload_words(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const uint32_t* sw = static_cast<const uint32_t*>(src);
  uint32_t* dw = static_cast<uint32_t*>(dst);
  const size_t nw = bytes / 4;
  for (size_t w0 = 0; w0 < nw; w0 += 960) {
    UploadChunk c;
    c.nwords = (int32_t)((nw - w0) < 960 ? (nw - w0) : 960);
    for (int w = 0; w < c.nwords; ++w) c.words[w] = sw[w0 + w];
    hipLaunchKernelGGL(k_upload, dim3(1), dim3(256), 0, s, dw + w0, c);
  }
}

void launch_setup(const Dev& d, const float* theta0, const float* prev_cost0,
                  const int32_t* converged0, hipStream_t s) {
  hipLaunchKernelGGL(k_setup_obj, dim3(d.n_obj), dim3(256), 0, s, d);
  hipLaunchKernelGGL(k_setup_pre, dim3(d.n_pre), dim3(256), 0, s, d);
  // the cloud sorts (one workgroup per cloud) and, beside them, the SDF tables
  hipLaunchKernelGGL(k_sort_cloud, dim3(2 * d.n_obj + d.n_pre + d.n_pre * d.sdf_blocks), dim3(1024), 0, s, d);
  const int n = d.Ktot > d.G ? d.Ktot : d.G;
  hipLaunchKernelGGL(k_setup_state, dim3((n + 255) / 256), dim3(256), 0, s, d,
                     theta0, prev_cost0, converged0);
}

}  // namespace asicp
