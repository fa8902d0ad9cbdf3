// k_nn_forward.hip -- transform, forward nearest neighbour and contact-loss
// partial sums (Algorithm 1: transform the source cloud, pair it with the
// object cloud by eq. (1), accumulate the terms of eqs. (14), (16), (17)).
//
// One wavefront = one particle x 16*Q contact points (consecutive in the
// k-d ordered contact cloud, so spatially close), matched against the object
// cloud of its group with the MFMA core.  By default object chunks that
// provably cannot hold any of the wave's nearest neighbours are skipped.  Q
// (1, 2 or 4 blocks of 16 queries) and the chunk size CH (1 or 2 tile groups
// of 64 points) are launch choices: every combination returns the same
// nearest neighbours and partial sums.
// Partial sums per wavefront: [sum |e|^2, sum e (3), sum
// s' x e (3), points], e = s' - r_nn, s' relative to the object's centroid (the
// finaliser turns the moment into sum (R s) x e = sum s' x e - (t - CoM) x
// sum e, so no pose value stays live through the scan).
#include "nn_core.h"

namespace asicp {

// Hardware places workgroup b on XCD b % 8.  MAP 0 deals units of `unit`
// consecutive logical workgroups (one particle's forward work) round-robin
// over the XCDs: each particle's workgroups run in one L2 and every XCD gets
// a mix of near and far particles (workgroups past the last whole round of 8
// units keep their index, so the map is a bijection for any count).  MAP 1
// keeps the dispatch order (a particle's consecutive workgroups on different
// XCDs).  Neither changes any result.
template <int MAP>
__device__ __forceinline__ int xcd_logical(int b, int nwg, int unit) {
  if (MAP == 1) return b;
  const int full = nwg / (8 * unit) * (8 * unit);
  if (b >= full) return b;
  const int s = b >> 3;
  return ((s / unit) * 8 + (b & 7)) * unit + s % unit;
}

#if ASICP_NN_WPE > 0
#define NN_OCCUPANCY __attribute__((amdgpu_waves_per_eu(ASICP_NN_WPE)))
#else
#define NN_OCCUPANCY
#endif

template <int Q, int CH, bool PRUNE, int MAP, bool FINE>
__device__ __forceinline__ void nn_forward_body(const Dev& d) {
  constexpr int QI = Q == 1 ? 0 : (Q == 2 ? 1 : 2);
  static_assert(q_blocks(QI) == Q, "1, 2 or 4 query blocks per wave");
  const int total_waves = d.total_waves[QI];
  const int nwg = (total_waves + 3) >> 2;
  const int unit = max(1, (d.pres[0].waves[QI] + 3) >> 2);  // workgroups per particle (first preshape)
  const int logical = xcd_logical<MAP>(blockIdx.x, nwg, unit);
  if (logical >= nwg) return;
  const int wave = __builtin_amdgcn_readfirstlane(logical * 4 + (int)(threadIdx.x >> 6));
  if (wave >= total_waves) return;
  const int lane = lane_id();

  int lo = 0, hi = d.G - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d.groups[mid].wave_off[QI] <= wave) lo = mid; else hi = mid - 1;
  }
  const GroupInfo gi = d.groups[lo];
  const PreInfo& pi = d.pres[gi.pre];
  const ObjInfo& oi = d.objs[gi.obj];
  const int local = wave - gi.wave_off[QI];
  const int pw = pi.waves[QI];
  const int pj = local / pw, chunk = local - pj * pw;
  const int i = lo * d.K + pj;

  // the pose relative to the object's centroid: the object cloud is stored
  // relative to it, so every value below is centroid-relative
  float t[3], qv[4], R[9];
  load_pose(d.theta, d.Ktot, i, t, qv);
  quat_to_rot(qv[0], qv[1], qv[2], qv[3], R);
  const float* com = d.obj_com + 4 * gi.obj;
  for (int a = 0; a < 3; ++a) t[a] = uniform_f(t[a] - com[a]);

  constexpr int QPW = 16 * Q;
  const float4* spts = d.pre_pts + (size_t)pi.prep_tg_begin * 64;  // k-d ordered contact cloud
  const int comp = lane >> 4, j = lane & 15;
  // bq: the B operand (row a = component a of the block's 16 queries, row 3
  // = 1); own: the lane's own query, number j of block min(comp, Q - 1)
  const int qo = min(comp, Q - 1);
  float bq[Q], own[3];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    int n = chunk * QPW + q * 16 + j;
    if (n >= pi.n) n = chunk * QPW;  // padding queries repeat the wave's first point
    const float4 s = spts[n];
    const float px = R[0] * s.x + R[1] * s.y + R[2] * s.z + t[0];
    const float py = R[3] * s.x + R[4] * s.y + R[5] * s.z + t[1];
    const float pz = R[6] * s.x + R[7] * s.y + R[8] * s.z + t[2];
    bq[q] = comp == 0 ? px : comp == 1 ? py : comp == 2 ? pz : 1.0f;
    if (q == 0 || q == qo) {
      own[0] = px;
      own[1] = py;
      own[2] = pz;
    }
  }
  int idx[Q];
  const float4* prep = (d.minibatch ? d.obj_prep_mb : d.obj_prep) + (size_t)oi.prep_tg_begin * 64;
  long long pairs;
  if (PRUNE) {
    int vq[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) vq[q] = max(0, min(16, pi.n - (chunk * QPW + q * 16)));
    const float* box = CH == 1 ? d.obj_box1 + (size_t)oi.prep_tg_begin * 8
                               : d.obj_box + (size_t)oi.prep_tg_begin / 2 * 8;
    const float* blk = (CH == 1 ? d.obj_blk1 : d.obj_blk) + (size_t)oi.prep_tg_begin / 4 * 8;
    pairs = nn_scan_pruned<Q, true, FINE, CH>(prep, oi.ntg, oi.m, box, blk, bq, nullptr, own, vq, com[3], idx,
                                              d.flags + 1);
  } else {
    nn_scan<Q, CH>(prep, oi.ntg, bq, nullptr, idx, d.flags + 1);
    pairs = (long long)oi.m * min(QPW, pi.n - chunk * QPW);
  }

  // lane l < 16*Q now owns sorted contact point chunk*16Q + l (block l/16, query l%16)
  int my = idx[0];
#pragma unroll
  for (int q = 1; q < Q; ++q)
    if (comp == q) my = idx[q];
  const int n = chunk * QPW + lane;
  float e2 = 0.f, ex = 0.f, ey = 0.f, ez = 0.f, mx = 0.f, my_ = 0.f, mz = 0.f, cnt = 0.f;
  if (lane < QPW && n < pi.n) {
    if (my >= oi.m) {
      atomicOr(d.flags + 1, 2);
      my = oi.m - 1;
    }
    // the lane's transformed contact point s' is its own query (block comp)
    const float px = own[0], py = own[1], pz = own[2];
    const float4 r = d.obj_pts[(size_t)oi.prep_tg_begin * 64 + my];
    ex = px - r.x;
    ey = py - r.y;
    ez = pz - r.z;
    e2 = ex * ex + ey * ey + ez * ez;
    mx = py * ez - pz * ey;
    my_ = pz * ex - px * ez;
    mz = px * ey - py * ex;
    cnt = 1.f;
    if (d.dbg_nn) {
      const int n_orig = d.pre_perm[(size_t)pi.prep_tg_begin * 64 + n];
      d.dbg_nn[(size_t)i * d.n_max + n_orig] = d.obj_perm[(size_t)oi.prep_tg_begin * 64 + my];
    }
  }
  // one record per wave: each block of 16 contact points (a row of lanes) is
  // summed by a fixed tree, then blocks are added in pairs and pairs of
  // pairs, the same partial tree the finaliser completes for smaller waves,
  // so every launch choice gives the same totals
  const float sums[8] = {e2, ex, ey, ez, mx, my_, mz, cnt};
  float tot = row_sum8(sums);  // lane 4m + j of row r: total of sums[2m + j] over block r
  if (Q >= 2) {
    const RowPair a = swap16(tot);
    tot = a.even + a.odd;
  }
  if (Q == 4) {
    const RowPair b = swap32(tot);
    tot = b.even + b.odd;
  }
  if (lane < 16 && (lane & 2) == 0)
    d.nn_part[((size_t)i * d.max_waves_pp + chunk) * kPartStride + ((lane >> 2) << 1 | (lane & 1))] = tot;
  // the wave's own slot: launches are ordered on the stream, so a plain
  // read-modify-write accumulates over them without contention
  if (lane == 0 && d.wave_pairs) d.wave_pairs[wave] += (unsigned long long)pairs;
}

// The pruned scan keeps fewer registers live per wavefront and gains from
// more wavefronts per SIMD to hide its per-chunk loads.  The full scan folds
// one tile group's MFMA results at a time, which fits 3 wavefronts per SIMD
// at 4 query blocks (168 registers; 4 would spill heavily); it visits every
// chunk in index order, so its chunk is always 2 tile groups.
template <int Q, int CH, int MAP, bool FINE>
__global__ __launch_bounds__(256) NN_OCCUPANCY void k_nn_forward(Dev d) {
  nn_forward_body<Q, CH, true, MAP, FINE>(d);
}
template <int Q, int MAP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_nn_forward_full(Dev d) {
  nn_forward_body<Q, 2, false, MAP, false>(d);
}

template <int Q, int CH>
static void launch_pruned(const Dev& d, dim3 g, dim3 b, hipStream_t s) {
  if (d.xcd_map) {
    if (d.fine) hipLaunchKernelGGL((k_nn_forward<Q, CH, 1, true>), g, b, 0, s, d);
    else hipLaunchKernelGGL((k_nn_forward<Q, CH, 1, false>), g, b, 0, s, d);
  } else {
    if (d.fine) hipLaunchKernelGGL((k_nn_forward<Q, CH, 0, true>), g, b, 0, s, d);
    else hipLaunchKernelGGL((k_nn_forward<Q, CH, 0, false>), g, b, 0, s, d);
  }
}

template <int Q>
static void launch_shape(const Dev& d, dim3 g, dim3 b, hipStream_t s) {
  if (!d.prune) {
    if (d.xcd_map) hipLaunchKernelGGL((k_nn_forward_full<Q, 1>), g, b, 0, s, d);
    else hipLaunchKernelGGL((k_nn_forward_full<Q, 0>), g, b, 0, s, d);
  } else if (d.nn_ch == 1) {
    launch_pruned<Q, 1>(d, g, b, s);
  } else {
    launch_pruned<Q, 2>(d, g, b, s);
  }
}

void launch_nn_forward(const Dev& d, hipStream_t s) {
  const int nwg = (d.total_waves[d.nn_qi] + 3) / 4;
  const int grid = ((nwg + 7) / 8) * 8;
  const dim3 g(grid), b(256);
  if (d.nn_qi == 0) launch_shape<1>(d, g, b, s);
  else if (d.nn_qi == 1) launch_shape<2>(d, g, b, s);
  else launch_shape<4>(d, g, b, s);
}

}  // namespace asicp
