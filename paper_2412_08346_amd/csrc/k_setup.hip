// k_setup.hip -- per-object and per-preshape set-up (Algorithm 1
// preprocessing): centre of mass of each object cloud (its centroid), tool
// centre point of each contact cloud (its centroid, Sec. IV-B), the
// Gauss-Newton diagonal preconditioner of eq. (3), MFMA-ready augmented copies
// of the clouds, and the initial particle state.  Sums run in FP64 over a
// fixed order (strided per thread, then a fixed tree).
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

// one workgroup per object
__global__ __launch_bounds__(256) void k_setup_obj(Dev d) {
  __shared__ double sh[256][4];
  const int o = blockIdx.x, tid = threadIdx.x;
  const ObjInfo oi = d.objs[o];
  double v[4] = {0, 0, 0, 0};
  for (int m = tid; m < oi.m; m += 256) {
    v[0] += d.rx[oi.r_begin + m];
    v[1] += d.ry[oi.r_begin + m];
    v[2] += d.rz[oi.r_begin + m];
  }
  block_sum4(v, sh);
  if (tid == 0) {
    for (int a = 0; a < 3; ++a) d.obj_com[4 * o + a] = (float)(v[a] / (double)oi.m);
    d.obj_com[4 * o + 3] = 0.f;
  }
  float* prep = reinterpret_cast<float*>(d.obj_prep + (size_t)oi.prep_tg_begin * 64);
  for (int m = tid; m < oi.ntg * 64; m += 256) {
    if (m < oi.m) {
      const float x = d.rx[oi.r_begin + m], y = d.ry[oi.r_begin + m], z = d.rz[oi.r_begin + m];
      prep_store(prep, m, -2.f * x, -2.f * y, -2.f * z, __builtin_fmaf(z, z, __builtin_fmaf(y, y, x * x)));
    } else {
      prep_store(prep, m, 0.f, 0.f, 0.f, kDummyNorm);
    }
  }
}

// one workgroup per preshape
__global__ __launch_bounds__(256) void k_setup_pre(Dev d) {
  __shared__ double sh[256][4];
  const int p = blockIdx.x, tid = threadIdx.x;
  const PreInfo pi = d.pres[p];
  double v[4] = {0, 0, 0, 0};
  for (int n = tid; n < pi.n; n += 256) {
    const double x = d.sx[pi.s_begin + n], y = d.sy[pi.s_begin + n], z = d.sz[pi.s_begin + n];
    v[0] += x; v[1] += y; v[2] += z;
    v[3] += x * x + y * y + z * z;
  }
  block_sum4(v, sh);
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
    pc[4] = (float)at; pc[5] = (float)aw; pc[6] = 0.f; pc[7] = 0.f;
  }
  float* prep = reinterpret_cast<float*>(d.pre_prep + (size_t)pi.prep_tg_begin * 64);
  for (int n = tid; n < pi.ntg * 64; n += 256) {
    if (n < pi.n) {
      const float x = d.sx[pi.s_begin + n], y = d.sy[pi.s_begin + n], z = d.sz[pi.s_begin + n];
      prep_store(prep, n, -2.f * x, -2.f * y, -2.f * z, __builtin_fmaf(z, z, __builtin_fmaf(y, y, x * x)));
    } else {
      prep_store(prep, n, 0.f, 0.f, 0.f, kDummyNorm);
    }
  }
}

__global__ __launch_bounds__(256) void k_setup_state(Dev d, const float* theta0, const float* prev0,
                                                     const int32_t* conv0) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < d.G) d.h[i] = 0.f;
  if (i < 4) d.flags[i] = 0;
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
  const int n = d.Ktot > d.G ? d.Ktot : d.G;
  hipLaunchKernelGGL(k_setup_state, dim3((n + 255) / 256), dim3(256), 0, s, d,
                     theta0, prev_cost0, converged0);
}

}  // namespace asicp
