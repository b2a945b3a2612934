// Implicit-differentiation adjoint of libsca (dense A, l1 regulariser).
//
// At a fixed point x* = xh(x*) of the block update, on the support
// S = {j : xh_j != 0, |xh_j| < beta} the stationarity condition reads
// A_S^T (A_S x_S - b) - 2c x_S + lambda s = 0 (s = sign(xh_S)), and x is locally constant
// off S.  Hence dx_S = H_S^{-1} (A_S^T db - s dlambda) with H_S = A_S^T A_S - 2c I, and the
// vector-Jacobian product for an output cotangent xbar is
//     bbar = A_S w,  lambar = -s^T w,  where  H_S w = xbar_S.
// H_S is applied matrix-free (u = A_S p, then A_S^T u - 2c p) inside conjugate gradients
// with FP64 vectors and dot products; several instances run side by side, each with its
// own scalars and convergence flag.  Every sum has a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <vector>

#include "sca_batch_internal.h"

using namespace sca;

namespace {

constexpr int kAMaxGroups = 32;

struct AState {
  RoundState rs;  // compaction results (rs.J_cnt = |S| total), rs.n_all = Ntot
  int tiles;
  int pad[3];
};

// per-instance scalars
enum { SC_RR = 0, SC_RR0, SC_PV, SC_RRN, SC_ALPHA, SC_BETA, SC_LAMB, SC_N };

__device__ __forceinline__ int last_le(const int* __restrict__ off, int K, int v) {
  int lo = 0, hi = K - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= v)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// sgn[j] = sign(xh_j) on the support, 0 elsewhere (wave per column).
template <typename T>
__global__ void __launch_bounds__(256)
k_adj_support(int K, const BInst* __restrict__ inst, const int* __restrict__ col_off,
              long long Ntot, const double* __restrict__ r64, const T* __restrict__ x,
              const double* __restrict__ cn2, double* __restrict__ sgn) {
  const int lane = threadIdx.x & 63;
  const long long nw = (long long)gridDim.x * 4;
  for (long long j = blockIdx.x * 4ll + (threadIdx.x >> 6); j < Ntot; j += nw) {
    const int k = last_le(col_off, K, (int)j);
    const BInst& I = inst[k];
    const T* col = (const T*)I.A + (size_t)(j - I.col_off) * I.lda;
    const double dot = col_dot<T, double, double, 4>(col, r64 + I.row_off, I.m, lane);
    if (lane == 0) {
      const double xj = (double)x[j];
      const double g = dot - 2.0 * I.c * xj;
      const double q = cn2[j] + I.tau;
      const double xh = soft_clip<double>(xj - g / q, I.lam / q, I.beta);
      sgn[j] = (xh != 0.0 && fabs(xh) < I.beta) ? (xh > 0.0 ? 1.0 : -1.0) : 0.0;
    }
  }
}

// Support range of every instance in the ascending support list, fold grouping and tiles.
template <int VN>
__global__ void __launch_bounds__(1024)
k_adj_plan(int K, const BInst* __restrict__ inst, const int* __restrict__ S_idx,
           AState* __restrict__ st, int* __restrict__ S_lo, int* __restrict__ S_n,
           int* __restrict__ Gk, int* __restrict__ ngk, int* __restrict__ nrtk,
           int* __restrict__ tile_off) {
  __shared__ int sh[17];
  const int J = st->rs.J_cnt;
  int run = 0;
  for (int k0 = 0; k0 < K; k0 += 1024) {
    const int k = k0 + threadIdx.x;
    int tiles = 0;
    if (k < K) {
      const int c0 = inst[k].col_off, c1 = c0 + inst[k].n;
      int lo = 0, hi = J;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (S_idx[mid] < c0)
          lo = mid + 1;
        else
          hi = mid;
      }
      const int a = lo;
      hi = J;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (S_idx[mid] < c1)
          lo = mid + 1;
        else
          hi = mid;
      }
      const int cnt = lo - a;
      int G = (cnt + kAMaxGroups - 1) / kAMaxGroups;
      if (G < 16) G = 16;
      const int ng = (cnt + G - 1) / G;
      const int nrt = (inst[k].m + 256 * VN - 1) / (256 * VN);
      tiles = ng * nrt;
      S_lo[k] = a;
      S_n[k] = cnt;
      Gk[k] = G;
      ngk[k] = ng;
      nrtk[k] = nrt;
    }
    int tot;
    const int off = block_exclusive_scan_1024(tiles, sh, &tot);
    if (k < K) tile_off[k] = run + off;
    run += tot;
  }
  if (threadIdx.x == 0) {
    tile_off[K] = run;
    st->tiles = run;
  }
}

// part[g][row] = sum over support entries e of group g of A[row, S_idx[e]] * val[e] (FP64).
template <typename T>
__global__ void __launch_bounds__(256)
k_adj_fold_partial(int K, const BInst* __restrict__ inst, const int* __restrict__ S_idx,
                   const double* __restrict__ val, const int* __restrict__ S_lo,
                   const int* __restrict__ S_n, const int* __restrict__ Gk,
                   const int* __restrict__ nrtk, const int* __restrict__ tile_off,
                   const AState* __restrict__ st, double* __restrict__ part, long long Mtot) {
  typedef typename V16<T>::v VA;
  constexpr int VN = V16<T>::N;
  const int ntiles = st->tiles;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int k = last_le(tile_off, K, tile);
    const BInst& I = inst[k];
    const int lt = tile - tile_off[k];
    const int nrt = nrtk[k];
    const int g = lt / nrt, rt = lt - g * nrt;
    const int e0 = S_lo[k] + g * Gk[k];
    const int e1 = min(e0 + Gk[k], S_lo[k] + S_n[k]);
    const T* A = (const T*)I.A;
    const int m = I.m;
    const int row0 = rt * 256 * VN + threadIdx.x * VN;
    double acc[VN];
#pragma unroll
    for (int v = 0; v < VN; ++v) acc[v] = 0.0;
    if (row0 + VN <= m) {
      for (int e = e0; e < e1; ++e) {
        const double d = val[e];
        const VA a = *reinterpret_cast<const VA*>(A + (size_t)(S_idx[e] - I.col_off) * I.lda + row0);
#pragma unroll
        for (int v = 0; v < VN; ++v) acc[v] += (double)a[v] * d;
      }
    } else if (row0 < m) {
      for (int e = e0; e < e1; ++e) {
        const double d = val[e];
        const T* c = A + (size_t)(S_idx[e] - I.col_off) * I.lda;
        for (int v = 0; v < m - row0; ++v) acc[v] += (double)c[row0 + v] * d;
      }
    }
    if (row0 < m) {
      double* dst = part + (size_t)g * Mtot + I.row_off + row0;
      for (int v = 0; v < VN; ++v)
        if (row0 + v < m) dst[v] = acc[v];
    }
  }
}

// u[i] = sum_{g < ng(instance of row i)} part[g][i]; optionally also out (dtype).
template <typename TO>
__global__ void __launch_bounds__(256)
k_adj_fold_reduce(const double* __restrict__ part, long long Mtot, const int* __restrict__ row_off,
                  int K, const int* __restrict__ ngk, double* __restrict__ u,
                  TO* __restrict__ out) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < Mtot;
       i += (long long)gridDim.x * blockDim.x) {
    const int k = last_le(row_off, K, (int)i);
    const int ng = ngk[k];
    double s = 0.0;
    for (int g = 0; g < ng; ++g) s += part[(size_t)g * Mtot + i];
    if (u) u[i] = s;
    if (out) out[i] = (TO)s;
  }
}

// v[e] = a_{S_idx[e]}^T u - 2c p[e]: the workgroup walk over <= kBC support columns.
template <typename T>
__global__ void __launch_bounds__(256)
k_adj_dots(const BInst* __restrict__ inst, const BItem* __restrict__ items, int nitems,
           const int* __restrict__ S_idx, const double* __restrict__ u,
           const double* __restrict__ p, double* __restrict__ v, const int* __restrict__ done) {
  typedef typename V16<T>::v VA;
  constexpr int VN = V16<T>::N;
  constexpr int ROWS = 256 * VN;
  constexpr int C = kBC;
  __shared__ double red[4][C];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int item = blockIdx.x; item < nitems; item += gridDim.x) {
    const BItem it = items[item];
    if (done[it.inst]) continue;  // uniform across the workgroup
    const BInst& I = inst[it.inst];
    const T* A = (const T*)I.A;
    const double* uu = u + I.row_off;
    const T* col[C];
#pragma unroll
    for (int c = 0; c < C; ++c)
      col[c] = A + (size_t)(S_idx[it.pos + min(c, it.cnt - 1)] - I.col_off) * I.lda;
    double acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.0;
    const int nfull = I.m / ROWS;
    const int row_t = threadIdx.x * VN;
    for (int step = 0; step < nfull; ++step) {
      const int row = step * ROWS + row_t;
      double uv[VN];
#pragma unroll
      for (int e = 0; e < VN; ++e) uv[e] = uu[row + e];
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const VA a = *reinterpret_cast<const VA*>(col[c] + row);
#pragma unroll
        for (int e = 0; e < VN; ++e) acc[c] += (double)a[e] * uv[e];
      }
    }
    {
      const int row = nfull * ROWS + row_t;
      for (int e = 0; e < VN; ++e)
        if (row + e < I.m) {
          const double ur = uu[row + e];
#pragma unroll
          for (int c = 0; c < C; ++c) acc[c] += (double)col[c][row + e] * ur;
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const double w = wave_sum(acc[c]);
      if (lane == 0) red[wave][c] = w;
    }
    __syncthreads();
    if ((int)threadIdx.x < it.cnt) {
      const int c = threadIdx.x, e = it.pos + c;
      v[e] = (((red[0][c] + red[1][c]) + red[2][c]) + red[3][c]) - 2.0 * I.c * p[e];
    }
    __syncthreads();
  }
}

// out[k*SC_N + slot] = sum over entry range of instance k of a[e]*b[e] (fixed order).
__global__ void __launch_bounds__(256)
k_adj_segdot(int K, const int* __restrict__ S_lo, const int* __restrict__ S_n,
             const double* __restrict__ a, const double* __restrict__ b,
             double* __restrict__ sc, int slot, const int* __restrict__ done) {
  __shared__ double res[3];
  for (int k = blockIdx.x; k < K; k += gridDim.x) {
    if (done && done[k]) continue;
    double s = 0.0;
    for (int e = S_lo[k] + threadIdx.x; e < S_lo[k] + S_n[k]; e += 256) s += a[e] * b[e];
    block_sum3_256(s, 0.0, 0.0, res);
    __syncthreads();
    if (threadIdx.x == 0) sc[k * SC_N + slot] = res[0];
    __syncthreads();
  }
}

__global__ void k_adj_init(long long N, const int* __restrict__ S_idx, const AState* __restrict__ st,
                           const void* xbar, int dtype, double* __restrict__ w,
                           double* __restrict__ res, double* __restrict__ p) {
  const int S = st->rs.J_cnt;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < S; e += gridDim.x * blockDim.x) {
    const int j = S_idx[e];
    const double xb = dtype == 0 ? (double)((const float*)xbar)[j] : ((const double*)xbar)[j];
    w[e] = 0.0;
    res[e] = xb;
    p[e] = xb;
  }
  (void)N;
}

__global__ void k_adj_start(int K, double* __restrict__ sc, int* __restrict__ done,
                            int* __restrict__ nonpd) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x) {
    sc[k * SC_N + SC_RR0] = sc[k * SC_N + SC_RR];
    done[k] = sc[k * SC_N + SC_RR] == 0.0;
    nonpd[k] = 0;
  }
}

// alpha = rr/pv; w += alpha p; res -= alpha v.
__global__ void k_adj_update1(int K, const int* __restrict__ S_lo, const AState* __restrict__ st,
                              double* __restrict__ sc, const int* __restrict__ done,
                              int* __restrict__ nonpd, const double* __restrict__ p,
                              const double* __restrict__ v, double* __restrict__ w,
                              double* __restrict__ res) {
  const int S = st->rs.J_cnt;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < S; e += gridDim.x * blockDim.x) {
    const int k = last_le(S_lo, K, e);
    if (done[k]) continue;
    const double pv = sc[k * SC_N + SC_PV];
    if (!(pv > 0.0)) {
      if (e == S_lo[k]) nonpd[k] = 1;
      continue;
    }
    const double alpha = sc[k * SC_N + SC_RR] / pv;
    w[e] += alpha * p[e];
    res[e] -= alpha * v[e];
  }
}

// beta = rr_new/rr; p = res + beta p.
__global__ void k_adj_update2(int K, const int* __restrict__ S_lo, const AState* __restrict__ st,
                              const double* __restrict__ sc, const int* __restrict__ done,
                              const int* __restrict__ nonpd, const double* __restrict__ res,
                              double* __restrict__ p) {
  const int S = st->rs.J_cnt;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < S; e += gridDim.x * blockDim.x) {
    const int k = last_le(S_lo, K, e);
    if (done[k] || nonpd[k]) continue;
    const double beta = sc[k * SC_N + SC_RRN] / sc[k * SC_N + SC_RR];
    p[e] = res[e] + beta * p[e];
  }
}

// rr = rr_new; converged when rr_new <= tol^2 rr0 (or a non-positive curvature was met).
__global__ void k_adj_scalars(int K, double tol2, double* __restrict__ sc, int* __restrict__ done,
                              const int* __restrict__ nonpd, int* __restrict__ iters) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x) {
    if (done[k]) continue;
    iters[k] += 1;
    if (nonpd[k]) {
      done[k] = 1;
      continue;
    }
    sc[k * SC_N + SC_RR] = sc[k * SC_N + SC_RRN];
    if (sc[k * SC_N + SC_RRN] <= tol2 * sc[k * SC_N + SC_RR0]) done[k] = 1;
  }
}

__global__ void k_adj_init_state(AState* st, int Ntot) {
  st->rs.n_all = Ntot;
  st->rs.J_cnt = 0;
  st->tiles = 0;
}

struct AdjWork {
  int K = 0;
  long long Ntot = 0, Mtot = 0;
  AState* st = nullptr;
  double *sgn = nullptr, *S_sgn = nullptr, *w = nullptr, *res = nullptr, *p = nullptr,
         *v = nullptr, *u = nullptr, *part = nullptr, *sc = nullptr;
  int *chunk = nullptr, *S_idx = nullptr, *S_lo = nullptr, *S_n = nullptr, *G = nullptr,
      *ng = nullptr, *nrt = nullptr, *tile_off = nullptr, *done = nullptr, *nonpd = nullptr,
      *iters = nullptr, *col_off = nullptr, *row_off = nullptr;
  BItem* items = nullptr;
  long long items_cap = 0;
  BInst* inst = nullptr;  // owned only for a plain problem
  bool own_inst = false;
  bool fixed = false;     // carved out of the fixed scratch array: never (re)allocated

  void release() {
    void* ptrs[] = {st, sgn, S_sgn, w, res, p, v, u, part, sc, chunk, S_idx, S_lo, S_n, G, ng,
                    nrt, tile_off, done, nonpd, iters, col_off, row_off, items};
    for (void* q : ptrs)
      if (q) (void)hipFree(q);
    if (own_inst && inst) (void)hipFree(inst);
  }
};

sca_status adj_alloc(AdjWork* W, int K, long long Ntot, long long Mtot) {
  W->K = K;
  W->Ntot = Ntot;
  W->Mtot = Mtot;
  sca_status st = SCA_OK;
  const long long nch = (Ntot + kChunk - 1) / kChunk + 1;
#define AALLOC(ptr, bytes) \
  if (st == SCA_OK) st = dev_alloc((void**)&(ptr), (bytes));
  AALLOC(W->st, sizeof(AState));
  AALLOC(W->sgn, sizeof(double) * Ntot);
  AALLOC(W->S_sgn, sizeof(double) * Ntot);
  AALLOC(W->w, sizeof(double) * Ntot);
  AALLOC(W->res, sizeof(double) * Ntot);
  AALLOC(W->p, sizeof(double) * Ntot);
  AALLOC(W->v, sizeof(double) * Ntot);
  AALLOC(W->u, sizeof(double) * Mtot);
  AALLOC(W->part, sizeof(double) * kAMaxGroups * Mtot);
  AALLOC(W->sc, sizeof(double) * SC_N * K);
  AALLOC(W->chunk, sizeof(int) * nch);
  AALLOC(W->S_idx, sizeof(int) * Ntot);
  AALLOC(W->S_lo, sizeof(int) * K);
  AALLOC(W->S_n, sizeof(int) * K);
  AALLOC(W->G, sizeof(int) * K);
  AALLOC(W->ng, sizeof(int) * K);
  AALLOC(W->nrt, sizeof(int) * K);
  AALLOC(W->tile_off, sizeof(int) * (K + 1));
  AALLOC(W->done, sizeof(int) * K);
  AALLOC(W->nonpd, sizeof(int) * K);
  AALLOC(W->iters, sizeof(int) * K);
  AALLOC(W->col_off, sizeof(int) * (K + 1));
  AALLOC(W->row_off, sizeof(int) * (K + 1));
#undef AALLOC
  // rows that no fold tile writes (padding between instances) read as zero
  if (st == SCA_OK && hipMemset(W->part, 0, sizeof(double) * kAMaxGroups * Mtot) != hipSuccess)
    st = set_error(SCA_EHIP, "adjoint workspace clear failed");
  return st;
}

// The whole adjoint for K instances.  r64 must hold A x* - b (FP64) in the r layout.
// Zeroes count ints (a fill kernel rather than a memset node, for callers that capture).
__global__ void __launch_bounds__(256) k_adj_zero_int(int* __restrict__ a, int count) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < count; i += gridDim.x * 256) a[i] = 0;
}

template <typename T>
sca_status adjoint_core(AdjWork* W, int dtype, int ncu, const BInst* d_inst,
                        const std::vector<BInst>& hinst, const double* d_cn2, const double* r64,
                        const T* xstar, const T* xbar, T* bbar, double* lambar_host, double tol,
                        int64_t maxit, hipStream_t s, std::vector<int>* iters_out) {
  const int K = W->K;
  constexpr int VN = V16<T>::N;
  std::vector<int> co(K + 1), ro(K + 1);
  for (int k = 0; k < K; ++k) {
    co[k] = hinst[k].col_off;
    ro[k] = hinst[k].row_off;
  }
  co[K] = (int)W->Ntot;
  ro[K] = (int)W->Mtot;
  if (hipMemcpyAsync(W->col_off, co.data(), sizeof(int) * (K + 1), hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipMemcpyAsync(W->row_off, ro.data(), sizeof(int) * (K + 1), hipMemcpyHostToDevice, s) !=
          hipSuccess)
    return set_error(SCA_EHIP, "adjoint set-up copy failed");
  hipLaunchKernelGGL(k_adj_init_state, dim3(1), dim3(1), 0, s, W->st, (int)W->Ntot);
  // support and its ordered list
  hipLaunchKernelGGL(k_adj_support<T>, dim3(16 * ncu), dim3(256), 0, s, K, d_inst,
                     (const int*)W->col_off, W->Ntot, r64, xstar, d_cn2, W->sgn);
  int* N_ptr = (int*)((char*)W->st + offsetof(RoundState, n_all));
  const int nch = (int)((W->Ntot + kChunk - 1) / kChunk);
  const int cg = std::max(1, std::min(nch, 2 * ncu));
  hipLaunchKernelGGL(k_compact_count<double>, dim3(cg), dim3(1024), 0, s, (const double*)W->sgn,
                     (const int*)N_ptr, W->chunk);
  hipLaunchKernelGGL(k_compact_scatter<double>, dim3(cg), dim3(1024), 0, s,
                     (const double*)W->sgn, (const int*)nullptr, (const int*)N_ptr,
                     (const int*)W->chunk, W->S_idx, W->S_sgn, (RoundState*)W->st, 0);
  hipLaunchKernelGGL(k_adj_plan<VN>, dim3(1), dim3(1024), 0, s, K, d_inst, (const int*)W->S_idx,
                     W->st, W->S_lo, W->S_n, W->G, W->ng, W->nrt, W->tile_off);
  // work items of the dot kernel, built on the host from the per-instance ranges
  std::vector<int> hlo(K), hn(K);
  if (hipMemcpyAsync(hlo.data(), W->S_lo, sizeof(int) * K, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipMemcpyAsync(hn.data(), W->S_n, sizeof(int) * K, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(SCA_EHIP, "adjoint support: %s", hipGetErrorString(hipGetLastError()));
  std::vector<BItem> items;
  for (int k = 0; k < K; ++k)
    for (int e = 0; e < hn[k]; e += kBC) {
      BItem it;
      it.pos = hlo[k] + e;
      it.cnt = std::min(kBC, hn[k] - e);
      it.inst = k;
      items.push_back(it);
    }
  if ((long long)items.size() > W->items_cap) {
    if (W->fixed)
      return set_error(SCA_EINVAL, "adjoint: %zu work items exceed the scratch's %lld",
                       items.size(), W->items_cap);
    if (W->items) (void)hipFree(W->items);
    W->items = nullptr;
    W->items_cap = std::max<long long>(1024, (long long)items.size());
    sca_status st = dev_alloc((void**)&W->items, sizeof(BItem) * W->items_cap);
    if (st != SCA_OK) return st;
  }
  if (!items.empty() &&
      hipMemcpyAsync(W->items, items.data(), sizeof(BItem) * items.size(), hipMemcpyHostToDevice,
                     s) != hipSuccess)
    return set_error(SCA_EHIP, "adjoint items copy failed");
  const int nitems = (int)items.size();
  const int ntot_s = hlo.empty() ? 0 : (hlo[K - 1] + hn[K - 1]);
  const int eg = std::max(1, std::min(4 * ncu, (ntot_s + 255) / 256));
  const int kg = std::max(1, (K + 255) / 256);
  // CG start: w = 0, res = p = xbar_S
  hipLaunchKernelGGL(k_adj_init, dim3(eg), dim3(256), 0, s, W->Ntot, (const int*)W->S_idx,
                     (const AState*)W->st, (const void*)xbar, dtype, W->w, W->res, W->p);
  hipLaunchKernelGGL(k_adj_zero_int, dim3(kg), dim3(256), 0, s, W->iters, K);
  hipLaunchKernelGGL(k_adj_segdot, dim3(std::min(K, 4 * ncu)), dim3(256), 0, s, K,
                     (const int*)W->S_lo, (const int*)W->S_n, (const double*)W->res,
                     (const double*)W->res, W->sc, (int)SC_RR, (const int*)nullptr);
  hipLaunchKernelGGL(k_adj_start, dim3(kg), dim3(256), 0, s, K, W->sc, W->done, W->nonpd);
  const int fg = 8 * ncu;
  const int rg = (int)std::min<long long>((W->Mtot + 255) / 256, 16ll * ncu);
  const double tol2 = tol * tol;
  std::vector<int> hdone(K), hnonpd(K);
  int64_t it = 0;
  bool all_done = false;
  while (it < maxit && !all_done) {
    const int64_t chunk = std::min<int64_t>(10, maxit - it);
    for (int64_t q = 0; q < chunk; ++q) {
      hipLaunchKernelGGL(k_adj_fold_partial<T>, dim3(fg), dim3(256), 0, s, K, d_inst,
                         (const int*)W->S_idx, (const double*)W->p, (const int*)W->S_lo,
                         (const int*)W->S_n, (const int*)W->G, (const int*)W->nrt,
                         (const int*)W->tile_off, (const AState*)W->st, W->part, W->Mtot);
      hipLaunchKernelGGL(k_adj_fold_reduce<double>, dim3(rg), dim3(256), 0, s,
                         (const double*)W->part, W->Mtot, (const int*)W->row_off, K,
                         (const int*)W->ng, W->u, (double*)nullptr);
      hipLaunchKernelGGL(k_adj_dots<T>, dim3(std::max(1, std::min(nitems, 4 * ncu))), dim3(256),
                         0, s, d_inst, (const BItem*)W->items, nitems, (const int*)W->S_idx,
                         (const double*)W->u, (const double*)W->p, W->v, (const int*)W->done);
      hipLaunchKernelGGL(k_adj_segdot, dim3(std::min(K, 4 * ncu)), dim3(256), 0, s, K,
                         (const int*)W->S_lo, (const int*)W->S_n, (const double*)W->p,
                         (const double*)W->v, W->sc, (int)SC_PV, (const int*)W->done);
      hipLaunchKernelGGL(k_adj_update1, dim3(eg), dim3(256), 0, s, K, (const int*)W->S_lo,
                         (const AState*)W->st, W->sc, (const int*)W->done, W->nonpd,
                         (const double*)W->p, (const double*)W->v, W->w, W->res);
      hipLaunchKernelGGL(k_adj_segdot, dim3(std::min(K, 4 * ncu)), dim3(256), 0, s, K,
                         (const int*)W->S_lo, (const int*)W->S_n, (const double*)W->res,
                         (const double*)W->res, W->sc, (int)SC_RRN, (const int*)W->done);
      hipLaunchKernelGGL(k_adj_update2, dim3(eg), dim3(256), 0, s, K, (const int*)W->S_lo,
                         (const AState*)W->st, (const double*)W->sc, (const int*)W->done,
                         (const int*)W->nonpd, (const double*)W->res, W->p);
      hipLaunchKernelGGL(k_adj_scalars, dim3(kg), dim3(256), 0, s, K, tol2, W->sc, W->done,
                         (const int*)W->nonpd, W->iters);
    }
    it += chunk;
    if (hipMemcpyAsync(hdone.data(), W->done, sizeof(int) * K, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return set_error(SCA_EHIP, "adjoint CG: %s", hipGetErrorString(hipGetLastError()));
    all_done = true;
    for (int k = 0; k < K; ++k) all_done = all_done && hdone[k];
  }
  // bbar = A_S w (dtype, r layout); lambar = -s^T w
  hipLaunchKernelGGL(k_adj_fold_partial<T>, dim3(fg), dim3(256), 0, s, K, d_inst,
                     (const int*)W->S_idx, (const double*)W->w, (const int*)W->S_lo,
                     (const int*)W->S_n, (const int*)W->G, (const int*)W->nrt,
                     (const int*)W->tile_off, (const AState*)W->st, W->part, W->Mtot);
  hipLaunchKernelGGL(k_adj_fold_reduce<T>, dim3(rg), dim3(256), 0, s, (const double*)W->part,
                     W->Mtot, (const int*)W->row_off, K, (const int*)W->ng, (double*)nullptr,
                     bbar);
  hipLaunchKernelGGL(k_adj_segdot, dim3(std::min(K, 4 * ncu)), dim3(256), 0, s, K,
                     (const int*)W->S_lo, (const int*)W->S_n, (const double*)W->S_sgn,
                     (const double*)W->w, W->sc, (int)SC_LAMB, (const int*)nullptr);
  std::vector<double> hsc((size_t)SC_N * K);
  std::vector<int> hit(K);
  if (hipMemcpyAsync(hsc.data(), W->sc, sizeof(double) * SC_N * K, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipMemcpyAsync(hnonpd.data(), W->nonpd, sizeof(int) * K, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipMemcpyAsync(hit.data(), W->iters, sizeof(int) * K, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(SCA_EHIP, "adjoint result copy failed");
  for (int k = 0; k < K; ++k) lambar_host[k] = -hsc[(size_t)k * SC_N + SC_LAMB];
  if (iters_out) *iters_out = hit;
  for (int k = 0; k < K; ++k)
    if (hnonpd[k])
      return set_error(SCA_EINVAL, "instance %d: A_S^T A_S - 2c I is not positive definite", k);
  if (!all_done) return set_error(SCA_ENOTCONV, "CG did not reach the tolerance");
  return SCA_OK;
}

}  // namespace

// ------------------------------------------------------------------ plain problem
struct sca_adj_cache {
  AdjWork W;
};

extern "C" sca_status sca_adjoint(sca_problem* p, const sca_opts* o, const void* xstar,
                                  const void* xbar, void* bbar, double* lambar, double cg_tol,
                                  int64_t cg_maxit, void* stream) {
  if (!p) return set_error(SCA_EINVAL, "problem is NULL");
  sca_status st = validate_opts(o);
  if (st != SCA_OK) return st;
  if (!xstar || !xbar || !bbar || !lambar) return set_error(SCA_EINVAL, "NULL argument");
  if (p->sparse) return set_error(SCA_EINVAL, "the adjoint is built for dense problems");
  if (p->reg != 0) return set_error(SCA_EINVAL, "the adjoint is defined for the l1 regulariser");
  if (!(p->cn2_min + o->tau > 0.0)) return set_error(SCA_EINVAL, "q_j = 0 (zero column, tau = 0)");
  if (cg_tol <= 0.0) cg_tol = p->dtype == SCA_F64 ? 1e-12 : 1e-6;
  if (cg_maxit <= 0) cg_maxit = 10000;
  hipStream_t s = (hipStream_t)stream;
  if (!p->adj) {
    p->adj = new (std::nothrow) sca_adj_cache();
    if (!p->adj) return set_error(SCA_ENOMEM, "host allocation failed");
    if ((st = adj_alloc(&p->adj->W, 1, p->n, p->ldp)) != SCA_OK ||
        (st = dev_alloc((void**)&p->adj->W.inst, sizeof(BInst))) != SCA_OK) {
      p->adj->W.release();
      delete p->adj;
      p->adj = nullptr;
      return st;
    }
    p->adj->W.own_inst = true;
  }
  AdjWork* W = &p->adj->W;
  BInst I;
  I.A = p->A;
  I.lda = p->lda;
  I.m = (int)p->m;
  I.n = (int)p->n;
  I.row_off = 0;
  I.col_off = 0;
  I.blk_off = 0;
  I.nblk = (int)p->nblocks;
  I.lam = p->lam;
  I.c = p->c;
  I.beta = p->beta;
  I.tau = o->tau;
  I.F_star = 0;
  I.inst_id = o->instance;
  I.pad = 0;
  std::vector<BInst> hinst(1, I);
  if (hipMemcpyAsync(W->inst, &hinst[0], sizeof(BInst), hipMemcpyHostToDevice, s) != hipSuccess)
    return set_error(SCA_EHIP, "adjoint descriptor copy failed");
  W->Mtot = p->m;  // rows of this problem (the workspace holds ldp >= m)
  residual_any(p, xstar, nullptr, s);  // FP64 residual at x* into p->d_r64
  if (p->dtype == SCA_F32)
    st = adjoint_core<float>(W, 0, p->ncu, W->inst, hinst, p->d_cn2, p->d_r64,
                             (const float*)xstar, (const float*)xbar, (float*)bbar, lambar,
                             cg_tol, cg_maxit, s, nullptr);
  else
    st = adjoint_core<double>(W, 1, p->ncu, W->inst, hinst, p->d_cn2, p->d_r64,
                              (const double*)xstar, (const double*)xbar, (double*)bbar, lambar,
                              cg_tol, cg_maxit, s, nullptr);
  return st;
}

// ------------------------------------------------------------------ no-allocation variant
// sca_adjoint_noalloc keeps its workspace in this fixed device array instead of memory the
// problem allocates on its first adjoint call.  Each GPU holds its own copy, at its own
// address, until the process ends.  In host code the array's name is not a device
// address: the address comes from hipGetSymbolAddress, once per device (scratch_base).
constexpr size_t kAdjScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kAdjScratchBytes];

namespace {

constexpr int kScratchMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_base[kScratchMaxDevices] = {};

// Device address of the current device's scratch array (looked up on its first use).
sca_status scratch_base(unsigned char** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchMaxDevices)
    return set_error(SCA_EHIP, "no usable current device for the adjoint scratch");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_base[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return set_error(SCA_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    }
    g_scratch_base[dev] = (unsigned char*)ptr;
  }
  *out = g_scratch_base[dev];
  return SCA_OK;
}

// Lays the workspace of one instance of n columns and m rows out in the scratch from base
// (256-byte aligned pieces); returns the bytes used.  With base == nullptr only counts.
size_t adj_carve(AdjWork* W, unsigned char* base, long long n, long long m) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> void* {
    off = (off + 255) & ~size_t(255);
    void* q = base ? (void*)(base + off) : nullptr;
    off += std::max<size_t>(bytes, 16);
    return q;
  };
  const long long nch = (n + kChunk - 1) / kChunk + 1;
  const long long nitems = (n + kBC - 1) / kBC + 1;
  W->st = (AState*)take(sizeof(AState));
  W->sgn = (double*)take(sizeof(double) * n);
  W->S_sgn = (double*)take(sizeof(double) * n);
  W->w = (double*)take(sizeof(double) * n);
  W->res = (double*)take(sizeof(double) * n);
  W->p = (double*)take(sizeof(double) * n);
  W->v = (double*)take(sizeof(double) * n);
  W->u = (double*)take(sizeof(double) * m);
  W->part = (double*)take(sizeof(double) * kAMaxGroups * m);
  W->sc = (double*)take(sizeof(double) * SC_N);
  W->chunk = (int*)take(sizeof(int) * nch);
  W->S_idx = (int*)take(sizeof(int) * n);
  W->S_lo = (int*)take(sizeof(int));
  W->S_n = (int*)take(sizeof(int));
  W->G = (int*)take(sizeof(int));
  W->ng = (int*)take(sizeof(int));
  W->nrt = (int*)take(sizeof(int));
  W->tile_off = (int*)take(sizeof(int) * 2);
  W->done = (int*)take(sizeof(int));
  W->nonpd = (int*)take(sizeof(int));
  W->iters = (int*)take(sizeof(int));
  W->col_off = (int*)take(sizeof(int) * 2);
  W->row_off = (int*)take(sizeof(int) * 2);
  W->items = (BItem*)take(sizeof(BItem) * nitems);
  W->inst = (BInst*)take(sizeof(BInst));
  W->items_cap = nitems;
  return off;
}

__global__ void k_adj_zero(double* __restrict__ a, long long count) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x)
    a[i] = 0.0;
}

}  // namespace

extern "C" sca_status sca_adjoint_noalloc(sca_problem* p, const sca_opts* o, const void* xstar,
                                          const void* xbar, void* bbar, double* lambar,
                                          double cg_tol, int64_t cg_maxit, void* stream) {
  if (!p) return set_error(SCA_EINVAL, "problem is NULL");
  sca_status st = validate_opts(o);
  if (st != SCA_OK) return st;
  if (!xstar || !xbar || !bbar || !lambar) return set_error(SCA_EINVAL, "NULL argument");
  if (p->sparse) return set_error(SCA_EINVAL, "the adjoint is built for dense problems");
  if (p->reg != 0) return set_error(SCA_EINVAL, "the adjoint is defined for the l1 regulariser");
  if (!(p->cn2_min + o->tau > 0.0)) return set_error(SCA_EINVAL, "q_j = 0 (zero column, tau = 0)");
  AdjWork W;
  const size_t need = adj_carve(&W, nullptr, p->n, p->m);
  if (need > kAdjScratchBytes)
    return set_error(SCA_EINVAL,
                     "sca_adjoint_noalloc: a problem of %lld rows and %lld columns needs %zu "
                     "bytes of workspace, beyond the fixed %zu (use sca_adjoint)",
                     (long long)p->m, (long long)p->n, need, kAdjScratchBytes);
  if (cg_tol <= 0.0) cg_tol = p->dtype == SCA_F64 ? 1e-12 : 1e-6;
  if (cg_maxit <= 0) cg_maxit = 10000;
  unsigned char* base = nullptr;
  if ((st = scratch_base(&base)) != SCA_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  adj_carve(&W, base, p->n, p->m);
  W.K = 1;
  W.Ntot = p->n;
  W.Mtot = p->m;
  W.fixed = true;
  // the array keeps the previous call's contents: the fold partials must start at zero
  // (rows no fold tile writes are read as zero); everything else is written before it is read
  const long long npart = (long long)kAMaxGroups * p->m;
  hipLaunchKernelGGL(k_adj_zero, dim3((unsigned)std::min<long long>((npart + 255) / 256, 1024)),
                     dim3(256), 0, s, W.part, npart);
  BInst I;
  I.A = p->A;
  I.lda = p->lda;
  I.m = (int)p->m;
  I.n = (int)p->n;
  I.row_off = 0;
  I.col_off = 0;
  I.blk_off = 0;
  I.nblk = (int)p->nblocks;
  I.lam = p->lam;
  I.c = p->c;
  I.beta = p->beta;
  I.tau = o->tau;
  I.F_star = 0;
  I.inst_id = o->instance;
  I.pad = 0;
  std::vector<BInst> hinst(1, I);
  if (hipMemcpyAsync(W.inst, &hinst[0], sizeof(BInst), hipMemcpyHostToDevice, s) != hipSuccess)
    return set_error(SCA_EHIP, "adjoint descriptor copy failed");
  residual_any(p, xstar, nullptr, s);  // FP64 residual at x* into the problem's workspace
  if (p->dtype == SCA_F32)
    return adjoint_core<float>(&W, 0, p->ncu, W.inst, hinst, p->d_cn2, p->d_r64,
                               (const float*)xstar, (const float*)xbar, (float*)bbar, lambar,
                               cg_tol, cg_maxit, s, nullptr);
  return adjoint_core<double>(&W, 1, p->ncu, W.inst, hinst, p->d_cn2, p->d_r64,
                              (const double*)xstar, (const double*)xbar, (double*)bbar, lambar,
                              cg_tol, cg_maxit, s, nullptr);
}

void sca::adjoint_release(sca_adj_cache* c) {
  if (!c) return;
  c->W.release();
  delete c;
}

// ------------------------------------------------------------------ batch
extern "C" sca_status sca_batch_adjoint(sca_batch* B, const sca_opts* o, const void* xstar_all,
                                        const void* xbar_all, void* bbar_all,
                                        double* lambar_host, double cg_tol, int64_t cg_maxit,
                                        void* stream) {
  if (!B) return set_error(SCA_EINVAL, "batch is NULL");
  sca_status st = validate_opts(o);
  if (st != SCA_OK) return st;
  if (!xstar_all || !xbar_all || !bbar_all || !lambar_host)
    return set_error(SCA_EINVAL, "NULL argument");
  if (B->reg != 0) return set_error(SCA_EINVAL, "the adjoint is defined for the l1 regulariser");
  if (cg_tol <= 0.0) cg_tol = B->dtype == SCA_F64 ? 1e-12 : 1e-6;
  if (cg_maxit <= 0) cg_maxit = 10000;
  hipStream_t s = (hipStream_t)stream;
  if (!B->adj) {
    B->adj = new (std::nothrow) sca_adj_cache();
    if (!B->adj) return set_error(SCA_ENOMEM, "host allocation failed");
    if ((st = adj_alloc(&B->adj->W, B->K, B->Ntot, B->Mtot)) != SCA_OK) {
      B->adj->W.release();
      delete B->adj;
      B->adj = nullptr;
      return st;
    }
  }
  batch_fresh_residual(B, xstar_all, s);
  if (B->dtype == SCA_F32)
    st = adjoint_core<float>(&B->adj->W, 0, B->ncu, B->d_inst, B->hinst, B->d_cn2, B->d_r64,
                             (const float*)xstar_all, (const float*)xbar_all, (float*)bbar_all,
                             lambar_host, cg_tol, cg_maxit, s, nullptr);
  else
    st = adjoint_core<double>(&B->adj->W, 1, B->ncu, B->d_inst, B->hinst, B->d_cn2, B->d_r64,
                              (const double*)xstar_all, (const double*)xbar_all,
                              (double*)bbar_all, lambar_host, cg_tol, cg_maxit, s, nullptr);
  return st;
}
