// Batched engine of libsca: many dense instances of uneven size run as one block-diagonal
// problem.  A device descriptor table holds each instance's A (borrowed), sizes, offsets
// into the concatenated x / r / b, lambda, c, beta, tau, F* and its Philox instance word.
// Per round the drawn blocks of every active instance, the gradient work items (<= C
// columns of one block), the moved-coordinate list and the fold tiles are all built on the
// device; convergence flags are updated on the device, so a graph of E rounds plus a
// check is replayed without host decisions in between.  Instance k follows exactly the
// trajectory of the plain path run with instance word k.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <new>
#include <vector>

#include "sca_batch_internal.h"

using namespace sca;

namespace {


__device__ __forceinline__ int upper_idx(const int* __restrict__ off, int K, int v) {
  // largest k in [0, K) with off[k] <= v (off ascending, off[0] = 0)
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

// ------------------------------------------------------------------ S.1 over all instances
__global__ void __launch_bounds__(1024)
k_bsel_count(int Btot, const int* __restrict__ blk_inst, const int* __restrict__ blk_len,
             const BInst* __restrict__ inst, const int* __restrict__ active, uint64_t seed,
             uint64_t T, const BState* __restrict__ st, int* __restrict__ blk_cols,
             int* __restrict__ chunk_cols, int* __restrict__ chunk_items,
             long long* __restrict__ inst_upd) {
  __shared__ int sh[2][16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long k = st->rs.k;
  for (int c = blockIdx.x; c * kChunk < Btot; c += gridDim.x) {
    const int b = c * kChunk + threadIdx.x;
    int cols = 0, items = 0;
    if (b < Btot) {
      const int q = blk_inst[b];
      if (active[q] &&
          block_drawn((uint32_t)(b - inst[q].blk_off), (uint64_t)k, inst[q].inst_id, seed, T)) {
        cols = blk_len[b];
        items = (cols + kBC - 1) / kBC;
        atomicAdd((unsigned long long*)&inst_upd[q], (unsigned long long)cols);
      }
      blk_cols[b] = cols;
    }
    const int wc = wave_sum(cols), wi = wave_sum(items);
    if (lane == 0) {
      sh[0][wave] = wc;
      sh[1][wave] = wi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int a = 0, i = 0;
      for (int w = 0; w < 16; ++w) {
        a += sh[0][w];
        i += sh[1][w];
      }
      chunk_cols[c] = a;
      chunk_items[c] = i;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(1024)
k_bsel_scatter(int Btot, const int* __restrict__ blk_inst, const int* __restrict__ blk_col0,
               const int* __restrict__ blk_cols, const int* __restrict__ chunk_cols,
               const int* __restrict__ chunk_items, BState* __restrict__ st,
               int* __restrict__ sel_cols, BItem* __restrict__ items) {
  __shared__ int sh[17];
  __shared__ int s_base[2];
  const int nch = (Btot + kChunk - 1) / kChunk;
  for (int c = blockIdx.x; c < nch; c += gridDim.x) {
    int pc = 0, pi = 0;
    for (int q = threadIdx.x; q < c; q += 1024) {
      pc += chunk_cols[q];
      pi += chunk_items[q];
    }
    int tc, ti;
    (void)block_exclusive_scan_1024(pc, sh, &tc);
    (void)block_exclusive_scan_1024(pi, sh, &ti);
    if (threadIdx.x == 0) {
      s_base[0] = tc;
      s_base[1] = ti;
    }
    __syncthreads();
    const int b = c * kChunk + threadIdx.x;
    const int cols = b < Btot ? blk_cols[b] : 0;
    const int nit = (cols + kBC - 1) / kBC;
    int totc, toti;
    const int oc = s_base[0] + block_exclusive_scan_1024(cols, sh, &totc);
    const int oi = s_base[1] + block_exclusive_scan_1024(nit, sh, &toti);
    if (cols) {
      const int c0 = blk_col0[b], q = blk_inst[b];
      for (int u = 0; u < cols; ++u) sel_cols[oc + u] = c0 + u;
      for (int u = 0; u < nit; ++u) {
        BItem it;
        it.pos = oc + u * kBC;
        it.cnt = min(kBC, cols - u * kBC);
        it.inst = q;
        items[oi + u] = it;
      }
    }
    if (c == nch - 1 && threadIdx.x == 0) {
      st->rs.S_cnt = s_base[0] + totc;
      st->items = s_base[1] + toti;
    }
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (Btot == 0) {
      st->rs.S_cnt = 0;
      st->items = 0;
    }
    st->rs.work_ctr = 0;
    st->rs.k += 1;
    const double g = st->rs.gamma_next;
    st->rs.gamma_cur = g;
    st->rs.gamma_next = g * (1.0 - st->rs.gamma_mu * g);
  }
}

// ------------------------------------------------------------------ S.2 + S.4
// The workgroup walk of the plain path, one work item (<= kBC columns of one block) at a time.
template <typename T, int U>
__global__ void __launch_bounds__(256)
k_bgrad(const BInst* __restrict__ inst, const BItem* __restrict__ items,
        const int* __restrict__ sel_cols, const T* __restrict__ r_all, T* __restrict__ x_all,
        const double* __restrict__ cn2, BState* __restrict__ st, T* __restrict__ dx_sel,
        BRParams bp0) {
  typedef typename V16<T>::v VA;
  constexpr int VN = V16<T>::N;
  constexpr int ROWS = 256 * VN;
  constexpr int C = kBC;
  __shared__ T red[4][C];
  __shared__ int s_item;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nitems = st->items;
  const T gamma = (T)st->rs.gamma_cur;
  const int GR = max(1, nitems / (int)(8 * gridDim.x));  // items taken per counter update
  int item = 0, left = 0;
  for (;;) {
    if (left == 0) {
      if (threadIdx.x == 0) s_item = atomicAdd(&st->rs.work_ctr, GR);
      __syncthreads();
      item = s_item;
      left = GR;
      __syncthreads();
    } else {
      ++item;
    }
    --left;
    if (item >= nitems) break;
    const BItem it = items[item];
    const BInst& I = inst[it.inst];
    const T* A = (const T*)I.A;
    const int m = I.m;
    const T* r = r_all + I.row_off;
    const T* col[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const int t = it.pos + min(c, it.cnt - 1);
      col[c] = A + (size_t)(sel_cols[t] - I.col_off) * I.lda;
    }
    T acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = (T)0;
    const int nfull = m / ROWS;
    const int row_t = threadIdx.x * VN;
    int step = 0;
    for (; step + U <= nfull; step += U) {
      VA a[U][C], rv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int row = (step + u) * ROWS + row_t;
        rv[u] = *reinterpret_cast<const VA*>(r + row);
#pragma unroll
        for (int c = 0; c < C; ++c)
          a[u][c] = __builtin_nontemporal_load(reinterpret_cast<const VA*>(col[c] + row));
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < C; ++c)
#pragma unroll
          for (int e = 0; e < VN; ++e) acc[c] += a[u][c][e] * rv[u][e];
    }
    for (; step < nfull; ++step) {
      const int row = step * ROWS + row_t;
      const VA rv = *reinterpret_cast<const VA*>(r + row);
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const VA a = __builtin_nontemporal_load(reinterpret_cast<const VA*>(col[c] + row));
#pragma unroll
        for (int e = 0; e < VN; ++e) acc[c] += a[e] * rv[e];
      }
    }
    {
      const int row = nfull * ROWS + row_t;
      for (int e = 0; e < VN; ++e) {
        if (row + e < m) {
          const T rr = r[row + e];
#pragma unroll
          for (int c = 0; c < C; ++c) acc[c] += col[c][row + e] * rr;
        }
      }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
      const T v = wave_sum(acc[c]);
      if (lane == 0) red[wave][c] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < it.cnt) {
      const int c = threadIdx.x;
      const int t = it.pos + c;
      const int j = sel_cols[t];
      BRParams bp = bp0;
      bp.tau = I.tau;
      bp.lam = I.lam;
      bp.lam_eta = I.lam * bp0.eta;
      bp.c2 = 2.0 * I.c;
      bp.beta = I.beta;
      const T dot = ((red[0][c] + red[1][c]) + red[2][c]) + red[3][c];
      const T xj = x_all[j];
      T g = dot - (T)bp.c2 * xj;
      if (bp.reg) g -= (T)bp.lam * dh_minus<T>(xj, bp);
      const T q = (T)(cn2[j] + bp.tau);
      const T xh = soft_clip<T>(xj - g / q, (T)bp.lam_eta / q, (T)bp.beta);
      const T d = gamma * (xh - xj);
      x_all[j] = xj + d;
      dx_sel[t] = d;
    }
  }
}

// ------------------------------------------------------------------ fold plan / tiles
// One workgroup: per instance, the range of the listed (ascending global) columns that
// belong to it, its column grouping and its tile count; tile offsets by a block scan.
template <int VN>
__global__ void __launch_bounds__(1024)
k_bfold_plan(int K, const BInst* __restrict__ inst, const int* __restrict__ J_idx,
             BState* __restrict__ st, int* __restrict__ J_lo, int* __restrict__ Jn,
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
      int lo = 0, hi = J;  // first listed entry >= c0
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (J_idx[mid] < c0)
          lo = mid + 1;
        else
          hi = mid;
      }
      const int a = lo;
      hi = J;  // first listed entry >= c1
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (J_idx[mid] < c1)
          lo = mid + 1;
        else
          hi = mid;
      }
      const int cnt = lo - a;
      int G = (cnt + kBMaxGroups - 1) / kBMaxGroups;
      if (G < 16) G = 16;
      const int ng = (cnt + G - 1) / G;
      const int nrt = (inst[k].m + 256 * VN - 1) / (256 * VN);
      tiles = ng * nrt;
      J_lo[k] = a;
      Jn[k] = cnt;
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

template <typename T, typename Acc>
__global__ void __launch_bounds__(256)
k_bfold_partial(int K, const BInst* __restrict__ inst, const int* __restrict__ J_idx,
                const T* __restrict__ J_val, const int* __restrict__ J_lo,
                const int* __restrict__ Jn, const int* __restrict__ Gk,
                const int* __restrict__ ngk, const int* __restrict__ nrtk,
                const int* __restrict__ tile_off, const BState* __restrict__ st,
                Acc* __restrict__ part, long long Mtot) {
  typedef typename V16<T>::v VA;
  constexpr int VN = V16<T>::N;
  const int ntiles = st->tiles;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int k = upper_idx(tile_off, K, tile);
    const BInst& I = inst[k];
    const int lt = tile - tile_off[k];
    const int nrt = nrtk[k];
    const int g = lt / nrt, rt = lt - g * nrt;
    const int G = Gk[k];
    const int e0 = J_lo[k] + g * G;
    const int e1 = min(e0 + G, J_lo[k] + Jn[k]);
    const T* A = (const T*)I.A;
    const int m = I.m;
    const int row0 = rt * 256 * VN + threadIdx.x * VN;
    Acc acc[VN];
#pragma unroll
    for (int v = 0; v < VN; ++v) acc[v] = (Acc)0;
    if (row0 + VN <= m) {
      int e = e0;
      for (; e + 4 <= e1; e += 4) {
        VA a[4];
        Acc d[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = J_idx[e + u] - I.col_off;
          d[u] = (Acc)J_val[e + u];
          a[u] = __builtin_nontemporal_load(
              reinterpret_cast<const VA*>(A + (size_t)j * I.lda + row0));
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < VN; ++v) acc[v] += (Acc)a[u][v] * d[u];
      }
      for (; e < e1; ++e) {
        const int j = J_idx[e] - I.col_off;
        const Acc d = (Acc)J_val[e];
        const VA a = __builtin_nontemporal_load(
            reinterpret_cast<const VA*>(A + (size_t)j * I.lda + row0));
#pragma unroll
        for (int v = 0; v < VN; ++v) acc[v] += (Acc)a[v] * d;
      }
    } else if (row0 < m) {
      for (int e = e0; e < e1; ++e) {
        const int j = J_idx[e] - I.col_off;
        const Acc d = (Acc)J_val[e];
        for (int v = 0; v < m - row0; ++v) acc[v] += (Acc)A[(size_t)j * I.lda + row0 + v] * d;
      }
    }
    if (row0 < m) {
      Acc* dst = part + (size_t)g * Mtot + I.row_off + row0;
      for (int v = 0; v < VN; ++v)
        if (row0 + v < m) dst[v] = acc[v];
    }
  }
}

template <typename TB, typename Acc, typename TO>
__global__ void __launch_bounds__(256)
k_bfold_reduce(const TB* __restrict__ base, double base_scale, const Acc* __restrict__ part,
               long long Mtot, const int* __restrict__ row_inst, const int* __restrict__ ngk,
               TO* __restrict__ out, double* __restrict__ out64) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < Mtot;
       i += (long long)gridDim.x * blockDim.x) {
    const int ng = ngk[row_inst[i]];
    Acc s = (Acc)(base_scale * (double)base[i]);
    for (int g = 0; g < ng; ++g) s += part[(size_t)g * Mtot + i];
    if (out) out[i] = (TO)s;
    if (out64) out64[i] = (double)s;
  }
}

// ------------------------------------------------------------------ checks
// One workgroup per instance: F_k from the FP64 residual, then the stopping test.
template <typename T>
__global__ void __launch_bounds__(256)
k_bobj_check(int K, const BInst* __restrict__ inst, const double* __restrict__ r64,
             const T* __restrict__ x_all, BRParams bp0, double tol, const BState* __restrict__ st,
             double* __restrict__ Fk, int* __restrict__ active, long long* __restrict__ done_round) {
  __shared__ double res[3];
  for (int k = blockIdx.x; k < K; k += gridDim.x) {
    const BInst& I = inst[k];
    BRParams bp = bp0;
    double sr = 0.0, sx = 0.0, sh = 0.0;
    for (int i = threadIdx.x; i < I.m; i += 256) {
      const double v = r64[I.row_off + i];
      sr += v * v;
    }
    for (int j = threadIdx.x; j < I.n; j += 256) {
      const double v = (double)x_all[I.col_off + j];
      sx += v * v;
      sh += h_value<double>(v, bp);
    }
    block_sum3_256(sr, sx, sh, res);
    __syncthreads();
    if (threadIdx.x == 0) {
      const double F = 0.5 * res[0] - I.c * res[1] + I.lam * res[2];
      Fk[k] = F;
      if (active[k]) {
        bool stop = !isfinite(F);
        if (tol > 0.0 && I.F_star != 0.0 && (F - I.F_star) / fabs(I.F_star) <= tol) stop = true;
        if (stop) {
          active[k] = 0;
          done_round[k] = st->rs.k;
        }
      }
    }
    __syncthreads();
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_bprobe(const BInst* __restrict__ inst, const int* __restrict__ col_inst, long long Ntot,
         const double* __restrict__ r64, const T* __restrict__ x_all,
         const double* __restrict__ cn2, BRParams bp0, double* __restrict__ cm,
         double* __restrict__ cs, int* __restrict__ cz) {
  const int lane = threadIdx.x & 63;
  const long long nw = (long long)gridDim.x * 4;
  for (long long j = blockIdx.x * 4ll + (threadIdx.x >> 6); j < Ntot; j += nw) {
    const BInst& I = inst[col_inst[j]];
    const T* col = (const T*)I.A + (size_t)(j - I.col_off) * I.lda;
    const double dot = col_dot<T, double, double, 4>(col, r64 + I.row_off, I.m, lane);
    if (lane == 0) {
      BRParams bp = bp0;
      bp.lam = I.lam;
      bp.lam_eta = I.lam * bp0.eta;
      bp.c2 = 2.0 * I.c;
      bp.beta = I.beta;
      const double xj = (double)x_all[j];
      double g = dot - bp.c2 * xj;
      if (bp.reg) g -= bp.lam * dh_minus<double>(xj, bp);
      const double q = cn2[j] + I.tau;
      const double xh = soft_clip<double>(xj - g / q, bp.lam_eta / q, bp.beta);
      const double y = soft_clip<double>(xj - g, bp.lam_eta, bp.beta);
      cm[j] = fabs(xh - xj);
      cs[j] = (xj - y) * (xj - y);
      cz[j] = xh != 0.0;
    }
  }
}

__global__ void __launch_bounds__(256)
k_bprobe_reduce(int K, const BInst* __restrict__ inst, const double* __restrict__ cm,
                const double* __restrict__ cs, const int* __restrict__ cz,
                double* __restrict__ out /* 3 per instance */) {
  __shared__ double res[3];
  __shared__ double shm[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int k = blockIdx.x; k < K; k += gridDim.x) {
    const BInst& I = inst[k];
    double mx = 0.0, sm = 0.0, nz = 0.0;
    for (int j = threadIdx.x; j < I.n; j += 256) {
      mx = fmax(mx, cm[I.col_off + j]);
      sm += cs[I.col_off + j];
      nz += (double)cz[I.col_off + j];
    }
    const double wm = wave_max(mx);
    if (lane == 0) shm[wave] = wm;
    block_sum3_256(sm, nz, 0.0, res);
    __syncthreads();
    if (threadIdx.x == 0) {
      out[3 * k] = fmax(fmax(shm[0], shm[1]), fmax(shm[2], shm[3]));
      out[3 * k + 1] = sqrt(res[0]);
      out[3 * k + 2] = res[1];
    }
    __syncthreads();
  }
}

// Per-instance merit test after a probe: deactivate instances with merit <= tol.
__global__ void k_bmerit_check(int K, const double* __restrict__ pr, double tol,
                               const BState* __restrict__ st, int* __restrict__ active,
                               long long* __restrict__ done_round) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x) {
    if (active[k] && pr[3 * k] <= tol) {
      active[k] = 0;
      done_round[k] = st->rs.k;
    }
  }
}

__global__ void k_binit(BState* st, long long k, double gamma, double mu, int Ntot, int K,
                        int* active, long long* done_round, long long* inst_upd, int reset) {
  for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < K; q += gridDim.x * blockDim.x) {
    if (reset) {
      active[q] = 1;
      done_round[q] = -1;
      inst_upd[q] = 0;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->rs.k = k;
    if (reset) {
      st->rs.coord_updates = 0;
      st->rs.moved_updates = 0;
    }
    st->rs.gamma_cur = gamma;
    st->rs.gamma_next = gamma;
    st->rs.gamma_mu = mu;
    st->rs.S_cnt = 0;
    st->rs.work_ctr = 0;
    st->rs.J_cnt = 0;
    st->rs.n_all = Ntot;
    st->items = 0;
    st->tiles = 0;
  }
}

template <typename T>
__global__ void k_bcolnorm2(const BInst* __restrict__ inst, const int* __restrict__ col_inst,
                            long long Ntot, double* __restrict__ cn2) {
  const int lane = threadIdx.x & 63;
  const long long nw = (long long)gridDim.x * 4;
  for (long long j = blockIdx.x * 4ll + (threadIdx.x >> 6); j < Ntot; j += nw) {
    const BInst& I = inst[col_inst[j]];
    const T* col = (const T*)I.A + (size_t)(j - I.col_off) * I.lda;
    double s = 0.0;
    for (int i = lane; i < I.m; i += 64) {
      const double v = (double)col[i];
      s += v * v;
    }
    s = wave_sum(s);
    if (lane == 0) cn2[j] = s;
  }
}

}  // namespace

namespace {

void batch_free(sca_batch* B) {
  void* ptrs[] = {B->d_inst, B->d_blk_inst, B->d_blk_col0, B->d_blk_len, B->d_blk_cols,
                  B->d_row_inst, B->d_col_inst, B->d_chunk_a, B->d_chunk_b, B->d_chunk_cnt,
                  B->d_cn2, B->d_b, B->d_r64, B->d_rrun, B->d_sel_cols, B->d_items,
                  B->d_dx_sel, B->d_J_idx, B->d_J_val, B->d_J_lo, B->d_Jn, B->d_G, B->d_ng, B->d_nrt,
                  B->d_tile_off, B->d_part, B->d_state, B->d_active, B->d_done, B->d_upd,
                  B->d_F, B->d_cm, B->d_cs, B->d_cz, B->d_pr};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  if (B->graph) (void)hipGraphExecDestroy(B->graph);
  if (B->cap) (void)hipStreamDestroy(B->cap);
  adjoint_release(B->adj);
  B->adj = nullptr;
}

int* N_total_ptr(sca_batch* B) { return (int*)((char*)B->d_state + offsetof(RoundState, n_all)); }
int* S_ptr(sca_batch* B) { return (int*)((char*)B->d_state + offsetof(RoundState, S_cnt)); }

// Fold of the listed (J_idx, J_val) columns into out = base_scale*base + A_J d.
template <typename T, typename Acc, typename TB, typename TO>
void batch_fold(sca_batch* B, const TB* base, double base_scale, TO* out, double* out64,
                hipStream_t s) {
  constexpr int VN = V16<T>::N;
  hipLaunchKernelGGL(k_bfold_plan<VN>, dim3(1), dim3(1024), 0, s, B->K, (const BInst*)B->d_inst,
                     (const int*)B->d_J_idx, B->d_state, B->d_J_lo, B->d_Jn, B->d_G, B->d_ng,
                     B->d_nrt, B->d_tile_off);
  hipLaunchKernelGGL((k_bfold_partial<T, Acc>), dim3(8 * B->ncu), dim3(256), 0, s, B->K,
                     (const BInst*)B->d_inst, (const int*)B->d_J_idx, (const T*)B->d_J_val,
                     (const int*)B->d_J_lo, (const int*)B->d_Jn, (const int*)B->d_G,
                     (const int*)B->d_ng, (const int*)B->d_nrt, (const int*)B->d_tile_off,
                     (const BState*)B->d_state, (Acc*)B->d_part, B->Mtot);
  const int g = (int)std::min<long long>((B->Mtot + 255) / 256, 16ll * B->ncu);
  hipLaunchKernelGGL((k_bfold_reduce<TB, Acc, TO>), dim3(g), dim3(256), 0, s, base, base_scale,
                     (const Acc*)B->d_part, B->Mtot, (const int*)B->d_row_inst,
                     (const int*)B->d_ng, out, out64);
}

template <typename T>
void batch_compact(sca_batch* B, const T* v, const int* idx, const int* N_ptr, long long Nmax,
                   int count_moved, hipStream_t s) {
  const int nch = (int)((Nmax + kChunk - 1) / kChunk);
  const int cg = std::max(1, std::min(nch, 2 * B->ncu));
  hipLaunchKernelGGL(k_compact_count<T>, dim3(cg), dim3(1024), 0, s, v, N_ptr, B->d_chunk_cnt);
  hipLaunchKernelGGL(k_compact_scatter<T>, dim3(cg), dim3(1024), 0, s, v, idx, N_ptr,
                     (const int*)B->d_chunk_cnt, B->d_J_idx, (T*)B->d_J_val,
                     (RoundState*)B->d_state, count_moved);
}

template <typename T>
void batch_round(sca_batch* B, const sca_opts* o, T* x, T* r, hipStream_t s) {
  const uint64_t Tthr = selection_threshold(o->select_p);
  BRParams bp;
  bp.tau = 0;
  bp.lam = 0;
  bp.lam_eta = 0;
  bp.c2 = 0;
  bp.beta = INFINITY;
  bp.theta = B->theta;
  bp.eta = B->eta;
  bp.reg = B->reg;
  const int nch = (B->Btot + kChunk - 1) / kChunk;
  const int cg = std::max(1, std::min(nch, 2 * B->ncu));
  hipLaunchKernelGGL(k_bsel_count, dim3(cg), dim3(1024), 0, s, B->Btot, (const int*)B->d_blk_inst,
                     (const int*)B->d_blk_len, (const BInst*)B->d_inst, (const int*)B->d_active,
                     o->seed, Tthr, (const BState*)B->d_state, B->d_blk_cols, B->d_chunk_a,
                     B->d_chunk_b, B->d_upd);
  hipLaunchKernelGGL(k_bsel_scatter, dim3(cg), dim3(1024), 0, s, B->Btot,
                     (const int*)B->d_blk_inst, (const int*)B->d_blk_col0,
                     (const int*)B->d_blk_cols, (const int*)B->d_chunk_a,
                     (const int*)B->d_chunk_b, B->d_state, B->d_sel_cols, B->d_items);
  hipLaunchKernelGGL((k_bgrad<T, 2>), dim3(2 * B->ncu), dim3(256), 0, s, (const BInst*)B->d_inst,
                     (const BItem*)B->d_items, (const int*)B->d_sel_cols, (const T*)r, x,
                     (const double*)B->d_cn2, B->d_state, (T*)B->d_dx_sel, bp);
  batch_compact<T>(B, (const T*)B->d_dx_sel, (const int*)B->d_sel_cols, (const int*)S_ptr(B),
                   B->Ntot, 1, s);
  batch_fold<T, T, T, T>(B, (const T*)r, 1.0, r, (double*)nullptr, s);
}

template <typename T>
void batch_residual(sca_batch* B, const T* x, T* r_out, hipStream_t s) {
  batch_compact<T>(B, x, (const int*)nullptr, (const int*)N_total_ptr(B), B->Ntot, 0, s);
  batch_fold<T, double, T, T>(B, (const T*)B->d_b, -1.0, r_out, B->d_r64, s);
}

BRParams batch_brparams(const sca_batch* B) {
  BRParams bp;
  bp.tau = 0;
  bp.lam = 0;
  bp.lam_eta = 0;
  bp.c2 = 0;
  bp.beta = INFINITY;
  bp.theta = B->theta;
  bp.eta = B->eta;
  bp.reg = B->reg;
  return bp;
}

template <typename T>
void batch_check(sca_batch* B, const T* x, double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_bobj_check<T>, dim3(std::min(B->K, 4 * B->ncu)), dim3(256), 0, s, B->K,
                     (const BInst*)B->d_inst, (const double*)B->d_r64, x, batch_brparams(B), tol,
                     (const BState*)B->d_state, B->d_F, B->d_active, B->d_done);
}

template <typename T>
void batch_probe(sca_batch* B, const T* x, hipStream_t s) {
  hipLaunchKernelGGL(k_bprobe<T>, dim3(16 * B->ncu), dim3(256), 0, s, (const BInst*)B->d_inst,
                     (const int*)B->d_col_inst, B->Ntot, (const double*)B->d_r64, x,
                     (const double*)B->d_cn2, batch_brparams(B), B->d_cm, B->d_cs, B->d_cz);
  hipLaunchKernelGGL(k_bprobe_reduce, dim3(std::min(B->K, 4 * B->ncu)), dim3(256), 0, s, B->K,
                     (const BInst*)B->d_inst, (const double*)B->d_cm, (const double*)B->d_cs,
                     (const int*)B->d_cz, B->d_pr);
}

void batch_init(sca_batch* B, const sca_opts* o, int64_t k0, int reset, hipStream_t s) {
  const double g = gamma_at_round(o->gamma, o->gamma_mu, k0);
  hipLaunchKernelGGL(k_binit, dim3(std::max(1, (B->K + 255) / 256)), dim3(256), 0, s, B->d_state,
                     (long long)k0, g, o->gamma_mu, (int)B->Ntot, B->K, B->d_active, B->d_done,
                     B->d_upd, reset);
}

template <typename T>
void batch_rounds(sca_batch* B, const sca_opts* o, int64_t n, void* x, void* r, hipStream_t s) {
  for (int64_t i = 0; i < n; ++i) batch_round<T>(B, o, (T*)x, (T*)r, s);
}

sca_status check_hip(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(SCA_EHIP, "%s: %s", what, hipGetErrorString(e));
  return SCA_OK;
}

}  // namespace

void sca::batch_fresh_residual(sca_batch* B, const void* x, hipStream_t s) {
  if (B->dtype == SCA_F32)
    batch_residual<float>(B, (const float*)x, (float*)nullptr, s);
  else
    batch_residual<double>(B, (const double*)x, (double*)nullptr, s);
}

// ------------------------------------------------------------------ public entry points
extern "C" sca_status sca_batch_create(sca_batch** out, sca_dtype dtype, int64_t count,
                                       const sca_batch_item* items, void* stream) {
  if (!out) return set_error(SCA_EINVAL, "out is NULL");
  *out = nullptr;
  if (dtype != SCA_F32 && dtype != SCA_F64) return set_error(SCA_EINVAL, "unknown dtype");
  if (count <= 0 || count > (1 << 20) || !items)
    return set_error(SCA_EINVAL, "count must lie in [1, 2^20] and items must not be NULL");
  const size_t es = dtype == SCA_F32 ? 4 : 8;
  const int64_t rpad = 16 / (int64_t)es;  // r offsets stay 16-byte aligned
  long long Mtot = 0, Ntot = 0, Btot = 0;
  for (int64_t k = 0; k < count; ++k) {
    const sca_batch_item& it = items[k];
    if (it.struct_size != sizeof(sca_batch_item))
      return set_error(SCA_EINVAL, "item %lld: struct_size mismatch", (long long)k);
    sca_status st = validate_problem_args(dtype, it.m, it.n, it.b_dev, it.lambda, it.c, it.beta,
                                          it.block_ptr_host, it.nblocks);
    if (st != SCA_OK) return set_error(st, "item %lld: %s", (long long)k, sca_last_error());
    if (!it.A_dev || ((uintptr_t)it.A_dev) % 16 || it.lda < it.m || (it.lda * (int64_t)es) % 16)
      return set_error(SCA_EINVAL, "item %lld: A must be 16-byte aligned, lda >= m, "
                       "lda*sizeof(element) a multiple of 16", (long long)k);
    if (!(it.tau >= 0.0) || !std::isfinite(it.tau))
      return set_error(SCA_EINVAL, "item %lld: tau must be finite and >= 0", (long long)k);
    if (!std::isfinite(it.F_star)) return set_error(SCA_EINVAL, "item %lld: F_star", (long long)k);
    Mtot += (it.m + rpad - 1) / rpad * rpad;
    Ntot += it.n;
    Btot += it.nblocks;
  }
  if (Mtot > INT32_MAX / 2 || Ntot > INT32_MAX / 2 || Btot > INT32_MAX / 2)
    return set_error(SCA_EINVAL, "batch too large (totals must stay below 2^30)");
  sca_batch* B = new (std::nothrow) sca_batch();
  if (!B) return set_error(SCA_ENOMEM, "host allocation failed");
  B->dtype = dtype;
  B->esize = es;
  B->K = (int)count;
  B->Mtot = Mtot;
  B->Ntot = Ntot;
  B->Btot = (int)Btot;
  B->ncu = device_cu_count();
  hipStream_t s = (hipStream_t)stream;
  std::vector<int> blk_inst, blk_col0, blk_len, row_inst(Mtot), col_inst(Ntot);
  blk_inst.reserve(Btot);
  blk_col0.reserve(Btot);
  blk_len.reserve(Btot);
  long long ro = 0, co = 0;
  int bo = 0;
  B->xoff.push_back(0);
  B->roff.push_back(0);
  for (int64_t k = 0; k < count; ++k) {
    const sca_batch_item& it = items[k];
    BInst I;
    I.A = it.A_dev;
    I.lda = it.lda;
    I.m = (int)it.m;
    I.n = (int)it.n;
    I.row_off = (int)ro;
    I.col_off = (int)co;
    I.blk_off = bo;
    I.nblk = (int)it.nblocks;
    I.lam = it.lambda;
    I.c = it.c;
    I.beta = it.beta;
    I.tau = it.tau;
    I.F_star = it.F_star;
    I.inst_id = it.instance;
    I.pad = 0;
    B->hinst.push_back(I);
    for (int64_t i = 0; i < it.nblocks; ++i) {
      blk_inst.push_back((int)k);
      blk_col0.push_back((int)(co + it.block_ptr_host[i]));
      blk_len.push_back((int)(it.block_ptr_host[i + 1] - it.block_ptr_host[i]));
    }
    const int64_t mp = (it.m + rpad - 1) / rpad * rpad;
    for (int64_t i = 0; i < mp; ++i) row_inst[ro + i] = (int)k;
    for (int64_t j = 0; j < it.n; ++j) col_inst[co + j] = (int)k;
    ro += mp;
    co += it.n;
    bo += (int)it.nblocks;
    B->xoff.push_back(co);
    B->roff.push_back(ro);
  }
  sca_status st = SCA_OK;
  const int nchB = (int)((Btot + kChunk - 1) / kChunk) + 1;
  const int nchN = (int)((Ntot + kChunk - 1) / kChunk) + 1;
#define BALLOC(ptr, bytes)                                              \
  if (st == SCA_OK) st = dev_alloc((void**)&(ptr), (bytes));
  BALLOC(B->d_inst, sizeof(BInst) * count);
  BALLOC(B->d_blk_inst, sizeof(int) * Btot);
  BALLOC(B->d_blk_col0, sizeof(int) * Btot);
  BALLOC(B->d_blk_len, sizeof(int) * Btot);
  BALLOC(B->d_blk_cols, sizeof(int) * Btot);
  BALLOC(B->d_row_inst, sizeof(int) * Mtot);
  BALLOC(B->d_col_inst, sizeof(int) * Ntot);
  BALLOC(B->d_chunk_a, sizeof(int) * nchB);
  BALLOC(B->d_chunk_b, sizeof(int) * nchB);
  BALLOC(B->d_chunk_cnt, sizeof(int) * nchN);
  BALLOC(B->d_cn2, sizeof(double) * Ntot);
  BALLOC(B->d_b, es * Mtot);
  BALLOC(B->d_r64, sizeof(double) * Mtot);
  BALLOC(B->d_rrun, es * Mtot + 16);
  BALLOC(B->d_sel_cols, sizeof(int) * Ntot);
  BALLOC(B->d_items, sizeof(BItem) * Ntot);
  BALLOC(B->d_dx_sel, es * Ntot);
  BALLOC(B->d_J_idx, sizeof(int) * Ntot);
  BALLOC(B->d_J_val, es * Ntot);
  BALLOC(B->d_J_lo, sizeof(int) * count);
  BALLOC(B->d_Jn, sizeof(int) * count);
  BALLOC(B->d_G, sizeof(int) * count);
  BALLOC(B->d_ng, sizeof(int) * count);
  BALLOC(B->d_nrt, sizeof(int) * count);
  BALLOC(B->d_tile_off, sizeof(int) * (count + 1));
  BALLOC(B->d_part, sizeof(double) * kBMaxGroups * Mtot);
  BALLOC(B->d_state, sizeof(BState));
  BALLOC(B->d_active, sizeof(int) * count);
  BALLOC(B->d_done, sizeof(long long) * count);
  BALLOC(B->d_upd, sizeof(long long) * count);
  BALLOC(B->d_F, sizeof(double) * count);
  BALLOC(B->d_cm, sizeof(double) * Ntot);
  BALLOC(B->d_cs, sizeof(double) * Ntot);
  BALLOC(B->d_cz, sizeof(int) * Ntot);
  BALLOC(B->d_pr, sizeof(double) * 3 * count);
#undef BALLOC
  if (st == SCA_OK) {
    bool ok = hipMemcpy(B->d_inst, B->hinst.data(), sizeof(BInst) * count,
                        hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(B->d_blk_inst, blk_inst.data(), sizeof(int) * Btot,
                        hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(B->d_blk_col0, blk_col0.data(), sizeof(int) * Btot,
                        hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(B->d_blk_len, blk_len.data(), sizeof(int) * Btot,
                        hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(B->d_row_inst, row_inst.data(), sizeof(int) * Mtot,
                        hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(B->d_col_inst, col_inst.data(), sizeof(int) * Ntot,
                        hipMemcpyHostToDevice) == hipSuccess;
    // padding rows of b, r and the fold partials stay zero
    ok = ok && hipMemsetAsync(B->d_b, 0, es * Mtot, s) == hipSuccess &&
         hipMemsetAsync(B->d_rrun, 0, es * Mtot + 16, s) == hipSuccess &&
         hipMemsetAsync(B->d_part, 0, sizeof(double) * kBMaxGroups * Mtot, s) == hipSuccess &&
         hipMemsetAsync(B->d_r64, 0, sizeof(double) * Mtot, s) == hipSuccess;
    for (int64_t k = 0; ok && k < count; ++k)
      ok = hipMemcpyAsync((char*)B->d_b + es * B->roff[k], items[k].b_dev, es * items[k].m,
                          hipMemcpyDeviceToDevice, s) == hipSuccess;
    if (!ok) st = set_error(SCA_EHIP, "batch set-up copies failed");
  }
  if (st == SCA_OK) {
    hipLaunchKernelGGL(k_binit, dim3(std::max(1, (B->K + 255) / 256)), dim3(256), 0, s,
                       B->d_state, 0ll, 1.0, 0.0, (int)B->Ntot, B->K, B->d_active, B->d_done,
                       B->d_upd, 1);
    if (dtype == SCA_F32)
      hipLaunchKernelGGL(k_bcolnorm2<float>, dim3(16 * B->ncu), dim3(256), 0, s,
                         (const BInst*)B->d_inst, (const int*)B->d_col_inst, B->Ntot, B->d_cn2);
    else
      hipLaunchKernelGGL(k_bcolnorm2<double>, dim3(16 * B->ncu), dim3(256), 0, s,
                         (const BInst*)B->d_inst, (const int*)B->d_col_inst, B->Ntot, B->d_cn2);
    std::vector<double> cn2(Ntot);
    if (hipMemcpyAsync(cn2.data(), B->d_cn2, sizeof(double) * Ntot, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      st = set_error(SCA_EHIP, "batch column norms failed");
    for (int64_t k = 0; st == SCA_OK && k < count; ++k) {
      for (long long j = B->xoff[k]; j < B->xoff[k + 1]; ++j) {
        if (!std::isfinite(cn2[j])) {
          st = set_error(SCA_EINVAL, "item %lld: A holds NaN or Inf", (long long)k);
          break;
        }
        if (!(cn2[j] + B->hinst[k].tau > 0.0)) {
          st = set_error(SCA_EINVAL, "item %lld: a zero column with tau = 0", (long long)k);
          break;
        }
      }
    }
  }
  if (st == SCA_OK && hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking) != hipSuccess)
    st = set_error(SCA_EHIP, "stream creation failed");
  if (st != SCA_OK) {
    batch_free(B);
    delete B;
    return st;
  }
  *out = B;
  return SCA_OK;
}

extern "C" void sca_batch_destroy(sca_batch* B) {
  if (!B) return;
  batch_free(B);
  delete B;
}

extern "C" sca_status sca_batch_layout(sca_batch* B, int64_t* x_off, int64_t* r_off) {
  if (!B) return set_error(SCA_EINVAL, "batch is NULL");
  for (int k = 0; k <= B->K; ++k) {
    if (x_off) x_off[k] = B->xoff[k];
    if (r_off) r_off[k] = B->roff[k];
  }
  return SCA_OK;
}

extern "C" sca_status sca_batch_set_regularizer(sca_batch* B, sca_reg reg, double theta) {
  if (!B) return set_error(SCA_EINVAL, "batch is NULL");
  if (reg == SCA_REG_L1) {
    B->reg = 0;
    B->theta = 0;
    B->eta = 1;
  } else if (reg == SCA_REG_EXP || reg == SCA_REG_LOG) {
    if (!(theta > 0.0) || !std::isfinite(theta)) return set_error(SCA_EINVAL, "theta must be > 0");
    B->reg = (int)reg;
    B->theta = theta;
    B->eta = reg == SCA_REG_EXP ? theta : theta / std::log1p(theta);
  } else {
    return set_error(SCA_EINVAL, "unknown regulariser");
  }
  if (B->graph) {
    (void)hipGraphExecDestroy(B->graph);
    B->graph = nullptr;
  }
  return SCA_OK;
}

extern "C" sca_status sca_batch_residual(sca_batch* B, const void* x, void* r, void* stream) {
  if (!B || !x || !r) return set_error(SCA_EINVAL, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  if (B->dtype == SCA_F32)
    batch_residual<float>(B, (const float*)x, (float*)r, s);
  else
    batch_residual<double>(B, (const double*)x, (double*)r, s);
  return check_hip("sca_batch_residual");
}

extern "C" sca_status sca_batch_step(sca_batch* B, const sca_opts* o, int64_t round_begin,
                                     int64_t nrounds, void* x, void* r, void* stream) {
  if (!B) return set_error(SCA_EINVAL, "batch is NULL");
  sca_status st = validate_opts(o);
  if (st != SCA_OK) return st;
  if (o->delay_chunks > 1)
    return set_error(SCA_EINVAL, "bounded-delay rounds need the single-problem dense path");
  if (round_begin < 0 || nrounds < 0 || !x || !r)
    return set_error(SCA_EINVAL, "bad round range or NULL x / r");
  if (((uintptr_t)r) % 16 || ((uintptr_t)x) % B->esize)
    return set_error(SCA_EINVAL, "x or r misaligned");
  hipStream_t s = (hipStream_t)stream;
  batch_init(B, o, round_begin, 1, s);
  if (B->dtype == SCA_F32)
    batch_rounds<float>(B, o, nrounds, x, r, s);
  else
    batch_rounds<double>(B, o, nrounds, x, r, s);
  return check_hip("sca_batch_step");
}

extern "C" sca_status sca_batch_objective(sca_batch* B, const sca_opts* o, const void* x,
                                          double* F, double* merit, double* MF, int64_t* nnz,
                                          void* stream) {
  if (!B || !x) return set_error(SCA_EINVAL, "NULL argument");
  sca_status st = validate_opts(o);
  if (st != SCA_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (B->dtype == SCA_F32) {
    batch_residual<float>(B, (const float*)x, (float*)nullptr, s);
    batch_check<float>(B, (const float*)x, 0.0, s);
    batch_probe<float>(B, (const float*)x, s);
  } else {
    batch_residual<double>(B, (const double*)x, (double*)nullptr, s);
    batch_check<double>(B, (const double*)x, 0.0, s);
    batch_probe<double>(B, (const double*)x, s);
  }
  std::vector<double> hF(B->K), hp(3 * B->K);
  if (hipMemcpyAsync(hF.data(), B->d_F, sizeof(double) * B->K, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipMemcpyAsync(hp.data(), B->d_pr, sizeof(double) * 3 * B->K, hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(SCA_EHIP, "batch objective: %s", hipGetErrorString(hipGetLastError()));
  for (int k = 0; k < B->K; ++k) {
    if (F) F[k] = hF[k];
    if (merit) merit[k] = hp[3 * k];
    if (MF) MF[k] = hp[3 * k + 1];
    if (nnz) nnz[k] = (int64_t)hp[3 * k + 2];
  }
  return SCA_OK;
}

// E rounds followed by a fresh FP64 residual and the per-instance stopping tests
// (relative objective error, and the merit when tol_merit > 0).
template <typename T>
static void batch_cycle(sca_batch* B, const sca_opts* o, T* x, T* r, hipStream_t s) {
  for (int64_t i = 0; i < o->check_every; ++i) batch_round<T>(B, o, x, r, s);
  batch_residual<T>(B, x, r, s);
  batch_check<T>(B, x, o->tol_rel_obj, s);
  if (o->tol_merit > 0.0) {
    batch_probe<T>(B, x, s);
    hipLaunchKernelGGL(k_bmerit_check, dim3(std::max(1, (B->K + 255) / 256)), dim3(256), 0, s,
                       B->K, (const double*)B->d_pr, o->tol_merit, (const BState*)B->d_state,
                       B->d_active, B->d_done);
  }
}

extern "C" sca_status sca_batch_solve(sca_batch* B, const sca_opts* o, void* x,
                                      sca_stats* stats, void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!B || !x) return set_error(SCA_EINVAL, "NULL argument");
  sca_status st = validate_opts(o);
  if (st != SCA_OK) return st;
  if (o->delay_chunks > 1)
    return set_error(SCA_EINVAL, "bounded-delay rounds need the single-problem dense path");
  if (o->max_rounds < 0 || o->check_every < 1)
    return set_error(SCA_EINVAL, "max_rounds >= 0 and check_every >= 1");
  if (stats)
    for (int k = 0; k < B->K; ++k)
      if (stats[k].struct_size != sizeof(sca_stats))
        return set_error(SCA_EINVAL, "stats[%d].struct_size mismatch", k);
  if (o->tol_rel_obj > 0.0)
    for (int k = 0; k < B->K; ++k)
      if (B->hinst[k].F_star == 0.0)
        return set_error(SCA_EINVAL, "instance %d: tol_rel_obj needs a nonzero F_star", k);
  hipStream_t s = (hipStream_t)stream;
  void* r = B->d_rrun;
  batch_init(B, o, 0, 1, s);
  if (B->dtype == SCA_F32)
    batch_residual<float>(B, (const float*)x, (float*)r, s);
  else
    batch_residual<double>(B, (const double*)x, (double*)r, s);
  // one graph = check_every rounds + check; built once per (x, check_every, tol)
  if (!B->graph || B->graph_rounds != o->check_every || B->graph_x != x ||
      B->graph_tol != o->tol_rel_obj || B->graph_tol_merit != o->tol_merit ||
      B->graph_p != o->select_p || B->graph_seed != o->seed) {
    if (B->graph) {
      (void)hipGraphExecDestroy(B->graph);
      B->graph = nullptr;
    }
    hipGraph_t g;
    if (hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return set_error(SCA_EHIP, "graph capture failed to start");
    if (B->dtype == SCA_F32)
      batch_cycle<float>(B, o, (float*)x, (float*)r, B->cap);
    else
      batch_cycle<double>(B, o, (double*)x, (double*)r, B->cap);
    if (hipStreamEndCapture(B->cap, &g) != hipSuccess)
      return set_error(SCA_EHIP, "graph capture failed");
    const hipError_t e = hipGraphInstantiate(&B->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      B->graph = nullptr;
      return set_error(SCA_EHIP, "graph instantiation failed");
    }
    B->graph_rounds = (int)o->check_every;
    B->graph_x = x;
    B->graph_tol = o->tol_rel_obj;
    B->graph_tol_merit = o->tol_merit;
    B->graph_p = o->select_p;
    B->graph_seed = o->seed;
  }
  std::vector<int> act(B->K);
  int64_t k = 0;
  int checks = 0;
  int nact = B->K;
  while (k < o->max_rounds && nact > 0) {
    if (hipGraphLaunch(B->graph, s) != hipSuccess)
      return set_error(SCA_EHIP, "graph launch failed");
    k += o->check_every;
    ++checks;
    if (hipMemcpyAsync(act.data(), B->d_active, sizeof(int) * B->K, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return set_error(SCA_EHIP, "batch solve: %s", hipGetErrorString(hipGetLastError()));
    nact = 0;
    for (int q = 0; q < B->K; ++q) nact += act[q];
  }
  // final report
  std::vector<double> F(B->K), mer(B->K), mf(B->K);
  std::vector<int64_t> nnz(B->K);
  if ((st = sca_batch_objective(B, o, x, F.data(), mer.data(), mf.data(), nnz.data(), stream)) !=
      SCA_OK)
    return st;
  std::vector<long long> done(B->K), upd(B->K);
  long long moved_all = 0;
  if (hipMemcpy(done.data(), B->d_done, sizeof(long long) * B->K, hipMemcpyDeviceToHost) !=
          hipSuccess ||
      hipMemcpy(upd.data(), B->d_upd, sizeof(long long) * B->K, hipMemcpyDeviceToHost) !=
          hipSuccess ||
      hipMemcpy(&moved_all, (char*)B->d_state + offsetof(RoundState, moved_updates),
                sizeof(long long), hipMemcpyDeviceToHost) != hipSuccess)
    return set_error(SCA_EHIP, "batch stats copy failed");
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  int notconv = 0;
  for (int q = 0; q < B->K; ++q) {
    const bool conv = done[q] >= 0;
    const bool fin = std::isfinite(F[q]);
    const bool want = o->tol_rel_obj > 0.0 || o->tol_merit > 0.0;
    if (!conv && want) ++notconv;
    if (stats) {
      sca_stats& S = stats[q];
      S.rounds = conv ? done[q] : k;
      S.coord_updates = upd[q];
      S.moved_updates = moved_all;
      S.F = F[q];
      S.merit = mer[q];
      S.MF = mf[q];
      const double fs = B->hinst[q].F_star;
      S.rel_err = fs != 0.0 ? (F[q] - fs) / std::fabs(fs) : 0.0;
      S.seconds = secs;
      S.nnz = nnz[q];
      S.status = !fin ? SCA_ENONFINITE : ((!conv && want) ? SCA_ENOTCONV : SCA_OK);
      S.checks = checks;
    }
  }
  if (notconv) return set_error(SCA_ENOTCONV, "%d instances did not reach the tolerance", notconv);
  return SCA_OK;
}

extern "C" sca_status sca_batch_update_rhs(sca_batch* B, const void* b_all, const double* lambda,
                                           void* stream) {
  if (!B || !b_all || !lambda) return set_error(SCA_EINVAL, "NULL argument");
  for (int k = 0; k < B->K; ++k)
    if (!(lambda[k] >= 0.0) || !std::isfinite(lambda[k]))
      return set_error(SCA_EINVAL, "lambda[%d] must be finite and >= 0", k);
  hipStream_t s = (hipStream_t)stream;
  for (int k = 0; k < B->K; ++k) {  // copy the valid rows only; padding stays zero
    const size_t off = B->esize * (size_t)B->roff[k];
    if (hipMemcpyAsync((char*)B->d_b + off, (const char*)b_all + off,
                       B->esize * (size_t)B->hinst[k].m, hipMemcpyDeviceToDevice, s) !=
        hipSuccess)
      return set_error(SCA_EHIP, "rhs copy failed");
    B->hinst[k].lam = lambda[k];
  }
  if (hipMemcpyAsync(B->d_inst, B->hinst.data(), sizeof(BInst) * B->K, hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return set_error(SCA_EHIP, "descriptor update failed");
  return SCA_OK;
}

extern "C" sca_status sca_batch_set_fstar(sca_batch* B, const double* F_star) {
  if (!B || !F_star) return set_error(SCA_EINVAL, "NULL argument");
  for (int k = 0; k < B->K; ++k) {
    if (!std::isfinite(F_star[k])) return set_error(SCA_EINVAL, "F_star[%d] not finite", k);
    B->hinst[k].F_star = F_star[k];
  }
  if (hipMemcpy(B->d_inst, B->hinst.data(), sizeof(BInst) * B->K, hipMemcpyHostToDevice) !=
      hipSuccess)
    return set_error(SCA_EHIP, "descriptor update failed");
  return SCA_OK;
}
