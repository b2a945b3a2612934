// Sparse path of libsca: A given in CSR is converted once to a library-owned CSC
// (rows ascending inside every column); a round then reads, per drawn coordinate, the
// nonzeros of its column (value + row index) and gathers r from L2.  The residual fold is
// a scatter-add into r; it is accumulated in 128-bit fixed point with integer atomics, so
// the sum is exact at 2^-72 resolution and independent of the order of the additions
// (bitwise reproducible), then added to r in one rounding.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "sca_internal.h"

using namespace sca;

namespace {

constexpr int kFixFrac = 72;  // fixed-point fraction bits: value = (hi * 2^64 + lo) * 2^-72

// ------------------------------------------------------------------ CSR -> CSC
__global__ void k_count_cols(const int32_t* __restrict__ colidx, long long nnz, int n,
                             int* __restrict__ colcnt, int* __restrict__ bad) {
  for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < nnz;
       k += (long long)gridDim.x * blockDim.x) {
    const int j = colidx[k];
    if (j < 0 || j >= n) {
      atomicOr(bad, 1);
    } else {
      atomicAdd(&colcnt[j], 1);
    }
  }
}

// One wave per CSR row: every entry goes to the next free slot of its column (slot
// order is arbitrary; the per-column sort below fixes it).
template <typename T>
__global__ void k_scatter_cols(const long long* __restrict__ rowptr,
                               const int32_t* __restrict__ colidx, const T* __restrict__ vals,
                               int m, const long long* __restrict__ colptr,
                               int* __restrict__ cursor, int* __restrict__ tmp_row,
                               long long* __restrict__ tmp_src) {
  const int lane = threadIdx.x & 63;
  const int nw = gridDim.x * (blockDim.x >> 6);
  for (int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < m; i += nw) {
    for (long long k = rowptr[i] + lane; k < rowptr[i + 1]; k += 64) {
      const int j = colidx[k];
      const long long pos = colptr[j] + atomicAdd(&cursor[j], 1);
      tmp_row[pos] = i;
      tmp_src[pos] = k;
    }
  }
}

// One wave per column: rank of each entry by (row, source position) = its final slot.
template <typename T>
__global__ void k_sort_cols(const long long* __restrict__ colptr, int n,
                            const int* __restrict__ tmp_row, const long long* __restrict__ tmp_src,
                            const T* __restrict__ vals, int* __restrict__ rowidx,
                            T* __restrict__ cvals, int* __restrict__ dup) {
  const int lane = threadIdx.x & 63;
  const int nw = gridDim.x * (blockDim.x >> 6);
  for (int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); j < n; j += nw) {
    const long long b = colptr[j], e = colptr[j + 1];
    for (long long p = b + lane; p < e; p += 64) {
      const int rp = tmp_row[p];
      const long long sp = tmp_src[p];
      long long rank = 0;
      for (long long q = b; q < e; ++q) {
        const int rq = tmp_row[q];
        if (rq < rp || (rq == rp && tmp_src[q] < sp)) ++rank;
        if (rq == rp && q != p) atomicOr(dup, 1);
      }
      rowidx[b + rank] = rp;
      cvals[b + rank] = vals[sp];
    }
  }
}

template <typename T>
__global__ void k_colnorm2_csc(const long long* __restrict__ colptr, const T* __restrict__ v,
                               int n, double* __restrict__ cn2) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (long long k = colptr[j]; k < colptr[j + 1]; ++k) {
      const double a = (double)v[k];
      s += a * a;
    }
    cn2[j] = s;
  }
}

// ------------------------------------------------------------------ round kernels
// 16 lanes per drawn coordinate (4 per wave): g_j = sum_k v_k r[row_k], then the best
// response and the step (the same closed form as the dense path).
template <typename T, typename TR, typename Acc>
__device__ __forceinline__ Acc csc_col_dot(const long long* __restrict__ colptr,
                                           const int* __restrict__ rowidx,
                                           const T* __restrict__ v, const TR* __restrict__ r,
                                           int j, int sub) {
  Acc s = (Acc)0;
  const long long b = colptr[j], e = colptr[j + 1];
  for (long long k = b + sub; k < e; k += 16) s += (Acc)v[k] * (Acc)r[rowidx[k]];
#pragma unroll
  for (int off = 8; off > 0; off >>= 1) s += __shfl_xor(s, off, 16);
  return s;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_grad_br_csc(const long long* __restrict__ colptr, const int* __restrict__ rowidx,
              const T* __restrict__ v, const T* __restrict__ r, T* __restrict__ x,
              const double* __restrict__ cn2, const int* __restrict__ sel_cols,
              const RoundState* __restrict__ st, T* __restrict__ dx_sel, BRParams bp) {
  const int sub = threadIdx.x & 15;
  const int S = st->S_cnt;
  const T gamma = (T)st->gamma_cur;
  const int ngroup = gridDim.x * 16;
  for (int t = blockIdx.x * 16 + (threadIdx.x >> 4); t < S; t += ngroup) {
    const int j = sel_cols[t];
    const T dot = csc_col_dot<T, T, T>(colptr, rowidx, v, r, j, sub);
    if (sub == 0) {
      const T xj = x[j];
      T g = dot - (T)bp.c2 * xj;
      if (bp.reg) g -= (T)bp.lam * dh_minus<T>(xj, bp);
      const T q = (T)(cn2[j] + bp.tau);
      const T xh = soft_clip<T>(xj - g / q, (T)bp.lam_eta / q, (T)bp.beta);
      const T d = gamma * (xh - xj);
      x[j] = xj + d;
      dx_sel[t] = d;
    }
  }
}

// Exact fixed-point accumulation of a double into a 128-bit two's-complement cell
// (cell[0] = low 64 bits, cell[1] = high 64 bits; unit 2^-72).  |val| is split into an
// integer part (units of 2^-8) and an exact fraction, negated in 128 bits when val < 0;
// the carry out of the low word is derived from the value the atomic returns, so the
// final cell is the exact sum whatever the order of the additions.
__device__ __forceinline__ void fix_add(unsigned long long* cell, double val) {
  const double a = ldexp(fabs(val), kFixFrac - 64);
  const double hi_d = floor(a);
  unsigned long long hi = (unsigned long long)hi_d;
  unsigned long long lo = (unsigned long long)ldexp(a - hi_d, 64);
  if (val < 0.0) {
    lo = ~lo + 1ull;
    hi = ~hi + (lo == 0ull ? 1ull : 0ull);
  }
  if (lo == 0ull && hi == 0ull) return;
  const unsigned long long old = atomicAdd(&cell[0], lo);
  const unsigned long long h = hi + ((old + lo < old) ? 1ull : 0ull);
  if (h != 0ull) atomicAdd(&cell[1], h);
}

// 16 lanes per listed column: every nonzero adds a_ij * d_j to the cell of row i.
template <typename T>
__global__ void __launch_bounds__(256)
k_fold_csc(const long long* __restrict__ colptr, const int* __restrict__ rowidx,
           const T* __restrict__ v, const int* __restrict__ J_idx, const T* __restrict__ J_val,
           const RoundState* __restrict__ st, unsigned long long* __restrict__ acc) {
  const int sub = threadIdx.x & 15;
  const int J = st->J_cnt;
  const int ngroup = gridDim.x * 16;
  for (int e = blockIdx.x * 16 + (threadIdx.x >> 4); e < J; e += ngroup) {
    const int j = J_idx[e];
    const double d = (double)J_val[e];
    for (long long k = colptr[j] + sub; k < colptr[j + 1]; k += 16)
      fix_add(acc + 2 * (size_t)rowidx[k], (double)v[k] * d);
  }
}

// out[i] = base_scale*base[i] + cell_i (one rounding); clears the cells for the next use.
template <typename TB, typename TO>
__global__ void __launch_bounds__(256)
k_fold_csc_finish(const TB* __restrict__ base, double base_scale, unsigned long long* acc, int m,
                  TO* __restrict__ out, double* __restrict__ out64) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    const unsigned long long lo = acc[2 * (size_t)i];
    const long long hi = (long long)acc[2 * (size_t)i + 1];
    acc[2 * (size_t)i] = 0ull;
    acc[2 * (size_t)i + 1] = 0ull;
    const double add = ldexp((double)hi, 64 - kFixFrac) + ldexp((double)lo, -kFixFrac);
    const double s = base_scale * (double)base[i] + add;
    if (out) out[i] = (TO)s;
    if (out64) out64[i] = s;
  }
}

template <typename T>
__global__ void __launch_bounds__(256)
k_probe_csc(const long long* __restrict__ colptr, const int* __restrict__ rowidx,
            const T* __restrict__ v, const double* __restrict__ r64, const T* __restrict__ x,
            int n, const double* __restrict__ cn2, BRParams bp, double* __restrict__ wmax,
            double* __restrict__ wsum, int* __restrict__ wcnt) {
  const int sub = threadIdx.x & 15;
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * 4 + (threadIdx.x >> 6);
  double mx = 0.0, sm = 0.0;
  int cnt = 0;
  const int ngroup = gridDim.x * 16;
  for (int j = blockIdx.x * 16 + (threadIdx.x >> 4); j < n; j += ngroup) {
    const double dot = csc_col_dot<T, double, double>(colptr, rowidx, v, r64, j, sub);
    if (sub == 0) {
      const double xj = (double)x[j];
      double g = dot - bp.c2 * xj;
      if (bp.reg) g -= bp.lam * dh_minus<double>(xj, bp);
      const double q = cn2[j] + bp.tau;
      const double xh = soft_clip<double>(xj - g / q, bp.lam_eta / q, bp.beta);
      const double y = soft_clip<double>(xj - g, bp.lam_eta, bp.beta);
      mx = fmax(mx, fabs(xh - xj));
      sm += (xj - y) * (xj - y);
      cnt += (xh != 0.0);
    }
  }
  // lanes 0, 16, 32, 48 hold values; fixed-order combination inside the wave
  mx = wave_max(mx);
  sm = wave_sum(sm);
  const int c = (int)wave_sum_i64((long long)cnt);
  if (lane == 0) {
    wmax[gw] = mx;
    wsum[gw] = sm;
    wcnt[gw] = c;
  }
}

template <typename T>
void fold_launch(sca_problem* p, hipStream_t s) {
  hipLaunchKernelGGL(k_fold_csc<T>, dim3(8 * p->ncu), dim3(256), 0, s,
                     (const long long*)p->csc_colptr, (const int*)p->csc_rowidx,
                     (const T*)p->csc_vals, (const int*)p->d_J_idx, (const T*)p->d_J_val,
                     (const RoundState*)p->d_state, (unsigned long long*)p->csr_tmp);
}

template <typename T>
void round_csc(sca_problem* p, const sca_opts* o, T* x, T* r, hipStream_t s, uint64_t Tthr,
               const BRParams& bp) {
  const int m = (int)p->m, n = (int)p->n;
  prof_begin(p, s, SCA_K_SELECT);
  hipLaunchKernelGGL(k_select, dim3(1), dim3(1024), 0, s, (int)p->nblocks, p->d_bp, o->seed,
                     o->instance, Tthr, p->d_state, p->d_sel_cols);
  prof_end(p, s, 0.0);
  prof_begin(p, s, SCA_K_GRAD);
  hipLaunchKernelGGL(k_grad_br_csc<T>, dim3(8 * p->ncu), dim3(256), 0, s,
                     (const long long*)p->csc_colptr, (const int*)p->csc_rowidx,
                     (const T*)p->csc_vals, (const T*)r, x, p->d_cn2, p->d_sel_cols,
                     (const RoundState*)p->d_state, (T*)p->d_dx_sel, bp);
  prof_end(p, s, 0.0);
  prof_begin(p, s, SCA_K_COMPACT);
  const int nch = (n + kChunk - 1) / kChunk;
  const int cgrid = std::max(1, std::min(nch, 2 * p->ncu));
  int* S_ptr = (int*)((char*)p->d_state + offsetof(RoundState, S_cnt));
  hipLaunchKernelGGL(k_compact_count<T>, dim3(cgrid), dim3(1024), 0, s, (const T*)p->d_dx_sel,
                     (const int*)S_ptr, p->d_chunk_cnt);
  hipLaunchKernelGGL(k_compact_scatter<T>, dim3(cgrid), dim3(1024), 0, s,
                     (const T*)p->d_dx_sel, (const int*)p->d_sel_cols, (const int*)S_ptr,
                     (const int*)p->d_chunk_cnt, p->d_J_idx, (T*)p->d_J_val, p->d_state, 1);
  prof_end(p, s, 0.0);
  prof_begin(p, s, SCA_K_FOLD);
  fold_launch<T>(p, s);
  hipLaunchKernelGGL((k_fold_csc_finish<T, T>), dim3((m + 255) / 256), dim3(256), 0, s,
                     (const T*)r, 1.0, (unsigned long long*)p->csr_tmp, m, r, (double*)nullptr);
  prof_end(p, s, 0.0);
}

template <typename T>
void residual_csc(sca_problem* p, const T* x, T* r_out, hipStream_t s) {
  const int m = (int)p->m, n = (int)p->n;
  int* N_ptr = (int*)((char*)p->d_state + offsetof(RoundState, n_all));
  const int nch = (n + kChunk - 1) / kChunk;
  const int cgrid = std::max(1, std::min(nch, 2 * p->ncu));
  hipLaunchKernelGGL(k_compact_count<T>, dim3(cgrid), dim3(1024), 0, s, x, (const int*)N_ptr,
                     p->d_chunk_cnt);
  hipLaunchKernelGGL(k_compact_scatter<T>, dim3(cgrid), dim3(1024), 0, s, x, (const int*)nullptr,
                     (const int*)N_ptr, (const int*)p->d_chunk_cnt, p->d_J_idx, (T*)p->d_J_val,
                     p->d_state, 0);
  fold_launch<T>(p, s);
  hipLaunchKernelGGL((k_fold_csc_finish<T, T>), dim3((m + 255) / 256), dim3(256), 0, s,
                     (const T*)p->b, -1.0, (unsigned long long*)p->csr_tmp, m, r_out, p->d_r64);
}

}  // namespace

// ------------------------------------------------------------------ hooks used by the API
void sca::launch_colnorm2_csc(sca_problem* p, hipStream_t s) {
  const int grid = std::max(1, std::min<int>((int)((p->n + 255) / 256), 8 * p->ncu));
  if (p->dtype == SCA_F32)
    hipLaunchKernelGGL(k_colnorm2_csc<float>, dim3(grid), dim3(256), 0, s,
                       (const long long*)p->csc_colptr, (const float*)p->csc_vals, (int)p->n,
                       p->d_cn2);
  else
    hipLaunchKernelGGL(k_colnorm2_csc<double>, dim3(grid), dim3(256), 0, s,
                       (const long long*)p->csc_colptr, (const double*)p->csc_vals, (int)p->n,
                       p->d_cn2);
}

void sca::launch_round_csc(sca_problem* p, const sca_opts* o, void* x, void* r, hipStream_t s,
                           uint64_t Tthr, const BRParams& bp) {
  if (p->dtype == SCA_F32)
    round_csc<float>(p, o, (float*)x, (float*)r, s, Tthr, bp);
  else
    round_csc<double>(p, o, (double*)x, (double*)r, s, Tthr, bp);
}

void sca::launch_residual_csc(sca_problem* p, const void* x, void* r_out, hipStream_t s) {
  if (p->dtype == SCA_F32)
    residual_csc<float>(p, (const float*)x, (float*)r_out, s);
  else
    residual_csc<double>(p, (const double*)x, (double*)r_out, s);
}

void sca::launch_probe_csc(sca_problem* p, const void* x, const BRParams& bp, hipStream_t s) {
  const int grid = p->probe_waves / 4;
  if (p->dtype == SCA_F32)
    hipLaunchKernelGGL(k_probe_csc<float>, dim3(grid), dim3(256), 0, s,
                       (const long long*)p->csc_colptr, (const int*)p->csc_rowidx,
                       (const float*)p->csc_vals, (const double*)p->d_r64, (const float*)x,
                       (int)p->n, (const double*)p->d_cn2, bp, p->d_wmax, p->d_wsum, p->d_wcnt);
  else
    hipLaunchKernelGGL(k_probe_csc<double>, dim3(grid), dim3(256), 0, s,
                       (const long long*)p->csc_colptr, (const int*)p->csc_rowidx,
                       (const double*)p->csc_vals, (const double*)p->d_r64, (const double*)x,
                       (int)p->n, (const double*)p->d_cn2, bp, p->d_wmax, p->d_wsum, p->d_wcnt);
}

// ------------------------------------------------------------------ create
template <typename T>
static sca_status build_csc(sca_problem* p, const long long* rowptr, const int32_t* colidx,
                            const T* vals, hipStream_t s) {
  const int m = (int)p->m, n = (int)p->n;
  const long long nnz = p->nnz;
  sca_status st;
  int *colcnt = nullptr, *flags = nullptr, *tmp_row = nullptr;
  long long* tmp_src = nullptr;
  auto cleanup = [&]() {
    if (colcnt) (void)hipFree(colcnt);
    if (flags) (void)hipFree(flags);
    if (tmp_row) (void)hipFree(tmp_row);
    if (tmp_src) (void)hipFree(tmp_src);
  };
  if ((st = dev_alloc((void**)&colcnt, sizeof(int) * (size_t)(n + 1))) != SCA_OK ||
      (st = dev_alloc((void**)&flags, sizeof(int) * 4)) != SCA_OK ||
      (st = dev_alloc((void**)&tmp_row, sizeof(int) * (size_t)std::max(1ll, nnz))) != SCA_OK ||
      (st = dev_alloc((void**)&tmp_src, sizeof(long long) * (size_t)std::max(1ll, nnz))) != SCA_OK ||
      (st = dev_alloc((void**)&p->csc_colptr, sizeof(long long) * (size_t)(n + 1))) != SCA_OK ||
      (st = dev_alloc((void**)&p->csc_rowidx, sizeof(int) * (size_t)std::max(1ll, nnz))) != SCA_OK ||
      (st = dev_alloc((void**)&p->csc_vals, sizeof(T) * (size_t)std::max(1ll, nnz))) != SCA_OK ||
      (st = dev_alloc((void**)&p->csr_tmp, 16 * (size_t)p->ldp)) != SCA_OK) {
    cleanup();
    return st;
  }
  // the row pointer is validated on the host
  std::vector<long long> hrp(m + 1);
  if (hipMemcpyAsync(hrp.data(), rowptr, sizeof(long long) * (m + 1), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    cleanup();
    return set_error(SCA_EHIP, "copy of rowptr failed");
  }
  if (hrp[0] != 0 || hrp[m] != nnz) {
    cleanup();
    return set_error(SCA_EINVAL, "rowptr must start at 0 and end at nnz");
  }
  for (int i = 0; i < m; ++i)
    if (hrp[i + 1] < hrp[i]) {
      cleanup();
      return set_error(SCA_EINVAL, "rowptr is not ascending");
    }
  (void)hipMemsetAsync(colcnt, 0, sizeof(int) * (size_t)(n + 1), s);
  (void)hipMemsetAsync(flags, 0, sizeof(int) * 4, s);
  (void)hipMemsetAsync(p->csr_tmp, 0, 16 * (size_t)p->ldp, s);
  const int g = 8 * p->ncu;
  hipLaunchKernelGGL(k_count_cols, dim3(g), dim3(256), 0, s, colidx, nnz, n, colcnt, flags);
  std::vector<int> hc(n + 1);
  int hbad = 0;
  if (hipMemcpyAsync(hc.data(), colcnt, sizeof(int) * n, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(&hbad, flags, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    cleanup();
    return set_error(SCA_EHIP, "column count failed");
  }
  if (hbad) {
    cleanup();
    return set_error(SCA_EINVAL, "colidx holds an index outside [0, n)");
  }
  std::vector<long long> hcp(n + 1);
  hcp[0] = 0;
  for (int j = 0; j < n; ++j) hcp[j + 1] = hcp[j] + hc[j];
  if (hipMemcpyAsync(p->csc_colptr, hcp.data(), sizeof(long long) * (n + 1),
                     hipMemcpyHostToDevice, s) != hipSuccess) {
    cleanup();
    return set_error(SCA_EHIP, "copy of colptr failed");
  }
  (void)hipMemsetAsync(colcnt, 0, sizeof(int) * (size_t)(n + 1), s);
  hipLaunchKernelGGL(k_scatter_cols<T>, dim3(g), dim3(256), 0, s, rowptr, colidx, vals, m,
                     (const long long*)p->csc_colptr, colcnt, tmp_row, tmp_src);
  hipLaunchKernelGGL(k_sort_cols<T>, dim3(g), dim3(256), 0, s, (const long long*)p->csc_colptr, n,
                     (const int*)tmp_row, (const long long*)tmp_src, vals, p->csc_rowidx,
                     (T*)p->csc_vals, flags + 1);
  int hdup = 0;
  if (hipMemcpyAsync(&hdup, flags + 1, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    cleanup();
    return set_error(SCA_EHIP, "CSC conversion failed: %s", hipGetErrorString(hipGetLastError()));
  }
  cleanup();
  if (hdup) return set_error(SCA_EINVAL, "CSR holds a repeated (row, column) entry");
  return SCA_OK;
}

extern "C" sca_status sca_problem_create_csr(sca_problem** out, sca_dtype dtype, int64_t m,
                                             int64_t n, int64_t nnz, const int64_t* rowptr,
                                             const int32_t* colidx, const void* vals,
                                             const void* b, double lambda, double c, double beta,
                                             const int64_t* block_ptr, int64_t nblocks,
                                             void* stream) {
  if (!out) return set_error(SCA_EINVAL, "out is NULL");
  *out = nullptr;
  sca_status st = validate_problem_args(dtype, m, n, b, lambda, c, beta, block_ptr, nblocks);
  if (st != SCA_OK) return st;
  if (nnz < 0 || nnz > (int64_t)INT32_MAX * 8)
    return set_error(SCA_EINVAL, "nnz out of range");
  if (!rowptr || (nnz > 0 && (!colidx || !vals)))
    return set_error(SCA_EINVAL, "rowptr, colidx or vals is NULL");
  sca_problem* p = new (std::nothrow) sca_problem();
  if (!p) return set_error(SCA_ENOMEM, "host allocation failed");
  p->dtype = dtype;
  p->esize = dtype == SCA_F32 ? 4 : 8;
  p->m = m;
  p->n = n;
  p->lda = 0;
  p->A = nullptr;
  p->b = b;
  p->lam = lambda;
  p->c = c;
  p->beta = beta;
  p->nblocks = nblocks;
  p->sparse = true;
  p->nnz = nnz;
  p->ncu = device_cu_count();
  hipStream_t s = (hipStream_t)stream;
  if ((st = alloc_workspace(p, block_ptr)) == SCA_OK) {
    st = dtype == SCA_F32
             ? build_csc<float>(p, (const long long*)rowptr, colidx, (const float*)vals, s)
             : build_csc<double>(p, (const long long*)rowptr, colidx, (const double*)vals, s);
  }
  if (st == SCA_OK) st = finish_create(p, s);
  if (st != SCA_OK) {
    free_workspace(p);
    delete p;
    return st;
  }
  *out = p;
  return SCA_OK;
}
