// Kernels of the dual iteration (paper section 4.3): the action of
// F = sum_i B_i K_i^+ B_i^T through the jump operators, the projection
// P = I - G (G^T G)^{-1} G^T, the scaled-row (B_D) preconditioners of
// section 4.4, deterministic dot products and the CG recurrences.
//
// All reductions use a fixed partition and a fixed summation order, so a
// solve gives bit-identical results whatever else runs on the device.
#include <algorithm>
#include <mutex>

#include "feti_impl.h"
#include "k_pcg.h"

namespace feti {

constexpr int LDV = TS + 1;

__device__ __forceinline__ bool halted(const PcgState* st) { return st != nullptr && st->done != 0; }
__device__ __forceinline__ int64_t tidx2(int i, int j) { return (int64_t)i * (i + 1) / 2 + j; }

// xb[b] = sum_{rows r touching b} coef * (w_r if weighted) * v[r]
__global__ void k_gather(int64_t NB, const int32_t* __restrict__ g_ptr, const int32_t* __restrict__ g_row,
                         const double* __restrict__ g_coef, const double* __restrict__ w, int weighted,
                         const double* __restrict__ v, double* __restrict__ xb, const PcgState* st) {
  if (halted(st)) return;
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= NB) return;
  double acc = 0.0;
  for (int k = g_ptr[b]; k < g_ptr[b + 1]; ++k) {
    const int r = g_row[k];
    acc += g_coef[k] * (weighted ? w[r] : 1.0) * v[r];
  }
  xb[b] = acc;
}

// out[r] = base[r] + sgn * (w_r if weighted) * (c0 y[b0] + c1 y[b1])   (base may be NULL)
__global__ void k_scatter(int64_t n_lam, const int64_t* __restrict__ b0, const double* __restrict__ c0,
                          const int64_t* __restrict__ b1, const double* __restrict__ c1,
                          const double* __restrict__ w, int weighted, const double* __restrict__ y,
                          const double* __restrict__ base, double sgn, double* __restrict__ out,
                          const PcgState* st) {
  if (halted(st)) return;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_lam) return;
  double v = c0[r] * y[b0[r]];
  if (b1[r] >= 0) v += c1[r] * y[b1[r]];
  if (weighted) v *= w[r];
  out[r] = (base ? base[r] : 0.0) + sgn * v;
}

// Block partial sums of up to two dot products over n entries (fixed partition).
__global__ __launch_bounds__(256) void k_dot_partial(int64_t n, const double* __restrict__ a,
                                                     const double* __restrict__ b,
                                                     const double* __restrict__ c,
                                                     const double* __restrict__ d, double* part,
                                                     const PcgState* st) {
  if (halted(st)) return;
  __shared__ double r1[256], r2[256];
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t k = lo + threadIdx.x; k < hi; k += 256) {
    s1 += a[k] * b[k];
    if (c) s2 += c[k] * d[k];
  }
  r1[threadIdx.x] = s1;
  r2[threadIdx.x] = s2;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      r1[threadIdx.x] += r1[threadIdx.x + h];
      r2[threadIdx.x] += r2[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = r1[0];
    part[2 * blockIdx.x + 1] = r2[0];
  }
}

__device__ void sum_parts(const double* part, int nparts, double* o1, double* o2) {
  __shared__ double r1[256], r2[256];
  double s1 = 0.0, s2 = 0.0;
  for (int k = threadIdx.x; k < nparts; k += 256) {
    s1 += part[2 * k];
    s2 += part[2 * k + 1];
  }
  r1[threadIdx.x] = s1;
  r2[threadIdx.x] = s2;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      r1[threadIdx.x] += r1[threadIdx.x + h];
      r2[threadIdx.x] += r2[threadIdx.x + h];
    }
    __syncthreads();
  }
  *o1 = r1[0];
  *o2 = r2[0];
}

// g[coarse_off + k] = rb_k . xb over the interface of every floating subdomain.
__global__ __launch_bounds__(256) void k_coarse_gt(const SubInfo* __restrict__ subs, const double* __restrict__ rb,
                                                   const double* __restrict__ xb, double* g,
                                                   const PcgState* st) {
  if (halted(st)) return;
  __shared__ double red[6][256];
  const SubInfo s = subs[blockIdx.x];
  if (s.n_modes == 0) return;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const int64_t n = (int64_t)s.nt_b * TS;
  for (int64_t b = threadIdx.x; b < n; b += 256) {
    const double x = xb[s.b_off + b];
    const double* R = rb + (s.b_off + b) * 6;
    for (int k = 0; k < 6; ++k) acc[k] += R[k] * x;
  }
  for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int k = 0; k < 6; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < s.n_modes) g[s.coarse_off + threadIdx.x] = red[threadIdx.x][0];
}

// Same over the full local space (e_i = R_i^T f_i).
__global__ __launch_bounds__(256) void k_coarse_gt_full(const SubInfo* __restrict__ subs,
                                                        const double* __restrict__ rf,
                                                        const double* __restrict__ xf, double* g) {
  __shared__ double red[6][256];
  const SubInfo s = subs[blockIdx.x];
  if (s.n_modes == 0) return;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const int64_t n = (int64_t)s.nt * TS;
  for (int64_t b = threadIdx.x; b < n; b += 256) {
    const double x = xf[s.full_off + b];
    const double* R = rf + (s.full_off + b) * 6;
    for (int k = 0; k < 6; ++k) acc[k] += R[k] * x;
  }
  for (int k = 0; k < 6; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int k = 0; k < 6; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < s.n_modes) g[s.coarse_off + threadIdx.x] = red[threadIdx.x][0];
}

// vb = Rb alpha (zero on subdomains without kernel)
__global__ void k_coarse_expand(int64_t NB, const int32_t* __restrict__ b_sub, const SubInfo* __restrict__ subs,
                                const double* __restrict__ rb, const double* __restrict__ alpha,
                                double* vb, const PcgState* st) {
  if (halted(st)) return;
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= NB) return;
  const SubInfo s = subs[b_sub[b]];
  double acc = 0.0;
  for (int k = 0; k < s.n_modes; ++k) acc += rb[b * 6 + k] * alpha[s.coarse_off + k];
  vb[b] = acc;
}

// u_full += R gamma on the full local space
__global__ void k_add_modes(int64_t NF, const int32_t* __restrict__ f_sub, const SubInfo* __restrict__ subs,
                            const double* __restrict__ rf, const double* __restrict__ gamma, double* u) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NF) return;
  const SubInfo s = subs[f_sub[p]];
  double acc = 0.0;
  for (int k = 0; k < s.n_modes; ++k) acc += rf[p * 6 + k] * gamma[s.coarse_off + k];
  u[p] += acc;
}

// Lumped preconditioner: yb = K_bb xb with the interface-interface block of
// every local stiffness stored slot-major (consecutive interface DOFs coalesce).
// Lumped preconditioner block y = K_bb x over the compact slot-major ELL of
// K_bb.  Four lanes share a row (lane q takes slots q, q+4, ...), so the
// launch has enough waves to hide the memory latency of the slot loads and
// the x gathers; the four partial sums are combined in a fixed order.
constexpr int LUMP_LANES = 4;
__global__ __launch_bounds__(256) void k_lumped(int64_t NB, int w_bb, const int32_t* __restrict__ bb_col,
                                                const double* __restrict__ bb_val, const double* __restrict__ xb,
                                                double* __restrict__ yb, const PcgState* st) {
  if (halted(st)) return;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t b = t / LUMP_LANES;
  const int q = (int)(t % LUMP_LANES);
  double acc = 0.0;
  if (b < NB) {
    constexpr int C = 4;   // slots per lane in flight
    for (int k0 = q; k0 < w_bb; k0 += C * LUMP_LANES) {
      int c[C];
      double v[C], x[C];
#pragma unroll
      for (int i = 0; i < C; ++i) {
        const int k = k0 + i * LUMP_LANES;
        const bool in = k < w_bb;
        c[i] = in ? bb_col[(int64_t)k * NB + b] : 0;
        v[i] = in ? bb_val[(int64_t)k * NB + b] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < C; ++i) x[i] = xb[c[i]];
#pragma unroll
      for (int i = 0; i < C; ++i) acc += v[i] * x[i];
    }
  }
  // lanes 4r..4r+3 of a wave hold row r's partial sums: ((q0 + q1) + (q2 + q3))
  acc += __shfl_xor(acc, 1, 64);
  acc += __shfl_xor(acc, 2, 64);
  if (b < NB && q == 0) yb[b] = acc;
}

// K_bb values from the assembled rows (after every factorisation).
__global__ void k_bb_fill(int64_t NB, int64_t NF, int w_bb, const int32_t* __restrict__ bb_slot,
                          const int64_t* __restrict__ b2full, const double* __restrict__ ell_val,
                          double* __restrict__ bb_val) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= NB * w_bb) return;
  const int64_t b = t % NB;
  const int k = (int)(t / NB);
  const int sl = bb_slot[t];
  bb_val[t] = sl >= 0 ? ell_val[(int64_t)sl * NF + b2full[b]] : 0.0;
}

// Multiplier right-hand side b: prescribed value of an all-floating Dirichlet row, else 0.
__global__ void k_bvec(int64_t n_lam, const int64_t* __restrict__ gdof, const double* __restrict__ dvals,
                       double* __restrict__ out) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_lam) return;
  out[r] = gdof[r] >= 0 ? dvals[gdof[r]] : 0.0;
}

// Global nodal result.  sum_mode 0: mean of the subdomain copies, Dirichlet
// DOFs take dvals.  sum_mode 1: sum of the copies (assembled vector), zero on
// Dirichlet DOFs.
__global__ void k_global(int64_t n_dof, const int32_t* __restrict__ uc_ptr, const int64_t* __restrict__ uc_idx,
                         const double* __restrict__ ufull, const uint8_t* __restrict__ dmask,
                         const double* __restrict__ dvals, double* out, int sum_mode) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_dof) return;
  if (dmask[g]) {
    out[g] = sum_mode ? 0.0 : dvals[g];
    return;
  }
  double acc = 0.0;
  const int n = uc_ptr[g + 1] - uc_ptr[g];
  for (int k = uc_ptr[g]; k < uc_ptr[g + 1]; ++k) acc += ufull[uc_idx[k]];
  out[g] = sum_mode ? acc : (n ? acc / n : 0.0);
}

// Dirichlet data of a Newton step: dvals = tau u_D - U on Dirichlet DOFs (U may be NULL).
__global__ void k_dirinc(int64_t n_dof, const uint8_t* __restrict__ dmask, const double* __restrict__ dirval,
                         double tau, const double* __restrict__ U, double* dvals) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_dof) return;
  dvals[g] = dmask[g] ? tau * dirval[g] - (U ? U[g] : 0.0) : 0.0;
}

// Block partial sums of the k dot products V_i . w (V_i = V + i ld) over the
// fixed partition of every dot product: part[i * DOT_PARTS + b].  One launch
// for all k (the Gram-Schmidt step of the GMRES iterations).
__global__ __launch_bounds__(256) void k_multi_dot(int64_t n, const double* __restrict__ V, int64_t ld,
                                                   const double* __restrict__ w, double* part) {
  __shared__ double r1[256];
  const double* a = V + (int64_t)blockIdx.y * ld;
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  double s1 = 0.0;
  for (int64_t k = lo + threadIdx.x; k < hi; k += 256) s1 += a[k] * w[k];
  r1[threadIdx.x] = s1;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) r1[threadIdx.x] += r1[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = r1[0];
}

// out[i] = sum of the DOT_PARTS partial sums of product i, in a fixed tree
// order (one workgroup per product).
__global__ __launch_bounds__(256) void k_multi_finish(const double* __restrict__ part, double* out) {
  static_assert(DOT_PARTS == 256, "one partial sum per thread");
  __shared__ double r1[256];
  r1[threadIdx.x] = part[(int64_t)blockIdx.x * DOT_PARTS + threadIdx.x];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) r1[threadIdx.x] += r1[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = r1[0];
}

// y -= sum_{i<k} h_i V_i, the products summed in order i = 0, 1, ...
__global__ void k_multi_axpy(int64_t n, const double* __restrict__ V, int64_t ld, int k,
                             const double* __restrict__ h, double* y) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double acc = 0.0;
  for (int i = 0; i < k; ++i) acc += h[i] * V[(int64_t)i * ld + r];
  y[r] -= acc;
}

__global__ void k_axpby(int64_t n, double a, const double* __restrict__ x, double b, double* y) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) y[k] = (b == 0.0) ? a * x[k] : a * x[k] + b * y[k];   // b == 0: y is not read
}

__global__ void k_fill(int64_t n, double v, double* y) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) y[k] = v;
}

__global__ void k_init_state(PcgState* st, double rtol, double atol, int max_it, int hist_cap) {
  st->rho = st->alpha = st->beta = st->w0 = st->wn = st->pq = 0.0;
  st->rtol = rtol;
  st->atol = atol;
  st->it = 0;
  st->max_it = max_it;
  st->done = 0;
  st->status = 0;
  st->hist_cap = hist_cap;
}

// ---------------------------------------------------------------------------
// Fused kernels of one PCG iteration (section 4.3 CG on P^T F with the
// projection P = I - G Q^{-1} G^T).  The search direction s = z + beta s is
// formed on the fly where it is read and written back by the per-row kernel
// that owns each multiplier; the dot products finish in the last workgroup to
// arrive (fixed partition and summation order, so results are deterministic).

// last-arriving block of a grid: thread 0 publishes the block's partial sums,
// fences and takes a ticket; the block that draws the last ticket reduces.
__device__ bool last_block(int* ticket, int nblocks = -1) {
  __shared__ bool last;
  if (nblocks < 0) nblocks = (int)gridDim.x;
  if (threadIdx.x == 0) {
    __threadfence();
    const int t = atomicAdd(ticket, 1);
    last = (t == nblocks - 1);
  }
  __syncthreads();
  if (last) __threadfence();
  return last;
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum of a and b over a 256-thread block (fixed order); result valid in every thread.
__device__ void block_reduce2(double& a, double& b, double* ra, double* rb) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    ra[w] = a;
    rb[w] = b;
  }
  __syncthreads();
  a = (ra[0] + ra[1]) + (ra[2] + ra[3]);
  b = (rb[0] + rb[1]) + (rb[2] + rb[3]);
}

constexpr int GT_CHUNKS = 4;

// One chunk of g = Rb^T (C v) for subdomain `sub`, with C a copy coupling
// (B^T B or B^T diag(w) B, CSR over b-space): the coarse right-hand side
// G^T (B v) straight from an interface vector v, without the row vector.
// Writes gpart[chunk][coarse_off + m].  Called by a whole block.
__device__ void gt_chunk(int sub, int chunk, const SubInfo* __restrict__ subs, const int32_t* __restrict__ c_ptr,
                         const int32_t* __restrict__ c_col, const double* __restrict__ cv,
                         const double* __restrict__ rbv, const double* __restrict__ v, double* gpart, int ldg) {
  __shared__ double red[6][4];
  const SubInfo s = subs[sub];
  if (s.n_modes == 0) return;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const int64_t nb = (int64_t)s.nt_b * TS;
  const int64_t lo = nb * chunk / GT_CHUNKS, hi = nb * (chunk + 1) / GT_CHUNKS;
  for (int64_t k = lo + threadIdx.x; k < hi; k += 256) {
    const int64_t b = s.b_off + k;
    const int e0 = c_ptr[b], e1 = c_ptr[b + 1];
    double u = 0.0;
    for (int e = e0; e < e1; ++e) u += cv[e] * v[c_col[e]];
    const double* R = rbv + b * 6;
#pragma unroll
    for (int m = 0; m < 6; ++m) acc[m] += R[m] * u;
  }
#pragma unroll
  for (int m = 0; m < 6; ++m) acc[m] = wave_sum(acc[m]);
  if ((threadIdx.x & 63) == 0)
    for (int m = 0; m < 6; ++m) red[m][threadIdx.x >> 6] = acc[m];
  __syncthreads();
  if (threadIdx.x < s.n_modes) {
    const int m = threadIdx.x;
    gpart[(int64_t)chunk * ldg + s.coarse_off + m] = (red[m][0] + red[m][1]) + (red[m][2] + red[m][3]);
  }
}

// xb = B^T (z + beta s)
__global__ void k_gather_s(int64_t NB, const int32_t* __restrict__ g_ptr, const int32_t* __restrict__ g_row,
                           const double* __restrict__ g_coef, const double* __restrict__ z,
                           const double* __restrict__ sv, double* __restrict__ xb, const PcgState* st) {
  if (halted(st)) return;
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= NB) return;
  const double beta = st->beta;
  double acc = 0.0;
  for (int k = g_ptr[b]; k < g_ptr[b + 1]; ++k) {
    const int r = g_row[k];
    acc += g_coef[k] * (z[r] + beta * sv[r]);
  }
  xb[b] = acc;
}

// Fused: blocks [0, nrow_blocks) do q = B yb, s <- z + beta s and the block
// partial sums of s.q (part[block]; alpha = rho / s.q is formed by the next
// kernel from them); the blocks after them form the coarse right-hand side
// G^T q = Rb^T (B^T B) yb by subdomain chunks.
__global__ __launch_bounds__(256) void k_scatter_dot_alpha_gt(
    int64_t n, int nrow_blocks, const int64_t* __restrict__ b0, const double* __restrict__ c0,
    const int64_t* __restrict__ b1, const double* __restrict__ c1, const double* __restrict__ yb,
    const double* __restrict__ z, double* sv, double* q, double* part, const PcgState* st,
    const SubInfo* __restrict__ subs, const int32_t* __restrict__ c_ptr, const int32_t* __restrict__ c_col,
    const double* __restrict__ cv, const double* __restrict__ rbv, double* gpart, int ldg) {
  if (st->done) return;
  if ((int)blockIdx.x >= nrow_blocks) {
    const int g = blockIdx.x - nrow_blocks;
    gt_chunk(g / GT_CHUNKS, g % GT_CHUNKS, subs, c_ptr, c_col, cv, rbv, yb, gpart, ldg);
    return;
  }
  __shared__ double ra[256], rb[256];
  double acc = 0.0, unused = 0.0;
  const double beta = st->beta;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)nrow_blocks * 256) {
    double v = c0[r] * yb[b0[r]];
    if (b1[r] >= 0) v += c1[r] * yb[b1[r]];
    const double sn = z[r] + beta * sv[r];
    sv[r] = sn;
    q[r] = v;
    acc += sn * v;
  }
  block_reduce2(acc, unused, ra, rb);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Fused: blocks [0, nrow_blocks) do the weighted scatter t = diag(w) B y;
// the blocks after them form G^T t = Rb^T (B^T diag(w) B) y by subdomain chunks.
__global__ __launch_bounds__(256) void k_scatter_w_gt(
    int64_t n, int nrow_blocks, const int64_t* __restrict__ b0, const double* __restrict__ c0,
    const int64_t* __restrict__ b1, const double* __restrict__ c1, const double* __restrict__ w,
    const double* __restrict__ y, double* __restrict__ out, const PcgState* st, const SubInfo* __restrict__ subs,
    const int32_t* __restrict__ c_ptr, const int32_t* __restrict__ c_col, const double* __restrict__ cv,
    const double* __restrict__ rbv, double* gpart, int ldg) {
  if (halted(st)) return;
  if ((int)blockIdx.x >= nrow_blocks) {
    const int g = blockIdx.x - nrow_blocks;
    gt_chunk(g / GT_CHUNKS, g % GT_CHUNKS, subs, c_ptr, c_col, cv, rbv, y, gpart, ldg);
    return;
  }
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)nrow_blocks * 256) {
    double v = c0[r] * y[b0[r]];
    if (b1[r] >= 0) v += c1[r] * y[b1[r]];
    out[r] = w[r] * v;
  }
}

// Partial g = Rb^T B^T x per floating subdomain, in GT_CHUNKS chunks of its
// interface (gpart[chunk][coarse index]); with_update: x is r - alpha q
// (formed on the fly).
__global__ __launch_bounds__(256) void k_proj_gt(const SubInfo* __restrict__ subs, const int32_t* __restrict__ g_ptr,
                                                 const int32_t* __restrict__ g_row, const double* __restrict__ g_coef,
                                                 const double* __restrict__ rbv, const double* __restrict__ x,
                                                 const double* __restrict__ q, int with_update, double* gpart,
                                                 int ldg, const PcgState* st) {
  if (halted(st)) return;
  __shared__ double red[6][4];
  const SubInfo s = subs[blockIdx.y];
  if (s.n_modes == 0) return;
  const double alpha = with_update ? st->alpha : 0.0;
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const int64_t nb = (int64_t)s.nt_b * TS;
  const int64_t lo = nb * blockIdx.x / GT_CHUNKS, hi = nb * (blockIdx.x + 1) / GT_CHUNKS;
  for (int64_t k = lo + threadIdx.x; k < hi; k += 256) {
    const int64_t b = s.b_off + k;
    double xv = 0.0;
    for (int e = g_ptr[b]; e < g_ptr[b + 1]; ++e) {
      const int r = g_row[e];
      xv += g_coef[e] * (with_update ? x[r] - alpha * q[r] : x[r]);
    }
    const double* R = rbv + b * 6;
    for (int m = 0; m < 6; ++m) acc[m] += R[m] * xv;
  }
  for (int m = 0; m < 6; ++m) acc[m] = wave_sum(acc[m]);
  if ((threadIdx.x & 63) == 0)
    for (int m = 0; m < 6; ++m) red[m][threadIdx.x >> 6] = acc[m];
  __syncthreads();
  if (threadIdx.x < s.n_modes) {
    const int m = threadIdx.x;
    gpart[(int64_t)blockIdx.x * ldg + s.coarse_off + m] = (red[m][0] + red[m][1]) + (red[m][2] + red[m][3]);
  }
}

// alpha_c = Qinv g with the dense symmetric inverse (leading dim ld); g is the
// sum of its GT_CHUNKS partials, formed once per block in LDS.  One wave per
// row: Qinv is symmetric, so row i is read as the contiguous column i; the
// lanes take columns lane, lane+64, ... and the wave sum fixes the order.
__global__ __launch_bounds__(256) void k_coarse_dense(int nc, int ld, const double* __restrict__ Qi,
                                                      const double* __restrict__ gpart, int ldg,
                                                      double* __restrict__ a, const PcgState* st) {
  if (halted(st)) return;
  extern __shared__ double g[];
  for (int j = threadIdx.x; j < nc; j += 256) {
    double v = 0.0;
#pragma unroll
    for (int c = 0; c < GT_CHUNKS; ++c) v += gpart[(int64_t)c * ldg + j];
    g[j] = v;
  }
  __syncthreads();
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= nc) return;
  const double* q = Qi + (int64_t)row * ld;
  double acc = 0.0;
  int j = lane;
  for (; j + 192 < nc; j += 256) {
    const double q0 = q[j], q1 = q[j + 64], q2 = q[j + 128], q3 = q[j + 192];
    acc += q0 * g[j];
    acc += q1 * g[j + 64];
    acc += q2 * g[j + 128];
    acc += q3 * g[j + 192];
  }
  for (; j < nc; j += 64) acc += q[j] * g[j];
  acc = wave_sum(acc);
  if (lane == 0) a[row] = acc;
}

// (G a)_r contribution of one row entry: Rb[b] . a[coarse block of b's
// subdomain], with co = coarse_off << 3 | n_modes of that subdomain (or -1)
__device__ __forceinline__ double g_alpha(int64_t b, int co, const double* rbv, const double* ac) {
  if (co < 0) return 0.0;
  const int nm = co & 7, off = co >> 3;
  double v = 0.0;
  for (int m = 0; m < nm; ++m) v += rbv[b * 6 + m] * ac[off + m];
  return v;
}

// bco[b] = coarse_off << 3 | n_modes of b's subdomain, or -1 without kernel
__global__ void k_fill_bco(int64_t NB, const int32_t* __restrict__ b_sub, const SubInfo* __restrict__ subs,
                           int32_t* bco) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= NB) return;
  const SubInfo s = subs[b_sub[b]];
  bco[b] = s.n_modes > 0 ? ((s.coarse_off << 3) | s.n_modes) : -1;
}

// rco[r] = (bco of the row's first entry, bco of its second entry or -1)
__global__ void k_fill_rco(int64_t n, const int64_t* __restrict__ b0, const int64_t* __restrict__ b1,
                           const int32_t* __restrict__ bco, int2* rco) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  rco[r] = make_int2(bco[b0[r]], b1[r] >= 0 ? bco[b1[r]] : -1);
}

// Per multiplier row:
//  mode 0: out = x - G ac
//  mode 1: r <- r - alpha q, lam <- lam + alpha s, w <- w - alpha (q - G ac) with
//          ac = Q^{-1} G^T q: the projected residual w = P r follows r (x is r,
//          out is w)
//  mode 2: out = x - G ac, then rho' = w.out, ||w||, beta, convergence (init: first evaluation)
__global__ __launch_bounds__(256) void k_proj_apply(
    int mode, int init, int64_t n, int coarse, const int64_t* __restrict__ b0, const double* __restrict__ c0,
    const int64_t* __restrict__ b1, const double* __restrict__ c1, const int2* __restrict__ rco,
    const double* __restrict__ rbv, const double* __restrict__ ac, double* x,
    const double* __restrict__ q, const double* __restrict__ sv, double* lam, double* out,
    const double* __restrict__ w, double* part, int* ticket, PcgState* st, double* hist,
    const double* __restrict__ apart, int napart) {
  if (st->done) return;
  __shared__ double ra[256], rb[256];
  double alpha = 0.0;
  if (mode == 1) {
    // alpha = rho / s.q from the scatter's block partials, summed in the same
    // order by every block; block 0 records it (or the breakdown)
    double pq = 0.0, unused = 0.0;
    for (int k = threadIdx.x; k < napart; k += 256) pq += apart[k];
    block_reduce2(pq, unused, ra, rb);
    if (!(pq > 0.0)) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->pq = pq;
        st->alpha = 0.0;
        st->status = FETI_EBREAKDOWN;
        st->done = 1;
      }
      return;
    }
    alpha = st->rho / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      st->pq = pq;
      st->alpha = alpha;
    }
  }
  double d1 = 0.0, d2 = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < n; r += (int64_t)gridDim.x * 256) {
    double ga = 0.0;
    if (coarse) {
      const int2 co = rco[r];
      ga = c0[r] * g_alpha(b0[r], co.x, rbv, ac);
      if (co.y >= 0) ga += c1[r] * g_alpha(b1[r], co.y, rbv, ac);
    }
    double o;
    if (mode == 1) {
      const double qr = q[r];
      x[r] -= alpha * qr;
      lam[r] += alpha * sv[r];
      o = out[r] - alpha * (qr - ga);
    } else {
      o = x[r] - ga;
    }
    out[r] = o;
    if (mode == 2) {
      d1 += w[r] * o;
      d2 += w[r] * w[r];
    }
  }
  if (mode != 2) return;
  block_reduce2(d1, d2, ra, rb);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = d1;
    part[2 * blockIdx.x + 1] = d2;
  }
  if (!last_block(ticket)) return;
  double wz = 0.0, ww = 0.0;
  for (int k = threadIdx.x; k < (int)gridDim.x; k += 256) {
    wz += part[2 * k];
    ww += part[2 * k + 1];
  }
  block_reduce2(wz, ww, ra, rb);
  if (threadIdx.x == 0) {
    *ticket = 0;
    const double wn = sqrt(ww);
    if (init) {
      st->rho = wz;
      st->w0 = wn;
      st->wn = wn;
      st->beta = 0.0;
      st->it = 0;
      if (!(wn > st->atol)) { st->done = 1; st->status = FETI_OK; }
    } else {
      const int it = st->it;
      if (hist && it < st->hist_cap) {
        hist[2 * it] = st->alpha;
        hist[2 * it + 1] = wz / st->rho;
      }
      st->beta = wz / st->rho;
      st->rho = wz;
      st->wn = wn;
      st->it = it + 1;
      if (wn <= st->rtol * st->w0 || !(wn > st->atol)) {
        st->done = 1;
        st->status = FETI_OK;
      } else if (st->it >= st->max_it) {
        st->done = 1;
        st->status = FETI_ENOCONV;
      }
    }
  }
}

// Dense column-major copy of a symmetric matrix stored as lower tiles (coarse inverse).
__global__ void k_tiles_to_dense(int nc, int ld, const double* __restrict__ tiles, double* __restrict__ D) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nc * nc) return;
  const int i = (int)(t % nc), j = (int)(t / nc);
  const int hi = i > j ? i : j, lo = i > j ? j : i;
  D[(int64_t)j * ld + i] = tiles[tidx2(hi / TS, lo / TS) * TS2 + (lo % TS) * TS + (hi % TS)];
}

// ---------------------------------------------------------------------------
// FP64 residual of the assembled problem for the mixed-precision refinement:
// the global displacement is restricted to every subdomain (k_restrict), the
// local residual f_i - K_i u_i is formed with the FP64 sparse rows of the
// local stiffness (free columns only: Dirichlet lifting is already in f_i),
// and summed over the subdomain copies afterwards.
// ul[q] = uglob[global DOF of local position q] (0 for padding)
__global__ void k_restrict(int64_t NF, const int32_t* __restrict__ fpos_lnode, const int8_t* __restrict__ fpos_comp,
                           const int64_t* __restrict__ loc_node, const double* __restrict__ uglob,
                           double* __restrict__ ul) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= NF) return;
  const int32_t ln = fpos_lnode[q];
  ul[q] = ln < 0 ? 0.0 : uglob[loc_node[ln] * 3 + fpos_comp[q]];
}

// One row per thread over the slot-major ELL; the column indices and values of
// RES_C slots are loaded before their products, so the loads overlap.  Empty
// slots add an exact zero, so the sum is that of the filled slots in slot order.
constexpr int RES_C = 9;
static_assert(ELLW_Q1 % RES_C == 0 && ELLW_Q2 % RES_C == 0, "whole groups of slots");
__global__ __launch_bounds__(256) void k_local_residual(
    int64_t NF, const int32_t* __restrict__ fpos_lnode, const int8_t* __restrict__ fpos_comp,
    const int64_t* __restrict__ loc_node, const int32_t* __restrict__ f_sub, const SubInfo* __restrict__ subs,
    const int32_t* __restrict__ ell_col, const double* __restrict__ ell_val, int ellw,
    const uint8_t* __restrict__ dmask, const double* __restrict__ ul, const double* __restrict__ f,
    double* __restrict__ r) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NF) return;
  // padding, and constrained DOFs (their residual is a reaction, absorbed by
  // the multipliers; the correction has zero Dirichlet data there)
  if (fpos_lnode[p] < 0 || dmask[loc_node[fpos_lnode[p]] * 3 + fpos_comp[p]]) {
    r[p] = 0.0;
    return;
  }
  const double* u = ul + subs[f_sub[p]].full_off;
  double acc = f ? f[p] : 0.0;   // f NULL: r = -K u
#pragma unroll 1
  for (int k0 = 0; k0 < ellw; k0 += RES_C) {
    int c[RES_C];
    double v[RES_C], x[RES_C];
#pragma unroll
    for (int i = 0; i < RES_C; ++i) c[i] = ell_col[(int64_t)(k0 + i) * NF + p];
    if (c[0] == -1) break;   // the filled slots of a row form a prefix: the rest add 0
#pragma unroll
    for (int i = 0; i < RES_C; ++i) {
      v[i] = c[i] >= 0 ? ell_val[(int64_t)(k0 + i) * NF + p] : 0.0;
      x[i] = c[i] >= 0 ? u[c[i]] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < RES_C; ++i) acc -= v[i] * x[i];
  }
  r[p] = acc;
}

// Assembled vector back to the subdomains, split evenly over the copies of each
// node: r_p = rg[g(p)] / (number of subdomains holding g).  Padding and
// constrained DOFs get 0.  Used for the loads of a refinement correction, whose
// interface forces then scale with the assembled residual.
__global__ void k_distribute(int64_t NF, const int32_t* __restrict__ fpos_lnode, const int8_t* __restrict__ fpos_comp,
                             const int64_t* __restrict__ loc_node, const int32_t* __restrict__ uc_ptr,
                             const uint8_t* __restrict__ dmask, const double* __restrict__ rg, double* __restrict__ r) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NF) return;
  if (fpos_lnode[p] < 0) {
    r[p] = 0.0;
    return;
  }
  const int64_t g = loc_node[fpos_lnode[p]] * 3 + fpos_comp[p];
  const int n = uc_ptr[g + 1] - uc_ptr[g];
  r[p] = (dmask[g] || n == 0) ? 0.0 : rg[g] / n;
}

// ---------------------------------------------------------------------------
// Local generalised inverse z = K^+ g on the full local vector of each
// subdomain, by the block formula of the interior-first elimination:
//   w_I = L_II^{-1} g_I,  w_b = g_b - L_bI w_I,  z_b = X w_b,
//   t_I = w_I - L_bI^T z_b,  z_I = L_II^{-T} t_I.
// The interior solves are k_kp_band; the two products with L_bI are
// k_kp_tiles (mode 1, one workgroup per interface tile row and subdomain) and
// k_kp_cols (mode 2, one per interior tile column); each workgroup reduces
// once at the end.  Both skip the factor tiles left of a tile row's envelope
// (env: first nonzero tile column per tile row), which are zero.
//   mode 1: yb_I = base_b - sum_{J<nt_i} L(nt_i+I, J) x_J   (rows I < nt_b)
//   mode 2: y_I = base_I - sum_{J<nt_b} L(nt_i+J, I)^T xb_J (cols I < nt_i)
template <typename T>
__global__ __launch_bounds__(256) void k_kp_tiles(int mode, const SubInfo* __restrict__ subs,
                                                  const int32_t* __restrict__ env,
                                                  const T* __restrict__ arena,
                                                  const double* __restrict__ x, const double* __restrict__ xb,
                                                  const double* __restrict__ base, double* y, double* yb) {
  __shared__ double red[4][TS];
  const SubInfo s = subs[blockIdx.y];
  const int I = blockIdx.x;
  if (I >= s.nt_b) return;
  const int tid = threadIdx.x;
  const int a = tid & 63, q = tid >> 6;   // output row, quarter of the reduction index
  double acc = 0.0;
  // tiles in pairs: both tiles' loads are in flight before the products
  // (same products, same order)
  int J = min(env[s.env_off + s.nt_i + I], s.nt_i);
  for (; J + 1 < s.nt_i; J += 2) {
    const T* t0 = arena + s.tile_off + tidx2(s.nt_i + I, J) * TS2;
    const T* t1 = arena + s.tile_off + tidx2(s.nt_i + I, J + 1) * TS2;
    T v0[16], v1[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v0[k] = t0[(16 * q + k) * TS + a];
#pragma unroll
    for (int k = 0; k < 16; ++k) v1[k] = t1[(16 * q + k) * TS + a];
    const double* x0 = x + s.full_off + (int64_t)J * TS;
    const double* x1 = x0 + TS;
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += (double)v0[k] * x0[16 * q + k];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += (double)v1[k] * x1[16 * q + k];
  }
  if (J < s.nt_i) {
    const T* tile = arena + s.tile_off + tidx2(s.nt_i + I, J) * TS2;
    const double* xs = x + s.full_off + (int64_t)J * TS;
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += (double)tile[(16 * q + k) * TS + a] * xs[16 * q + k];
  }
  red[q][a] = acc;
  __syncthreads();
  if (tid < TS) {
    const double v = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    yb[s.b_off + (int64_t)I * TS + tid] = base[s.full_off + (int64_t)(s.nt_i + I) * TS + tid] - v;
  }
}

// Mode 2 with coalesced loads: column tile I of L_bI is read
// tile row by tile row, each tile loaded with consecutive threads on
// consecutive elements and transposed through LDS (a column-wise read of a
// column-major tile makes every load touch 64 cache lines); the next tile's
// loads are in flight during this tile's products.
template <typename T>
__global__ __launch_bounds__(256) void k_kp_cols(const SubInfo* __restrict__ subs, const int32_t* __restrict__ env,
                                                 const T* __restrict__ arena, const double* __restrict__ xb,
                                                 const double* __restrict__ base, double* y) {
  __shared__ double tl[TS * (TS + 1)];   // tl[c * (TS + 1) + r] = L(r, c)
  __shared__ double red[4][TS];
  const SubInfo s = subs[blockIdx.y];
  const int I = blockIdx.x;
  if (I >= s.nt_i) return;
  const int tid = threadIdx.x;
  const int a = tid & 63, q = tid >> 6;   // column of the tile, quarter of its rows
  const int32_t* ev = env + s.env_off + s.nt_i;
  const T* Lb = arena + s.tile_off;
  int J = 0;
  while (J < s.nt_b && ev[J] > I) ++J;
  constexpr int N = TS2 / 256;
  double v[N];
  if (J < s.nt_b) {
    const T* tile = Lb + tidx2(s.nt_i + J, I) * TS2;
#pragma unroll
    for (int u = 0; u < N; ++u) v[u] = (double)tile[tid + 256 * u];
  }
  double acc = 0.0;
  while (J < s.nt_b) {
    int Jn = J + 1;
    while (Jn < s.nt_b && ev[Jn] > I) ++Jn;
    __syncthreads();   // the previous tile's reads of tl are done
#pragma unroll
    for (int u = 0; u < N; ++u) {
      const int e = tid + 256 * u;
      tl[(e >> 6) * (TS + 1) + (e & 63)] = v[u];
    }
    __syncthreads();
    if (Jn < s.nt_b) {
      const T* tile = Lb + tidx2(s.nt_i + Jn, I) * TS2;
#pragma unroll
      for (int u = 0; u < N; ++u) v[u] = (double)tile[tid + 256 * u];
    }
    const double* xs = xb + s.b_off + (int64_t)J * TS;
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += tl[a * (TS + 1) + 16 * q + k] * xs[16 * q + k];
    J = Jn;
  }
  red[q][a] = acc;
  __syncthreads();
  if (tid < TS) {
    const double r = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    y[s.full_off + (int64_t)I * TS + tid] = base[s.full_off + (int64_t)I * TS + tid] - r;
  }
}

// Interior solves with the interior factor itself, one workgroup of 1024
// threads per subdomain, tile by tile (no explicit inverse: the interior block
// is banded, so each step reads the few factor tiles inside the envelope):
//   mode 0: y = L_II^{-1} x   (forward: y_I = Linv_II (x_I - sum_{env(I)<=J<I} L_IJ y_J))
//   mode 3: y = L_II^{-T} x   (backward: y_I = Linv_II^T (x_I - sum_{J>I, env(J)<=I} L_JI^T y_J))
// x and y are full-space local vectors (interior tile rows only).  Each step
// loads its Linv_II values with its band tiles (they do not depend on the
// step's right-hand side), so a step waits for memory once.  The solved
// segments are kept in LDS (LDSY; else read back from y after a barrier).
constexpr int BAND_Q = 16;   // column (forward) or row (backward) groups of four per tile
template <typename T, bool LDSY>
__global__ __launch_bounds__(1024) void k_kp_band(int mode, const SubInfo* __restrict__ subs,
                                                  const int32_t* __restrict__ env, const T* __restrict__ arena,
                                                  const T* __restrict__ linv, const double* __restrict__ x,
                                                  double* y) {
  extern __shared__ double ylds[];   // nt_i * TS solved values (LDSY)
  __shared__ double red[BAND_Q][TS];
  __shared__ double rv[TS];
  const SubInfo s = subs[blockIdx.x];
  const int nti = s.nt_i, tid = threadIdx.x;
  const bool fwd = mode == 0;
  // forward: thread (a = row, q = columns 4q..4q+3); backward: (a = column, q = rows 4q..4q+3)
  const int a = fwd ? (tid & 63) : (tid >> 4);
  const int q = fwd ? (tid >> 6) : (tid & 15);
  const T* Lb = arena + s.tile_off;
  double* yg = y + s.full_off;
  const double* yr = LDSY ? ylds : yg;
  for (int step = 0; step < nti; ++step) {
    const int I = fwd ? step : nti - 1 - step;
    const T* Li = linv + s.linv_off + (int64_t)I * TS2;
    T li[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) li[k] = fwd ? Li[(4 * q + k) * TS + a] : Li[a * TS + 4 * q + k];
    double acc = 0.0;
    if (fwd) {
      for (int J = env[s.env_off + I]; J < I; ++J) {
        const T* tile = Lb + tidx2(I, J) * TS2;
#pragma unroll
        for (int k = 0; k < 4; ++k) acc += (double)tile[(4 * q + k) * TS + a] * yr[J * TS + 4 * q + k];
      }
    } else {
      for (int J = I + 1; J < nti; ++J) {
        if (env[s.env_off + J] > I) continue;
        const T* tile = Lb + tidx2(J, I) * TS2;
#pragma unroll
        for (int k = 0; k < 4; ++k) acc += (double)tile[a * TS + 4 * q + k] * yr[J * TS + 4 * q + k];
      }
    }
    red[q][a] = acc;
    __syncthreads();
    if (tid < TS) {
      double sum = 0.0;
#pragma unroll
      for (int g = 0; g < BAND_Q; ++g) sum += red[g][tid];
      rv[tid] = x[s.full_off + (int64_t)I * TS + tid] - sum;
    }
    __syncthreads();
    double acc2 = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) acc2 += (double)li[k] * rv[4 * q + k];
    red[q][a] = acc2;
    __syncthreads();
    if (tid < TS) {
      double v = 0.0;
#pragma unroll
      for (int g = 0; g < BAND_Q; ++g) v += red[g][tid];
      yg[(int64_t)I * TS + tid] = v;
      if (LDSY) ylds[I * TS + tid] = v;
    }
    // the segment is visible for the next steps; red is free again
    __syncthreads();
  }
}

// full[b2full[k]] = b[k]
__global__ void k_set_b2f(int64_t NB, const int64_t* __restrict__ b2full, const double* __restrict__ b,
                          double* full) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < NB) full[b2full[k]] = b[k];
}

// ---------------------------------------------------------------------------
static inline dim3 grid1(int64_t n, int bs = 256) { return dim3((unsigned)((n + bs - 1) / bs)); }

void pcg_gather(const DevIdx& d, int weighted, const double* v, double* xb, const PcgState* st, hipStream_t s) {
  if (d.NB) hipLaunchKernelGGL(k_gather, grid1(d.NB), dim3(256), 0, s, d.NB, d.g_ptr, d.g_row, d.g_coef, d.r_w, weighted, v, xb, st);
}
void pcg_scatter(const DevIdx& d, int weighted, const double* y, const double* base, double sgn, double* out,
                 const PcgState* st, hipStream_t s) {
  if (d.n_lam) hipLaunchKernelGGL(k_scatter, grid1(d.n_lam), dim3(256), 0, s, d.n_lam, d.r_b0, d.r_c0, d.r_b1, d.r_c1, d.r_w, weighted, y, base, sgn, out, st);
}
void pcg_dot(int64_t n, const double* a, const double* b, const double* c, const double* d, double* part,
             const PcgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partial, dim3(DOT_PARTS), dim3(256), 0, s, n, a, b, c, d, part, st);
}
void pcg_coarse_gt(int n_sub, const SubInfo* subs, const double* rb, const double* xb, double* g,
                   const PcgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_gt, dim3(n_sub), dim3(256), 0, s, subs, rb, xb, g, st);
}
void pcg_coarse_gt_full(int n_sub, const SubInfo* subs, const double* rf, const double* xf, double* g,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_coarse_gt_full, dim3(n_sub), dim3(256), 0, s, subs, rf, xf, g);
}
void pcg_coarse_expand(const DevIdx& d, const SubInfo* subs, const double* rb, const double* alpha, double* vb,
                       const PcgState* st, hipStream_t s) {
  if (d.NB) hipLaunchKernelGGL(k_coarse_expand, grid1(d.NB), dim3(256), 0, s, d.NB, d.b_sub, subs, rb, alpha, vb, st);
}
void pcg_add_modes(int64_t NF, const int32_t* f_sub, const SubInfo* subs, const double* rf, const double* gamma,
                   double* u, hipStream_t s) {
  hipLaunchKernelGGL(k_add_modes, grid1(NF), dim3(256), 0, s, NF, f_sub, subs, rf, gamma, u);
}
void pcg_lumped(const DevIdx& d, int w_bb, const int32_t* bb_col, const double* bb_val, const double* xb,
                double* yb, const PcgState* st, hipStream_t s) {
  if (d.NB) hipLaunchKernelGGL(k_lumped, grid1(d.NB * LUMP_LANES), dim3(256), 0, s, d.NB, w_bb, bb_col, bb_val, xb, yb, st);
}
void lumped_fill(const DevIdx& d, int w_bb, const int32_t* bb_slot, const double* ell_val, double* bb_val,
                 hipStream_t s) {
  if (d.NB && w_bb) hipLaunchKernelGGL(k_bb_fill, grid1(d.NB * w_bb), dim3(256), 0, s, d.NB, d.NF, w_bb, bb_slot, d.b2full, ell_val, bb_val);
}
void vec_bvec(const DevIdx& d, const double* dvals, double* out, hipStream_t s) {
  if (d.n_lam) hipLaunchKernelGGL(k_bvec, grid1(d.n_lam), dim3(256), 0, s, d.n_lam, d.r_gdof, dvals, out);
}
void vec_global(int64_t n_dof, const int32_t* uc_ptr, const int64_t* uc_idx, const double* ufull,
                const uint8_t* dmask, const double* dvals, double* out, int sum_mode, hipStream_t s) {
  hipLaunchKernelGGL(k_global, grid1(n_dof), dim3(256), 0, s, n_dof, uc_ptr, uc_idx, ufull, dmask, dvals, out, sum_mode);
}
void vec_dirinc(int64_t n_dof, const uint8_t* dmask, const double* dirval, double tau, const double* U,
                double* dvals, hipStream_t s) {
  hipLaunchKernelGGL(k_dirinc, grid1(n_dof), dim3(256), 0, s, n_dof, dmask, dirval, tau, U, dvals);
}
void vec_multi_dot(int64_t n, const double* V, int64_t ld, int k, const double* w, double* part, double* out,
                   hipStream_t s) {
  if (k <= 0) return;
  hipLaunchKernelGGL(k_multi_dot, dim3(DOT_PARTS, k), dim3(256), 0, s, n, V, ld, w, part);
  hipLaunchKernelGGL(k_multi_finish, dim3(k), dim3(256), 0, s, part, out);
}
void vec_multi_axpy(int64_t n, const double* V, int64_t ld, int k, const double* h, double* y, hipStream_t s) {
  if (n > 0 && k > 0) hipLaunchKernelGGL(k_multi_axpy, grid1(n), dim3(256), 0, s, n, V, ld, k, h, y);
}
void vec_axpby(int64_t n, double a, const double* x, double b, double* y, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_axpby, grid1(n), dim3(256), 0, s, n, a, x, b, y);
}
void vec_fill(int64_t n, double v, double* y, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_fill, grid1(n), dim3(256), 0, s, n, v, y);
}
void pcg_init_state(PcgState* st, double rtol, double atol, int max_it, int hist_cap, hipStream_t s) {
  hipLaunchKernelGGL(k_init_state, dim3(1), dim3(1), 0, s, st, rtol, atol, max_it, hist_cap);
}
void local_residual(int64_t NF, const int32_t* fpos_lnode, const int8_t* fpos_comp, const int64_t* loc_node,
                    const int32_t* f_sub, const SubInfo* subs, const int32_t* ell_col, const double* ell_val,
                    int ellw, const uint8_t* dmask, const double* uglob, double* ul, const double* f, double* r,
                    hipStream_t s) {
  if (!NF) return;
  hipLaunchKernelGGL(k_restrict, grid1(NF), dim3(256), 0, s, NF, fpos_lnode, fpos_comp, loc_node, uglob, ul);
  hipLaunchKernelGGL(k_local_residual, grid1(NF), dim3(256), 0, s, NF, fpos_lnode, fpos_comp, loc_node, f_sub, subs,
                     ell_col, ell_val, ellw, dmask, ul, f, r);
}
void vec_distribute(int64_t NF, const int32_t* fpos_lnode, const int8_t* fpos_comp, const int64_t* loc_node,
                    const int32_t* uc_ptr, const uint8_t* dmask, const double* rg, double* r, hipStream_t s) {
  hipLaunchKernelGGL(k_distribute, grid1(NF), dim3(256), 0, s, NF, fpos_lnode, fpos_comp, loc_node, uc_ptr, dmask, rg, r);
}
// Row blocks of the fused per-multiplier kernels: up to FUSE_BLOCKS (eight
// per compute unit, so that the gathers of a row overlap), fewer for short
// vectors.  The block partial sums of their reductions are then summed in a
// fixed order.
int fuse_rows(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>(FUSE_BLOCKS, (n + 255) / 256)); }
void pcg_gather_s(const DevIdx& d, const double* z, const double* sv, double* xb, const PcgState* st,
                  hipStream_t s) {
  if (d.NB) hipLaunchKernelGGL(k_gather_s, grid1(d.NB), dim3(256), 0, s, d.NB, d.g_ptr, d.g_row, d.g_coef, z, sv, xb, st);
}
void pcg_scatter_dot_alpha_gt(const DevIdx& d, int n_sub, int coarse, const SubInfo* subs, const double* rbv,
                              const double* yb, const double* z, double* sv, double* q, double* part,
                              PcgState* st, double* gpart, int ldg, hipStream_t s) {
  const int nrow = fuse_rows(d.n_lam);
  const int nb = nrow + (coarse ? GT_CHUNKS * n_sub : 0);
  hipLaunchKernelGGL(k_scatter_dot_alpha_gt, dim3(nb), dim3(256), 0, s, d.n_lam, nrow, d.r_b0, d.r_c0, d.r_b1,
                     d.r_c1, yb, z, sv, q, part, st, subs, d.c_ptr, d.c_col, d.c_v0, rbv, gpart, ldg);
}
void pcg_scatter_w_gt(const DevIdx& d, int n_sub, int coarse, const SubInfo* subs, const double* rbv,
                      const double* y, double* out, const PcgState* st, double* gpart, int ldg, hipStream_t s) {
  const int nrow = fuse_rows(d.n_lam);
  const int nb = nrow + (coarse ? GT_CHUNKS * n_sub : 0);
  if (nb) hipLaunchKernelGGL(k_scatter_w_gt, dim3(nb), dim3(256), 0, s, d.n_lam, nrow, d.r_b0, d.r_c0, d.r_b1, d.r_c1,
                             d.r_w, y, out, st, subs, d.c_ptr, d.c_col, d.c_v1, rbv, gpart, ldg);
}
void pcg_proj_gt(int n_sub, const SubInfo* subs, const DevIdx& d, const double* rbv, const double* x,
                 const double* q, int with_update, double* gpart, int ldg, const PcgState* st, hipStream_t s) {
  hipLaunchKernelGGL(k_proj_gt, dim3(GT_CHUNKS, n_sub), dim3(256), 0, s, subs, d.g_ptr, d.g_row, d.g_coef, rbv, x, q, with_update, gpart, ldg, st);
}
void pcg_coarse_dense(int nc, int ld, const double* Qi, const double* gpart, int ldg, double* a, const PcgState* st,
                      hipStream_t s) {
  if (nc) hipLaunchKernelGGL(k_coarse_dense, dim3((nc + 3) / 4), dim3(256), nc * sizeof(double), s, nc, ld, Qi, gpart, ldg, a, st);
}
void pcg_proj_apply(int mode, int init, const DevIdx& d, int coarse, const int2* rco, const double* rbv,
                    const double* ac, double* x, const double* q, const double* sv, double* lam, double* out,
                    const double* w, double* part, int* ticket, PcgState* st, double* hist, hipStream_t s,
                    const double* apart) {
  const int nrow = fuse_rows(d.n_lam);
  hipLaunchKernelGGL(k_proj_apply, dim3(nrow), dim3(256), 0, s, mode, init, d.n_lam, coarse, d.r_b0, d.r_c0, d.r_b1, d.r_c1, rco, rbv, ac, x, q, sv, lam, out, w, part, ticket, st, hist, apart, nrow);
}
void fill_bco(const DevIdx& d, const SubInfo* subs, int32_t* bco, int2* rco, hipStream_t s) {
  if (d.NB) hipLaunchKernelGGL(k_fill_bco, grid1(d.NB), dim3(256), 0, s, d.NB, d.b_sub, subs, bco);
  if (d.n_lam) hipLaunchKernelGGL(k_fill_rco, grid1(d.n_lam), dim3(256), 0, s, d.n_lam, d.r_b0, d.r_b1, bco, rco);
}
void coarse_to_dense(int nc, int ld, const double* tiles, double* D, hipStream_t s) {
  if (nc) hipLaunchKernelGGL(k_tiles_to_dense, grid1((int64_t)nc * nc), dim3(256), 0, s, nc, ld, tiles, D);
}

template <typename T>
void local_kp_tiles(int mode, int n_sub, int max_rows, const SubInfo* subs, const int32_t* env, const T* arena,
                    const double* x, const double* xb, const double* base, double* y, double* yb, hipStream_t s) {
  if (max_rows <= 0) return;
  if (mode == 2)
    hipLaunchKernelGGL(k_kp_cols<T>, dim3(max_rows, n_sub), dim3(256), 0, s, subs, env, arena, xb, base, y);
  else
    hipLaunchKernelGGL(k_kp_tiles<T>, dim3(max_rows, n_sub), dim3(256), 0, s, mode, subs, env, arena, x, xb, base,
                       y, yb);
}
template void local_kp_tiles<double>(int, int, int, const SubInfo*, const int32_t*, const double*, const double*,
                                     const double*, const double*, double*, double*, hipStream_t);
template void local_kp_tiles<float>(int, int, int, const SubInfo*, const int32_t*, const float*, const double*,
                                    const double*, const double*, double*, double*, hipStream_t);
template <typename T>
void local_kp_band(int mode, int n_sub, int max_nt_i, const SubInfo* subs, const int32_t* env, const T* arena,
                   const T* linv, const double* x, double* y, hipStream_t s) {
  if (n_sub <= 0 || max_nt_i <= 0) return;
  const size_t ybytes = (size_t)max_nt_i * TS * sizeof(double);
  if (ybytes <= 48 * 1024)
    hipLaunchKernelGGL((k_kp_band<T, true>), dim3(n_sub), dim3(1024), ybytes, s, mode, subs, env, arena, linv, x, y);
  else
    hipLaunchKernelGGL((k_kp_band<T, false>), dim3(n_sub), dim3(1024), 0, s, mode, subs, env, arena, linv, x, y);
}
template void local_kp_band<double>(int, int, int, const SubInfo*, const int32_t*, const double*, const double*,
                                    const double*, double*, hipStream_t);
template void local_kp_band<float>(int, int, int, const SubInfo*, const int32_t*, const float*, const float*,
                                   const double*, double*, hipStream_t);
void vec_set_b2f(const DevIdx& d, const double* b, double* full, hipStream_t s) {
  if (d.NB) hipLaunchKernelGGL(k_set_b2f, grid1(d.NB), dim3(256), 0, s, d.NB, d.b2full, b, full);
}

// ---------------------------------------------------------------------------
// Scratch of feti_solve_noalloc: one static array per device, holding the
// dual iteration's scratch set (PcgScratch) for callers that cannot allocate.
// Host code never passes the array's name to a kernel: its device address on
// each device comes from hipGetSymbolAddress, once per device, and only that
// address is used.  Every call on a device shares the array; calls that
// overlap on one device race.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

void* noalloc_scratch(int device) {
  constexpr int kMaxDev = 64;
  static std::mutex mu;
  static void* addr[kMaxDev] = {};
  if (device < 0 || device >= kMaxDev) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device) {
      (void)hipGetLastError();
      return nullptr;   // the device must be current
    }
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    addr[device] = ptr;
  }
  return addr[device];
}

PcgScratch noalloc_layout(void* base, int n_sub) {
  auto* b = static_cast<unsigned char*>(base);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* q = b + off;
    off += (bytes + 255) / 256 * 256;
    return q;
  };
  PcgScratch sc;
  sc.state = reinterpret_cast<PcgState*>(take(sizeof(PcgState)));
  sc.ticket = reinterpret_cast<int*>(take(4 * sizeof(int)));
  sc.fpart = reinterpret_cast<double*>(take(2 * FUSE_BLOCKS * sizeof(double)));
  sc.apart = reinterpret_cast<double*>(take(FUSE_BLOCKS * sizeof(double)));
  sc.dots = reinterpret_cast<double*>(take(2 * DOT_PARTS * sizeof(double)));
  sc.gpart = reinterpret_cast<double*>(take((size_t)4 * 6 * std::max(n_sub, 1) * sizeof(double)));
  sc.hist = reinterpret_cast<double*>(take((size_t)2 * kNoAllocMaxIt * sizeof(double)));
  sc.hist_cap = kNoAllocMaxIt;
  return sc;
}
static_assert(sizeof(PcgState) <= 256, "state slot");
static_assert(256 + 256 + 2 * FUSE_BLOCKS * 8 + FUSE_BLOCKS * 8 + 2 * DOT_PARTS * 8 + (size_t)4 * 6 * kMaxSub * 8 + 256 +
                  (size_t)2 * kNoAllocMaxIt * 8 <= kNoAllocScratchBytes,
              "the largest scratch set fits the static array");

}  // namespace feti
