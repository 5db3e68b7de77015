// Packed-symmetric tile GEMV y = M x over the interface blocks of all
// subdomains: the per-iteration action of the local interface inverses in the
// dual operator F = sum_i B_i K_i^+ B_i^T (paper section 4.3, eq.
// (classicalFetiF)), and the Dirichlet preconditioner's Schur complements
// (section 4.4, eq. (DirichletVK)).  HBM-bound: every stored tile is read once
// per launch.
#include "feti_impl.h"
#include "k_pcg.h"

namespace feti {

constexpr int LDV = TS + 1;

__device__ __forceinline__ bool halted(const PcgState* st) { return st != nullptr && st->done != 0; }
__device__ __forceinline__ int64_t tidx2(int i, int j) { return (int64_t)i * (i + 1) / 2 + j; }
static inline dim3 grid1(int64_t n, int bs = 256) { return dim3((unsigned)((n + bs - 1) / bs)); }

// Symmetric tile matrix-vector product, phase 1: every stored lower tile
// (I, J) of a symmetric matrix contributes M_IJ x_J to block row I and,
// off the diagonal, M_IJ^T x_I to block row J.  Partial sums go to
// part[part_off + (row*nt + col)*TS + .] and are summed in order afterwards.
//
// Persistent and software-pipelined: a workgroup walks the tasks
// blockIdx.x, blockIdx.x + gridDim.x, ... (gridDim.x a multiple of 8, so a
// workgroup stays on the XCD the task order was laid out for) and issues
// the 16-byte loads of its next tile before it computes the current one from
// LDS, so every resident workgroup keeps a tile of HBM reads in flight.
template <typename T>
struct SymvTile {
  static constexpr int W = 16 / sizeof(T);          // elements per 16-byte load
  static constexpr int NV = TS2 / (256 * W);         // loads per thread per tile
  using V = __attribute__((ext_vector_type(W))) T;
};

// Rows of tile (t.i, t.j) that take part: rows beyond the last real DOF of
// the block are not read (the padding of the last tile row meets zero inputs
// and its outputs are dropped; with iface_only, in the dual operator, so do
// trailing-block DOFs without multipliers), nor is the upper half of a
// diagonal tile (the lower half is mirrored).
__device__ __forceinline__ int symv_rows(const Task& t, const SubInfo& s, int iface_only) {
  const int nreal = iface_only ? s.n_if : s.n_b;
  return t.i == s.nt_b - 1 ? nreal - TS * (s.nt_b - 1) : TS;
}

// Issue the 16-byte loads of a tile (W consecutive rows of one column each);
// a load none of whose rows takes part is skipped.  The values are masked
// when they are stored to LDS, so the loads stay in flight meanwhile.
template <typename T>
__device__ __forceinline__ void symv_fetch(const Task& t, const SubInfo& s, const T* __restrict__ M, int iface_only,
                                           typename SymvTile<T>::V (&v)[SymvTile<T>::NV]) {
  using ST = SymvTile<T>;
  using V = typename ST::V;
  const int rows = symv_rows(t, s, iface_only);
  const V* tile = reinterpret_cast<const V*>(M + s.x_off + tidx2(t.i, t.j) * TS2);
  const bool diag = t.i == t.j;
#pragma unroll
  for (int u = 0; u < ST::NV; ++u) {
    const int e0 = (threadIdx.x + 256 * u) * ST::W;
    const int col = e0 >> 6, row0 = e0 & 63;
    const int lo = diag ? (row0 > col ? row0 : col) : row0;   // first row that takes part
    v[u] = (lo < rows && lo < row0 + ST::W) ? tile[threadIdx.x + 256 * u] : V{};
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_symv_tiles(const Task* __restrict__ tasks, int count,
                                                    const SubInfo* __restrict__ subs,
                                                    const T* __restrict__ M,
                                                    const double* __restrict__ xb, double* part,
                                                    const PcgState* st, int iface_only) {
  using ST = SymvTile<T>;
  if (halted(st)) return;
  __shared__ T sM[TS * LDV];
  __shared__ double xI[TS], xJ[TS];
  __shared__ double red[4][TS], red2[4][TS];
  const int tid = threadIdx.x;
  int task = blockIdx.x;
  if (task >= count) return;
  Task t = tasks[task];
  SubInfo s = subs[t.sub];
  typename ST::V v[ST::NV];
  double xi = 0.0, xj = 0.0;   // x_I, x_J of the tile in flight (threads < TS)
  symv_fetch<T>(t, s, M, iface_only, v);
  if (tid < TS) {
    xi = xb[s.b_off + (int64_t)t.i * TS + tid];
    xj = xb[s.b_off + (int64_t)t.j * TS + tid];
  }
  for (; task < count; task += gridDim.x) {
    const Task tc = t;
    const SubInfo sc = s;
    const int next = task + gridDim.x;
    if (next < count) {   // descriptors of the next tile (scalar loads)
      t = tasks[next];
      s = subs[t.sub];
    }
    __syncthreads();      // the previous tile's readers of sM, xI, xJ are done
    {
      const int rows = symv_rows(tc, sc, iface_only);
      const bool diag = tc.i == tc.j;
#pragma unroll
      for (int u = 0; u < ST::NV; ++u) {
        const int e0 = (tid + 256 * u) * ST::W;
        const int col = e0 >> 6;
#pragma unroll
        for (int w = 0; w < ST::W; ++w) {
          const int row = (e0 & 63) + w;
          const bool need = row < rows && (!diag || row >= col);
          sM[col * LDV + row] = need ? v[u][w] : T(0);
        }
      }
    }
    if (tid < TS) {
      xI[tid] = xi;
      xJ[tid] = xj;
    }
    __syncthreads();
    if (next < count) {   // in flight during the compute below
      symv_fetch<T>(t, s, M, iface_only, v);
      if (tid < TS) {
        xi = xb[s.b_off + (int64_t)t.i * TS + tid];
        xj = xb[s.b_off + (int64_t)t.j * TS + tid];
      }
    }
    const int a = tid & 63, q = tid >> 6;
    double s1 = 0.0, s2 = 0.0;
    if (tc.i != tc.j) {
#pragma unroll 4
      for (int k = 0; k < 16; ++k) {
        const int c = 16 * q + k;
        s1 += (double)sM[c * LDV + a] * xJ[c];     // (M x_J)[a]
        s2 += (double)sM[a * LDV + c] * xI[c];     // (M^T x_I)[a], column a row c
      }
    } else {
      // diagonal tile: only its lower triangle is meaningful; mirror it
#pragma unroll 4
      for (int k = 0; k < 16; ++k) {
        const int c = 16 * q + k;
        const int hi = a > c ? a : c, lo = a > c ? c : a;
        s1 += (double)sM[lo * LDV + hi] * xJ[c];
      }
    }
    red[q][a] = s1;
    red2[q][a] = s2;
    __syncthreads();
    if (tid < TS) {
      const int nt = sc.nt_b;
      part[sc.part_off + ((int64_t)tc.i * nt + tc.j) * TS + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
      if (tc.i != tc.j)
        part[sc.part_off + ((int64_t)tc.j * nt + tc.i) * TS + tid] =
            red2[0][tid] + red2[1][tid] + red2[2][tid] + red2[3][tid];
    }
  }
}

// Phase 2: yb[b] = sum_J part[row I of b][J] in order (loads of a chunk of
// eight partials in flight together).
__global__ void k_symv_reduce(int64_t NB, const int32_t* __restrict__ b_sub, const SubInfo* __restrict__ subs,
                              const double* __restrict__ part, double* __restrict__ yb, const PcgState* st) {
  if (halted(st)) return;
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= NB) return;
  const SubInfo s = subs[b_sub[b]];
  const int64_t loc = b - s.b_off;
  const int I = (int)(loc / TS), r = (int)(loc % TS);
  const double* p = part + s.part_off + (int64_t)I * s.nt_b * TS + r;
  const int nt = s.nt_b;
  double acc = 0.0;
  for (int J0 = 0; J0 < nt; J0 += 8) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = J0 + k < nt ? p[(int64_t)(J0 + k) * TS] : 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) acc += v[k];
  }
  yb[b] = acc;
}

template <typename T>
void pcg_symv(const Task* tasks, int count, const SubInfo* subs, const T* M, const double* xb, double* part,
              int64_t NB, const int32_t* b_sub, double* yb, const PcgState* st, hipStream_t s, int iface_only) {
  if (count <= 0) return;
  // resident workgroups: four per CU (LDS), 256 CUs
  constexpr int kResident = 4 * 256;
  const int grid = count < kResident ? count : kResident;
  hipLaunchKernelGGL(k_symv_tiles<T>, dim3(grid), dim3(256), 0, s, tasks, count, subs, M, xb, part, st, iface_only);
  if (yb) hipLaunchKernelGGL(k_symv_reduce, grid1(NB), dim3(256), 0, s, NB, b_sub, subs, (const double*)part, yb, st);
}
template void pcg_symv<double>(const Task*, int, const SubInfo*, const double*, const double*, double*, int64_t, const int32_t*, double*, const PcgState*, hipStream_t, int);
template void pcg_symv<float>(const Task*, int, const SubInfo*, const float*, const double*, double*, int64_t, const int32_t*, double*, const PcgState*, hipStream_t, int);

}  // namespace feti
