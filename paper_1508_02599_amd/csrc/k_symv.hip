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
__host__ __device__ __forceinline__ int64_t tidx2(int i, int j) { return (int64_t)i * (i + 1) / 2 + j; }
static inline dim3 grid1(int64_t n, int bs = 256) { return dim3((unsigned)((n + bs - 1) / bs)); }

// Symmetric tile matrix-vector product, phase 1: every stored lower tile
// (I, J) of a symmetric matrix contributes M_IJ x_J to block row I and,
// off the diagonal, M_IJ^T x_I to block row J.  Partial sums go to
// part[part_off + (row*nt + col)*TS + .] and are summed in order afterwards.
template <typename T>
__global__ __launch_bounds__(256) void k_symv_tiles(const Task* __restrict__ tasks,
                                                    const SubInfo* __restrict__ subs,
                                                    const T* __restrict__ M,
                                                    const double* __restrict__ xb, double* part,
                                                    const PcgState* st, int iface_only) {
  if (halted(st)) return;
  __shared__ T sM[TS * LDV];
  __shared__ double xI[TS], xJ[TS];
  __shared__ double red[4][TS], red2[4][TS];
  const Task t = tasks[blockIdx.x];
  const SubInfo s = subs[t.sub];
  const T* tile = M + s.x_off + tidx2(t.i, t.j) * TS2;
  const int tid = threadIdx.x;
  {
    // only the stored entries that take part are read: rows beyond the last
    // real DOF of the block (the padding of the last tile row meets zero
    // inputs and its outputs are dropped; with iface_only, in the dual
    // operator, so do trailing-block DOFs without multipliers) and the upper
    // half of a diagonal tile (the lower half is mirrored) are not fetched
    const int nreal = iface_only ? s.n_if : s.n_b;
    const int rows = t.i == s.nt_b - 1 ? nreal - TS * (s.nt_b - 1) : TS;
    const int row = tid & 63;
    T v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int col = (tid >> 6) + 4 * i;
      const bool need = row < rows && (t.i != t.j || row >= col);
      v[i] = need ? tile[tid + 256 * i] : T(0);   // all loads in flight first
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int e = tid + 256 * i;
      sM[(e >> 6) * LDV + (e & 63)] = v[i];
    }
  }
  if (tid < TS) {
    xI[tid] = xb[s.b_off + (int64_t)t.i * TS + tid];
    xJ[tid] = xb[s.b_off + (int64_t)t.j * TS + tid];
  }
  __syncthreads();
  const int a = tid & 63, q = tid >> 6;
  double s1 = 0.0, s2 = 0.0;
  if (t.i != t.j) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int c = 16 * q + k;
      s1 += (double)sM[c * LDV + a] * xJ[c];     // (M x_J)[a]
      s2 += (double)sM[a * LDV + c] * xI[c];     // (M^T x_I)[a], column a row c
    }
  } else {
    // diagonal tile: only its lower triangle is meaningful; mirror it
#pragma unroll
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
    const int nt = s.nt_b;
    part[s.part_off + ((int64_t)t.i * nt + t.j) * TS + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    if (t.i != t.j)
      part[s.part_off + ((int64_t)t.j * nt + t.i) * TS + tid] =
          red2[0][tid] + red2[1][tid] + red2[2][tid] + red2[3][tid];
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
  hipLaunchKernelGGL(k_symv_tiles<T>, dim3(count), dim3(256), 0, s, tasks, subs, M, xb, part, st, iface_only);
  if (yb) hipLaunchKernelGGL(k_symv_reduce, grid1(NB), dim3(256), 0, s, NB, b_sub, subs, (const double*)part, yb, st);
}
// Descriptor of one interface tile for k_symv_one: eight int64 fields, read
// by lanes 0..7 of each wave as one vector load, in place of two dependent
// scalar loads (task, then its subdomain).  See gemv_descriptors.
constexpr int GD_TILE = 0, GD_XI = 1, GD_XJ = 2, GD_PIJ = 3, GD_PJI = 4, GD_ROWS_B = 5, GD_ROWS_IF = 6,
              GD_DIAG = 7;

template <typename T>
struct SymvTile {
  static constexpr int W = 16 / sizeof(T);          // elements per 16-byte load
  static constexpr int NV = TS2 / (256 * W);         // loads per thread per tile
  using V = __attribute__((ext_vector_type(W))) T;
};

// Uniform field f of the descriptor held by lanes 0..7 of the wave.
__device__ __forceinline__ int64_t gd_field(int64_t mine, int f) {
  const int lo = __builtin_amdgcn_readlane((int)(mine & 0xffffffff), f);
  const int hi = __builtin_amdgcn_readlane((int)(mine >> 32), f);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Issue the 16-byte loads of a tile (W consecutive rows of one column each);
// a load none of whose rows takes part is skipped.  Rows beyond the last
// real DOF of the block (the padding of the last tile row, and with
// iface_only the trailing-block DOFs without multipliers) and the upper half
// of a diagonal tile (mirrored from the lower half) do not take part; the
// values are masked when stored to LDS, so the loads stay in flight.
template <typename T>
__device__ __forceinline__ void symv_fetch(const T* __restrict__ M, int64_t tile_off, int rows, bool diag,
                                           typename SymvTile<T>::V (&v)[SymvTile<T>::NV]) {
  using ST = SymvTile<T>;
  using V = typename ST::V;
  const V* tile = reinterpret_cast<const V*>(M + tile_off);
#pragma unroll
  for (int u = 0; u < ST::NV; ++u) {
    const int e0 = (threadIdx.x + 256 * u) * ST::W;
    const int col = e0 >> 6, row0 = e0 & 63;
    const int lo = diag ? (row0 > col ? row0 : col) : row0;   // first row that takes part
    v[u] = (lo < rows && lo < row0 + ST::W) ? tile[threadIdx.x + 256 * u] : V{};
  }
}

// k_symv_tiles over the tile descriptors, for the interface tiles of the dual
// operator and of the Dirichlet preconditioner: one tile per workgroup; the
// descriptor is one vector load, then the tile's 16-byte loads and its x
// blocks are issued together.
template <typename T>
__global__ __launch_bounds__(256) void k_symv_one(const int64_t* __restrict__ desc, const T* __restrict__ M,
                                                  const double* __restrict__ xb, double* part, const PcgState* st,
                                                  int iface_only) {
  using ST = SymvTile<T>;
  if (halted(st)) return;
  __shared__ T sM[TS * LDV];
  __shared__ double xI[TS], xJ[TS];
  __shared__ double red[4][TS], red2[4][TS];
  const int tid = threadIdx.x, lane = tid & 63;
  const int64_t d = desc[(int64_t)blockIdx.x * 8 + (lane & 7)];
  const int rows = (int)gd_field(d, iface_only ? GD_ROWS_IF : GD_ROWS_B);
  const bool diag = gd_field(d, GD_DIAG) != 0;
  typename ST::V v[ST::NV];
  symv_fetch<T>(M, gd_field(d, GD_TILE), rows, diag, v);
  if (tid < TS) {
    xI[tid] = xb[gd_field(d, GD_XI) + tid];
    xJ[tid] = xb[gd_field(d, GD_XJ) + tid];
  }
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
  __syncthreads();
  const int a = tid & 63, q = tid >> 6;
  double s1 = 0.0, s2 = 0.0;
  if (!diag) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int c = 16 * q + k;
      s1 += (double)sM[c * LDV + a] * xJ[c];
      s2 += (double)sM[a * LDV + c] * xI[c];
    }
  } else {
#pragma unroll
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
    part[gd_field(d, GD_PIJ) + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
    if (!diag) part[gd_field(d, GD_PJI) + tid] = red2[0][tid] + red2[1][tid] + red2[2][tid] + red2[3][tid];
  }
}

// Descriptors of the tiles tasks[0..count) for k_symv_one (host side).
void gemv_descriptors(const Task* tasks, int count, const SubInfo* subs, std::vector<int64_t>& out) {
  out.assign((size_t)count * 8, 0);
  for (int k = 0; k < count; ++k) {
    const Task& t = tasks[k];
    const SubInfo& s = subs[t.sub];
    int64_t* d = out.data() + (size_t)k * 8;
    const int nt = s.nt_b;
    d[GD_TILE] = s.x_off + tidx2(t.i, t.j) * TS2;
    d[GD_XI] = s.b_off + (int64_t)t.i * TS;
    d[GD_XJ] = s.b_off + (int64_t)t.j * TS;
    d[GD_PIJ] = s.part_off + ((int64_t)t.i * nt + t.j) * TS;
    d[GD_PJI] = s.part_off + ((int64_t)t.j * nt + t.i) * TS;
    d[GD_ROWS_B] = t.i == nt - 1 ? s.n_b - TS * (nt - 1) : TS;
    d[GD_ROWS_IF] = t.i == nt - 1 ? s.n_if - TS * (nt - 1) : TS;
    d[GD_DIAG] = t.i == t.j;
  }
}

template <typename T>
void pcg_symv_desc(const int64_t* desc, int count, const T* M, const double* xb, double* part, int64_t NB,
                   const int32_t* b_sub, const SubInfo* subs, double* yb, const PcgState* st, hipStream_t s,
                   int iface_only) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_symv_one<T>, dim3(count), dim3(256), 0, s, desc, M, xb, part, st, iface_only);
  if (yb) hipLaunchKernelGGL(k_symv_reduce, grid1(NB), dim3(256), 0, s, NB, b_sub, subs, (const double*)part, yb, st);
}
template void pcg_symv_desc<double>(const int64_t*, int, const double*, const double*, double*, int64_t,
                                    const int32_t*, const SubInfo*, double*, const PcgState*, hipStream_t, int);
template void pcg_symv_desc<float>(const int64_t*, int, const float*, const double*, double*, int64_t,
                                   const int32_t*, const SubInfo*, double*, const PcgState*, hipStream_t, int);

template void pcg_symv<double>(const Task*, int, const SubInfo*, const double*, const double*, double*, int64_t, const int32_t*, double*, const PcgState*, hipStream_t, int);
template void pcg_symv<float>(const Task*, int, const SubInfo*, const float*, const double*, double*, int64_t, const int32_t*, double*, const PcgState*, hipStream_t, int);

}  // namespace feti
