// Batched dense tile kernels for the local generalised inverses (gfx950).
//
// Every subdomain matrix K_i is stored interior-first as a lower-triangular
// array of 64x64 column-major tiles.  A blocked left-looking Cholesky runs over
// all subdomains at once: each launch processes one tile column of every
// subdomain that has it (a task list built on the host), so subdomains of
// different sizes share launches.  The contractions run on 16x16x4 MFMA
// (FP64 for the FP64 path, FP32 with FP32 accumulation for the mixed path).
//
// The factorisation realises the generalised inverse of the paper's
// eq. (localSolutions) by interior-first elimination (section 4, eq.
// (reordered) orders interior DOFs before coupling DOFs): after the interior
// columns the trailing block is the Schur complement S_i of eq. (DirichletVK);
// it is regularised on its rigid-body kernel, factored, and inverted
// explicitly (X_i = S~_i^{-1}) so that every PCG iteration applies the local
// pseudo-inverse restricted to the interface as one dense matrix-vector product.
#include "feti_impl.h"

namespace feti {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
template <typename T> struct V4;
template <> struct V4<double> { typedef d4 type; };
template <> struct V4<float> { typedef f4 type; };

constexpr int LD = TS + 1;   // LDS leading dimension (odd: conflict-free transposed stores)

__device__ __forceinline__ d4 mfma4(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma4(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
// Row of accumulator register r held by lane l (column is l & 15).
__device__ __forceinline__ int out_row(double, int l, int r) { return 4 * r + (l >> 4); }
__device__ __forceinline__ int out_row(float, int l, int r) { return 4 * (l >> 4) + r; }

__device__ __forceinline__ int64_t tidx(int i, int j) { return (int64_t)i * (i + 1) / 2 + j; }

// Task of this workgroup.  Workgroups of a launch are handed to the eight
// XCDs in turn (workgroup b to XCD b mod 8), each XCD with its own L2.  Task
// lists run subdomain by subdomain, and the tasks of one subdomain share
// operand tiles (the column panel of a column step, the rows of W in X = W^T W),
// so XCD x takes the contiguous run of tasks [x n/8, (x+1) n/8) in order:
// neighbouring tasks, and the tiles they share, stay in one L2.  A bijection
// of [0, n), whatever the order the hardware actually dispatches in.
__device__ __forceinline__ int xcd_map(int l, int n) {
  const int q = n >> 3, r = n & 7, x = l & 7;
  return x * q + min(x, r) + (l >> 3);
}
__device__ __forceinline__ int xcd_task() { return xcd_map((int)blockIdx.x, (int)gridDim.x); }
// Launches that carry tasks of several kinds remap each range on its own, so
// that every kind spreads over all XCDs: l in [0, n), the first n_first of
// them one range, the rest another.
__device__ __forceinline__ int xcd_split(int l, int n, int n_first) {
  return l < n_first ? xcd_map(l, n_first) : n_first + xcd_map(l - n_first, n - n_first);
}

// The elements e = threadIdx.x + NT u (u < TS2 / NT) of a tile that one thread
// of an NT-thread block handles.  The loops below have a compile-time trip
// count, so every load of a tile is issued before the first use; a loop
// bounded by threadIdx.x is kept rolled and waits on each load in turn.
// tile_rmw: C[e] = f(e, C[e]) for every element.
template <int NT = 256, typename T, typename F>
__device__ __forceinline__ void tile_rmw(T* C, F f) {
  constexpr int N = TS2 / NT;
  T c[N];
#pragma unroll
  for (int u = 0; u < N; ++u) c[u] = C[threadIdx.x + NT * u];
#pragma unroll
  for (int u = 0; u < N; ++u) {
    const int e = threadIdx.x + NT * u;
    C[e] = f(e, c[u]);
  }
}
// tile_copy: dst[e] = src[e] for every element.
template <typename T>
__device__ __forceinline__ void tile_copy(T* dst, const T* __restrict__ src) {
  constexpr int N = TS2 / 256;
  T c[N];
#pragma unroll
  for (int u = 0; u < N; ++u) c[u] = src[threadIdx.x + 256 * u];
#pragma unroll
  for (int u = 0; u < N; ++u) dst[threadIdx.x + 256 * u] = c[u];
}

// LDS operand layout: s[k*LD + m] holds op(A)(m, k) (or op(B)(k, m)).
// Tiles are read with 16-byte vector loads, all issued before any LDS store,
// so that a workgroup keeps a whole 64x64 tile of loads in flight.
template <typename T> struct Vec16;
template <> struct Vec16<double> { typedef double2 type; static constexpr int n = 2; };
template <> struct Vec16<float> { typedef float4 type; static constexpr int n = 4; };

template <typename T, bool TRANS>
__device__ __forceinline__ void lds_load(T* s, const T* __restrict__ g) {
  typedef typename Vec16<T>::type V;
  constexpr int EPV = Vec16<T>::n;
  constexpr int NV = TS2 / EPV / 256;
  const V* gv = reinterpret_cast<const V*>(g);
  V v[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = gv[threadIdx.x + 256 * i];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int e0 = (threadIdx.x + 256 * i) * EPV;
#pragma unroll
    for (int u = 0; u < EPV; ++u) {
      const int e = e0 + u;
      const T x = reinterpret_cast<const T*>(&v[i])[u];
      if (TRANS) s[(e & 63) * LD + (e >> 6)] = x;
      else s[(e >> 6) * LD + (e & 63)] = x;
    }
  }
}
// A tile held in registers between its global load and its LDS store, so the
// load of the next k-step's tiles can be in flight during this step's MFMAs.
template <typename T, int NT = 256>
struct TileRegs {
  typedef typename Vec16<T>::type V;
  static constexpr int EPV = Vec16<T>::n;
  static constexpr int NV = TS2 / EPV / NT;
  V v[NV];
  __device__ __forceinline__ void fetch(const T* __restrict__ g) {
    const V* gv = reinterpret_cast<const V*>(g);
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = gv[threadIdx.x + NT * i];
  }
  template <bool TRANS>
  __device__ __forceinline__ void store(T* s) const {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int e0 = (threadIdx.x + NT * i) * EPV;
#pragma unroll
      for (int u = 0; u < EPV; ++u) {
        const int e = e0 + u;
        const T x = reinterpret_cast<const T*>(&v[i])[u];
        if (TRANS) s[(e & 63) * LD + (e >> 6)] = x;
        else s[(e >> 6) * LD + (e & 63)] = x;
      }
    }
  }
};

// direct: s[k][m] = g[k*TS + m]   (A not transposed, or B transposed)
template <typename T>
__device__ __forceinline__ void lds_direct(T* s, const T* __restrict__ g) { lds_load<T, false>(s, g); }
// transposed: s[k][m] = g[m*TS + k]   (A transposed, or B not transposed)
template <typename T>
__device__ __forceinline__ void lds_trans(T* s, const T* __restrict__ g) { lds_load<T, true>(s, g); }

template <typename T>
struct Acc {
  typename V4<T>::type c[2][2];
  __device__ void zero() {
    for (int x = 0; x < 2; ++x)
      for (int y = 0; y < 2; ++y)
        for (int r = 0; r < 4; ++r) c[x][y][r] = T(0);
  }
};

// acc += opA * opB for one 64x64x64 product; wave w owns the 32x32 block (w>>1, w&1).
// LDX: leading dimension of the LDS operands.
// KC: number of k-values held (a multiple of 4; 64 = the whole tile).
template <typename T, int LDX = LD, int KC = TS>
__device__ __forceinline__ void mma64w(Acc<T>& acc, const T* sA, const T* sB, int w) {
  const int lane = threadIdx.x & 63;
  const int wr = w >> 1, wc = w & 1, lr = lane & 15, lk = lane >> 4;
  // fully unrolled, so the LDS reads of later k-slices issue ahead of the
  // MFMAs that consume earlier ones
#pragma unroll
  for (int kk = 0; kk < KC / 4; ++kk) {
    const int k = 4 * kk + lk;
    const T a0 = sA[k * LDX + 32 * wr + lr], a1 = sA[k * LDX + 32 * wr + 16 + lr];
    const T b0 = sB[k * LDX + 32 * wc + lr], b1 = sB[k * LDX + 32 * wc + 16 + lr];
    acc.c[0][0] = mfma4(a0, b0, acc.c[0][0]);
    acc.c[0][1] = mfma4(a0, b1, acc.c[0][1]);
    acc.c[1][0] = mfma4(a1, b0, acc.c[1][0]);
    acc.c[1][1] = mfma4(a1, b1, acc.c[1][1]);
  }
}

template <typename T>
__device__ __forceinline__ void mma64(Acc<T>& acc, const T* sA, const T* sB) {
  mma64w(acc, sA, sB, (int)(threadIdx.x >> 6));
}

// Scatter scale*acc into LDS.  colmajor: s[col*LD + row]; else s[row*LD + col].
template <typename T>
__device__ __forceinline__ void acc_to_lds_w(T* s, const Acc<T>& acc, T scale, bool colmajor, int w) {
  const int lane = threadIdx.x & 63;
  const int wr = w >> 1, wc = w & 1;
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y)
      for (int r = 0; r < 4; ++r) {
        const int row = 32 * wr + 16 * x + out_row(T(0), lane, r);
        const int col = 32 * wc + 16 * y + (lane & 15);
        s[colmajor ? col * LD + row : row * LD + col] = scale * acc.c[x][y][r];
      }
}
template <typename T>
__device__ __forceinline__ void acc_to_lds(T* s, const Acc<T>& acc, T scale, bool colmajor) {
  acc_to_lds_w(s, acc, scale, colmajor, (int)(threadIdx.x >> 6));
}

// ---------------------------------------------------------------------------
// C_ij <- C_ij - sum_{k0<=k<k1} L_ik L_jk^T   (left-looking update)
// acc = sum_{k0<=k<k1} L_ik L_jk^T, software-pipelined: the tiles of step k+1
// load while step k multiplies
template <typename T>
__device__ __forceinline__ void accumulate_tile(Acc<T>& acc, const T* __restrict__ base, int i, int j, int k0,
                                                int k1, T* sA,
                                                T* sB) {
  acc.zero();
  TileRegs<T> ra, rb;
  if (k0 < k1) {
    ra.fetch(base + tidx(i, k0) * TS2);
    rb.fetch(base + tidx(j, k0) * TS2);
  }
  for (int k = k0; k < k1; ++k) {
    ra.template store<false>(sA);
    rb.template store<false>(sB);
    __syncthreads();
    if (k + 1 < k1) {
      ra.fetch(base + tidx(i, k + 1) * TS2);
      rb.fetch(base + tidx(j, k + 1) * TS2);
    }
    mma64(acc, sA, sB);
    __syncthreads();
  }
}

template <typename T>
__device__ __forceinline__ void update_tile(const Task& t, const SubInfo* __restrict__ subs, T* arena, T* sA,
                                            T* sB) {
  T* base = arena + subs[t.sub].tile_off;
  Acc<T> acc;
  accumulate_tile(acc, base, t.i, t.j, t.k0, t.k1, sA, sB);
  acc_to_lds(sA, acc, T(-1), true);
  __syncthreads();
  T* C = base + tidx(t.i, t.j) * TS2;
  tile_rmw(C, [&](int e, T c) { return c + sA[(e >> 6) * LD + (e & 63)]; });
}

template <typename T>
__device__ void trtri_tile(const Task& t, const SubInfo* __restrict__ subs, const T* __restrict__ arena,
                           const T* __restrict__ linv, T* W, T* sA, T* sB);

// Blocked factorisation of a diagonal tile (diag_block): 16x16 blocks.
constexpr int DB = 16;
// FP64 LDS scratch of a diagonal block, in doubles: the tile (TS LD), the
// inverses of its four diagonal 16x16 blocks, and three 16x16 partial products
constexpr int DIAG_SMEM = TS * LD + 4 * DB * DB + 3 * DB * DB;
// LDS of a kernel whose blocks hold `elems` elements of T or a diagonal
// block's scratch, in doubles
template <typename T>
constexpr int smem_doubles(int elems) {
  return (elems * (int)sizeof(T) > DIAG_SMEM * 8 ? elems * (int)sizeof(T) : DIAG_SMEM * 8) / 8;
}

template <typename T>
__device__ __forceinline__ void diag_block(const Task& t, const SubInfo* __restrict__ subs, T* arena, T* linv,
                                           int* err, T* sA, T* sB, double* scratch);

// One launch per column step.  Blocks below n_diag take the diagonal tiles
// of the column (diag_block: the tile's last update term, its factorisation
// and inverse); the hardware dispatches them first.  Blocks from n_diag to
// n_upd update the tiles below (update_tile); the blocks after them, if any,
// compute one block row of the inverse of the factor (trtri_tile), whose
// inputs are complete once the previous column step is done.  Fusing them
// keeps the serial chain of launches short and needs no second stream.
template <typename T>
__global__ __launch_bounds__(256) void k_update(const Task* __restrict__ tasks, int n_diag, int n_upd,
                                                const SubInfo* __restrict__ subs, T* arena,
                                                T* linv, T* W, int* err) {
  __shared__ double smem[smem_doubles<T>(2 * TS * LD)];
  T* sA = reinterpret_cast<T*>(smem);
  T* sB = sA + TS * LD;
  const int b0 = (int)blockIdx.x;
  if (b0 < n_diag) {
    diag_block<T>(tasks[b0], subs, arena, linv, err, sA, sB, smem);
    return;
  }
  const int b = n_diag + xcd_split(b0 - n_diag, (int)gridDim.x - n_diag, n_upd - n_diag);
  const Task t = tasks[b];
  if (b < n_upd) update_tile<T>(t, subs, arena, sA, sB);
  else trtri_tile<T>(t, subs, arena, linv, W, sA, sB);
}

// Copy N consecutive elements from global memory into LDS unchanged
// (s[e] = g[e]) with the direct global-to-LDS loads of gfx950: each
// instruction moves 16 bytes per lane, 1 KiB per wave, to consecutive LDS
// addresses from a wave-uniform base, without passing through registers.
// Their completion is counted by vmcnt.
template <typename T, int N>
__device__ __forceinline__ void dma_copy(T* s, const T* __restrict__ g) {
  constexpr int RUNS = N * (int)sizeof(T) / 1024;   // 1 KiB runs
  constexpr int PER_WAVE = RUNS / 4;
  static_assert(PER_WAVE * 4 * 1024 == N * (int)sizeof(T), "whole 1 KiB runs per wave");
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < PER_WAVE; ++q) {
    const int run = w * PER_WAVE + q;
    __builtin_amdgcn_global_load_lds(
        (const __attribute__((address_space(1))) void*)((const char*)g + run * 1024 + lane * 16),
        (__attribute__((address_space(3))) void*)((char*)s + run * 1024), 16, 0, 0);
  }
}

// s_waitcnt vmcnt(0): every global (and global-to-LDS) load of this wave done
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Double-buffered form of k_update: the operands advance in chunks of KC
// k-values (KC consecutive columns of a column-major tile: 64 KC contiguous
// elements).  The next chunk of both operands streams straight into the other
// LDS buffer (dma_copy) while this chunk's MFMAs read the current one, with
// one barrier per chunk.  LDS rows are unpadded (64 elements): each 16-lane
// group of an operand read takes 16 consecutive elements.  Same products in
// the same order as update_tile, so the results are bit-identical.  With
// KC = 32 the buffers take 64 KiB in FP64, two workgroups per compute unit.
// Occupancy asked of the double-buffered update: three waves per SIMD in
// FP32 (its LDS allows three workgroups per compute unit), two in FP64.  The
// PLAIN form (launches of update tasks only, KC = 16) needs no LDS for the
// diagonal blocks or the inverse rows: about 33 KiB in FP64, four
// workgroups per compute unit.
template <typename T, bool PLAIN = false>
struct UpdOcc { static constexpr int waves = PLAIN ? 4 : (sizeof(T) == 4 ? 3 : 2); };
template <typename T, int KC, bool PLAIN = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(UpdOcc<T, PLAIN>::waves))) void k_update_db(const Task* __restrict__ tasks, int n_diag, int n_upd,
                                                   const SubInfo* __restrict__ subs, T* arena,
                                                   T* linv, T* W, int* err) {
  constexpr int CH = TS * KC;                 // elements per chunk
  constexpr int PARTS = TS / KC;              // chunks per tile
  // [buffer][A, B][chunk]; the result tile uses TS LD; the inverse rows 2 TS LD,
  // the diagonal blocks their scratch
  constexpr int NFIX = PLAIN ? TS * LD : 2 * TS * LD;
  constexpr int NLDS = 4 * CH > NFIX ? 4 * CH : NFIX;
  __shared__ double smem[PLAIN ? (NLDS * (int)sizeof(T) + 7) / 8 : smem_doubles<T>(NLDS)];
  T* lds = reinterpret_cast<T*>(smem);
  const int b0 = (int)blockIdx.x;
  int b = b0;
  if constexpr (!PLAIN) {
    if (b0 < n_diag) {
      diag_block<T>(tasks[b0], subs, arena, linv, err, lds, lds + TS * LD, smem);
      return;
    }
    b = n_diag + xcd_split(b0 - n_diag, (int)gridDim.x - n_diag, n_upd - n_diag);
  } else {
    b = xcd_task();
  }
  const Task t = tasks[b];
  if constexpr (!PLAIN) {
    if (b >= n_upd) {
      trtri_tile<T>(t, subs, arena, linv, W, lds, lds + TS * LD);
      return;
    }
  }
  T* base = arena + subs[t.sub].tile_off;
  const int w = threadIdx.x >> 6;
  const int steps = (t.k1 - t.k0) * PARTS;
  Acc<T> acc;
  acc.zero();
  if (steps > 0) {
    dma_copy<T, CH>(lds, base + tidx(t.i, t.k0) * TS2);
    dma_copy<T, CH>(lds + CH, base + tidx(t.j, t.k0) * TS2);
  }
  for (int st = 0; st < steps; ++st) {
    const int cur = st & 1;
    // this chunk has landed (every wave's share), and every wave is done
    // reading the other buffer
    wait_vm();
    __syncthreads();
    if (st + 1 < steps) {
      const int k = t.k0 + (st + 1) / PARTS, part = (st + 1) % PARTS;
      T* nxt = lds + (cur ^ 1) * 2 * CH;
      dma_copy<T, CH>(nxt, base + tidx(t.i, k) * TS2 + part * CH);
      dma_copy<T, CH>(nxt + CH, base + tidx(t.j, k) * TS2 + part * CH);
    }
    const T* sa = lds + cur * 2 * CH;
    mma64w<T, TS, KC>(acc, sa, sa + CH, w);
  }
  __syncthreads();
  acc_to_lds(lds, acc, T(-1), true);
  __syncthreads();
  T* C = base + tidx(t.i, t.j) * TS2;
  tile_rmw(C, [&](int e, T c) { return c + lds[(e >> 6) * LD + (e & 63)]; });
}

// Wide form: one workgroup of eight waves updates output tiles (i, j) and
// (i+1, j) (t.n = 2; t.n = 1: only (i, j)), sharing the column panel L_jk:
// three tiles staged per k-step for two tiles of output, 27% less memory
// traffic per flop than the 64x64 form, with two waves per SIMD.  Waves 0-3
// compute tile i, waves 4-7 tile i+1, each a 32x32 block as in mma64, so every
// output element sums the same products in the same order as in update_tile:
// both forms give bit-identical factors.
template <typename T>
__global__ __launch_bounds__(512) void k_update_wide(const Task* __restrict__ tasks,
                                                     const SubInfo* __restrict__ subs, T* arena) {
  __shared__ T sA0[TS * LD], sA1[TS * LD], sB[TS * LD];
  const Task t = tasks[xcd_task()];
  T* base = arena + subs[t.sub].tile_off;
  const int w = threadIdx.x >> 6;
  const int h = w >> 2, wl = w & 3;
  const bool two = t.n == 2;
  const bool active = h == 0 || two;
  Acc<T> acc;
  acc.zero();
  TileRegs<T, 512> ra0, ra1, rb;
  if (t.k0 < t.k1) {
    ra0.fetch(base + tidx(t.i, t.k0) * TS2);
    if (two) ra1.fetch(base + tidx(t.i + 1, t.k0) * TS2);
    rb.fetch(base + tidx(t.j, t.k0) * TS2);
  }
  for (int k = t.k0; k < t.k1; ++k) {
    ra0.template store<false>(sA0);
    if (two) ra1.template store<false>(sA1);
    rb.template store<false>(sB);
    __syncthreads();
    if (k + 1 < t.k1) {
      ra0.fetch(base + tidx(t.i, k + 1) * TS2);
      if (two) ra1.fetch(base + tidx(t.i + 1, k + 1) * TS2);
      rb.fetch(base + tidx(t.j, k + 1) * TS2);
    }
    if (active) mma64w(acc, h ? sA1 : sA0, sB, wl);
    __syncthreads();
  }
  if (active) acc_to_lds_w(h ? sA1 : sA0, acc, T(-1), true, wl);
  __syncthreads();
  T* C0 = base + tidx(t.i, t.j) * TS2;
  tile_rmw<512>(C0, [&](int e, T c) { return c + sA0[(e >> 6) * LD + (e & 63)]; });
  if (two) {
    T* C1 = base + tidx(t.i + 1, t.j) * TS2;
    tile_rmw<512>(C1, [&](int e, T c) { return c + sA1[(e >> 6) * LD + (e & 63)]; });
  }
}

// Broadcast lane `lane`'s value of v to the whole wave (two v_readlane_b32).
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Diagonal tile of a column step: C_jj = L_jj L_jj^T (in place, FP64
// arithmetic) and the explicit inverse L_jj^{-1}, by all four waves of the
// workgroup on the tile held in LDS, in 16x16 blocks.  For each block column p:
// wave 0 factors the diagonal block in registers (lane r holds row r; pivots
// read from the owning lane with readlane; a correctly rounded square root and
// its reciprocal per pivot) and inverts it; the rows below are solved against
// that inverse (one thread per row); the trailing lower triangle takes the
// rank-16 update.  The off-diagonal blocks of the inverse follow block
// diagonal by block diagonal: X_qp = -X_qq sum_{p<=k<q} L_qk X_kp, stored
// transposed in the unused upper triangle of the tile.  The serial chain is
// 4 x 16 pivots instead of 64.  A non-positive or non-finite pivot records
// the subdomain in err[0] -- unless err[2] allows modified pivots (a factor
// used only as the preconditioner of a refinement against the exact
// operator): then a finite non-positive pivot d is replaced by
// max(|d|, 1e-12 s), s the largest diagonal magnitude of the tile, as in a
// modified Cholesky factorisation, and err[3] counts the replacements.
// scratch: DIAG_SMEM doubles of LDS.
template <typename T>
__device__ __forceinline__ void diag_blocked(const Task& t, const SubInfo* __restrict__ subs, T* arena, T* linv,
                                             int* err, double* scratch) {
  double* A = scratch;                    // A(r, c) = A[c * LD + r]
  double* Dinv = scratch + TS * LD;       // Dinv_p(i, k) = Dinv[p * 256 + i * 16 + k]
  double* Tmp = Dinv + 4 * DB * DB;       // [3][16 * 16]
  const SubInfo s = subs[t.sub];
  T* C = arena + s.tile_off + tidx(t.j, t.j) * TS2;
  T* Li = linv + s.linv_off + (int64_t)t.j * TS2;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  {
    constexpr int N = TS2 / 256;
    T c[N];
#pragma unroll
    for (int u = 0; u < N; ++u) c[u] = C[tid + 256 * u];
#pragma unroll
    for (int u = 0; u < N; ++u) {
      const int e = tid + 256 * u;
      A[(e >> 6) * LD + (e & 63)] = (double)c[u];
    }
  }
  __syncthreads();
  const int allow_mod = err[2];
  double dscale = 0.0;   // largest diagonal magnitude of the tile (wave 0)
  if (w == 0) {
    dscale = fabs(A[lane * LD + lane]);
    for (int o = 32; o > 0; o >>= 1) dscale = fmax(dscale, __shfl_xor(dscale, o, 64));
  }
  int nmod = 0;
  bool bad = false;
  for (int p = 0; p < 4; ++p) {
    const int p0 = DB * p;
    if (w == 0) {
      // lane r holds row p0 + (r & 15) of the diagonal block; lanes 16..63
      // repeat the rows of lanes 0..15 and write nothing
      const int r = lane & 15;
      double a[DB];
#pragma unroll
      for (int c = 0; c < DB; ++c) a[c] = A[(p0 + c) * LD + p0 + r];
      double my_inv = 1.0;
#pragma unroll
      for (int c = 0; c < DB; ++c) {
        const double d = readlane_d(a[c], c);
        const bool ok = (d > 0.0) && (d < 1e300);
        double dd = ok ? d : 1.0;
        if (!ok && allow_mod && fabs(d) < 1e300 && dscale > 0.0) {
          dd = fmax(fabs(d), 1e-12 * dscale);
          ++nmod;
        } else {
          bad |= !ok;
        }
        // L(c, c) = sqrt(d) and its reciprocal, both correctly rounded, so that
        // the block inverse built from inv is the inverse of the stored factor
        // to rounding
        const double sd = sqrt(dd);
        const double inv = 1.0 / sd;
        double l = a[c] * inv;
        l = r > c ? l : 0.0;
        l = r == c ? sd : l;
        my_inv = r == c ? inv : my_inv;
        a[c] = l;
#pragma unroll
        for (int cc = c + 1; cc < DB; ++cc) a[cc] -= l * readlane_d(l, cc);
      }
      // inverse of the block: lane j holds column j,
      // X(i, j) = (delta_ij - sum_{k<i} L(i, k) X(k, j)) / L(i, i)
      const int j = r;
      double x[DB];
#pragma unroll
      for (int i = 0; i < DB; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < i; ++k) acc += readlane_d(a[k], i) * x[k];
        const double xi = ((i == j ? 1.0 : 0.0) - acc) * readlane_d(my_inv, i);
        x[i] = i < j ? 0.0 : xi;
      }
      if (lane < DB) {
#pragma unroll
        for (int c = 0; c < DB; ++c) A[(p0 + c) * LD + p0 + r] = c > r ? 0.0 : a[c];
#pragma unroll
        for (int i = 0; i < DB; ++i) Dinv[p * DB * DB + i * DB + j] = x[i];
      }
    }
    __syncthreads();
    const int n = TS - p0 - DB;   // rows below the block column
    if (n > 0) {
      // L(r, p0 + c) = sum_{k <= c} A(r, p0 + k) X_pp(c, k), one thread per row
      if (tid < n) {
        const int r = p0 + DB + tid;
        double a[DB];
#pragma unroll
        for (int k = 0; k < DB; ++k) a[k] = A[(p0 + k) * LD + r];
#pragma unroll
        for (int c = 0; c < DB; ++c) {
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k <= c; ++k) acc += a[k] * Dinv[p * DB * DB + c * DB + k];
          A[(p0 + c) * LD + r] = acc;
        }
      }
      __syncthreads();
      // A(r, c) -= sum_k L(r, p0 + k) L(c, p0 + k) for p0 + 16 <= c <= r
      for (int e = tid; e < n * n; e += 256) {
        const int r = p0 + DB + e / n, c = p0 + DB + e % n;
        if (c <= r) {
          double acc = 0.0;
#pragma unroll
          for (int k = 0; k < DB; ++k) acc += A[(p0 + k) * LD + r] * A[(p0 + k) * LD + c];
          A[c * LD + r] -= acc;
        }
      }
      __syncthreads();
    }
  }
  // off-diagonal blocks of X = L^{-1}, block diagonal d = q - p at a time;
  // X(R, C) for block(R) > block(C) is kept at A[R * LD + C]
  {
    const int i = tid >> 4, jj = tid & 15;
    for (int d = 1; d < 4; ++d) {
      for (int p = 0; p + d < 4; ++p) {
        const int q = p + d;
        // T(i, jj) = sum_{k=p}^{q-1} sum_m L_qk(i, m) X_kp(m, jj)
        double acc = 0.0;
        for (int k = p; k < q; ++k)
#pragma unroll
          for (int m = 0; m < DB; ++m) {
            const double l = A[(DB * k + m) * LD + DB * q + i];
            const double xv = k == p ? Dinv[p * DB * DB + m * DB + jj] : A[(DB * k + m) * LD + DB * p + jj];
            acc += l * xv;
          }
        Tmp[p * DB * DB + i * DB + jj] = acc;
      }
      __syncthreads();
      for (int p = 0; p + d < 4; ++p) {
        const int q = p + d;
        // X_qp(i, jj) = -sum_{m <= i} X_qq(i, m) T(m, jj)
        double acc = 0.0;
#pragma unroll
        for (int m = 0; m < DB; ++m)
          acc += (m <= i ? Dinv[q * DB * DB + i * DB + m] : 0.0) * Tmp[p * DB * DB + m * DB + jj];
        A[(DB * q + i) * LD + DB * p + jj] = -acc;
      }
      __syncthreads();
    }
  }
  // L to the tile (upper triangle zero) and X to the inverse arena, column-major
  for (int e = tid; e < TS2; e += 256) {
    const int row = e & 63, col = e >> 6;
    C[e] = (T)(row >= col ? A[col * LD + row] : 0.0);
    double xv = 0.0;
    if (row >= col) {
      const int br = row >> 4, bc = col >> 4;
      xv = br == bc ? Dinv[br * DB * DB + (row & 15) * DB + (col & 15)] : A[row * LD + col];
    }
    Li[e] = (T)xv;
  }
  if (w == 0 && lane == 0) {   // wave 0 ran the pivots; lane 0 reports them
    if (bad) atomicMin(err, t.sub);
    if (nmod) atomicAdd(err + 3, nmod);
  }
}

// A diagonal task (j, j, k0, k1) of a 256-thread block: the four waves
// subtract the update terms k0 <= k < k1 (update_tile, usually the one term
// k = j - 1, the others having been subtracted by the previous column step),
// then factor and invert the tile (diag_blocked) with `scratch`, which may
// alias sA and sB.
template <typename T>
__device__ __forceinline__ void diag_block(const Task& t, const SubInfo* __restrict__ subs, T* arena, T* linv,
                                           int* err, T* sA, T* sB, double* scratch) {
  if (t.k0 < t.k1) {
    update_tile<T>(t, subs, arena, sA, sB);
    __syncthreads();   // the updated tile is in memory and sA, sB are free
  }
  diag_blocked<T>(t, subs, arena, linv, err, scratch);
}

// Diagonal tasks alone (the first column of a stage, and the launches whose
// update form cannot host them).
template <typename T>
__global__ __launch_bounds__(256) void k_diag(const Task* __restrict__ tasks,
                                              const SubInfo* __restrict__ subs, T* arena, T* linv,
                                              int* err) {
  __shared__ double smem[smem_doubles<T>(2 * TS * LD)];
  T* sA = reinterpret_cast<T*>(smem);
  diag_block<T>(tasks[blockIdx.x], subs, arena, linv, err, sA, sA + TS * LD, smem);
}

// L_ij <- C_ij L_jj^{-T}   (panel solve by the explicit diagonal inverse)
template <typename T>
__global__ __launch_bounds__(256) void k_trsm(const Task* __restrict__ tasks,
                                              const SubInfo* __restrict__ subs, T* arena,
                                              const T* __restrict__ linv) {
  // One 64x64x64 product per workgroup: each wave reads the MFMA operands of
  // its 32x32 block straight from the column-major tiles (16 lanes take 16
  // consecutive rows of one column, 128 bytes), all before the first MFMA;
  // only the result passes through LDS.  Same operands and order as mma64.
  __shared__ T sC[TS * LD];
  const Task t = tasks[xcd_task()];
  const SubInfo s = subs[t.sub];
  T* C = arena + s.tile_off + tidx(t.i, t.j) * TS2;
  const T* Li = linv + s.linv_off + (int64_t)t.j * TS2;   // B(k,n) = Linv(n,k)
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wr = w >> 1, wc = w & 1, lr = lane & 15, lk = lane >> 4;
  T a0[TS / 4], a1[TS / 4], b0[TS / 4], b1[TS / 4];
#pragma unroll
  for (int kk = 0; kk < TS / 4; ++kk) {
    const int k = 4 * kk + lk;
    a0[kk] = C[k * TS + 32 * wr + lr];
    a1[kk] = C[k * TS + 32 * wr + 16 + lr];
    b0[kk] = Li[k * TS + 32 * wc + lr];
    b1[kk] = Li[k * TS + 32 * wc + 16 + lr];
  }
  Acc<T> acc;
  acc.zero();
#pragma unroll
  for (int kk = 0; kk < TS / 4; ++kk) {
    acc.c[0][0] = mfma4(a0[kk], b0[kk], acc.c[0][0]);
    acc.c[0][1] = mfma4(a0[kk], b1[kk], acc.c[0][1]);
    acc.c[1][0] = mfma4(a1[kk], b0[kk], acc.c[1][0]);
    acc.c[1][1] = mfma4(a1[kk], b1[kk], acc.c[1][1]);
  }
  acc_to_lds(sC, acc, T(1), true);
  // every wave has read its operands from C before C is overwritten
  __syncthreads();
  for (int e = threadIdx.x; e < TS2; e += 256) C[e] = sC[(e >> 6) * LD + (e & 63)];
}

// One tile of the inverse W of the interface factor, block row i given rows
// < i (tile indices local to the interface block):
// W_ii = L_ii^{-1};  W_ij = -L_ii^{-1} sum_{k=k0}^{i-1} L_ik W_kj for j < i
// (the tasks carry k0 = j: all terms).  W tiles are stored row-major
// (element (r, c) at r * TS + c), so that X = W^T W streams both of its
// operands as contiguous row chunks (k_lauum_db).
template <typename T>
__device__ void trtri_tile(const Task& t, const SubInfo* __restrict__ subs, const T* __restrict__ arena,
                           const T* __restrict__ linv, T* W, T* sA, T* sB) {
  const SubInfo s = subs[t.sub];
  const int ni = s.nt_i;
  const T* Lbase = arena + s.tile_off;
  T* Wbase = W + s.x_off;
  T* out = Wbase + tidx(t.i, t.j) * TS2;
  const T* Lii_inv = linv + s.linv_off + (int64_t)(ni + t.i) * TS2;
  if (t.i == t.j) {
    lds_direct(sA, Lii_inv);   // sA[c * LD + r] = Linv(r, c)
    __syncthreads();
    for (int e = threadIdx.x; e < TS2; e += 256) out[e] = sA[(e & 63) * LD + (e >> 6)];
    return;
  }
  Acc<T> acc;
  acc.zero();
  TileRegs<T> ra, rb;
  if (t.k0 < t.i) {
    ra.fetch(Lbase + tidx(ni + t.i, ni + t.k0) * TS2);
    rb.fetch(Wbase + tidx(t.k0, t.j) * TS2);
  }
  for (int k = t.k0; k < t.i; ++k) {
    ra.template store<false>(sA);
    rb.template store<false>(sB);   // row-major W_kj: B(k, n) = W_kj(k, n)
    __syncthreads();
    if (k + 1 < t.i) {
      ra.fetch(Lbase + tidx(ni + t.i, ni + k + 1) * TS2);
      rb.fetch(Wbase + tidx(k + 1, t.j) * TS2);
    }
    mma64(acc, sA, sB);
    __syncthreads();
  }
  acc_to_lds(sB, acc, T(1), false);   // B(k, n) = acc(k, n)
  lds_direct(sA, Lii_inv);            // A(m, k) = Linv(m, k)
  __syncthreads();
  Acc<T> acc2;
  acc2.zero();
  mma64(acc2, sA, sB);
  __syncthreads();
  acc_to_lds(sA, acc2, T(-1), false);   // row-major
  __syncthreads();
  for (int e = threadIdx.x; e < TS2; e += 256) out[e] = sA[(e >> 6) * LD + (e & 63)];
}

// One block row of the inverse per launch (the rows not fused into updates).
template <typename T>
__global__ __launch_bounds__(256) void k_trtri(const Task* __restrict__ tasks,
                                               const SubInfo* __restrict__ subs,
                                               const T* __restrict__ arena,
                                               const T* __restrict__ linv, T* W) {
  __shared__ T sA[TS * LD], sB[TS * LD];
  const Task t = tasks[xcd_task()];
  trtri_tile<T>(t, subs, arena, linv, W, sA, sB);
}

// X_IJ = sum_{k>=I} W_kI^T W_kJ  (I >= J): X = W^T W = (L L^T)^{-1}.
// With the row-major tiles of W both operands are contiguous chunks of KC
// rows, streamed into two LDS buffers by the direct global-to-LDS loads as in
// k_update_db.  X tiles are written column-major.
template <typename T, int KC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(UpdOcc<T>::waves))) void k_lauum_db(
    const Task* __restrict__ tasks, const SubInfo* __restrict__ subs, const T* __restrict__ W, T* X) {
  constexpr int CH = TS * KC;
  constexpr int PARTS = TS / KC;
  constexpr int NLDS = 4 * CH > TS * LD ? 4 * CH : TS * LD;
  __shared__ double smem[(NLDS * (int)sizeof(T) + 7) / 8];
  T* lds = reinterpret_cast<T*>(smem);
  const Task t = tasks[xcd_task()];
  const SubInfo s = subs[t.sub];
  const T* Wb = W + s.x_off;
  const int w = threadIdx.x >> 6;
  const int steps = (t.k1 - t.k0) * PARTS;
  Acc<T> acc;
  acc.zero();
  if (steps > 0) {
    dma_copy<T, CH>(lds, Wb + tidx(t.k0, t.i) * TS2);
    dma_copy<T, CH>(lds + CH, Wb + tidx(t.k0, t.j) * TS2);
  }
  for (int st = 0; st < steps; ++st) {
    const int cur = st & 1;
    wait_vm();
    __syncthreads();
    if (st + 1 < steps) {
      const int k = t.k0 + (st + 1) / PARTS, part = (st + 1) % PARTS;
      T* nxt = lds + (cur ^ 1) * 2 * CH;
      dma_copy<T, CH>(nxt, Wb + tidx(k, t.i) * TS2 + part * CH);
      dma_copy<T, CH>(nxt + CH, Wb + tidx(k, t.j) * TS2 + part * CH);
    }
    const T* sa = lds + cur * 2 * CH;
    mma64w<T, TS, KC>(acc, sa, sa + CH, w);
  }
  __syncthreads();
  acc_to_lds(lds, acc, T(1), true);
  __syncthreads();
  T* out = X + s.x_off + tidx(t.i, t.j) * TS2;
  for (int e = threadIdx.x; e < TS2; e += 256) out[e] = lds[(e >> 6) * LD + (e & 63)];
}

// Copy of the interface Schur complement (for the Dirichlet preconditioner).
template <typename T>
__global__ __launch_bounds__(256) void k_copy_iface(const Task* __restrict__ tasks,
                                                    const SubInfo* __restrict__ subs,
                                                    const T* __restrict__ arena, T* S) {
  const Task t = tasks[blockIdx.x];
  const SubInfo s = subs[t.sub];
  const T* src = arena + s.tile_off + tidx(s.nt_i + t.i, s.nt_i + t.j) * TS2;
  T* dst = S + s.x_off + tidx(t.i, t.j) * TS2;
  tile_copy(dst, src);
}

// rho_s = mean of the diagonal of the interface Schur complement (real DOFs).
template <typename T>
__global__ __launch_bounds__(256) void k_rho(const SubInfo* __restrict__ subs,
                                             const T* __restrict__ arena, double* rho) {
  __shared__ double red[256];
  const SubInfo s = subs[blockIdx.x];
  double acc = 0.0;
  for (int d = threadIdx.x; d < s.n_b; d += 256) {
    const int I = d / TS, r = d % TS;
    acc += (double)arena[s.tile_off + tidx(s.nt_i + I, s.nt_i + I) * TS2 + r * TS + r];
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) rho[blockIdx.x] = s.n_b > 0 ? red[0] / s.n_b : 0.0;
}

// S~ = S + rho Rb Rb^T on the interface tiles of floating subdomains, with all
// six rigid modes (rb: interface-space vectors, 6 interleaved orthonormal
// columns, kernel modes first).  For a stressed tangent whose kernel holds
// only some of them, the inverse is corrected afterwards (k_wb_*).
template <typename T>
__global__ __launch_bounds__(256) void k_regularise(const Task* __restrict__ tasks,
                                                    const SubInfo* __restrict__ subs,
                                                    const double* __restrict__ rb,
                                                    const double* __restrict__ rho, T* arena) {
  const Task t = tasks[blockIdx.x];
  const SubInfo s = subs[t.sub];
  if (!s.floating) return;
  const double r0 = rho[t.sub];
  T* C = arena + s.tile_off + tidx(s.nt_i + t.i, s.nt_i + t.j) * TS2;
  const double* Ri = rb + (s.b_off + (int64_t)t.i * TS) * 6;
  const double* Rj = rb + (s.b_off + (int64_t)t.j * TS) * 6;
  tile_rmw(C, [&](int e, T cv) {
    const int c = e >> 6, r = e & 63;
    double acc = 0.0;
    for (int k = 0; k < 6; ++k) acc += Ri[r * 6 + k] * Rj[c * 6 + k];
    return (T)((double)cv + r0 * acc);
  });
}

// Exact generalised inverse for stressed floating subdomains.  With V the
// regularised rigid modes that are not in ker K_i (columns n_modes..5 of rb),
// S~_k = S + rho Rk Rk^T (kernel modes only) equals S~_6 - rho V V^T, so by the
// Woodbury identity X_k = X_6 + Y M Y^T with Y = X_6 V and
// M = (I/rho - V^T Y)^{-1}.  X_k is then a generalised inverse of S, as the
// local solution formula (eq. (localSolutions)) requires.
template <typename T>
__device__ __forceinline__ double xsym(const T* X, int64_t x_off, int I, int J, int r, int c) {
  if (I > J) return (double)X[x_off + tidx(I, J) * TS2 + c * TS + r];
  if (I < J) return (double)X[x_off + tidx(J, I) * TS2 + r * TS + c];
  return r >= c ? (double)X[x_off + tidx(I, I) * TS2 + c * TS + r] : (double)X[x_off + tidx(I, I) * TS2 + r * TS + c];
}

template <typename T>
__global__ __launch_bounds__(256) void k_wb_y(const SubInfo* __restrict__ subs, const T* __restrict__ X,
                                              const double* __restrict__ rb, double* Y) {
  __shared__ double red[4][TS][3];
  const SubInfo s = subs[blockIdx.y];
  const int I = blockIdx.x;
  if (s.floating != 1 || s.n_modes >= 6 || I >= s.nt_b) return;
  const int mk = s.n_modes, mv = 6 - mk;
  const int r = threadIdx.x & 63, q = threadIdx.x >> 6;
  double acc[3] = {0, 0, 0};
  for (int J = 0; J < s.nt_b; ++J)
    for (int c = 16 * q; c < 16 * q + 16; ++c) {
      const double x = xsym(X, s.x_off, I, J, r, c);
      const double* v = rb + (s.b_off + (int64_t)J * TS + c) * 6 + mk;
      for (int k = 0; k < mv; ++k) acc[k] += x * v[k];
    }
  for (int k = 0; k < 3; ++k) red[q][r][k] = acc[k];
  __syncthreads();
  if (threadIdx.x < TS)
    for (int k = 0; k < 3; ++k)
      Y[(s.b_off + (int64_t)I * TS + r) * 3 + k] = red[0][r][k] + red[1][r][k] + red[2][r][k] + red[3][r][k];
}

__global__ __launch_bounds__(256) void k_wb_m(const SubInfo* __restrict__ subs, const double* __restrict__ rb,
                                              const double* __restrict__ Y, const double* __restrict__ rho,
                                              double* Mout) {
  __shared__ double red[256];
  __shared__ double Cm[3][3];
  const SubInfo s = subs[blockIdx.x];
  if (s.floating != 1 || s.n_modes >= 6) return;
  const int mk = s.n_modes, mv = 6 - mk;
  const int64_t nb = (int64_t)s.nt_b * TS;
  for (int k = 0; k < mv; ++k)
    for (int l = 0; l < mv; ++l) {
      double acc = 0.0;
      for (int64_t b = threadIdx.x; b < nb; b += 256)
        acc += rb[(s.b_off + b) * 6 + mk + k] * Y[(s.b_off + b) * 3 + l];
      red[threadIdx.x] = acc;
      __syncthreads();
      for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
      }
      if (threadIdx.x == 0) Cm[k][l] = (k == l ? 1.0 / rho[blockIdx.x] : 0.0) - red[0];
      __syncthreads();
    }
  if (threadIdx.x == 0) {
    // Gauss-Jordan inverse of the mv x mv capacitance matrix
    double A[3][6];
    for (int k = 0; k < mv; ++k)
      for (int l = 0; l < 2 * mv; ++l) A[k][l] = l < mv ? Cm[k][l] : (l - mv == k ? 1.0 : 0.0);
    for (int c = 0; c < mv; ++c) {
      int piv = c;
      for (int k = c + 1; k < mv; ++k)
        if (fabs(A[k][c]) > fabs(A[piv][c])) piv = k;
      for (int l = 0; l < 2 * mv; ++l) {
        const double t = A[c][l];
        A[c][l] = A[piv][l];
        A[piv][l] = t;
      }
      const double d = A[c][c];
      for (int l = 0; l < 2 * mv; ++l) A[c][l] /= d;
      for (int k = 0; k < mv; ++k)
        if (k != c) {
          const double f = A[k][c];
          for (int l = 0; l < 2 * mv; ++l) A[k][l] -= f * A[c][l];
        }
    }
    for (int k = 0; k < 3; ++k)
      for (int l = 0; l < 3; ++l) Mout[blockIdx.x * 9 + 3 * k + l] = (k < mv && l < mv) ? A[k][mv + l] : 0.0;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_wb_update(const Task* __restrict__ tasks, const SubInfo* __restrict__ subs,
                                                   const double* __restrict__ Y, const double* __restrict__ Mm,
                                                   T* X) {
  const Task t = tasks[blockIdx.x];
  const SubInfo s = subs[t.sub];
  if (s.floating != 1 || s.n_modes >= 6) return;
  const double* M = Mm + t.sub * 9;
  T* C = X + s.x_off + tidx(t.i, t.j) * TS2;
  const double* Yi = Y + (s.b_off + (int64_t)t.i * TS) * 3;
  const double* Yj = Y + (s.b_off + (int64_t)t.j * TS) * 3;
  tile_rmw(C, [&](int e, T cv) {
    const int c = e >> 6, r = e & 63;
    double acc = 0.0;
    for (int k = 0; k < 3; ++k) {
      double mk = 0.0;
      for (int l = 0; l < 3; ++l) mk += M[3 * k + l] * Yj[c * 3 + l];
      acc += Yi[r * 3 + k] * mk;
    }
    return (T)((double)cv + acc);
  });
}

template <typename T>
void launch_woodbury(int n_sub, int max_nt_b, const Task* xtasks, int xcount, const SubInfo* subs, T* X,
                     const double* rb, const double* rho, double* Y, double* M, hipStream_t st) {
  if (max_nt_b <= 0) return;
  hipLaunchKernelGGL(k_wb_y<T>, dim3(max_nt_b, n_sub), dim3(256), 0, st, subs, (const T*)X, rb, Y);
  hipLaunchKernelGGL(k_wb_m, dim3(n_sub), dim3(256), 0, st, subs, rb, (const double*)Y, rho, M);
  if (xcount > 0) hipLaunchKernelGGL(k_wb_update<T>, dim3(xcount), dim3(256), 0, st, xtasks, subs, (const double*)Y, (const double*)M, X);
}
template void launch_woodbury<double>(int, int, const Task*, int, const SubInfo*, double*, const double*, const double*, double*, double*, hipStream_t);
template void launch_woodbury<float>(int, int, const Task*, int, const SubInfo*, float*, const double*, const double*, double*, double*, hipStream_t);

// Zero every factor tile, with unit diagonal on padding positions.
template <typename T>
__global__ __launch_bounds__(256) void k_init_arena(const Task* __restrict__ tasks,
                                                    const SubInfo* __restrict__ subs, T* arena) {
  const Task t = tasks[blockIdx.x];
  const SubInfo s = subs[t.sub];
  T* C = arena + s.tile_off + tidx(t.i, t.j) * TS2;
  for (int e = threadIdx.x; e < TS2; e += 256) {
    const int c = e >> 6, r = e & 63;
    T v = T(0);
    if (t.i == t.j && r == c) {
      const int p = t.i * TS + r;
      const bool pad = (p >= s.n_ii && p < s.nt_i * TS) || (p >= s.nt_i * TS + s.n_b);
      if (pad) v = T(1);
    }
    C[e] = v;
  }
}

// ---------------------------------------------------------------------------
// launchers
template <typename T>
void launch_dense(int kind, const Task* tasks, int count, const SubInfo* subs, T* arena, T* linv,
                  T* W, T* X, int* err, hipStream_t st, int split, int form, int ndiag) {
  if (count <= 0) return;
  if (is_update_kind(kind)) {
    const int nupd = kind == K_UPDATE ? count : split;   // diagonal and update tasks
    if (form == 3 && ndiag == 0 && nupd == count) {
      // update tasks only: the 16-wide chunks at four workgroups per CU
      hipLaunchKernelGGL((k_update_db<T, 16, true>), dim3(count), dim3(256), 0, st, tasks, 0, count, subs, arena,
                         linv, W, err);
    } else if (form == 2 || form == 3) {
      hipLaunchKernelGGL((k_update_db<T, 32>), dim3(count), dim3(256), 0, st, tasks, ndiag, nupd, subs, arena,
                         linv, W, err);
    } else if (form == 1) {
      // the task list is the wide form: diagonal tasks, two-tile updates, inverse rows
      if (ndiag > 0) hipLaunchKernelGGL(k_diag<T>, dim3(ndiag), dim3(256), 0, st, tasks, subs, arena, linv, err);
      if (nupd > ndiag)
        hipLaunchKernelGGL(k_update_wide<T>, dim3(nupd - ndiag), dim3(512), 0, st, tasks + ndiag, subs, arena);
      if (count > nupd)
        hipLaunchKernelGGL(k_trtri<T>, dim3(count - nupd), dim3(256), 0, st, tasks + nupd, subs, (const T*)arena,
                           (const T*)linv, W);
    } else {
      hipLaunchKernelGGL(k_update<T>, dim3(count), dim3(256), 0, st, tasks, ndiag, nupd, subs, arena, linv, W, err);
    }
    return;
  }
  switch (kind) {
    case K_DIAG: hipLaunchKernelGGL(k_diag<T>, dim3(count), dim3(256), 0, st, tasks, subs, arena, linv, err); break;
    case K_TRSM: hipLaunchKernelGGL(k_trsm<T>, dim3(count), dim3(256), 0, st, tasks, subs, arena, (const T*)linv); break;
    case K_TRTRI:
      hipLaunchKernelGGL(k_trtri<T>, dim3(count), dim3(256), 0, st, tasks, subs, (const T*)arena, (const T*)linv, W);
      break;
    case K_LAUUM:
      hipLaunchKernelGGL((k_lauum_db<T, 32>), dim3(count), dim3(256), 0, st, tasks, subs, (const T*)W, X);
      break;
  }
}
template void launch_dense<double>(int, const Task*, int, const SubInfo*, double*, double*, double*, double*, int*, hipStream_t, int, int, int);
template void launch_dense<float>(int, const Task*, int, const SubInfo*, float*, float*, float*, float*, int*, hipStream_t, int, int, int);

template <typename T>
void launch_init_arena(const Task* tasks, int count, const SubInfo* subs, T* arena, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_init_arena<T>, dim3(count), dim3(256), 0, st, tasks, subs, arena);
}
template void launch_init_arena<double>(const Task*, int, const SubInfo*, double*, hipStream_t);
template void launch_init_arena<float>(const Task*, int, const SubInfo*, float*, hipStream_t);

template <typename T>
void launch_copy_iface(const Task* tasks, int count, const SubInfo* subs, const T* arena, T* S, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_copy_iface<T>, dim3(count), dim3(256), 0, st, tasks, subs, arena, S);
}
template void launch_copy_iface<double>(const Task*, int, const SubInfo*, const double*, double*, hipStream_t);
template void launch_copy_iface<float>(const Task*, int, const SubInfo*, const float*, float*, hipStream_t);

template <typename T>
void launch_rho(int n_sub, const SubInfo* subs, const T* arena, double* rho, hipStream_t st) {
  hipLaunchKernelGGL(k_rho<T>, dim3(n_sub), dim3(256), 0, st, subs, arena, rho);
}
template void launch_rho<double>(int, const SubInfo*, const double*, double*, hipStream_t);
template void launch_rho<float>(int, const SubInfo*, const float*, double*, hipStream_t);

template <typename T>
void launch_regularise(const Task* tasks, int count, const SubInfo* subs, const double* rb,
                       const double* rho, T* arena, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_regularise<T>, dim3(count), dim3(256), 0, st, tasks, subs, rb, rho, arena);
}
template void launch_regularise<double>(const Task*, int, const SubInfo*, const double*, const double*, double*, hipStream_t);
template void launch_regularise<float>(const Task*, int, const SubInfo*, const double*, const double*, float*, hipStream_t);

}  // namespace feti
