// Kernels over the n cells: K-step stencil stages, stencil projections,
// Gram reductions and tall-skinny updates (gfx950, wave64).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>

#include "kernels.hpp"

namespace dlra {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxPartialBlocks = 1024;   // partial-sum blocks of one contraction
constexpr int kContractWaves = 8192;      // waves a contraction launch aims for
constexpr int kSumsqBlocks = 2048;

__device__ __forceinline__ void cell_coords(const GridDev &g, int x, int c[3]) {
  c[0] = x % g.nx;
  int t = x / g.nx;
  c[1] = t % g.ny;
  c[2] = t / g.ny;
}

// ------------------------------------------------------------------ 1/S
template <typename T>
__global__ void k_inverse_stop(GridDev g, const T *__restrict__ w, int n_mat,
                               const double *__restrict__ Si, T *__restrict__ s, Ctl *ctl) {
  int x = blockIdx.x * kBlock + threadIdx.x;
  if (x >= g.n) return;
  double st = 0.0;
  for (int i = 0; i < n_mat; ++i) st += double(w[size_t(i) * g.n + x]) * Si[i];
  if (!(st > 0.0)) {
    atomicOr(&ctl->flags, kFlagStop);
    st = 1.0;
  }
  s[x] = T(1.0 / st);
}

template <typename T>
struct YMat {
  const T *Y;
  int ld;
  __device__ T operator()(int x, int c) const { return Y[size_t(c) * ld + x]; }
};
// source column c = b n_mat + i of a context's beams: w_i(x) psi_b(x)
template <typename T>
struct YSrc {
  const T *w;
  const T *psi;
  int n, n_mat;
  size_t pstride;
  __device__ T operator()(int x, int c) const {
    const int b = c / n_mat, i = c - b * n_mat;
    return w[size_t(i) * n + x] * psi[size_t(b) * pstride + x];
  }
};
template <typename T>
struct WOne {
  __device__ T operator()(int) const { return T(1); }
};
template <typename T>
struct WMatS {
  const T *w;
  const T *s;
  __device__ T operator()(int x) const { return w[x] * s[x]; }
};

// ------------------------------------------------------------------ K-step stage

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d4v __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
// Accumulator layouts of the 16x16x4 MFMAs (lane l, register v, column
// l % 16): row 4 (l / 16) + v for f32, row l / 16 + 4 v for f64.
template <>
struct Mfma<float> {
  using acc_t = f4v;
  static __device__ __forceinline__ int row(int q, int v) { return 4 * q + v; }
  static __device__ __forceinline__ acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <>
struct Mfma<double> {
  using acc_t = d4v;
  static __device__ __forceinline__ int row(int q, int v) { return q + 4 * v; }
  static __device__ __forceinline__ acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

// One RK4 stage of the K-step as a dense contraction on the matrix cores:
//   out(x, j) = K0(x, j) - coef * sum_{dk, k} D_dk(x, k) B_dk(k, j),
// D_dk = second-order one-sided differences of s o W.  Each wave owns 16
// consecutive cells and all r <= 16 NJ outputs.  The 16x16x4 MFMA computes
// the transposed tile out^T = B^T D^T: A(j, kk) = Bp(4t + kk, 16 jt + j) from
// lane j + 16 kk and B(kk, i) = D(cell x0 + i, 4t + kk) from lane i + 16 kk
// (computed in registers from W and s); accumulator rows (outputs j) follow
// Mfma<T>::row, columns are the cells.
// Tile -> cells map of the stage kernel.  A tile is 64 cells: 4 waves of 16
// consecutive cells.  When nx is a multiple of 16 the 64 cells are a 16 (x) x
// 4 (y) patch and the tile order sweeps columns of 32 x 32 cells through all
// z before moving on, so the +-2-plane stencil halo of the tiles in flight
// stays in L2.  Otherwise tiles are 64 consecutive cells.  Returns the first
// cell of wave `wave` of tile L, or -1.
__device__ __forceinline__ int tile_wave_cell(const GridDev &g, int L, int wave, int tiled) {
  if (!tiled) {
    const int x0 = (L * 4 + wave) * 16;
    return x0 < g.n ? x0 : -1;
  }
  const int px = g.nx >> 4, py = (g.ny + 3) >> 2;
  const int tpx = min(2, px), tpy = min(8, py);
  const int ntx = (px + tpx - 1) / tpx;
  const int per_col = tpx * tpy * g.nz;
  const int col = L / per_col, rc = L % per_col;
  const int z = rc / (tpx * tpy), pin = rc % (tpx * tpy);
  const int tx = col % ntx, ty = col / ntx;
  const int ix = tx * tpx + pin % tpx, iy = ty * tpy + pin / tpx;
  if (ix >= px || iy >= py) return -1;
  const int y = iy * 4 + wave;
  if (y >= g.ny) return -1;
  return (z * g.ny + y) * g.nx + ix * 16;
}

// Persistent launch: gridDim.x is a multiple of 8, the hardware hands block b
// to XCD b % 8, and XCD i's blocks walk the i-th eighth of the tile order
// together (block b takes tiles lo + b / 8, lo + b / 8 + gridDim.x / 8, ...),
// so the tiles in flight on one XCD are neighbours and share its L2.  The
// couplings are staged in LDS once per block when BLDS.
template <typename T, int NJ, bool BLDS>
__global__ __launch_bounds__(256) void k_kstage_mfma(GridDev g, const T *__restrict__ s,
                                                    const T *__restrict__ W,
                                                    const T *__restrict__ K0,
                                                    T *__restrict__ out, int ld, int r,
                                                    const T *__restrict__ Bp, double coef,
                                                    int tiled, int ntiles) {
  constexpr int RB = 16 * NJ;
  constexpr int KS = 4 * NJ;           // MFMA k-steps per difference operator
  constexpr int KU = KS < 8 ? KS : 8;  // k-steps whose loads are issued together
  using acc_t = typename Mfma<T>::acc_t;
  extern __shared__ unsigned char smem_raw[];
  T *Bs = reinterpret_cast<T *>(smem_raw);
  if constexpr (BLDS) {
    const int nbk = 2 * g.dim * RB * RB;
    for (int e = threadIdx.x; e < nbk; e += blockDim.x) Bs[e] = Bp[e];
    __syncthreads();
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int c = lane & 15, q = lane >> 4;
  const int xcd = blockIdx.x & 7, nper = gridDim.x >> 3;
  const int lo = int((long long)xcd * ntiles / 8), hi = int((long long)(xcd + 1) * ntiles / 8);
  const int size[3] = {g.nx, g.ny, g.nz};
  const int ksteps = (r + 3) >> 2;
  for (int L = lo + (blockIdx.x >> 3); L < hi; L += nper) {
    const int x0 = tile_wave_cell(g, L, wave, tiled);
    if (x0 < 0) continue;
    const int x = x0 + c;
    const bool valid = x < g.n;
    // Every load below uses an in-range (clamped) index and is unconditional;
    // masked terms are zeroed by their stencil weight or a select.  A load
    // inside a divergent branch would be followed by a full wait.
    const int xc = valid ? x : g.n - 1;
    int cc[3] = {0, 0, 0};
    cell_coords(g, xc, cc);
    acc_t acc[NJ];
#pragma unroll
    for (int jt = 0; jt < NJ; ++jt) acc[jt] = acc_t{0, 0, 0, 0};
    for (int d = 0; d < g.dim; ++d) {
      const int st = d == 0 ? 1 : (d == 1 ? g.nx : g.nx * g.ny);
      const bool m1 = valid && cc[d] >= 1, m2 = valid && cc[d] >= 2;
      const bool p1 = valid && cc[d] + 1 < size[d], p2 = valid && cc[d] + 2 < size[d];
      const int im1 = m1 ? xc - st : xc, im2 = m2 ? xc - 2 * st : xc;
      const int ip1 = p1 ? xc + st : xc, ip2 = p2 ? xc + 2 * st : xc;
      // s at the stencil points, zero outside the grid (zero ghost cells)
      T s0 = s[xc], sm1 = s[im1], sm2 = s[im2], sp1 = s[ip1], sp2 = s[ip2];
      s0 = valid ? s0 : T(0);
      sm1 = m1 ? sm1 : T(0);
      sm2 = m2 ? sm2 : T(0);
      sp1 = p1 ? sp1 : T(0);
      sp2 = p2 ? sp2 : T(0);
      const T ih = T(g.inv2h[d]);
      const int ob = 2 * d * RB * RB, of = ob + RB * RB;
      for (int k0 = 0; k0 < ksteps; k0 += KU) {
        T db[KU], df[KU];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
          const int k = 4 * (k0 + u) + q;
          const T *col = W + size_t(min(k, r - 1)) * ld;
          const T a0 = col[xc], am1 = col[im1], am2 = col[im2], ap1 = col[ip1],
                  ap2 = col[ip2];
          const T w0 = s0 * a0;
          const T bk = (T(3) * w0 - T(4) * (sm1 * am1) + sm2 * am2) * ih;
          const T fk = (T(4) * (sp1 * ap1) - T(3) * w0 - sp2 * ap2) * ih;
          db[u] = k < r ? bk : T(0);
          df[u] = k < r ? fk : T(0);
        }
#pragma unroll
        for (int u = 0; u < KU; ++u) {
          if (k0 + u < ksteps) {
            const int brow = (4 * (k0 + u) + q) * RB + c;
#pragma unroll
            for (int jt = 0; jt < NJ; ++jt) {
              T bb, bf;
              if constexpr (BLDS) {
                bb = Bs[ob + brow + 16 * jt];
                bf = Bs[of + brow + 16 * jt];
              } else {
                bb = Bp[ob + brow + 16 * jt];
                bf = Bp[of + brow + 16 * jt];
              }
              acc[jt] = Mfma<T>::op(bb, db[u], acc[jt]);
              acc[jt] = Mfma<T>::op(bf, df[u], acc[jt]);
            }
          }
        }
      }
    }
    // the accumulator holds the transposed tile (rows = outputs j, columns =
    // cells), so 16 consecutive lanes store 16 consecutive cells of one column
    T k0v[NJ][4];
#pragma unroll
    for (int jt = 0; jt < NJ; ++jt)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        k0v[jt][v] = K0[size_t(min(16 * jt + Mfma<T>::row(q, v), r - 1)) * ld + xc];
#pragma unroll
    for (int jt = 0; jt < NJ; ++jt) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = 16 * jt + Mfma<T>::row(q, v);
        if (valid && j < r)
          out[size_t(j) * ld + x] = T(double(k0v[jt][v]) - coef * double(acc[jt][v]));
      }
    }
  }
}

// K-step stage with an LDS z-march (r <= 32 in FP32, r <= 16 in FP64).  A
// block owns a brick column of 16 (x) x 4 (y) cells and a chunk of z planes
// and marches through z.  The LDS holds a ring of 5 + A planes of W (each
// brick row with a 2-cell x halo; planes z-2..z+2 in use, z+3 .. z+2+A landed
// or arriving), 1 + A buffers of the 2-row y halo, the matching values of s
// and 1 + A tiles of K0, all filled by direct buffer->LDS loads issued A = 2
// steps ahead of their use (130 KiB of LDS at r <= 32 in FP32).  No global load returns to registers inside the march,
// so the only waits on memory are the explicit ones before the per-step
// barrier, which leave the newest loads in flight.  Cells outside the grid
// are read clamped into range and their s is masked to zero when used (the
// zero ghost cells of the stencil).  Every difference operand comes from
// LDS, so each input value is read from L2 about twice instead of once per
// stencil use.  Wave w computes row w of the centre plane: the transposed
// tile out^T = B^T D^T on 16x16x4 MFMAs with the couplings in registers,
// each difference of s o W formed as an s-weighted sum of W.
constexpr bool kUseBrick = true;
constexpr int kBrickBY = 4;                    // rows per brick = waves per block
constexpr int kBrickRW = 16 + 4;               // row width with the x halo
constexpr int kBrickPC = kBrickBY * kBrickRW;  // cells per ring plane
constexpr int kBrickHC = 4 * 16;               // y-halo cells (4 rows of 16)
constexpr int kBrickHS = 80;                   // y-halo stride per column of W
constexpr int kBrickKS = 68;                   // K0-tile stride per column
// steps between a load and its use, ring planes, y-halo / K0-tile buffers.
// Step z (after the barrier that ended step z - 1) loads ring plane z+1+AH
// into the slot of plane z - 3 and the y halo / K0 tile of step z+AH-1 into
// the buffers of step z - 1, interleaved with its MFMAs.
__host__ __device__ constexpr int brick_ahead(int) { return 3; }
__host__ __device__ constexpr int brick_slots(int tsize) { return 4 + brick_ahead(tsize); }
__host__ __device__ constexpr int brick_bufs(int tsize) { return brick_ahead(tsize); }
constexpr unsigned kBufWord3 = 0x00020000u;    // raw (untyped) buffer resource
// byte offset beyond every buffer the z-march reads (their sizes stay below
// it), so a load with it returns zero; offset + plane base stays below 2^32
constexpr int kOobOffset = 0x7F000000;
// waves per brick row for two output tiles (FP32, 16 < r <= 32): with two,
// each wave computes one tile and two waves share every SIMD
constexpr int kBrickSplit = 2;
static_assert(kBrickPC % 32 == 16 && kBrickHS % 32 == 16, "LDS strides avoid bank conflicts");
static_assert(kBrickPC == kBrickHS, "one column stride for ring and halo");

// dwords of the s region of one ring plane (a whole number of 64-dword loads)
__host__ __device__ constexpr int brick_s_dwords(int dpe) {
  return (kBrickPC * dpe + 63) / 64 * 64;
}

__host__ __device__ constexpr size_t brick_lds_bytes(int rb, int tsize, int js) {
  return size_t(4) * (size_t(brick_slots(tsize)) * rb * kBrickPC * (tsize / 4) +
                      size_t(brick_bufs(tsize)) * rb * kBrickHS * (tsize / 4) +
                      size_t(brick_slots(tsize)) * brick_s_dwords(tsize / 4) +
                      size_t(brick_bufs(tsize)) * kBrickHC * (tsize / 4) +
                      size_t(brick_bufs(tsize)) * rb * kBrickKS * (tsize / 4) + 64) +
         (js == 2 ? size_t(2) * kBrickBY * 2 * 256 * tsize : 0);   // partial-sum exchange
}

// s_waitcnt vmcnt(N) (expcnt and lgkmcnt not waited for): at most N of this
// wave's vector memory operations are still outstanding, i.e. all but the
// newest N have completed (direct buffer->LDS loads included)
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Workgroup barrier without the memory fence of __syncthreads(), whose
// release would wait for every outstanding load of the wave, including the
// direct buffer->LDS loads meant to stay in flight.  The LDS data the barrier
// publishes is written only by those loads, and their landing is ensured by
// an explicit wait_vm before it; the signal fences keep the compiler from
// moving LDS accesses across it.
__device__ __forceinline__ void block_barrier() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_barrier();
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, size_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), short(0), int(bytes),
                                           int(kBufWord3));
}

// one dword per lane from the buffer (byte offset vo + so) into LDS at
// dst + 4 * lane (dst wave-uniform)
__device__ __forceinline__ void dma_dword(__amdgpu_buffer_rsrc_t rs, void *dst, int vo, int so) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (__attribute__((address_space(3))) void *)dst, 4,
                                           vo, so, 0, 0);
}

template <typename T>
__device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t r, int vo, int so) {
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, vo, so, 0);
  } else {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, vo, so, 0);
  }
}

template <typename T, int NJ, int DIM, int JS>
__global__ __launch_bounds__(64 * kBrickBY * JS) void k_kstage_brick(
    GridDev g, const T *__restrict__ s, const T *__restrict__ W, const T *__restrict__ K0,
    T *__restrict__ out, int ld, int r, const T *__restrict__ Bp, double coef, int nzc,
    int zchunk) {
  constexpr int RB = 16 * NJ, KS = 4 * NJ, DPE = int(sizeof(T)) / 4, TB = int(sizeof(T));
  constexpr int BY = kBrickBY, RW = kBrickRW, PC = kBrickPC, HC = kBrickHC, HS = kBrickHS;
  constexpr int KST = kBrickKS, NW = BY * JS;
  // JS = 2: the two waves of a brick row split the column blocks kq (the
  // contraction) and swap their partial sums of each other's output tile
  // through LDS once per plane; each stores one output tile
  constexpr bool KSPLIT = JS == 2;
  constexpr int KSW = KS / JS;                       // column blocks per wave
  constexpr int NOUT = KSPLIT ? 1 : NJ;              // output tiles stored per wave
  static_assert(JS == 1 || (JS == 2 && NJ == 2), "column split for two output tiles");
  constexpr int AH = brick_ahead(TB), NS = brick_slots(TB), NB = brick_bufs(TB);
  static_assert(brick_lds_bytes(RB, TB, JS) <= 160 * 1024, "fits the LDS");
  constexpr int SPD = brick_s_dwords(DPE);           // dwords of one s ring plane
  constexpr int SP = SPD / DPE;                      // ... in elements
  constexpr int NPI = RB * PC * DPE / (64 * NW);     // W-plane loads per wave and step
  constexpr int NHI = RB * HC * DPE / (64 * NW);     // W y-halo loads ...
  constexpr int NKI = RB * 64 * DPE / (64 * NW);     // K0-tile loads ...
  constexpr int NSX = SPD / 64 + HC * DPE / 64;      // s loads (plane + y halo)
  constexpr int NSI = (NSX + NW - 1) / NW;           // ... per wave (padded with dummies)
  static_assert((RB * PC * DPE) % (64 * NW) == 0 && (RB * HC * DPE) % (64 * NW) == 0 &&
                    (RB * 64 * DPE) % (64 * NW) == 0,
                "equal whole 64-dword loads per wave");
  constexpr int NLOADS = NPI + NHI + NKI + NSI;      // per wave and step
  static_assert(AH >= 2 && (AH - 2) * NLOADS < 64, "fits vmcnt");
  using acc_t = typename Mfma<T>::acc_t;
  extern __shared__ unsigned char smem_raw[];
  T *ringW = reinterpret_cast<T *>(smem_raw);        // [NS][RB][PC]
  T *haloW = ringW + NS * RB * PC;                   // [NB][RB][HS]
  T *ringS = haloW + NB * RB * HS;                   // [NS][SP]
  T *haloS = ringS + NS * SP;                        // [NB][HC]
  T *K0t = haloS + NB * HC;                          // [NB][RB][KST]
  unsigned char *pad = reinterpret_cast<unsigned char *>(K0t + NB * RB * KST);   // 64 dwords
  T *xbuf = reinterpret_cast<T *>(pad + 256);        // [2][BY][2][256] (KSPLIT)
  // block -> (brick column, z chunk); the hardware's round-robin of blocks
  // over the 8 XCDs gets one contiguous range of this order per XCD
  const int nblk = gridDim.x, b = blockIdx.x;
  const int xcd = b & 7, per = nblk >> 3, rem = nblk & 7;
  const int L = xcd * per + min(xcd, rem) + (b >> 3);
  // columns in x-fastest order: an XCD's range covers whole rows of bricks,
  // so the 128-byte lines shared by x neighbours (x halos, K0 and output
  // rows) are fetched from HBM once into that XCD's L2
  const int zc = L % nzc, col = L / nzc;
  const int nbx = (g.nx + 15) >> 4;
  const int bx = col % nbx, by = col / nbx;
  const int gx0 = 16 * bx, gy0 = BY * by;
  const int z0 = zc * zchunk, z1 = min(g.nz, z0 + zchunk);
  if (z0 >= z1) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int row = wave % BY;                    // brick row of this wave
  const int jh = wave / BY;                     // KSPLIT: its half of the kq, its tile
  const int kq0 = jh * KSW;                     // first column block of this wave
  const int c = lane & 15, q = lane >> 4;
  const int nx = g.nx, ny = g.ny, nz = g.nz, plane = nx * ny;
  const size_t tall_bytes = size_t(ld) * r * TB;
  const __amdgpu_buffer_rsrc_t rW = make_rsrc(W, tall_bytes), rK = make_rsrc(K0, tall_bytes);
  const __amdgpu_buffer_rsrc_t rO = make_rsrc(out, tall_bytes);
  const __amdgpu_buffer_rsrc_t rS = make_rsrc(s, size_t(g.n) * TB);
  auto clampy = [&](int y) { return min(max(y, 0), ny - 1); };
  auto clampx = [&](int x) { return min(max(x, 0), nx - 1); };
  auto clampz = [&](int z) { return min(max(z, 0), nz - 1); };
  auto halo_y = [&](int hr) { return gy0 + (hr < 2 ? hr - 2 : BY + hr - 2); };
  // couplings: the A operands of all MFMAs of this lane
  T bq[DIM][KSW][NJ][2];
#pragma unroll
  for (int d = 0; d < DIM; ++d)
#pragma unroll
    for (int kq = 0; kq < KSW; ++kq)
#pragma unroll
      for (int jt = 0; jt < NJ; ++jt)
#pragma unroll
        for (int f = 0; f < 2; ++f)
          bq[d][kq][jt][f] =
              Bp[size_t(2 * d + f) * RB * RB + (4 * (kq0 + kq) + q) * RB + 16 * jt + c];
  // per-lane byte offsets (within one z plane) of every load of the march
  int poff[NPI], hoff[NHI], koff[NKI], soff[NSI];
#pragma unroll
  for (int i = 0; i < NPI; ++i) {
    const int dw = 64 * (wave + NW * i) + lane;
    const int e = dw / DPE, k = e / PC, cell = e % PC;
    const int gy = clampy(gy0 + cell / RW), gx = clampx(gx0 + cell % RW - 2);
    poff[i] = ((min(k, r - 1) * ld + gy * nx + gx) * DPE + dw % DPE) * 4;
  }
#pragma unroll
  for (int i = 0; i < NHI; ++i) {
    const int dw = 64 * (wave + NW * i) + lane;
    const int k = dw / (HC * DPE), hd = dw % (HC * DPE), hc = hd / DPE;
    const int gy = clampy(halo_y(hc >> 4)), gx = clampx(gx0 + (hc & 15));
    hoff[i] = ((min(k, r - 1) * ld + gy * nx + gx) * DPE + hd % DPE) * 4;
  }
#pragma unroll
  for (int i = 0; i < NKI; ++i) {
    const int dw = 64 * (wave + NW * i) + lane;
    const int j = dw / (64 * DPE), cd = dw % (64 * DPE), cell = cd / DPE;
    const int gy = clampy(gy0 + (cell >> 4)), gx = clampx(gx0 + (cell & 15));
    koff[i] = ((min(j, r - 1) * ld + gy * nx + gx) * DPE + cd % DPE) * 4;
  }
#pragma unroll
  for (int i = 0; i < NSI; ++i) {
    const int idx = wave + NW * i;   // s load: plane part, y-halo part or dummy
    int gy = 0, gx = 0, half = 0;
    if (idx < SPD / 64) {
      const int dw = 64 * idx + lane, cell = min(dw / DPE, PC - 1);
      half = dw % DPE;
      gy = gy0 + cell / RW;
      gx = gx0 + cell % RW - 2;
    } else if (idx < NSX) {
      const int dw = 64 * (idx - SPD / 64) + lane, hc = dw / DPE;
      half = dw % DPE;
      gy = halo_y(hc >> 4);
      gx = gx0 + (hc & 15);
    }
    const bool in_grid = gx >= 0 && gx < nx && gy >= 0 && gy < ny;
    soff[i] = in_grid ? ((gy * nx + gx) * DPE + half) * 4 : kOobOffset;
  }
  static_assert(NB == AH, "one y-halo / K0 buffer per step in flight");
  auto slot = [](int z) { return (z % NS + NS) % NS; };   // prologue only
  // W of ring plane zp, W y halo of plane zh, K0 tile of plane zh, s of both
  // loads lo .. hi-1 of the NLOADS of one step (W plane, W y halo, K0 tile,
  // s), so that a step's loads can be spread over the column blocks
  auto issue_part = [&](int lo, int hi, int zp, int zh, int hbuf, int sl) {
    const int pb = clampz(zp) * plane * TB, hb = clampz(zh) * plane * TB;
    // s planes outside the grid read as zero (out-of-range buffer loads)
    const int pbs = (zp >= 0 && zp < nz) ? pb : kOobOffset;
    const int hbs = (zh >= 0 && zh < nz) ? hb : kOobOffset;
    unsigned char *dp = reinterpret_cast<unsigned char *>(ringW + sl * RB * PC);
    unsigned char *dh = reinterpret_cast<unsigned char *>(haloW + hbuf * RB * HS);
    unsigned char *dk = reinterpret_cast<unsigned char *>(K0t + hbuf * RB * KST);
    unsigned char *dsp = reinterpret_cast<unsigned char *>(ringS + sl * SP);
    unsigned char *dsh = reinterpret_cast<unsigned char *>(haloS + hbuf * HC);
    auto in = [&](int i) { return i >= lo && i < hi; };
#pragma unroll
    for (int i = 0; i < NPI; ++i)
      if (in(i)) dma_dword(rW, dp + 256 * (wave + NW * i), poff[i], pb);
#pragma unroll
    for (int i = 0; i < NHI; ++i) {
      const int dw0 = 64 * (wave + NW * i);
      if (in(NPI + i))
        dma_dword(rW, dh + 4 * ((dw0 / (HC * DPE)) * HS * DPE + dw0 % (HC * DPE)), hoff[i], hb);
    }
#pragma unroll
    for (int i = 0; i < NKI; ++i) {
      const int dw0 = 64 * (wave + NW * i);
      if (in(NPI + NHI + i))
        dma_dword(rK, dk + 4 * ((dw0 / (64 * DPE)) * KST * DPE + dw0 % (64 * DPE)), koff[i],
                  hb);
    }
#pragma unroll
    for (int i = 0; i < NSI; ++i) {
      const int idx = wave + NW * i;
      if (!in(NPI + NHI + NKI + i)) continue;
      if (idx < SPD / 64) dma_dword(rS, dsp + 256 * idx, soff[i], pbs);
      else if (idx < NSX) dma_dword(rS, dsh + 256 * (idx - SPD / 64), soff[i], hbs);
      else dma_dword(rS, pad, soff[i], 0);
    }
  };
  auto issue = [&](int zp, int zh) { issue_part(0, NLOADS, zp, zh, zh % NB, slot(zp)); };
  // prologue: ring planes z0-2 .. z0+AH, y halos / K0 tiles of z0 .. z0+AH-2;
  // step z loads ring plane z+1+AH and the y halo / K0 tile / s of z+AH-1,
  // spread over its column blocks
  for (int i = 0; i < AH + 3; ++i) issue(z0 - 2 + i, z0 + min(i, AH - 2));
  wait_vm<0>();
  __syncthreads();
  T ih[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) ih[d] = T(g.inv2h[d]);
  const T tcoef = T(coef);
  const int gx = gx0 + c, gy = gy0 + row;
  const bool valid = gx < nx && gy < ny;
  const int xyo = (clampy(gy) * nx + clampx(gx)) * TB;
  const int base = row * RW + c + 2;
  // outputs of the previous step, stored during this one (KSPLIT: own partial
  // sums and K0, combined with the partner's partial sums at the store)
  T pend[NOUT][4], pk0[NOUT][4];
  // this lane's column offset in a ring plane or halo (PC == HS): column
  // 4 kq0 + q; the column blocks kq then add compile-time offsets
  const int qoff = (4 * kq0 + q) * PC;
  auto xslot = [&](int zz, int writer) {
    return xbuf + (((zz & 1) * BY + row) * 2 + writer) * 256 + lane;
  };
  auto out_value = [&](int jt, int v, int zz) {
    if constexpr (KSPLIT) return pk0[jt][v] - tcoef * (pend[jt][v] + xslot(zz, 1 - jh)[64 * v]);
    else return pend[jt][v];
  };
  auto out_col = [&](int jt, int v) {
    return 16 * (KSPLIT ? jh : jt) + Mfma<T>::row(q, v);
  };
  // ring slots of the planes z - 2 .. z + 2 and z + 1 + AH, and the y-halo /
  // K0 buffer of step z, all stepped below (no division)
  int hb = z0 % NB, sc = slot(z0), sdma = slot(z0 + 1 + AH);
  int zsl[4] = {slot(z0 - 2), slot(z0 - 1), slot(z0 + 1), slot(z0 + 2)};
  for (int z = z0; z < z1; ++z) {
    const int hbl = hb == 0 ? NB - 1 : hb - 1;   // buffer of step z + AH - 1 (NB == AH)
    const T *Wc = ringW + sc * RB * PC, *Sc = ringS + sc * SP;
    const T *wp[DIM][4];
    T sv[DIM][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int o = t < 2 ? t - 2 : t - 1;
      wp[0][t] = Wc + base + o + qoff;
      sv[0][t] = Sc[base + o];   // zero outside the grid
      const int yr = row + o;
      const bool inb = yr >= 0 && yr < BY;
      const int hr = yr < 0 ? yr + 2 : yr - BY + 2;
      wp[1][t] = (inb ? Wc + yr * RW + c + 2 : haloW + hb * RB * HS + hr * 16 + c) + qoff;
      const T sy_in = Sc[min(max(yr, 0), BY - 1) * RW + c + 2];
      const T sy_h = haloS[hb * HC + min(max(hr, 0), 3) * 16 + c];
      sv[1][t] = inb ? sy_in : sy_h;
      if constexpr (DIM == 3) {
        wp[2][t] = ringW + zsl[t] * RB * PC + base + qoff;
        sv[2][t] = ringS[zsl[t] * SP + base];
      }
    }
    // s-weights of the one-sided differences (ih folded in)
    const T s0 = Sc[base];
    T cb[DIM][3], cf[DIM][3];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      cb[d][0] = T(3) * ih[d] * s0;
      cb[d][1] = T(-4) * ih[d] * sv[d][1];
      cb[d][2] = ih[d] * sv[d][0];
      cf[d][0] = T(-3) * ih[d] * s0;
      cf[d][1] = T(4) * ih[d] * sv[d][2];
      cf[d][2] = -ih[d] * sv[d][3];
    }
    acc_t acc[NJ];
    // stores of the previous step's outputs, spread over this step's column
    // blocks like the loads
    auto store_part = [&](int lo, int hi) {
#pragma unroll
      for (int u = 0; u < NOUT * 4; ++u) {
        const int jt = u / 4, v = u % 4;
        const int j = out_col(jt, v);
        if (u >= lo && u < hi && z > z0 && valid && j < r)
          buf_store(out_value(jt, v, z - 1), rO, xyo + j * ld * TB, (z - 1) * plane * TB);
      }
    };
#pragma unroll
    for (int jt = 0; jt < NJ; ++jt) acc[jt] = acc_t{0, 0, 0, 0};
    // software pipeline over the column blocks kq: the LDS reads of block
    // kq + 1 are issued before the MFMAs of block kq and its differences are
    // formed after them, so the reads complete under the matrix work
    T sten[1 + 4 * DIM];
    const T *wc0 = Wc + base + qoff;
    auto read_sten = [&](int kq) {
      const int ok = 4 * kq * PC;   // column block offset (PC == HS)
      sten[0] = wc0[ok];
#pragma unroll
      for (int d = 0; d < DIM; ++d)
#pragma unroll
        for (int t = 0; t < 4; ++t) sten[1 + 4 * d + t] = wp[d][t][ok];
    };
    T db[DIM], df[DIM];
    // the centre terms of the two differences are negatives of each other
    // (cf0 = -cb0 exactly), so one product serves both
    auto diffs = [&]() {
      const T w0 = sten[0];
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const T wm2 = sten[1 + 4 * d], wm1 = sten[2 + 4 * d];
        const T wp1 = sten[3 + 4 * d], wp2 = sten[4 + 4 * d];
        const T t0 = cb[d][0] * w0;
        db[d] = cb[d][2] * wm2 + (cb[d][1] * wm1 + t0);
        df[d] = cf[d][2] * wp2 + (cf[d][1] * wp1 - t0);
      }
    };
    read_sten(0);
    diffs();
#pragma unroll
    for (int kq = 0; kq < KSW; ++kq) {
      if (kq + 1 < KSW) read_sten(kq + 1);
      issue_part(kq * NLOADS / KSW, (kq + 1) * NLOADS / KSW, z + 1 + AH, z + AH - 1, hbl,
                 sdma);
      store_part(kq * NOUT * 4 / KSW, (kq + 1) * NOUT * 4 / KSW);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        // the output tiles alternate, so consecutive MFMAs never depend on
        // each other (same accumulation order per tile)
#pragma unroll
        for (int jt = 0; jt < NJ; ++jt) acc[jt] = Mfma<T>::op(bq[d][kq][jt][0], db[d], acc[jt]);
#pragma unroll
        for (int jt = 0; jt < NJ; ++jt) acc[jt] = Mfma<T>::op(bq[d][kq][jt][1], df[d], acc[jt]);
      }
      __builtin_amdgcn_sched_barrier(0);
      if (kq + 1 < KSW) diffs();
    }
    const T *Kt = K0t + hb * RB * KST + row * 16 + c;
    if constexpr (KSPLIT) {
      // partial sums of the partner's tile to LDS (read after the barrier);
      // own partial sums and K0 of the own tile kept for the next step
      T *xs = xslot(z, jh);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        xs[64 * v] = jh ? acc[0][v] : acc[1][v];
        pend[0][v] = jh ? acc[1][v] : acc[0][v];
        pk0[0][v] = Kt[out_col(0, v) * KST];
      }
      // the LDS writes complete before the barrier
      __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0)
    } else {
#pragma unroll
      for (int jt = 0; jt < NJ; ++jt) {
#pragma unroll
        for (int v = 0; v < 4; ++v)
          pend[jt][v] = Kt[out_col(jt, v) * KST] - tcoef * acc[jt][v];
      }
    }
    // the loads of step z + 1 (issued during step z + 2 - AH) must have
    // landed before the barrier, those of the later AH - 2 steps may stay in
    // flight (past the chunk end they are clamped into the grid and fill
    // buffers no later step reads)
    wait_vm<(AH - 2) * NLOADS>();
    block_barrier();
    hb = hb + 1 == NB ? 0 : hb + 1;
    zsl[0] = zsl[1];
    zsl[1] = sc;
    sc = zsl[2];
    zsl[2] = zsl[3];
    zsl[3] = zsl[3] + 1 == NS ? 0 : zsl[3] + 1;
    sdma = sdma + 1 == NS ? 0 : sdma + 1;
  }
#pragma unroll
  for (int jt = 0; jt < NOUT; ++jt) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = out_col(jt, v);
      if (valid && j < r)
        buf_store(out_value(jt, v, z1 - 1), rO, xyo + j * ld * TB, (z1 - 1) * plane * TB);
    }
  }
  wait_vm<0>();   // no load into LDS outlives the block
}

// General weighted Gram P(a, b) = sum_x X(x, a) wt(x) Y(x, b) on the matrix
// cores (any p, q <= 112; k_gram_mfma covers the common shapes).  Per block a
// chunk of cells in tiles of 64: the tiles of X (64 x p) and of Y (64 x q)
// are staged in LDS with coalesced loads (consecutive threads read
// consecutive cells of one column), then each wave (one 16-column tile b of
// Y) runs the 16x16x4 MFMAs over the 16 groups of 4 cells for all 16-row
// tiles a of X.  Partial sums of block bx go to partial[bx * pq].
constexpr int kCT = 64;   // cells per staged tile

template <typename T, typename Tc, int NA, typename YF, typename WF>
__global__ __launch_bounds__(512) void k_contract_mfma(GridDev g, const T *__restrict__ X,
                                                      int ldx, int p,
                                                      YF yf, int q, WF wf, int chunk,
                                                      double *__restrict__ partial) {
  using acc_t = typename Mfma<Tc>::acc_t;
  extern __shared__ unsigned char smem_raw[];
  const int pa = 16 * NA + 1;                        // row lengths (odd: no bank conflicts)
  const int nbw = (q + 15) >> 4;
  const int pb = 16 * nbw + 1;
  Tc *Xs = reinterpret_cast<Tc *>(smem_raw);         // [kCT][pa]
  Tc *Ys = Xs + kCT * pa;                            // [kCT][pb]
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int w = tid >> 6, lane = tid & 63;
  const int c = lane & 15, qq = lane >> 4;
  acc_t acc[NA];
#pragma unroll
  for (int at = 0; at < NA; ++at) acc[at] = acc_t{0, 0, 0, 0};
  const int x_begin = blockIdx.x * chunk;
  const int x_end = min(g.n, x_begin + chunk);
  for (int x0 = x_begin; x0 < x_end; x0 += kCT) {
    __syncthreads();
    // staging: clamped, unconditional loads, zeroed by a select
#pragma unroll 4
    for (int e = tid; e < kCT * 16 * NA; e += nthr) {
      const int cc_ = e % kCT, a = e / kCT;
      const int x = x0 + cc_;
      const int xc = min(x, x_end - 1);
      const Tc v = Tc(X[size_t(min(a, p - 1)) * ldx + xc]) * Tc(wf(xc));
      Xs[cc_ * pa + a] = (x < x_end && a < p) ? v : Tc(0);
    }
#pragma unroll 4
    for (int e = tid; e < kCT * 16 * nbw; e += nthr) {
      const int cc_ = e % kCT, b = e / kCT;
      const int x = x0 + cc_;
      const int xc = min(x, x_end - 1), bc = min(b, q - 1);
      const Tc v = Tc(yf(xc, bc));
      Ys[cc_ * pb + b] = (x < x_end && b < q) ? v : Tc(0);
    }
    __syncthreads();
#pragma unroll 4
    for (int k4 = 0; k4 < kCT / 4; ++k4) {
      const int cell = 4 * k4 + qq;
      const Tc bv = Ys[cell * pb + w * 16 + c];
#pragma unroll
      for (int at = 0; at < NA; ++at)
        acc[at] = Mfma<Tc>::op(Xs[cell * pa + at * 16 + c], bv, acc[at]);
    }
  }
  const size_t pq = size_t(p) * q;
  double *out = partial + size_t(blockIdx.x) * pq;
  const int b = w * 16 + c;
#pragma unroll
  for (int at = 0; at < NA; ++at) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = at * 16 + Mfma<Tc>::row(qq, v);
      if (a < p && b < q) out[a + size_t(b) * p] = double(acc[at][v]);
    }
  }
}

// Stencil projections C_dk = X^T D_dk(s o X) of one direction d (blockIdx.y)
// on the matrix cores: both one-sided differences (dk = 2d, 2d + 1) come from
// the same five stencil points, so a block stages the X tile once and the two
// difference tiles from one set of loads.  The X tile carries a 2-cell halo
// on each side (for d = 0 the x neighbours then come from LDS, and for every
// d the centre value is the tile's own), s at the five stencil points of
// each tile cell is staged once per tile, and only the y or z neighbours of
// W = X are loaded per element (clamped, unconditional, masked by a select).
// Four waves; wave w owns the 16-column tiles w, w + 4 of the right factor
// for all 16-row tiles of the left one.  With one or two such tiles the 4 / NA
// waves of a tile split the cells of each staged tile instead, and their sums
// are added in wave order at the end.  Partial sums of block bx go to
// partial[(bx * 2 dim + dk) * p * p].
template <typename T, typename Tc, int NA>
__global__ __launch_bounds__(256) void k_stencil_proj(GridDev g, const T *__restrict__ s,
                                                     const T *__restrict__ X, int ldx, int p,
                                                     int chunk, int nchunk,
                                                     double *__restrict__ partial) {
  using acc_t = typename Mfma<Tc>::acc_t;
  constexpr int CT = sizeof(Tc) == 8 ? 32 : 64;   // cells per staged tile
  constexpr int CH = CT + 4;                      // with a 2-cell halo on each side
  constexpr int PA = 16 * NA + 1;                 // row length (odd: no bank conflicts)
  constexpr int NBT = (NA + 3) / 4;               // right-factor tiles per wave
  constexpr int KSP = NA <= 2 ? 4 / NA : 1;       // waves splitting the cells of a tile
  static_assert(KSP == 1 || (CH * PA + 5 * CT) * sizeof(T) % (4 * sizeof(Tc)) == 0,
                "wave-sum exchange aligned");
  constexpr int PER = CT * 16 * NA / 256;         // staged elements per thread
  constexpr int PERH = (CH * 16 * NA + 255) / 256;
  static_assert((CT * 16 * NA) % 256 == 0, "whole staging rounds");
  extern __shared__ unsigned char smem_raw[];
  T *Xh = reinterpret_cast<T *>(smem_raw);        // [CH][PA] X with halo (storage type)
  T *Sw = Xh + CH * PA;                           // [5][CT] s at the stencil points (0 outside)
  Tc *Yb = reinterpret_cast<Tc *>(Sw + 5 * CT);   // [CT][PA]
  Tc *Yf = Yb + CT * PA;                          // [CT][PA]
  // the left factor is read from the tile's own rows of Xh: beyond the chunk
  // end the differences are zero, and rows a >= p are never written out
  static_assert(sizeof(T) == sizeof(Tc), "left factor read in the storage type");
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
  const int c = lane & 15, qq = lane >> 4;
  // block -> (direction, chunk): the hardware deals blocks round-robin over
  // the 8 XCDs; each XCD gets one contiguous range of chunks of a direction,
  // so the y / z neighbours a chunk reads are mostly its L2's own lines
  const int nblk = gridDim.x, xcd = blockIdx.x & 7;
  const int L = xcd * (nblk >> 3) + min(xcd, nblk & 7) + (blockIdx.x >> 3);
  const int d = L / nchunk, bx = L % nchunk;
  const int st = d == 0 ? 1 : (d == 1 ? g.nx : g.nx * g.ny);
  const int size = d == 0 ? g.nx : (d == 1 ? g.ny : g.nz);
  const T ih = T(g.inv2h[d]);
  acc_t ab[NBT][NA], af[NBT][NA];
#pragma unroll
  for (int bt = 0; bt < NBT; ++bt)
#pragma unroll
    for (int at = 0; at < NA; ++at) ab[bt][at] = af[bt][at] = acc_t{0, 0, 0, 0};
  const int x_begin = bx * chunk;
  const int x_end = min(g.n, x_begin + chunk);
  // The loads of tile x0 + CT (X with halo, s at the stencil points and, for
  // d != 0 and small NA, the y / z neighbours) are issued into registers
  // before the MFMAs of tile x0; all loads are clamped and unconditional.
  constexpr bool EARLY = NA <= 2;
  constexpr int NSW = (5 * CT + 255) / 256;        // s values per thread
  T xr[PERH], sr[NSW];
  T nbv[EARLY ? PER : 1][4];
  // cell offset of stencil point t (0, -1, -2, +1, +2) of tile cell cc; in grid?
  auto s_point = [&](int x0, int e, int &src) {
    const int t = e / CT, cc = e % CT;
    const int xc = min(x0 + cc, x_end - 1);
    const int cd = d == 0 ? xc % g.nx : (d == 1 ? (xc / g.nx) % g.ny : xc / (g.nx * g.ny));
    const int o = t == 0 ? 0 : (t < 3 ? -t : t - 2);
    const bool in = cd + o >= 0 && cd + o < size;
    src = in ? xc + o * st : xc;
    return in;
  };
  auto fetch = [&](int x0) {
#pragma unroll
    for (int i = 0; i < PERH; ++i) {
      const int e = min(tid + 256 * i, CH * 16 * NA - 1);
      const int hc = e % CH, a = e / CH;
      const int xc = min(max(x0 - 2 + hc, 0), g.n - 1);
      xr[i] = X[size_t(min(a, p - 1)) * ldx + xc];
    }
#pragma unroll
    for (int u = 0; u < NSW; ++u) {
      int src;
      (void)s_point(x0, min(tid + 256 * u, 5 * CT - 1), src);
      sr[u] = s[src];
    }
    if constexpr (EARLY) {
      const int cc = tid % CT, xc = min(x0 + cc, x_end - 1);
      const int im1 = max(xc - st, 0), im2 = max(xc - 2 * st, 0);
      const int ip1 = min(xc + st, g.n - 1), ip2 = min(xc + 2 * st, g.n - 1);
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int b = tid / CT + (256 / CT) * i;
        const T *col = X + size_t(min(b, p - 1)) * ldx;
        nbv[i][0] = col[im1];
        nbv[i][1] = col[im2];
        nbv[i][2] = col[ip1];
        nbv[i][3] = col[ip2];
      }
    }
  };
  fetch(x_begin);
  for (int x0 = x_begin; x0 < x_end; x0 += CT) {
    __syncthreads();
    // X on cells x0-2 .. x0+CT+1 (clamped into the grid; only in-tile cells
    // and, for d = 0, in-grid x neighbours of in-tile cells are used)
#pragma unroll
    for (int i = 0; i < PERH; ++i) {
      const int e = tid + 256 * i;
      if (e < CH * 16 * NA) Xh[(e % CH) * PA + e / CH] = xr[i];
    }
    // s at the stencil points of every tile cell, zero outside the grid
#pragma unroll
    for (int u = 0; u < NSW; ++u) {
      const int e = tid + 256 * u;
      int src;
      const bool in = s_point(x0, min(e, 5 * CT - 1), src);
      if (e < 5 * CT) Sw[e] = in ? sr[u] : T(0);
    }
    __syncthreads();
    // each thread keeps one cell (cc = tid % CT) and walks the columns b
    {
      const int cc = tid % CT, x = x0 + cc, xc = min(x, x_end - 1);
      const bool xin = x < x_end;
      // s-weights of the one-sided differences with 1 / (2 Delta) folded in,
      // formed once per cell; the centre terms of the two differences are
      // negatives of each other, so one product serves both
      const T cb0 = T(3) * ih * Sw[cc], cb1 = T(-4) * ih * Sw[CT + cc];
      const T cb2 = ih * Sw[2 * CT + cc];
      const T cf1 = T(4) * ih * Sw[3 * CT + cc], cf2 = -ih * Sw[4 * CT + cc];
      auto put = [&](int b, T w0, T wm1, T wm2, T wp1, T wp2) {
        const T t0 = cb0 * w0;
        const T db = cb2 * wm2 + (cb1 * wm1 + t0);
        const T df = cf2 * wp2 + (cf1 * wp1 - t0);
        const bool ok = xin && b < p;
        Yb[cc * PA + b] = ok ? Tc(db) : Tc(0);
        Yf[cc * PA + b] = ok ? Tc(df) : Tc(0);
      };
      if (d == 0) {   // x neighbours from the halo'd tile
#pragma unroll
        for (int i = 0; i < PER; ++i) {
          const int b = tid / CT + (256 / CT) * i;
          put(b, Xh[(cc + 2) * PA + b], Xh[(cc + 1) * PA + b], Xh[cc * PA + b],
              Xh[(cc + 3) * PA + b], Xh[(cc + 4) * PA + b]);
        }
      } else if constexpr (EARLY) {   // y or z neighbours loaded above
#pragma unroll
        for (int i = 0; i < PER; ++i) {
          const int b = tid / CT + (256 / CT) * i;
          put(b, Xh[(cc + 2) * PA + b], nbv[i][0], nbv[i][1], nbv[i][2], nbv[i][3]);
        }
      } else {        // y or z neighbours from memory (clamped; masked by s = 0)
        const int im1 = max(xc - st, 0), im2 = max(xc - 2 * st, 0);
        const int ip1 = min(xc + st, g.n - 1), ip2 = min(xc + 2 * st, g.n - 1);
#pragma unroll
        for (int i = 0; i < PER; ++i) {
          const int b = tid / CT + (256 / CT) * i;
          const T *col = X + size_t(min(b, p - 1)) * ldx;
          put(b, Xh[(cc + 2) * PA + b], col[im1], col[im2], col[ip1], col[ip2]);
        }
      }
    }
    fetch(x0 + CT);   // past the chunk end: clamped, unused
    __syncthreads();
#pragma unroll 2
    for (int k4 = KSP > 1 ? w / NA : 0; k4 < CT / 4; k4 += KSP) {
      const int cell = 4 * k4 + qq;
#pragma unroll
      for (int bt = 0; bt < NBT; ++bt) {
        // a wave without a tile of its own repeats the last one (no branch
        // around the MFMAs; its sums are not written out)
        const int btile = KSP > 1 ? w % NA : min(w + 4 * bt, NA - 1);
        const Tc yb = Yb[cell * PA + btile * 16 + c], yf = Yf[cell * PA + btile * 16 + c];
#pragma unroll
        for (int at = 0; at < NA; ++at) {
          const Tc xa = Xh[(cell + 2) * PA + at * 16 + c];
          ab[bt][at] = Mfma<Tc>::op(xa, yb, ab[bt][at]);
          af[bt][at] = Mfma<Tc>::op(xa, yf, af[bt][at]);
        }
      }
    }
  }
  if constexpr (KSP > 1) {
    // sums of the waves w >= NA through LDS (the staging buffers are free
    // once every wave is past its last MFMA), added in wave order
    acc_t *xb = reinterpret_cast<acc_t *>(Yb);
    __syncthreads();
    if (w >= NA) {
#pragma unroll
      for (int at = 0; at < NA; ++at) {
        xb[((w - NA) * NA + at) * 2 * 64 + lane] = ab[0][at];
        xb[(((w - NA) * NA + at) * 2 + 1) * 64 + lane] = af[0][at];
      }
    }
    __syncthreads();
    if (w < NA) {
      for (int kp = 1; kp < KSP; ++kp) {
        const int o = kp * NA + w - NA;
#pragma unroll
        for (int at = 0; at < NA; ++at) {
          const acc_t vb = xb[(o * NA + at) * 2 * 64 + lane];
          const acc_t vf = xb[((o * NA + at) * 2 + 1) * 64 + lane];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            ab[0][at][v] += vb[v];
            af[0][at][v] += vf[v];
          }
        }
      }
    }
  }
  const size_t pq = size_t(p) * p;
  double *outb = partial + (size_t(bx) * 2 * g.dim + 2 * d) * pq;
  double *outf = outb + pq;
#pragma unroll
  for (int bt = 0; bt < NBT; ++bt) {
    // >= p for a repeated tile or a wave whose sums went to another
    const int b = (KSP > 1 && w >= NA) ? p : (w + 4 * bt) * 16 + c;
#pragma unroll
    for (int at = 0; at < NA; ++at) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = at * 16 + Mfma<Tc>::row(qq, v);
        if (a < p && b < p) {
          outb[a + size_t(b) * p] = double(ab[bt][at][v]);
          outf[a + size_t(b) * p] = double(af[bt][at][v]);
        }
      }
    }
  }
}

// dynamic LDS of k_stencil_proj
template <typename T, typename Tc, int NA>
constexpr size_t stencil_proj_lds() {
  constexpr int CT = sizeof(Tc) == 8 ? 32 : 64;
  // the two difference tiles; the wave-sum exchange of NA <= 2 reuses them
  // (extended where it needs more room)
  constexpr size_t diff = size_t(2) * CT * (16 * NA + 1) * sizeof(Tc);
  constexpr size_t xchg = NA <= 2 ? size_t(4 - NA) * NA * 2 * 64 * 4 * sizeof(Tc) : 0;
  return size_t(CT + 4) * (16 * NA + 1) * sizeof(T) + size_t(5) * CT * sizeof(T) +
         (diff > xchg ? diff : xchg);
}

// Weighted Grams G(a, b) = sum_x X(x, a) wt(x) Y(x, b) on the matrix cores
// (Y = yf(x, b), wt = wf(x)).  Per block a chunk of cells in tiles of 64:
// every thread stages one cell of the tile (the weight is evaluated once per
// cell) for a fixed stride of columns, all loads of the tile in flight
// together; then the 4 waves share the NA x NB output tiles (a wave without a
// tile of its own repeats the last one and does not write it).  Partial sums
// of block bx go to partial[bx * p * q].  With same (Y is X, unit weights,
// square tiles) only X is loaded and its staged tile is both operands.
constexpr int kGramBlocks = 2048;

template <typename T, typename Tc, int NA, int NB, typename YF, typename WF>
__global__ __launch_bounds__(256) void k_gram_mfma(int n, const T *__restrict__ X, int ldx, int p,
                                                  YF yf, int q, WF wf, int chunk,
                                                  double *__restrict__ partial, bool same) {
  using acc_t = typename Mfma<Tc>::acc_t;
  constexpr int CT = 64;
  constexpr int PA = 16 * NA + 1, PB = 16 * NB + 1;   // odd row lengths
  constexpr int NT = NA * NB, TPW = (NT + 3) / 4;     // output tiles, per wave
  constexpr int PERA = CT * 16 * NA / 256, PERB = CT * 16 * NB / 256;
  extern __shared__ unsigned char smem_raw[];
  Tc *Xs = reinterpret_cast<Tc *>(smem_raw);          // [CT][PA]
  Tc *Ys = Xs + CT * PA;                              // [CT][PB]
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c = lane & 15, qq = lane >> 4;
  acc_t acc[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u) acc[u] = acc_t{0, 0, 0, 0};
  const int x_begin = blockIdx.x * chunk;
  const int x_end = min(n, x_begin + chunk);
  const int cc = tid % CT, col0 = tid / CT;
  // the loads of the next tile are issued before the MFMAs of this one
  T xr[PERA], yr[PERB], wr;
  auto fetch = [&](int x0) {
    const int xc = min(x0 + cc, x_end - 1);   // clamped: loads stay unconditional
    wr = wf(xc);
#pragma unroll
    for (int i = 0; i < PERA; ++i) xr[i] = X[size_t(min(col0 + 4 * i, p - 1)) * ldx + xc];
    if (!same)
#pragma unroll
      for (int i = 0; i < PERB; ++i) yr[i] = yf(xc, min(col0 + 4 * i, q - 1));
  };
  fetch(x_begin);
  for (int x0 = x_begin; x0 < x_end; x0 += CT) {
    __syncthreads();
    {
      const bool xin = x0 + cc < x_end;
      const Tc wt = Tc(wr);
#pragma unroll
      for (int i = 0; i < PERA; ++i) {
        const int a = col0 + 4 * i;
        const Tc v = Tc(xr[i]) * wt;
        Xs[cc * PA + a] = (xin && a < p) ? v : Tc(0);
      }
      if (!same)
#pragma unroll
        for (int i = 0; i < PERB; ++i) {
          const int b = col0 + 4 * i;
          Ys[cc * PB + b] = (xin && b < q) ? Tc(yr[i]) : Tc(0);
        }
    }
    __syncthreads();
    fetch(x0 + CT);
    // the right factor: its own staged tile, or X's when it is X (same values)
    const Tc *Yt = same ? Xs : Ys;
    const int pb = same ? PA : PB;
#pragma unroll 2
    for (int k4 = 0; k4 < CT / 4; ++k4) {
      const int cell = 4 * k4 + qq;
#pragma unroll
      for (int u = 0; u < TPW; ++u) {
        const int t = min(w + 4 * u, NT - 1), ta = t % NA, tb = t / NA;
        acc[u] = Mfma<Tc>::op(Xs[cell * PA + ta * 16 + c], Yt[cell * pb + tb * 16 + c], acc[u]);
      }
    }
  }
  double *out = partial + size_t(blockIdx.x) * p * q;
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int t = w + 4 * u;
    if (t < NT) {
      const int ta = t % NA, tb = t / NA, b = tb * 16 + c;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int a = ta * 16 + Mfma<Tc>::row(qq, v);
        if (a < p && b < q) out[a + size_t(b) * p] = double(acc[u][v]);
      }
    }
  }
}

// Bp[(dk RB + k) RB + j] = B_dk(k, j) (zero padded to RB), from the
// column-major double couplings (leading dimension ldb, blocks ldb^2 apart).
template <typename T>
__global__ void k_pack_couplings(int ndk, int r, int RB, const double *__restrict__ B, int ldb,
                                 T *__restrict__ Bp) {
  int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= ndk * RB * RB) return;
  int j = e % RB, k = (e / RB) % RB, dk = e / (RB * RB);
  double v = (k < r && j < r) ? B[size_t(dk) * ldb * ldb + k + size_t(j) * ldb] : 0.0;
  Bp[e] = T(v);
}

// ------------------------------------------------------------------ reductions
// out[e] = sum_b partial[b * elems + e] in a fixed order: 8 groups of threads
// take every 8th block for 32 consecutive elements, then group sums combine.
constexpr int kRedE = 32, kRedG = 8;
__global__ __launch_bounds__(kRedE * kRedG) void k_reduce_partials(
    const double *__restrict__ partial, int nblocks, int elems, double *__restrict__ out) {
  __shared__ double red[kRedG][kRedE];
  const int el = threadIdx.x % kRedE, grp = threadIdx.x / kRedE;
  const int e = blockIdx.x * kRedE + el;
  double s = 0.0;
  if (e < elems)
    for (int b = grp; b < nblocks; b += kRedG) s += partial[size_t(b) * elems + e];
  red[grp][el] = s;
  __syncthreads();
  if (grp == 0 && e < elems) {
    double t = 0.0;
    for (int g = 0; g < kRedG; ++g) t += red[g][el];
    out[e] = t;
  }
}

// doubles of a buffer of `total` left after `blocks` blocks of `per`
static size_t room_after(size_t total, size_t blocks, size_t per) {
  return total > blocks * per ? total - blocks * per : 0;
}

// First level of the partial-sum reduction: segment blockIdx.y of the
// nblocks partial blocks, 64 elements per workgroup, the four waves take
// every fourth block of the segment (four independent sums per lane).
__global__ __launch_bounds__(256) void k_reduce_partials_seg(const double *__restrict__ partial,
                                                             int nblocks, int elems, int nseg,
                                                             double *__restrict__ seg_out) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + lane, sg = blockIdx.y;
  const int b0 = int(int64_t(sg) * nblocks / nseg), b1 = int(int64_t(sg + 1) * nblocks / nseg);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  if (e < elems) {
    const double *src = partial + e;
    int b = b0 + w;
    for (; b + 12 < b1; b += 16) {
      s0 += src[size_t(b) * elems];
      s1 += src[size_t(b + 4) * elems];
      s2 += src[size_t(b + 8) * elems];
      s3 += src[size_t(b + 12) * elems];
    }
    for (; b < b1; b += 4) s0 += src[size_t(b) * elems];
  }
  red[w][lane] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  if (w == 0 && e < elems)
    seg_out[size_t(sg) * elems + e] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// out[e] = sum_b partial[b * elems + e] in a fixed order.  Given room for
// scratch_elems doubles at scratch (disjoint from partial and out), the
// blocks are first summed in up to 64 segments (many workgroups), then the
// segment sums.
void reduce_partials(const double *partial, int nblocks, int elems, double *out, hipStream_t st,
                     double *scratch = nullptr, size_t scratch_elems = 0) {
  if (elems <= 0) return;
  int nseg = std::min(64, nblocks / 16);
  if (scratch == nullptr) nseg = 0;
  nseg = int(std::min<size_t>(size_t(std::max(nseg, 0)), scratch_elems / size_t(elems)));
  if (nseg >= 2) {
    double *seg = scratch;
    k_reduce_partials_seg<<<dim3((elems + 63) / 64, nseg), 256, 0, st>>>(partial, nblocks, elems,
                                                                        nseg, seg);
    partial = seg;
    nblocks = nseg;
  }
  k_reduce_partials<<<(elems + kRedE - 1) / kRedE, kRedE * kRedG, 0, st>>>(partial, nblocks,
                                                                         elems, out);
}

// scatter a reduced p x q block into a col-major matrix with leading dim ldc
__global__ void k_scatter(const double *__restrict__ src, int p, int q, int nblk,
                          double *__restrict__ dst, int ldc, size_t dst_stride) {
  int e = blockIdx.x * kBlock + threadIdx.x;
  int pq = p * q;
  if (e >= pq * nblk) return;
  int blk = e / pq, o = e % pq;
  int a = o % p, b = o / p;
  dst[blk * dst_stride + a + size_t(b) * ldc] = src[e];
}

template <typename T>
__global__ void k_sumsq(int n, const T *__restrict__ X, int ld, int q, double *partial) {
  __shared__ double red[kBlock];
  double acc = 0.0;
  // FP32 with aligned columns: 16-byte loads of four cells, scalar tail
  if (sizeof(T) == 4 && ld % 4 == 0 && (reinterpret_cast<uintptr_t>(X) & 15) == 0) {
    const int n4 = n >> 2;
    for (int c = 0; c < q; ++c) {
      const float4 *col = reinterpret_cast<const float4 *>(X + size_t(c) * ld);
#pragma unroll 4
      for (int x = blockIdx.x * kBlock + threadIdx.x; x < n4; x += gridDim.x * kBlock) {
        const float4 v = col[x];
        acc += double(v.x) * v.x + double(v.y) * v.y + double(v.z) * v.z + double(v.w) * v.w;
      }
      for (int x = 4 * n4 + blockIdx.x * kBlock + threadIdx.x; x < n; x += gridDim.x * kBlock) {
        const double v = double(X[size_t(c) * ld + x]);
        acc += v * v;
      }
    }
  } else {
    for (int c = 0; c < q; ++c)
#pragma unroll 4
      for (int x = blockIdx.x * kBlock + threadIdx.x; x < n; x += gridDim.x * kBlock) {
        const double v = double(X[size_t(c) * ld + x]);
        acc += v * v;
      }
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// ------------------------------------------------------------------ updates
// Tall-skinny update on the matrix cores:
//   Z(x, j) = alpha Y(x, j) + beta sum_a X(x, a) G(a, j) + sum_i src_i(x) sC(j, i),
// src_i(x) = sdt w_i(x) psi(x) (only when sw != nullptr), and optionally
// dose(x) += dscale sum_j Z(x, j) dc(j).  The coefficient matrix (beta G with
// the rows sC^T appended, as T, rows padded to a multiple of 4) is staged in
// LDS once per block; the waves then take 32-cell tiles (two 16-cell halves)
// and compute per half the transposed tile Z^T = Gs^T X^T: A(j, kk) = Gs(4t + kk, 16 jt + j) from LDS,
// B(kk, i) = X(x0 + i, 4t + kk) from lane i + 16 kk, so the stores of 16
// consecutive lanes are 16 consecutive cells of one column.  Y may alias Z
// (each element is read and written by the same lane); X must not.
constexpr int kUpdBlocks = 2048;
constexpr int kUpdChunk = 8;      // MFMA k-steps whose loads are issued together

template <typename T, int NQ, bool HY>
__global__ __launch_bounds__(256) void k_update_mfma(
    int n, const T *__restrict__ X, int ldx, int p, const double *__restrict__ G, int ldg,
    double beta, const T *Y, int ldy, double alpha, T *Z, int ldz, int q,
    double *__restrict__ dose, const double *__restrict__ dc, double dscale,
    const T *__restrict__ sw, int n_mat, int n_src, const T *__restrict__ spsi, size_t pstride,
    const double *__restrict__ sC, int ldsc, double sdt) {
  using acc_t = typename Mfma<T>::acc_t;
  constexpr int QS = 16 * NQ;
  extern __shared__ unsigned char smem_raw[];
  const int ne = p + (sw != nullptr ? n_src : 0);
  const int nk = (ne + 3) & ~3;
  T *Gs = reinterpret_cast<T *>(smem_raw);                 // [nk][QS]
  double *dcs = reinterpret_cast<double *>(Gs + nk * QS);  // [QS]
  for (int e = threadIdx.x; e < nk * QS; e += blockDim.x) {
    const int a = e / QS, j = e % QS;
    double v = 0.0;
    if (j < q) {
      if (a < p) v = beta * G[size_t(j) * ldg + a];
      else if (a < ne) v = sC[j + size_t(a - p) * ldsc];
    }
    Gs[e] = T(v);
  }
  if (dose != nullptr)
    for (int j = threadIdx.x; j < QS; j += blockDim.x) dcs[j] = j < q ? dc[j] : 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int c = lane & 15, qd = lane >> 4;
  const int waves = gridDim.x * (blockDim.x >> 6);
  // 32-cell tiles: a wave takes two 16-cell halves at once, so that the loads
  // of both (and the Y loads, issued first) are in flight together
  const int ntiles = (n + 31) >> 5;
  for (int tile = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); tile < ntiles;
       tile += waves) {
    int x[2], xc[2];
    bool valid[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      x[h] = 32 * tile + 16 * h + c;
      valid[h] = x[h] < n;
      xc[h] = valid[h] ? x[h] : n - 1;   // clamped: loads stay unconditional
    }
    T yraw[2][NQ][4];
    if constexpr (HY) {
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int jt = 0; jt < NQ; ++jt)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            yraw[h][jt][v] = Y[size_t(min(16 * jt + Mfma<T>::row(qd, v), q - 1)) * ldy + xc[h]];
    }
    acc_t acc[2][NQ];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int jt = 0; jt < NQ; ++jt) acc[h][jt] = acc_t{0, 0, 0, 0};
    for (int k0 = 0; k0 < nk; k0 += 4 * kUpdChunk) {
      T b[2][kUpdChunk];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int u = 0; u < kUpdChunk; ++u) {
          const int k = k0 + 4 * u + qd;
          T v = X[size_t(min(k, p - 1)) * ldx + xc[h]];
          // source column e = b n_mat + i: sdt w_i(x) psi_b(x), loaded only
          // in the column blocks that hold source columns (wave-uniform test)
          if (sw != nullptr && k0 + 4 * u + 3 >= p) {
            const int e = min(max(k - p, 0), n_src - 1);
            const int b = e / n_mat, i = e - b * n_mat;
            const double src = sdt * double(spsi[size_t(b) * pstride + xc[h]]);
            const T sv = T(double(sw[size_t(i) * n + xc[h]]) * src);
            v = k < p ? v : sv;
          }
          b[h][u] = (valid[h] && k < ne) ? v : T(0);
        }
#pragma unroll
      for (int u = 0; u < kUpdChunk; ++u) {
        if (k0 + 4 * u < nk) {
          const T *ga = Gs + (k0 + 4 * u + qd) * QS + c;
#pragma unroll
          for (int jt = 0; jt < NQ; ++jt) {
            const T gv = ga[16 * jt];
#pragma unroll
            for (int h = 0; h < 2; ++h) acc[h][jt] = Mfma<T>::op(gv, b[h][u], acc[h][jt]);
          }
        }
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double dsum = 0.0;
#pragma unroll
      for (int jt = 0; jt < NQ; ++jt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int j = 16 * jt + Mfma<T>::row(qd, v);
          double yv = 0.0;
          if constexpr (HY) yv = alpha * double(yraw[h][jt][v]);
          if (valid[h] && j < q) {
            const T zv = T(double(acc[h][jt][v]) + yv);
            Z[size_t(j) * ldz + x[h]] = zv;
            if (dose != nullptr) dsum += double(zv) * dcs[j];
          }
        }
      }
      if (dose != nullptr) {
        dsum += __shfl_xor(dsum, 16);
        dsum += __shfl_xor(dsum, 32);
        if (qd == 0 && valid[h]) dose[x[h]] += dscale * dsum;
      }
    }
  }
}

// FP32 form with 16-byte accesses: a wave takes 64 cells and lane (c, qd)
// loads the four consecutive cells 64 t + 4 c .. 64 t + 4 c + 3 of a column at
// once; MFMA i (i = 0..3) takes the cells 64 t + 4 c + i, so the four
// accumulators of one output row are again four consecutive cells (one
// 16-byte store).  Each output is formed by the same MFMA sequence as in
// k_update_mfma.  A tile that ends past n takes clamped scalar accesses.
template <int NQ, bool HY>
__global__ __launch_bounds__(256) void k_update_vec(
    int n, const float *__restrict__ X, int ldx, int p, const double *__restrict__ G, int ldg,
    double beta, const float *Y, int ldy, double alpha, float *Z, int ldz, int q,
    double *__restrict__ dose, const double *__restrict__ dc, double dscale,
    const float *__restrict__ sw, int n_mat, int n_src, const float *__restrict__ spsi,
    size_t pstride, const double *__restrict__ sC, int ldsc, double sdt) {
  using acc_t = typename Mfma<float>::acc_t;
  constexpr int QS = 16 * NQ;
  extern __shared__ unsigned char smem_raw[];
  const int ne = p + (sw != nullptr ? n_src : 0);
  const int nk = (ne + 3) & ~3;
  float *Gs = reinterpret_cast<float *>(smem_raw);             // [nk][QS]
  double *dcs = reinterpret_cast<double *>(Gs + nk * QS);      // [QS]
  for (int e = threadIdx.x; e < nk * QS; e += blockDim.x) {
    const int a = e / QS, j = e % QS;
    double v = 0.0;
    if (j < q) {
      if (a < p) v = beta * G[size_t(j) * ldg + a];
      else if (a < ne) v = sC[j + size_t(a - p) * ldsc];
    }
    Gs[e] = float(v);
  }
  if (dose != nullptr)
    for (int j = threadIdx.x; j < QS; j += blockDim.x) dcs[j] = j < q ? dc[j] : 0.0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int c = lane & 15, qd = lane >> 4;
  const int waves = gridDim.x * (blockDim.x >> 6);
  const int ntiles = (n + 63) >> 6;
  for (int tile = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); tile < ntiles;
       tile += waves) {
    const int xb = 64 * tile + 4 * c;
    const bool full = 64 * tile + 64 <= n;   // wave-uniform
    bool valid[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) valid[i] = xb + i < n;
    // four consecutive cells of one column
    auto ld4 = [&](const float *col) {
      if (full) return *reinterpret_cast<const float4 *>(col + xb);
      float4 v;
      v.x = col[min(xb, n - 1)];
      v.y = col[min(xb + 1, n - 1)];
      v.z = col[min(xb + 2, n - 1)];
      v.w = col[min(xb + 3, n - 1)];
      return v;
    };
    float4 yraw[NQ][4];
    if constexpr (HY) {
#pragma unroll
      for (int jt = 0; jt < NQ; ++jt)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          yraw[jt][v] = ld4(Y + size_t(min(16 * jt + Mfma<float>::row(qd, v), q - 1)) * ldy);
    }
    acc_t acc[4][NQ];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int jt = 0; jt < NQ; ++jt) acc[i][jt] = acc_t{0, 0, 0, 0};
    for (int k0 = 0; k0 < nk; k0 += 4 * kUpdChunk) {
      float b[kUpdChunk][4];
#pragma unroll
      for (int u = 0; u < kUpdChunk; ++u) {
        const int k = k0 + 4 * u + qd;
        const float4 xv = ld4(X + size_t(min(k, p - 1)) * ldx);
        float v[4] = {xv.x, xv.y, xv.z, xv.w};
        // source column e = b n_mat + i: sdt w_i(x) psi_b(x), loaded only in
        // the column blocks that hold source columns (wave-uniform test)
        if (sw != nullptr && k0 + 4 * u + 3 >= p) {
          const int e = min(max(k - p, 0), n_src - 1);
          const int b = e / n_mat, im = e - b * n_mat;
          const float4 wv = ld4(sw + size_t(im) * n);
          const float4 ps = ld4(spsi + size_t(b) * pstride);
          const float wa[4] = {wv.x, wv.y, wv.z, wv.w};
          const float pa[4] = {ps.x, ps.y, ps.z, ps.w};
#pragma unroll
          for (int i = 0; i < 4; ++i)
            v[i] = k < p ? v[i] : float(double(wa[i]) * (sdt * double(pa[i])));
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) b[u][i] = (valid[i] && k < ne) ? v[i] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < kUpdChunk; ++u) {
        if (k0 + 4 * u < nk) {
          const float *ga = Gs + (k0 + 4 * u + qd) * QS + c;
#pragma unroll
          for (int jt = 0; jt < NQ; ++jt) {
            const float gv = ga[16 * jt];
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i][jt] = Mfma<float>::op(gv, b[u][i], acc[i][jt]);
          }
        }
      }
    }
    double dsum[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int jt = 0; jt < NQ; ++jt) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = 16 * jt + Mfma<float>::row(qd, v);
        if (j < q) {
          float zv[4];
          const float yr[4] = {HY ? yraw[jt][v].x : 0.0f, HY ? yraw[jt][v].y : 0.0f,
                               HY ? yraw[jt][v].z : 0.0f, HY ? yraw[jt][v].w : 0.0f};
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double yv = HY ? alpha * double(yr[i]) : 0.0;
            zv[i] = float(double(acc[i][jt][v]) + yv);
            if (dose != nullptr) dsum[i] += double(zv[i]) * dcs[j];
          }
          float *zc = Z + size_t(j) * ldz;
          if (full) {
            *reinterpret_cast<float4 *>(zc + xb) = make_float4(zv[0], zv[1], zv[2], zv[3]);
          } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
              if (valid[i]) zc[xb + i] = zv[i];
          }
        }
      }
    }
    if (dose != nullptr) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        dsum[i] += __shfl_xor(dsum[i], 16);
        dsum[i] += __shfl_xor(dsum[i], 32);
        if (qd == 0 && valid[i]) dose[xb + i] += dscale * dsum[i];
      }
    }
  }
}


}  // namespace

// ================================================================== launchers

template <typename T>
void launch_inverse_stop(const GridDev &g, const T *w, int n_mat, const double *Si, T *s,
                         Ctl *ctl, hipStream_t st) {
  k_inverse_stop<T><<<(g.n + kBlock - 1) / kBlock, kBlock, 0, st>>>(g, w, n_mat, Si, s, ctl);
}

template <typename T>
void launch_pack_couplings(int ndk, int r, const double *B, int ldb, T *Bp, hipStream_t st) {
  const int RB = ((r + 15) / 16) * 16;
  const int tot = ndk * RB * RB;
  k_pack_couplings<T><<<(tot + kBlock - 1) / kBlock, kBlock, 0, st>>>(ndk, r, RB, B, ldb, Bp);
}

template <typename T, int NJ>
static void kstage_launch(const GridDev &g, const T *s, const T *W, const T *K0, T *out, int ld,
                          int r, const T *Bp, double coef, int tiled, int ntiles,
                          hipStream_t st) {
  const size_t shm = size_t(2) * g.dim * (16 * NJ) * (16 * NJ) * sizeof(T);
  const bool lds = shm <= 65536;
  auto kern = lds ? k_kstage_mfma<T, NJ, true> : k_kstage_mfma<T, NJ, false>;
  // resident blocks per CU and CU count, queried once per instantiation
  static std::atomic<int> per_cu_cache[2] = {0, 0};
  static std::atomic<int> n_cu_cache{0};
  int n_cu = n_cu_cache.load(std::memory_order_relaxed);
  if (n_cu <= 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n_cu <= 0)
      n_cu = 256;
    n_cu_cache.store(n_cu, std::memory_order_relaxed);
  }
  int pc = per_cu_cache[lds ? 1 : 0].load(std::memory_order_relaxed);
  if (pc <= 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, reinterpret_cast<const void *>(kern),
                                                     256, lds ? shm : 0) != hipSuccess ||
        pc <= 0)
      pc = 1;
    per_cu_cache[lds ? 1 : 0].store(pc, std::memory_order_relaxed);
  }
  const int cap = std::max(1, pc * n_cu / 8);
  const int blocks = 8 * std::min(cap, std::max(1, (ntiles + 7) / 8));
  kern<<<blocks, 256, lds ? shm : 0, st>>>(g, s, W, K0, out, ld, r, Bp, coef, tiled, ntiles);
}

template <typename T, int NJ, int DIM, int JS = 1>
static void kstage_brick_launch(const GridDev &g, const T *s, const T *W, const T *K0, T *out,
                                int ld, int r, const T *Bp, double coef, hipStream_t st) {

  constexpr int NT = 64 * kBrickBY * JS;
  const size_t shm = brick_lds_bytes(16 * NJ, int(sizeof(T)), JS);
  auto kern = k_kstage_brick<T, NJ, DIM, JS>;
  static std::atomic<int> blocks_cache{0};
  int cap = blocks_cache.load(std::memory_order_relaxed);
  if (cap <= 0) {
    if (shm > 65536)
      (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
    int dev = 0, n_cu = 0, pc = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n_cu <= 0)
      n_cu = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&pc, reinterpret_cast<const void *>(kern),
                                                     NT, shm) != hipSuccess ||
        pc <= 0)
      pc = 1;
    cap = pc * n_cu;
    blocks_cache.store(cap, std::memory_order_relaxed);
  }
  const int nbx = (g.nx + 15) / 16, nby = (g.ny + kBrickBY - 1) / kBrickBY;
  const int ncol = nbx * nby;
  int nzc = std::max(1, std::min(g.nz, (cap + ncol - 1) / ncol));
  const int zchunk = (g.nz + nzc - 1) / nzc;
  nzc = (g.nz + zchunk - 1) / zchunk;
  kern<<<ncol * nzc, NT, shm, st>>>(g, s, W, K0, out, ld, r, Bp, coef, nzc, zchunk);
}

template <typename T>
void launch_kstep_stage(const GridDev &g, const T *s, const T *W, const T *K0, T *out, int ld,
                        int r, const T *Bp, double coef, hipStream_t st) {
  // z-march kernel where its LDS fits (r <= 32 in FP32, r <= 16 in FP64) and
  // its buffers end below the out-of-range offset of its zero loads
  if (kUseBrick && r <= (sizeof(T) == 4 ? 32 : 16) &&
      size_t(ld) * 16 * ((r + 15) / 16) * sizeof(T) < size_t(kOobOffset)) {
    const bool three = g.dim == 3;
    if (r <= 16 && three) kstage_brick_launch<T, 1, 3>(g, s, W, K0, out, ld, r, Bp, coef, st);
    else if (r <= 16) kstage_brick_launch<T, 1, 2>(g, s, W, K0, out, ld, r, Bp, coef, st);
    else if constexpr (sizeof(T) == 4) {
      if (three) kstage_brick_launch<T, 2, 3, kBrickSplit>(g, s, W, K0, out, ld, r, Bp, coef, st);
      else kstage_brick_launch<T, 2, 2, kBrickSplit>(g, s, W, K0, out, ld, r, Bp, coef, st);
    }
    return;
  }
  const int tiled = (g.nx % 16 == 0) ? 1 : 0;
  int ntiles;
  if (tiled) {
    const int px = g.nx / 16, py = (g.ny + 3) / 4;
    const int tpx = std::min(2, px), tpy = std::min(8, py);
    const int ncol = ((px + tpx - 1) / tpx) * ((py + tpy - 1) / tpy);
    ntiles = ncol * tpx * tpy * g.nz;
  } else {
    ntiles = (g.n + 63) / 64;
  }
  switch ((r + 15) / 16) {
    case 1: kstage_launch<T, 1>(g, s, W, K0, out, ld, r, Bp, coef, tiled, ntiles, st); break;
    case 2: kstage_launch<T, 2>(g, s, W, K0, out, ld, r, Bp, coef, tiled, ntiles, st); break;
    case 3: kstage_launch<T, 3>(g, s, W, K0, out, ld, r, Bp, coef, tiled, ntiles, st); break;
    default: kstage_launch<T, 4>(g, s, W, K0, out, ld, r, Bp, coef, tiled, ntiles, st); break;
  }
}

template <typename T, typename Tc, typename YF, typename WF>
static void contract(const GridDev &g, const T *X, int ldx, int p, YF yf, int q, WF wf,
                     double *partial, size_t partial_elems, hipStream_t st, int &nb_out) {
  const size_t pq = size_t(p) * q;
  const int na = (p + 15) / 16, nbw = (q + 15) / 16;
  int nb = (kContractWaves + nbw - 1) / nbw;
  nb = std::max(1, std::min({nb, kMaxPartialBlocks, (g.n + kCT - 1) / kCT}));
  // partial sums of nb blocks plus their sum behind them
  while (nb > 1 && size_t(nb + 1) * pq > partial_elems) nb /= 2;
  int chunk = (g.n + nb - 1) / nb;
  chunk = (chunk + 3) / 4 * 4;
  nb = (g.n + chunk - 1) / chunk;
  dim3 grid(nb), block(64 * nbw);
  const size_t shm = size_t(kCT) * (16 * na + 1 + 16 * nbw + 1) * sizeof(Tc);
#define DLRA_CONTRACT(NA)                                                                  \
  do {                                                                                     \
    auto kern = k_contract_mfma<T, Tc, NA, YF, WF>;                                        \
    if (shm > 65536)                                                                       \
      (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kern),                       \
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));    \
    kern<<<grid, block, shm, st>>>(g, X, ldx, p, yf, q, wf, chunk, partial);               \
  } while (0)
  switch (na) {
    case 1: DLRA_CONTRACT(1); break;
    case 2: DLRA_CONTRACT(2); break;
    case 3: DLRA_CONTRACT(3); break;
    case 4: DLRA_CONTRACT(4); break;
    case 5: DLRA_CONTRACT(5); break;
    case 6: DLRA_CONTRACT(6); break;
    default: DLRA_CONTRACT(7); break;
  }
#undef DLRA_CONTRACT
  nb_out = nb;
}

// Gram launch: SQUARE (q == p) uses NB = NA tiles, otherwise q <= 16 (NB = 1);
// p <= 112 (NA <= 7) in both cases, which the callers check.
template <typename T, typename Tc, int NA, int NB, typename YF, typename WF>
static void gram_launch_na(int n, const T *X, int ldx, int p, YF yf, int q, WF wf, int nb,
                           int chunk, double *partial, hipStream_t st, bool same) {
  const size_t shm = size_t(64) * (16 * NA + 1 + 16 * NB + 1) * sizeof(Tc);
  auto kern = k_gram_mfma<T, Tc, NA, NB, YF, WF>;
  if (shm > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
  kern<<<nb, 256, shm, st>>>(n, X, ldx, p, yf, q, wf, chunk, partial, same && NA == NB);
}

template <typename T, typename Tc, bool SQUARE, typename YF, typename WF>
static void gram(int n, const T *X, int ldx, int p, YF yf, int q, WF wf, double *partial,
                 size_t partial_elems, hipStream_t st, int &nb_out, bool same = false) {
  const size_t pq = size_t(p) * q;
  int nb = std::max(1, std::min(kGramBlocks, (n + 63) / 64));
  while (nb > 1 && size_t(nb + 1) * pq > partial_elems) nb /= 2;
  int chunk = std::max(1, (n + nb - 1) / nb);
  chunk = (chunk + 63) / 64 * 64;
  nb = (n + chunk - 1) / chunk;
  const int na = (p + 15) / 16;
#define DLRA_GRAM(NA)                                                                       \
  gram_launch_na<T, Tc, NA, SQUARE ? NA : 1>(n, X, ldx, p, yf, q, wf, nb, chunk, partial, st, \
                                             same)
  switch (na) {
    case 1: DLRA_GRAM(1); break;
    case 2: DLRA_GRAM(2); break;
    case 3: DLRA_GRAM(3); break;
    case 4: DLRA_GRAM(4); break;
    case 5: DLRA_GRAM(5); break;
    case 6: DLRA_GRAM(6); break;
    default: DLRA_GRAM(7); break;
  }
#undef DLRA_GRAM
  nb_out = nb;
}

template <typename T, typename Acc, int NA>
static void stencil_proj_launch(const GridDev &g, const T *s, const T *X, int ld, int p, int nb,
                                int chunk, double *partial, hipStream_t st) {
  const size_t shm = stencil_proj_lds<T, Acc, NA>();
  auto kern = k_stencil_proj<T, Acc, NA>;
  if (shm > 65536)
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));
  kern<<<nb * g.dim, 256, shm, st>>>(g, s, X, ld, p, chunk, nb, partial);
}

template <typename T, typename Acc>
void launch_stencil_projection(const GridDev &g, const T *s, const T *X, int ld, int p,
                               double *C, int ldc, double *partial, size_t partial_elems,
                               hipStream_t st) {
  const int ndk = 2 * g.dim;
  const size_t pq = size_t(p) * p;
  constexpr int CT = sizeof(Acc) == 8 ? 32 : 64;
  int nb = (kContractWaves + 4 * g.dim - 1) / (4 * g.dim);
  nb = std::max(1, std::min({nb, kMaxPartialBlocks, (g.n + CT - 1) / CT}));
  while (nb > 1 && size_t(nb + 1) * ndk * pq > partial_elems) nb /= 2;
  int chunk = (g.n + nb - 1) / nb;
  chunk = (chunk + CT - 1) / CT * CT;
  nb = (g.n + chunk - 1) / chunk;
#define DLRA_SPROJ(NA) stencil_proj_launch<T, Acc, NA>(g, s, X, ld, p, nb, chunk, partial, st)
  switch ((p + 15) / 16) {
    case 1: DLRA_SPROJ(1); break;
    case 2: DLRA_SPROJ(2); break;
    case 3: DLRA_SPROJ(3); break;
    case 4: DLRA_SPROJ(4); break;
    case 5: DLRA_SPROJ(5); break;
    case 6: DLRA_SPROJ(6); break;
    default: DLRA_SPROJ(7); break;
  }
#undef DLRA_SPROJ
  const size_t per = size_t(ndk) * p * p;
  double *red = partial + size_t(nb) * per;
  reduce_partials(partial, nb, int(per), red, st, red + per, room_after(partial_elems, nb + 1, per));
  k_scatter<<<(per + kBlock - 1) / kBlock, kBlock, 0, st>>>(red, p, p, ndk, C, ldc,
                                                            size_t(ldc) * ldc);
}

template <typename T, typename Acc>
void launch_gram(int n, const T *X, int ldx, int p, const T *Y, int ldy, int q, const T *wmat,
                 const T *s, double *G, int ldg, double *partial, size_t partial_elems,
                 hipStream_t st) {
  GridDev g{};
  g.n = n;
  int nb = 0;
  if (p == q && p <= 112) {
    if (wmat != nullptr)
      gram<T, Acc, true>(n, X, ldx, p, YMat<T>{Y, ldy}, q, WMatS<T>{wmat, s}, partial,
                         partial_elems, st, nb);
    else   // X^T X stages X once
      gram<T, Acc, true>(n, X, ldx, p, YMat<T>{Y, ldy}, q, WOne<T>{}, partial, partial_elems,
                         st, nb, Y == X && ldy == ldx);
  } else if (wmat != nullptr) {
    contract<T, Acc>(g, X, ldx, p, YMat<T>{Y, ldy}, q, WMatS<T>{wmat, s}, partial,
                     partial_elems, st, nb);
  } else {
    contract<T, Acc>(g, X, ldx, p, YMat<T>{Y, ldy}, q, WOne<T>{}, partial, partial_elems,
                     st, nb);
  }
  const size_t per = size_t(p) * q;
  double *red = partial + size_t(nb) * per;
  reduce_partials(partial, nb, int(per), red, st, red + per, room_after(partial_elems, nb + 1, per));
  k_scatter<<<(per + kBlock - 1) / kBlock, kBlock, 0, st>>>(red, p, q, 1, G, ldg, 0);
}

template <typename T, typename Acc>
void launch_xt_source(int n, const T *X, int ld, int p, const T *w, int n_mat, int n_beams,
                      const T *psi, size_t pstride, double *H, int ldh, double *partial,
                      size_t partial_elems, hipStream_t st) {
  int nb = 0;
  const int q = n_mat * n_beams;
  const YSrc<T> ys{w, psi, n, n_mat, pstride};
  if (p <= 112 && q <= 16) {
    gram<T, Acc, false>(n, X, ld, p, ys, q, WOne<T>{}, partial, partial_elems, st, nb);
  } else {
    GridDev g{};
    g.n = n;
    contract<T, Acc>(g, X, ld, p, ys, q, WOne<T>{}, partial, partial_elems, st, nb);
  }
  const size_t per = size_t(p) * q;
  double *red = partial + size_t(nb) * per;
  reduce_partials(partial, nb, int(per), red, st, red + per, room_after(partial_elems, nb + 1, per));
  k_scatter<<<(per + kBlock - 1) / kBlock, kBlock, 0, st>>>(red, p, q, 1, H, ldh, 0);
}

template <typename T>
void launch_sumsq(int n, const T *X, int ld, int q, double *out, double *partial,
                  size_t partial_elems, hipStream_t st) {
  int nb = std::min((n + kBlock - 1) / kBlock, kSumsqBlocks);
  if (size_t(nb) > partial_elems) nb = int(partial_elems);
  k_sumsq<T><<<nb, kBlock, 0, st>>>(n, X, ld, q, partial);
  reduce_partials(partial, nb, 1, out, st, partial + nb, room_after(partial_elems, nb, 1));
}

template <typename T>
static void update(int n, const T *X, int ldx, int p, const double *G, int ldg, double beta,
                   const T *Y, int ldy, double alpha, T *Z, int ldz, int q, double *dose,
                   const double *dc, double dscale, const T *sw, int n_mat, int n_beams,
                   const T *spsi, size_t pstride, const double *sC, int ldsc, double sdt,
                   hipStream_t st) {
  if (n <= 0 || q <= 0) return;
  const int nq = (q + 15) / 16;   // q <= 64: ranks are capped at 50
  const int n_src = n_mat * n_beams;
  const int ne = p + (sw != nullptr ? n_src : 0);
  const int nk = (ne + 3) & ~3;
  const size_t shm = size_t(nk) * 16 * nq * sizeof(T) + size_t(16) * nq * sizeof(double);
  const int blocks = std::max(1, std::min(kUpdBlocks, (n + 127) / 128));
  const bool HY = Y != nullptr && alpha != 0.0;
#define DLRA_UPDATE(NQ)                                                                     \
  do {                                                                                      \
    auto kern = HY ? k_update_mfma<T, NQ, true> : k_update_mfma<T, NQ, false>;              \
    if (shm > 65536)                                                                        \
      (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kern),                        \
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));     \
    kern<<<blocks, 256, shm, st>>>(n, X, ldx, p, G, ldg, beta, Y, ldy, alpha, Z, ldz, q,    \
                                   dose, dc, dscale, sw, n_mat, n_src, spsi, pstride, sC,   \
                                   ldsc, sdt);                                              \
  } while (0)
  auto a16 = [](const void *ptr) { return (reinterpret_cast<uintptr_t>(ptr) & 15) == 0; };
  if constexpr (sizeof(T) == 4) {
    // 16-byte form where every column start is 16-byte aligned
    const bool vec = ldx % 4 == 0 && ldz % 4 == 0 && a16(X) && a16(Z) &&
                     (!HY || (ldy % 4 == 0 && a16(Y))) &&
                     (sw == nullptr || (n % 4 == 0 && pstride % 4 == 0 && a16(sw) && a16(spsi)));
    if (vec) {
      const int vblocks = std::max(1, std::min(kUpdBlocks, (n + 255) / 256));
#define DLRA_UPDATE_VEC(NQ)                                                                 \
  do {                                                                                      \
    auto kern = HY ? k_update_vec<NQ, true> : k_update_vec<NQ, false>;                      \
    if (shm > 65536)                                                                        \
      (void)hipFuncSetAttribute(reinterpret_cast<const void *>(kern),                        \
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(shm));     \
    kern<<<vblocks, 256, shm, st>>>(n, X, ldx, p, G, ldg, beta, Y, ldy, alpha, Z, ldz, q,   \
                                    dose, dc, dscale, sw, n_mat, n_src, spsi, pstride, sC,  \
                                    ldsc, sdt);                                             \
  } while (0)
      switch (nq) {
        case 1: DLRA_UPDATE_VEC(1); break;
        case 2: DLRA_UPDATE_VEC(2); break;
        case 3: DLRA_UPDATE_VEC(3); break;
        default: DLRA_UPDATE_VEC(4); break;
      }
#undef DLRA_UPDATE_VEC
      return;
    }
  }
  switch (nq) {
    case 1: DLRA_UPDATE(1); break;
    case 2: DLRA_UPDATE(2); break;
    case 3: DLRA_UPDATE(3); break;
    default: DLRA_UPDATE(4); break;
  }
#undef DLRA_UPDATE
}

template <typename T>
void launch_update(int n, const T *X, int ldx, int p, const double *G, int ldg, double beta,
                   const T *Y, int ldy, double alpha, T *Z, int ldz, int q, double *dose,
                   const double *dc, double dscale, hipStream_t st) {
  update<T>(n, X, ldx, p, G, ldg, beta, Y, ldy, alpha, Z, ldz, q, dose, dc, dscale, nullptr, 1,
            1, nullptr, 0, nullptr, 0, 0.0, st);
}

template <typename T>
void launch_source_k(int n, const T *U, int ld, int r, const double *St, int lds, const T *w,
                     int n_mat, int n_beams, const T *psi, size_t pstride, const double *Cg,
                     int ldcg, double dt, T *K, hipStream_t st) {
  update<T>(n, U, ld, r, St, lds, 1.0, nullptr, 0, 0.0, K, ld, r, nullptr, nullptr, 0.0, w,
            n_mat, n_beams, psi, pstride, Cg, ldcg, dt, st);
}

// ------------------------------------------------------------------ plan objective
// D(x) = sum_b w_b D_b(x); J = sum_{x in T} (D - dhat)^2 + lam sum_{x not in T} D^2;
// dJ/dw_b = sum_x g(x) D_b(x) with g = dJ/dD (2 (D - dhat) on T, 2 lam D off it).
// Block k of both kernels covers the cells [k chunk, (k + 1) chunk); partial
// row k holds its J share (element 0) and its share of every dJ/dw_b.
__global__ __launch_bounds__(256) void k_plan_residual(int n, int nb, const double *__restrict__ doses,
                                                       PlanWeights pw,
                                                       const unsigned char *__restrict__ target,
                                                       double dhat, double lam, int chunk,
                                                       double *__restrict__ g,
                                                       double *__restrict__ partial) {
  __shared__ double red[4];
  const int x0 = blockIdx.x * chunk, x1 = min(n, x0 + chunk);
  double acc = 0.0;
  for (int x = x0 + threadIdx.x; x < x1; x += blockDim.x) {
    double D = 0.0;
    for (int b = 0; b < nb; ++b) D += pw.w[b] * doses[size_t(b) * n + x];
    const bool in = target[x] != 0;
    const double e = in ? D - dhat : D;
    acc += in ? e * e : lam * e * e;
    g[x] = in ? 2.0 * e : 2.0 * lam * e;
  }
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0)
    partial[size_t(blockIdx.x) * (nb + 1)] = (red[0] + red[1]) + (red[2] + red[3]);
}

__global__ __launch_bounds__(256) void k_plan_dots(int n, int nb, const double *__restrict__ doses,
                                                   const double *__restrict__ g, int chunk,
                                                   double *__restrict__ partial) {
  __shared__ double red[4];
  const int b = blockIdx.y;
  const int x0 = blockIdx.x * chunk, x1 = min(n, x0 + chunk);
  const double *Db = doses + size_t(b) * n;
  double acc = 0.0;
  for (int x = x0 + threadIdx.x; x < x1; x += blockDim.x) acc += g[x] * Db[x];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0)
    partial[size_t(blockIdx.x) * (nb + 1) + 1 + b] = (red[0] + red[1]) + (red[2] + red[3]);
}

static int plan_blocks(int n) { return std::max(1, std::min(kPlanBlocks, (n + 255) / 256)); }

size_t plan_objective_work(int n, int nb) {
  return size_t(n) + size_t(plan_blocks(n) + 1 + 64) * size_t(nb + 1);
}

void launch_plan_objective(int n, int nb, const double *doses, const PlanWeights &pw,
                           const unsigned char *target, double dhat, double lam, double *work,
                           double *out, hipStream_t st) {
  const int nblk = plan_blocks(n);
  const int chunk = (n + nblk - 1) / nblk;
  double *g = work, *partial = work + n;
  double *scratch = partial + size_t(nblk) * (nb + 1);
  k_plan_residual<<<nblk, 256, 0, st>>>(n, nb, doses, pw, target, dhat, lam, chunk, g, partial);
  k_plan_dots<<<dim3(nblk, nb), 256, 0, st>>>(n, nb, doses, g, chunk, partial);
  reduce_partials(partial, nblk, nb + 1, out, st, scratch, size_t(64) * (nb + 1));
}

// One-pass form: every block forms the residual g(x) of its cells and
// multiplies it into every beam's dose at once, so no n-sized buffer is
// needed; per-block arithmetic (cell order, reduction tree) is that of
// k_plan_residual followed by k_plan_dots.
__global__ __launch_bounds__(256) void k_plan_fused(int n, int nb, const double *__restrict__ doses,
                                                    PlanWeights pw,
                                                    const unsigned char *__restrict__ target,
                                                    double dhat, double lam, int chunk,
                                                    double *__restrict__ partial) {
  __shared__ double red[4][kPlanMaxBeams + 1];
  const int x0 = blockIdx.x * chunk, x1 = min(n, x0 + chunk);
  double acc[kPlanMaxBeams + 1];
#pragma unroll
  for (int b = 0; b <= kPlanMaxBeams; ++b) acc[b] = 0.0;
  for (int x = x0 + threadIdx.x; x < x1; x += blockDim.x) {
    double D = 0.0;
    for (int b = 0; b < nb; ++b) D += pw.w[b] * doses[size_t(b) * n + x];
    const bool in = target[x] != 0;
    const double e = in ? D - dhat : D;
    acc[0] += in ? e * e : lam * e * e;
    const double g = in ? 2.0 * e : 2.0 * lam * e;
#pragma unroll
    for (int b = 0; b < kPlanMaxBeams; ++b)
      if (b < nb) acc[1 + b] += g * doses[size_t(b) * n + x];
  }
#pragma unroll
  for (int b = 0; b <= kPlanMaxBeams; ++b) {
    if (b <= nb) {
      double v = acc[b];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][b] = v;
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b <= nb; b += blockDim.x)
    partial[size_t(blockIdx.x) * (nb + 1) + b] = (red[0][b] + red[1][b]) + (red[2][b] + red[3][b]);
}

size_t plan_objective_fused_scratch(int nb) {
  return size_t(kPlanBlocks + 64 + 1) * size_t(nb + 1);
}

void launch_plan_objective_fused(int n, int nb, const double *doses, const PlanWeights &pw,
                                 const unsigned char *target, double dhat, double lam,
                                 double *scratch, double *out, hipStream_t st) {
  const int nblk = plan_blocks(n);
  const int chunk = (n + nblk - 1) / nblk;
  double *partial = scratch;
  double *seg = partial + size_t(nblk) * (nb + 1);
  k_plan_fused<<<nblk, 256, 0, st>>>(n, nb, doses, pw, target, dhat, lam, chunk, partial);
  reduce_partials(partial, nblk, nb + 1, out, st, seg, size_t(64) * (nb + 1));
}

#define DLRA_INSTANTIATE(T, Acc)                                                              \
  template void launch_inverse_stop<T>(const GridDev &, const T *, int, const double *, T *,  \
                                       Ctl *, hipStream_t);                                   \
  template void launch_kstep_stage<T>(const GridDev &, const T *, const T *, const T *, T *,  \
                                      int, int, const T *, double, hipStream_t);              \
  template void launch_pack_couplings<T>(int, int, const double *, int, T *, hipStream_t);    \
  template void launch_stencil_projection<T, Acc>(const GridDev &, const T *, const T *, int, \
                                                  int, double *, int, double *, size_t,       \
                                                  hipStream_t);                               \
  template void launch_gram<T, Acc>(int, const T *, int, int, const T *, int, int, const T *, \
                                    const T *, double *, int, double *, size_t, hipStream_t); \
  template void launch_xt_source<T, Acc>(int, const T *, int, int, const T *, int, int,      \
                                         const T *, size_t, double *, int, double *, size_t,  \
                                         hipStream_t);                                        \
  template void launch_sumsq<T>(int, const T *, int, int, double *, double *, size_t,         \
                                hipStream_t);                                                 \
  template void launch_update<T>(int, const T *, int, int, const double *, int, double,       \
                                 const T *, int, double, T *, int, int, double *,             \
                                 const double *, double, hipStream_t);                        \
  template void launch_source_k<T>(int, const T *, int, int, const double *, int, const T *,  \
                                   int, int, const T *, size_t, const double *, int, double,  \
                                   T *, hipStream_t);

DLRA_INSTANTIATE(double, double)
DLRA_INSTANTIATE(float, float)
template void launch_gram<float, double>(int, const float *, int, int, const float *, int, int,
                                         const float *, const float *, double *, int, double *,
                                         size_t, hipStream_t);

}  // namespace dlra
