// HGKS hot path for MI355X (gfx950): kernels and the C ABI declared in hgks.h.
//
// Per S2O4 stage and direction d (local frame (n, t1, t2) = (d, d+1, d+2)):
//   recon_kernel<d>: normal WENO-Z sweep of a face tile (values and slopes of
//     the left/right states and the equilibrium slope), staged in LDS, then
//     the first tangential sweep to the two Gauss lines along t1 -> buffer B.
//   flux4_kernel<d> (FP64 x and z faces), flux4y_kernel (FP64 y faces),
//   flux_kernel<d> (FP32 face data): one lane per Gauss point: second
//     tangential sweep along t2 (the FP64 kernels from B rows staged in LDS),
//     the BGK flux of Eq. (flux) integrated over [0, dt] and [0, dt/2], the
//     2x2 Gauss sum by cross-lane swaps, F^n and dF^n/dt -> face buffer F_d.
// then update_kernel<stage>: L, dL/dt from the six faces of each cell and the
// two-stage update of Eq. (two-stage); stage 2 also reduces the wave speed of
// the new state for the next CFL time step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hgks.h"
#include "hgks_numerics.hpp"

namespace hgks {

// Quantities per face and Gauss line after the first tangential sweep, k the
// conserved component.  The flux kernel's Gauss-point pairs read two
// quantities together, and each such pair sits in adjacent planes:
// (Q^l_k, Q^r_k), (dQ^l_k/dn, dQ^l_k/dt1), (dQ^r_k/dn, dQ^r_k/dt1); then the
// equilibrium normal slopes dQ0_k/dn.
constexpr int b_ql(int k) { return 2 * k; }
constexpr int b_qr(int k) { return 2 * k + 1; }
constexpr int b_dln(int k) { return 10 + 2 * k; }
constexpr int b_dlt1(int k) { return 11 + 2 * k; }
constexpr int b_drn(int k) { return 20 + 2 * k; }
constexpr int b_drt1(int k) { return 21 + 2 * k; }
constexpr int b_d0(int k) { return 30 + k; }
constexpr int B_COUNT = 35;

struct Params {
  int n[3];
  int bc[3];
  int flags;  // hgks_config.flags
  double gamma, gm1, K, mu_ref, T_ref, mu_exp, pr_fix, T_wall;
  double iK3, iT_ref;  // 1/(K + 3); 1/T_ref (0 without a power law)
  double imu_ref;      // 1/mu_ref (0 for an inviscid gas)
  double force[3];
  const double* hcell[3];  // cell widths
  const double* dface[3];  // d(index)/dx at faces 0..n
  const double* dgp[3];    // d(index)/dx at the Gauss points, 2 per cell
  const double* dcen[3];   // d(index)/dx at cell centres
};

// Scalars kept on the device so that a step needs no host round trip.
struct Scalars {
  double dt;                 // time step of the current step
  double t;                  // simulated time
  double dt_residual;        // time step used by hgks_residual
  double steps;              // steps taken
  unsigned long long smax;   // bit pattern of max wave speed / h (positive double)
  double force_x;            // streamwise body force in effect (the controller's, with the mass-flux flag)
  double m_prev;             // volume mean of rho U after the last step (mass-flux controller)
  double dt_fixed;           // > 0: the time step of every step; <= 0: the CFL rule
};

// Global-memory view of a device pointer.  A pointer that a kernel reads out
// of memory (the batched kernels take theirs from the instance table) is a
// generic pointer to the compiler, which then emits flat accesses; flat loads
// share the wait counter of LDS traffic, so every LDS wait would also wait for
// outstanding HBM loads.  Accessing through an address-space-1 pointer gives
// global loads and stores.
#define HGKS_GLOBAL __attribute__((address_space(1)))
template <class T> __device__ __forceinline__ HGKS_GLOBAL T* gmem(T* p) { return (HGKS_GLOBAL T*)p; }

__host__ __device__ inline size_t cells(const Params& P) { return (size_t)P.n[0] * P.n[1] * P.n[2]; }

// Face extents of direction d: one more face than cells along d (on a
// periodic axis the last face repeats face 0 and is computed from the same
// data).
// Faces of direction d per axis: n along the tangential axes; along the
// normal n + 1 on a wall axis and n on a periodic one, where face n is face 0
// (the same stencil after the wrap, so the same flux): the update reads face
// 0 as the last cell's right face.
__host__ __device__ inline void face_extents(const Params& P, int d, int fe[3]) {
  for (int a = 0; a < 3; ++a) fe[a] = P.n[a] + (a == d && P.bc[d] != HGKS_BC_PERIODIC ? 1 : 0);
}

// Row pitch of the face arrays (buffer B and the face fluxes F): the x extent
// rounded up to 32 elements, so that every row starts on a 128-byte boundary
// and a tile's 16-face rows do not straddle cache lines.
__host__ __device__ inline int face_pitch(int nx) { return (nx + 31) & ~31; }

// Tile order across the grid of blocks: tile index `fast` varies fastest
// (neighbouring tiles along that axis share stencil data), and the blocks are
// remapped so that each of the 8 XCDs (which take blocks round robin and have
// their own L2) works through a contiguous run of tiles.
__device__ __forceinline__ int xcd_linear_block(int nblocks) {
  const int bid = blockIdx.x;
  const int full = (nblocks / 8) * 8;
  if (bid >= full) return bid;
  return (bid % 8) * (full / 8) + bid / 8;
}
__device__ __forceinline__ void tile_coords(int lin, const int nt[3], int fast, int t[3]) {
  const int a1 = fast == 0 ? 1 : 0;
  const int a2 = fast == 2 ? 1 : 2;
  t[fast] = lin % nt[fast];
  lin /= nt[fast];
  t[a1] = lin % nt[a1];
  t[a2] = lin / nt[a1];
}
// Extents of buffer B of direction d: faces, plus two ghost rows on each side
// of t2 when t2 is a wall axis (the second tangential sweep reads them).
__host__ __device__ inline void b_extents(const Params& P, int d, int be[3], int bo[3]) {
  int d2 = (d + 2) % 3;
  face_extents(P, d, be);
  for (int a = 0; a < 3; ++a) bo[a] = 0;
  if (P.bc[d2] == HGKS_BC_ISOTHERMAL_WALL) {
    be[d2] += 4;
    bo[d2] = -2;
  }
}

// t mod n for -n <= t < 2n: one correction either way, no integer division
// (which takes some 40 vector instructions).
__host__ __device__ __forceinline__ int wrap1(int t, int n) {
  t = t < 0 ? t + n : t;
  return t >= n ? t - n : t;
}

// One cell of the padded state, synthesised from the interior: periodic wrap,
// or the isothermal-wall mirror (velocity reversed, same pressure,
// temperature 2 T_w - T (not below 0.1 T_w), density p/T), all in FP64.
// Every caller passes coordinates within three cells of the grid, and every
// axis has at least 4 cells, so one wrap correction suffices.
template <class S>
__device__ __forceinline__ void load_cell(const S* __restrict__ q, const Params& P, int c0, int c1, int c2,
                                          double v[5]) {
  int c[3] = {c0, c1, c2};
  bool mirror = false;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int N = P.n[a];
    if (c[a] < 0 || c[a] >= N) {
      if (P.bc[a] == HGKS_BC_ISOTHERMAL_WALL) {
        mirror = true;
        c[a] = c[a] < 0 ? -c[a] - 1 : 2 * N - 1 - c[a];
      } else {
        c[a] = wrap1(c[a], N);
      }
    }
  }
  const size_t n3 = cells(P);
  const size_t idx = ((size_t)c[2] * P.n[1] + c[1]) * P.n[0] + c[0];
#pragma unroll
  for (int k = 0; k < 5; ++k) v[k] = double(gmem(q)[k * n3 + idx]);
  if (mirror) {
    double rho = v[0], ir = 1.0 / rho;
    double U = v[1] * ir, V = v[2] * ir, W = v[3] * ir;
    double p = P.gm1 * (v[4] - 0.5 * rho * (U * U + V * V + W * W));
    double Tg = fmax(2.0 * P.T_wall - p * ir, 0.1 * P.T_wall);
    double rg = p / Tg;
    v[0] = rg;
    v[1] = -rg * U;
    v[2] = -rg * V;
    v[3] = -rg * W;
    v[4] = p / P.gm1 + 0.5 * rg * (U * U + V * V + W * W);
  }
}

// Faces per reconstruction tile in the local frame (n, t1, t2).  x, the
// contiguous axis, runs across lanes in every direction, W faces wide: 16 for
// FP64 B (128-byte rows), 32 for FP32 B (also 128-byte rows).
// Where Gauss line g (of the two along t1) of face i sits within one quantity's
// 2 NB entries of B.  FP64 face data interleave the two lines, 2 i + g, so a
// 16-face tile row is one 256-byte run (the reconstruction's stores are the
// cost there: 2.7 vs 3.2 ms per launch at 256^3); FP32 face data keep them in
// two planes, g NB + i, which the FP32 flux kernel reads faster (6.0 vs 6.35 ms).
template <class R> constexpr bool B_INTERLEAVED = sizeof(R) == 8;
template <class R> __host__ __device__ constexpr size_t b_pos(size_t i, int g, size_t NB) {
  return B_INTERLEAVED<R> ? 2 * i + g : (size_t)g * NB + i;
}
// FP64 face data are tile-major: for each 16-face run along x of a row
// (z, y) of B, the 35 quantities' two Gauss lines sit together in one chunk
// of 35 x 32 doubles (8960 bytes), quantity q at 32 q, face x at 2 (x mod 16)
// + line.  A flux wave's loads of one stencil row then touch one chunk (the
// ten quantities of a phase: 2.5 KB contiguous) instead of 35 runs of 256
// bytes spread over 35 quantity planes, and a reconstruction wave's stores
// fill chunks.  FP32 face data keep quantity planes.
constexpr int B_CHUNK = B_COUNT * 32;  // doubles per (row, 16-face run)
// Index of quantity 0, line 0 of face (x, y, z) (B coordinates) in FP64 B,
// for row pitch bp (a multiple of 32) and be1 rows per z plane.
__host__ __device__ inline size_t b64_face(int x, int y, int z, int bp, int be1) {
  return (((size_t)z * be1 + y) * (size_t)(bp >> 4) + (size_t)(x >> 4)) * B_CHUNK + 2 * (size_t)(x & 15);
}

// Byte distance between a quantity of B and the next one (2 NB entries).
template <class R> __host__ __device__ inline uint32_t second_pair_offset(size_t NB) {
  return (uint32_t)(2 * NB * sizeof(R));
}

// The same pointer, declared uniform across the wave (it is: callers pass
// block-uniform values), so that loads from it plus a 32-bit lane offset take
// the scalar-base form instead of a 64-bit vector address per lane.
__device__ __forceinline__ const HGKS_GLOBAL char* uniform_ptr(const HGKS_GLOBAL char* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return reinterpret_cast<const HGKS_GLOBAL char*>(((uint64_t)hi << 32) | lo);
}

template <int DIR, int W> struct ReconTileW;
template <int W> struct ReconTileW<0, W> { static constexpr int TN = W, T1 = 8, T2 = 1; };
template <int W> struct ReconTileW<1, W> { static constexpr int TN = 1, T1 = 8, T2 = W; };
template <int W> struct ReconTileW<2, W> { static constexpr int TN = 1, T1 = W, T2 = 8; };
template <int DIR, class R> using ReconTile = ReconTileW<DIR, sizeof(R) == 8 ? 16 : 32>;

template <int DIR, class R> __host__ __device__ inline void recon_tile_extents(int S[3]) {
  constexpr int D1 = (DIR + 1) % 3, D2 = (DIR + 2) % 3;
  S[DIR] = ReconTile<DIR, R>::TN;
  S[D1] = ReconTile<DIR, R>::T1;
  S[D2] = ReconTile<DIR, R>::T2;
}
template <int DIR, class R> constexpr int recon_tile_faces() {
  return ReconTile<DIR, R>::TN * ReconTile<DIR, R>::T1 * ReconTile<DIR, R>::T2;
}

constexpr int RECON_THREADS = 256;

// Normal sweep and first tangential sweep for a tile of faces of direction DIR.
// LDS holds the 25 normal-sweep quantities of the tile plus a 2-face halo along
// t1.  Output: quantity q of B at B[q * 2 NB + b_pos(face, g1)] in the
// arithmetic type R.
template <int DIR, class R> constexpr int recon_lds_faces() {
  return ReconTile<DIR, R>::TN * (ReconTile<DIR, R>::T1 + 4) * ReconTile<DIR, R>::T2;
}

// Number of reconstruction tiles of direction DIR.
template <int DIR, class R> __host__ __device__ inline int recon_tiles(const Params& P) {
  int S[3], be[3], bo[3];
  recon_tile_extents<DIR, R>(S);
  b_extents(P, DIR, be, bo);
  return ((be[0] + S[0] - 1) / S[0]) * ((be[1] + S[1] - 1) / S[1]) * ((be[2] + S[2] - 1) / S[2]);
}

template <int DIR, class R, class ST = double>
__device__ __forceinline__ void recon_tile(const ST* __restrict__ q, const Params& P,
                                           const double* __restrict__ qref, R* __restrict__ B, int lin,
                                           R (*A)[recon_lds_faces<DIR, R>()]) {
  constexpr int D1 = (DIR + 1) % 3, D2 = (DIR + 2) % 3;
  constexpr int NA = recon_lds_faces<DIR, R>();
  constexpr int NF = recon_tile_faces<DIR, R>();  // 128 (FP64) or 256 (FP32)

  int S[3];
  recon_tile_extents<DIR, R>(S);
  int SA[3] = {S[0], S[1], S[2]};
  SA[D1] += 4;
  int be[3], bo[3];
  b_extents(P, DIR, be, bo);
  int nt[3], tc[3], org[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) nt[a] = (be[a] + S[a] - 1) / S[a];
  tile_coords(lin, nt, DIR, tc);  // normal tiles adjacent
#pragma unroll
  for (int a = 0; a < 3; ++a) org[a] = tc[a] * S[a] + bo[a];

  // reference state subtracted before the reconstruction (zero on the FP64 path)
  double ref[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) ref[k] = gmem(qref)[k];
  double rl[5];
  rl[0] = ref[0];
  rl[1] = ref[1 + DIR];
  rl[2] = ref[1 + D1];
  rl[3] = ref[1 + D2];
  rl[4] = ref[4];

  // ---- normal sweep on the tile and its t1 halo -------------------------
  for (int idx = threadIdx.x; idx < NA; idx += RECON_THREADS) {
    int l[3];
    l[0] = idx % SA[0];
    l[1] = (idx / SA[0]) % SA[1];
    l[2] = idx / (SA[0] * SA[1]);
    int f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) f[a] = org[a] + l[a] - (a == D1 ? 2 : 0);
    bool ok = f[DIR] < be[DIR] && f[D2] < bo[D2] + be[D2] && f[D1] >= -2 && f[D1] < P.n[D1] + 2;
    if (!ok) continue;
    R c[6][5];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      int cc[3] = {f[0], f[1], f[2]};
      cc[DIR] += m - 3;
      double v[5];
      load_cell(q, P, cc[0], cc[1], cc[2], v);
      c[m][0] = R(v[0] - rl[0]);
      c[m][1] = R(v[1 + DIR] - rl[1]);
      c[m][2] = R(v[1 + D1] - rl[2]);
      c[m][3] = R(v[1 + D2] - rl[3]);
      c[m][4] = R(v[4] - rl[4]);
    }
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      R cv[6] = {c[0][k], c[1][k], c[2][k], c[3][k], c[4][k], c[5][k]};
      R ql, qr, dl, dr, d0;
      normal_sweep(cv, ql, qr, dl, dr, d0);
      A[0 + k][idx] = ql;
      A[5 + k][idx] = qr;
      A[10 + k][idx] = dl;
      A[15 + k][idx] = dr;
      A[20 + k][idx] = d0;
    }
  }
  __syncthreads();

  // ---- first tangential sweep: both Gauss lines of a face per work item ----
  // Items (face, h): h = 0 the left-state quantities, h = 1 the right-state
  // ones (whole waves share h); the two Gauss lines share each stencil's
  // candidates and WENO-Z factors.  The linear equilibrium slopes split 3 + 2
  // components.
  const size_t NB = (size_t)face_pitch(be[0]) * be[1] * be[2];
  const size_t qstride = 2 * NB;
  for (int item = threadIdx.x; item < 2 * NF; item += RECON_THREADS) {
    const int o = item % NF, h = item / NF;
    int lo[3];
    lo[0] = o % S[0];
    lo[1] = (o / S[0]) % S[1];
    lo[2] = o / (S[0] * S[1]);
    int f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) f[a] = org[a] + lo[a];
    if (f[DIR] >= be[DIR] || f[D1] >= P.n[D1] || f[D2] >= bo[D2] + be[D2]) continue;  // this item only
    int ai[5];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      int l[3] = {lo[0], lo[1], lo[2]};
      l[D1] += j;  // A tile is offset by -2 along t1
      ai[j] = (l[2] * SA[1] + l[1]) * SA[0] + l[0];
    }
    const size_t bidx =
        ((size_t)(f[2] - bo[2]) * be[1] + (f[1] - bo[1])) * face_pitch(be[0]) + (f[0] - bo[0]);
    // B is written once and read once, by the flux kernel: non-temporal stores
    // (no L2 allocation for a stream many times the cache's size).
    HGKS_GLOBAL R* out =
        gmem(B) + (B_INTERLEAVED<R> ? b64_face(f[0] - bo[0], f[1] - bo[1], f[2] - bo[2], face_pitch(be[0]), be[1])
                                    : b_pos<R>(bidx, 0, NB));
    using R2 = R __attribute__((ext_vector_type(2)));
    auto put = [&](int q, const R val[2]) {
      if constexpr (B_INTERLEAVED<R>) {
        const R2 v2 = {val[0], val[1]};
        __builtin_nontemporal_store(v2, reinterpret_cast<HGKS_GLOBAL R2*>(&out[q * 32]));
      } else {
        __builtin_nontemporal_store(val[0], &out[q * qstride]);
        __builtin_nontemporal_store(val[1], &out[q * qstride + NB]);
      }
    };
    auto stencil = [&](int row, R v[5]) {
#pragma unroll
      for (int j = 0; j < 5; ++j) v[j] = A[row][ai[j]];
    };
    const int av = h ? 5 : 0, an = h ? 15 : 10;
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      R v[5], val[2], der[2];
      stencil(av + k, v);
      gauss_value_slope2(v, val, der);
      put(h ? b_qr(k) : b_ql(k), val);
      put(h ? b_drt1(k) : b_dlt1(k), der);
      stencil(an + k, v);
      gauss_value2(v, val);
      put(h ? b_drn(k) : b_dln(k), val);
    }
    const int k0 = h ? 3 : 0, k1 = h ? 5 : 3;
    for (int k = k0; k < k1; ++k) {
      R v[5], val[2];
      stencil(20 + k, v);
      gauss_linear2(v, val);
      put(b_d0(k), val);
    }
  }
}

template <int DIR, class R, class ST>
__global__ __launch_bounds__(RECON_THREADS) void recon_kernel(const ST* __restrict__ q, Params P,
                                                              const double* __restrict__ qref,
                                                              R* __restrict__ B) {
  __shared__ R A[25][recon_lds_faces<DIR, R>()];
  recon_tile<DIR, R, ST>(q, P, qref, B, xcd_linear_block(recon_tiles<DIR, R>(P)), A);
}

// Asynchronous copy of 16 bytes per lane from global memory into LDS (lane l's
// bytes land at lds + 16 l; lds must be the same on every lane of the wave).
// Completion is tracked by the wave's vector-memory counter.
__device__ __forceinline__ void dma16_to_lds(const HGKS_GLOBAL char* src, double* lds) {
  __builtin_amdgcn_global_load_lds(reinterpret_cast<const HGKS_GLOBAL void*>(src),
                                   (__attribute__((address_space(3))) void*)(lds), 16, 0, 0);
}
// Every outstanding vector-memory operation of the wave complete (the LDS
// copies above included); the compiler moves no memory access across it.
__device__ __forceinline__ void wait_vmem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
// The value counts as defined by this (empty) asm: no wait for the load that
// produced it is left to the compiler after this point (the vector-memory
// counter retires in order, so such a wait would also wait for every copy
// issued after the load).
template <class T> __device__ __forceinline__ void produced_here(T& x) { asm volatile("" : "+v"(x)); }

// Lane exchanges between the rows of a wavefront (row = 16 lanes), on the
// VALU (gfx950 permlane swaps), every lane active.  swap_rows16(x, y): on an
// even row x keeps its value and y takes the x of the odd row above it; on
// an odd row y keeps its value and x takes the y of the even row below it.
// swap_rows32(x, y): the same between the half-waves (rows 0-1 and 2-3): x
// of the upper half takes y of the lower half, y of the lower half takes x
// of the upper half.
template <bool kHalf> __device__ __forceinline__ void swap_rows_u32(uint32_t& x, uint32_t& y) {
  if constexpr (kHalf) {
    const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
    x = r[0];
    y = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
    x = r[0];
    y = r[1];
  }
}
template <bool kHalf> __device__ __forceinline__ void swap_rows(float& x, float& y) {
  uint32_t a = __float_as_uint(x), b = __float_as_uint(y);
  swap_rows_u32<kHalf>(a, b);
  x = __uint_as_float(a);
  y = __uint_as_float(b);
}
template <bool kHalf> __device__ __forceinline__ void swap_rows(double& x, double& y) {
  const uint64_t a = (uint64_t)__double_as_longlong(x), b = (uint64_t)__double_as_longlong(y);
  uint32_t al = (uint32_t)a, ah = (uint32_t)(a >> 32), bl = (uint32_t)b, bh = (uint32_t)(b >> 32);
  swap_rows_u32<kHalf>(al, bl);
  swap_rows_u32<kHalf>(ah, bh);
  x = __longlong_as_double((long long)(((uint64_t)ah << 32) | al));
  y = __longlong_as_double((long long)(((uint64_t)bh << 32) | bl));
}
template <class T> __device__ __forceinline__ void swap_rows16(T& x, T& y) { swap_rows<false>(x, y); }
template <class T> __device__ __forceinline__ void swap_rows32(T& x, T& y) { swap_rows<true>(x, y); }

// The face's 2x2 Gauss sum and its store.  Rows 0..3 of a wavefront hold the
// Gauss points (g1, g2) = (row >> 1, row & 1) of the same 16 faces; Fn, Fd
// are F^n and dF^n/dt at the lane's point (local frame).  Row pairs (0,1),
// (2,3) are summed first, then the half-waves, each value in the order
// (r0 + r1) + (r2 + r3).  Every sum ends on one row: rows 0..3 store F^n and
// dF^n/dt of components (0, 1) (t[0]), (2, 3) (t[1]), and rows 0, 1 those of
// component 4, each scaled by the quarter face area and rotated to the
// global frame.
template <int DIR, class R>
__device__ __forceinline__ void gauss_sum_store(const Params& P, double* __restrict__ F, const int f[3], bool valid,
                                                int gpi, const R Fn[5], const R Fd[5]) {
  constexpr int D1 = (DIR + 1) % 3, D2 = (DIR + 2) % 3;
  double s[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    double x = double(Fn[k]), y = double(Fd[k]);
    swap_rows16(x, y);
    s[k] = x + y;  // rows 0, 2: F^n over the row pair; rows 1, 3: dF^n/dt
  }
  double t[3];
  {
    double x = s[0], y = s[1];
    swap_rows32(x, y);
    t[0] = x + y;
  }
  {
    double x = s[2], y = s[3];
    swap_rows32(x, y);
    t[1] = x + y;
  }
  {
    double x = s[4], y = s[4];
    swap_rows32(x, y);
    t[2] = x + y;
  }
  if (!valid) return;
  int fe[3];
  face_extents(P, DIR, fe);
  const double qarea = 0.25 * gmem(P.hcell[D1])[f[D1]] * gmem(P.hcell[D2])[f[D2]];
  const int fpitch = face_pitch(fe[0]);
  const size_t NF = (size_t)fpitch * fe[1] * fe[2];
  const size_t fi = ((size_t)f[2] * fe[1] + f[1]) * fpitch + f[0];
  const int fd = (gpi & 1) * 5, hi = gpi >> 1;
  HGKS_GLOBAL double* Fg = gmem(F) + fi;
  // global component of local components 0/1, 2/3 (momentum rotated back)
  Fg[(fd + (hi ? 1 + DIR : 0)) * NF] = qarea * t[0];
  Fg[(fd + (hi ? 1 + D2 : 1 + D1)) * NF] = qarea * t[1];
  if (!hi) Fg[(fd + 4) * NF] = qarea * t[2];
}

constexpr int FLUX_THREADS = 256;  // 64 faces x 4 Gauss points
// At least two blocks (two waves per SIMD) resident per CU: the FP64 kernels
// fit 256 registers per lane without spills (the values that phase 4 needs
// from phase 1 wait in LDS), and the second wave hides each phase's LDS and
// memory latency.
constexpr int FLUX_MIN_BLOCKS = 2;

// Flux tiles: 64 faces, TX along x times 64/TX along y, one z plane.
template <int TX> __host__ __device__ inline void flux_tile_counts(const Params& P, int d, int nt[3]) {
  int fe[3];
  face_extents(P, d, fe);
  nt[0] = (fe[0] + TX - 1) / TX;
  nt[1] = (fe[1] + 64 / TX - 1) / (64 / TX);
  nt[2] = fe[2];
}
template <int TX> __host__ __device__ inline int flux_tiles(const Params& P, int d) {
  int nt[3];
  flux_tile_counts<TX>(P, d, nt);
  return nt[0] * nt[1] * nt[2];
}

// The flux of one lane's Gauss point and the face's 2x2 Gauss sum, in four
// phases, for the staged FP64 tiles (flux_tile4, flux_tile4y).  Lane layout
// in a wavefront: lanes 16 g .. 16 g + 15 hold Gauss point g of 16
// consecutive faces along x.  The stencils come from a caller-given source:
// begin(p) at the start of phase p (0..3), pair(qi0, v)
// the five stencil values of quantity qi0 + g2 (Gauss-point pairs: see below),
// plain(qi, v) those of quantity qi.  f is the lane's face (clamped to a real
// one for the lanes beyond the grid, valid false), sn, st1, st2 the metric
// factors of its normal slope and of its Gauss point's tangential slopes,
// rl the reference state (local frame) added back to the reconstructed
// deviations; NT threads per block.
template <int DIR, class R, int NT, bool kCarryLent, class Begin, class Pair, class Plain>
__device__ __forceinline__ void flux_lane(Begin&& begin, Pair&& pair, Plain&& plain, const Params& P, double dt,
                                          double* __restrict__ F, const int f[3], bool valid, int gpi, R sn, R st1,
                                          R st2, const double rl[5], double* carry_area) {
  constexpr int D1 = (DIR + 1) % 3, D2 = (DIR + 2) % 3;
  const int tid = threadIdx.x;
  GasParams<R> g;
  g.gm1 = R(P.gm1);
  g.K = R(P.K);
  g.K3 = R(P.K + 3.0);
  g.iK3 = R(P.iK3);
  g.mu_ref = R(P.mu_ref);
  g.iT_ref = R(P.iT_ref);
  g.imu_ref = R(P.imu_ref);
  g.mu_exp = R(P.mu_exp);
  g.pr_fix = R(P.pr_fix);
  // Gauss-point pairs: the lanes g2 = 0 and g2 = 1 of a Gauss line (lane and
  // lane ^ 16, an even row and the odd row above it) share every t2
  // stencil.  Each reconstructs one of two quantities at both points and the
  // pair exchanges the other point's values (swap_rows16).  The g2 = 0 lane
  // takes quantity qi0 (Q^l, the normal slopes), the g2 = 1 lane the next
  // one (Q^r, the t1 slopes).
  R pa[5][5];

  // phase 1: left/right values and their t2 slopes; equilibrium, tau, time integrals
  R ql[5], qr[5], tl2[5], tr2[5];
  begin(0);
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    R v[5], val[2], der[2];
    pair(b_ql(k), v);
    gauss_value_slope2(v, val, der);  // the lane's quantity at -s and +s
    swap_rows16(val[0], val[1]);       // Q^l and Q^r at the lane's point
    swap_rows16(der[0], der[1]);
    ql[k] = R(double(val[0]) + rl[k]);
    qr[k] = R(double(val[1]) + rl[k]);
    tl2[k] = der[0] * st2;
    tr2[k] = der[1] * st2;
  }
  FluxAcc<R> acc;
  flux_begin(ql, qr, g, R(dt), acc);
  // FP64: the equilibrium part's time coefficients and 1/(2 lambda0) are made
  // in phase 1 and read only in phase 4.  They wait in LDS (one slot per
  // lane) instead of occupying registers through the two side phases, where
  // the compiler would otherwise spill them to scratch memory (16-60 bytes
  // per lane; reloads wait on the vector-memory counter).  The empty asm with
  // a memory clobber keeps the stores and the reloads apart, so the values
  // really leave the registers.
  // The caller may lend LDS for them (kCarryLent: carry_area, 7 NT doubles
  // free from the start of phase 2 on).
  constexpr bool kCarry = sizeof(R) == 8;
  __shared__ double carry_own[kCarry && !kCarryLent ? 7 * NT : 1];
  double* const carry_lds = kCarryLent ? carry_area : carry_own;
  begin(1);
  if constexpr (kCarry) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      carry_lds[i * NT + tid] = acc.Cn[i];
      carry_lds[(3 + i) * NT + tid] = acc.Cd[i];
    }
    carry_lds[6 * NT + tid] = acc.ihl0;
    asm volatile("" ::: "memory");
  }

  // phase 2: left side
  {
    R dq[3][5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      pair(b_dln(k), pa[k]);
      R val[2];
      gauss_value2(pa[k], val);     // the lane's quantity at -s and +s
      swap_rows16(val[0], val[1]);  // normal and t1 slope at the lane's point
      dq[0][k] = val[0] * sn;
      dq[1][k] = val[1] * st1;
      dq[2][k] = tl2[k];
    }
    flux_side<R, true>(ql, dq, g, acc);
  }

  // phase 3: right side
  {
    R dq[3][5];
    begin(2);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      pair(b_drn(k), pa[k]);
      R val[2];
      gauss_value2(pa[k], val);     // the lane's quantity at -s and +s
      swap_rows16(val[0], val[1]);  // normal and t1 slope at the lane's point
      dq[0][k] = val[0] * sn;
      dq[1][k] = val[1] * st1;
      dq[2][k] = tr2[k];
    }
    flux_side<R, false>(qr, dq, g, acc);
  }

  // phase 4: equilibrium part and Prandtl correction
  R Fn[5], Fd[5];  // F^n and dF^n/dt at this lane's Gauss point
  {
    R dq0n[5];
    begin(3);
    const LinearWeights<R> lw(gpi & 1);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      plain(b_d0(k), pa[k]);
      dq0n[k] = gauss_linear(pa[k], lw) * sn;
    }
    if constexpr (kCarry) {
      asm volatile("" ::: "memory");
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        acc.Cn[i] = carry_lds[i * NT + tid];
        acc.Cd[i] = carry_lds[(3 + i) * NT + tid];
      }
      acc.ihl0 = carry_lds[6 * NT + tid];
    }
    flux_finish(dq0n, g, acc, Fn, Fd);
  }

  gauss_sum_store<DIR>(P, F, f, valid, gpi, Fn, Fd);
}

// Second tangential sweep, Gauss-point flux, Gauss sum, F^n and dF^n/dt for
// flux tile `lin` of direction DIR, FP32 face data: the phases of flux_lane
// with the stencils read straight from B.  Lane layout as there; the four
// waves of the block take four 16-face groups of the TX x (64/TX) tile.
template <int DIR, class R, int TX>
__device__ __forceinline__ void flux_tile(const R* __restrict__ B, const Params& P, const double* __restrict__ qref,
                                          double dt, double* __restrict__ F, int lin) {
  static_assert(sizeof(R) == 4, "FP64 face data use the staged tiles (flux_tile4, flux_tile4y)");
  constexpr int D1 = (DIR + 1) % 3, D2 = (DIR + 2) % 3;
  constexpr int GX = TX / 16;  // 16-face groups along x per tile row
  int fe[3], be[3], bo[3];
  face_extents(P, DIR, fe);
  b_extents(P, DIR, be, bo);
  int nt[3], tc[3];
  flux_tile_counts<TX>(P, DIR, nt);
  if (D2 != 0 && (nt[0] & 1) == 0) {
    // x-tile pairs, then t2: the two tiles of a pair read the two halves of
    // each 128-byte line of FP32 face data one after the other, and t2
    // neighbours (sharing four of five stencil rows) are two blocks apart
    const int xh = lin & 1;
    int r = lin >> 1;
    tc[D2] = r % nt[D2];
    r /= nt[D2];
    tc[0] = 2 * (r % (nt[0] >> 1)) + xh;
    tc[3 - D2] = r / (nt[0] >> 1);
  } else {
    tile_coords(lin, nt, D2, tc);  // t2 tiles adjacent
  }
  const int tid = threadIdx.x;
  const int w = tid >> 6;
  int f[3];
  f[0] = tc[0] * TX + (w % GX) * 16 + (tid & 15);
  f[1] = tc[1] * (64 / TX) + w / GX;
  f[2] = tc[2];
  const int gpi = (tid >> 4) & 3;
  const int g1 = gpi >> 1, g2 = gpi & 1;
  const bool valid = f[0] < fe[0] && f[1] < fe[1] && f[2] < fe[2];
  if (!valid) {  // keep the lane for the exchanges, on a valid face
    f[0] = min(f[0], fe[0] - 1);
    f[1] = min(f[1], fe[1] - 1);
  }

  // ---- second tangential sweep along t2 ----------------------------------
  const int bp = face_pitch(be[0]);
  const size_t NB = (size_t)bp * be[1] * be[2];
  const size_t qstride = 2 * NB;
  // Addressing of B (quantity planes): a load is a wave-uniform base held in
  // scalar registers plus a 32-bit lane offset.  Every face of a block lies
  // in one z plane of B for each stencil row j (z is the normal for y and z
  // faces, and t2 for x faces, whose z then depends on j only), so the base
  // is the quantity's start plus that plane's offset and the lane offset the
  // face's place in the plane, plus the partner quantity's plane for the
  // Gauss-point pairs (the lane offsets stay below 2^32, checked when the
  // configuration is validated).
  const size_t plane = (size_t)bp * be[1];
  const uint32_t pair_off = second_pair_offset<R>(NB);
  const size_t qbytes = qstride * sizeof(R);
  const bool second = g2 != 0;
  uint32_t off[5];     // lane offsets, pair partner included on the g2 = 1 lanes
  size_t zoff[5];      // byte offsets of the stencil rows (block-uniform z plane)
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    int b[3] = {f[0], f[1], f[2]};
    int t = f[D2] + j - 2;
    if (P.bc[D2] != HGKS_BC_ISOTHERMAL_WALL) t = t < 0 ? t + P.n[D2] : (t >= P.n[D2] ? t - P.n[D2] : t);
    b[D2] = t;
    zoff[j] = sizeof(R) * b_pos<R>((size_t)(b[2] - bo[2]) * plane, 0, NB);
    const uint32_t inplane = (uint32_t)(b[1] - bo[1]) * (uint32_t)bp + (uint32_t)(b[0] - bo[0]);
    off[j] = (uint32_t)sizeof(R) * (uint32_t)b_pos<R>(inplane, g1, NB) + (second ? pair_off : 0u);
  }
  const R sn = R(gmem(P.dface[DIR])[f[DIR]]);
  const R st1 = R(gmem(P.dgp[D1])[2 * f[D1] + g1]);
  const R st2 = R(gmem(P.dgp[D2])[2 * f[D2] + g2]);
  const HGKS_GLOBAL R* Bg = gmem(B);
  const HGKS_GLOBAL double* qrg = gmem(qref);
  double rl[5];
  rl[0] = qrg[0];
  rl[1] = qrg[1 + DIR];
  rl[2] = qrg[1 + D1];
  rl[3] = qrg[1 + D2];
  rl[4] = qrg[4];
  GasParams<R> g;
  g.gm1 = R(P.gm1);
  g.K = R(P.K);
  g.K3 = R(P.K + 3.0);
  g.iK3 = R(P.iK3);
  g.mu_ref = R(P.mu_ref);
  g.iT_ref = R(P.iT_ref);
  g.imu_ref = R(P.imu_ref);
  g.mu_exp = R(P.mu_exp);
  g.pr_fix = R(P.pr_fix);
  // Wave-uniform base of quantity qi and stencil row j.
  auto row_base = [&](int qi, int j) {
    return uniform_ptr(reinterpret_cast<const HGKS_GLOBAL char*>(Bg) + (size_t)qi * qbytes + zoff[j]);
  };
  // Five stencil values of quantity qi along t2 (qi the same on every lane).
  auto stencil = [&](int qi, R v[5]) {
#pragma unroll
    for (int j = 0; j < 5; ++j) {
      const uint32_t o = off[j] - (second ? pair_off : 0u);
      v[j] = *reinterpret_cast<const HGKS_GLOBAL R*>(row_base(qi, j) + o);
    }
  };
  // Gauss-point pairs: the lanes g2 = 0 and g2 = 1 of a Gauss line (lane and
  // lane ^ 16, an even row and the odd row above it) share every t2
  // stencil.  Each reconstructs one of two quantities at both points and the
  // pair exchanges the other point's values (swap_rows16).  The g2 = 0 lane
  // takes quantity qi0 (Q^l, the normal slopes), the g2 = 1 lane the next
  // one (Q^r, the t1 slopes).
  auto stencil_pair = [&](int qi0, R v[5]) {
#pragma unroll
    for (int j = 0; j < 5; ++j) v[j] = *reinterpret_cast<const HGKS_GLOBAL R*>(row_base(qi0, j) + off[j]);
  };

  // Each phase loads its own raw t2 stencils; the kernels run at least two
  // waves per SIMD (launch bounds), so the other wave covers their latency.
  R pa[5][5];

  // phase 1: left/right values and their t2 slopes; equilibrium, tau, time integrals
  R ql[5], qr[5], tl2[5], tr2[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    R v[5], val[2], der[2];
    stencil_pair(b_ql(k), v);
    gauss_value_slope2(v, val, der);  // the lane's quantity at -s and +s
    swap_rows16(val[0], val[1]);       // Q^l and Q^r at the lane's point
    swap_rows16(der[0], der[1]);
    ql[k] = R(double(val[0]) + rl[k]);
    qr[k] = R(double(val[1]) + rl[k]);
    tl2[k] = der[0] * st2;
    tr2[k] = der[1] * st2;
  }
  FluxAcc<R> acc;
  flux_begin(ql, qr, g, R(dt), acc);

  // phase 2: left side
  {
    R dq[3][5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      stencil_pair(b_dln(k), pa[k]);
      R val[2];
      gauss_value2(pa[k], val);     // the lane's quantity at -s and +s
      swap_rows16(val[0], val[1]);  // normal and t1 slope at the lane's point
      dq[0][k] = val[0] * sn;
      dq[1][k] = val[1] * st1;
      dq[2][k] = tl2[k];
    }
    flux_side<R, true>(ql, dq, g, acc);
  }

  // phase 3: right side
  {
    R dq[3][5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      stencil_pair(b_drn(k), pa[k]);
      R val[2];
      gauss_value2(pa[k], val);     // the lane's quantity at -s and +s
      swap_rows16(val[0], val[1]);  // normal and t1 slope at the lane's point
      dq[0][k] = val[0] * sn;
      dq[1][k] = val[1] * st1;
      dq[2][k] = tr2[k];
    }
    flux_side<R, false>(qr, dq, g, acc);
  }

  // phase 4: equilibrium part and Prandtl correction
  R Fn[5], Fd[5];  // F^n and dF^n/dt at this lane's Gauss point
  {
    R dq0n[5];
    const LinearWeights<R> lw(g2);
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      stencil(b_d0(k), pa[k]);
      dq0n[k] = gauss_linear(pa[k], lw) * sn;
    }
    flux_finish(dq0n, g, acc, Fn, Fd);
  }

  gauss_sum_store<DIR>(P, F, f, valid, gpi, Fn, Fd);
}

// ---- FP64 flux tiles with the t2 stencil rows shared in LDS (x and z faces) --
// For x and z faces t2 is z or y.  A flux block takes 16 faces along x at 4
// consecutive t2 positions (256 threads: wave w holds position w), so it
// needs 8 rows of B per quantity instead of 4 x 5.  At its start the block
// copies all 35 quantities of those rows into LDS (asynchronous global -> LDS
// loads, 16 bytes per lane: one face's two Gauss lines; 70 KB), then every
// phase reads its stencils from there; the other block on the CU computes
// meanwhile.  y faces: flux_tile4y below.
constexpr int FLUX4_X = 16, FLUX4_P = 4, FLUX4_ROWS = FLUX4_P + 4;
__host__ __device__ inline void flux4_tile_counts(const Params& P, int d, int nt[3]) {
  int fe[3];
  face_extents(P, d, fe);
  const int d2 = (d + 2) % 3;
  for (int a = 0; a < 3; ++a) nt[a] = fe[a];
  nt[0] = (fe[0] + FLUX4_X - 1) / FLUX4_X;
  nt[d2] = (fe[d2] + FLUX4_P - 1) / FLUX4_P;
}
__host__ __device__ inline int flux4_tiles(const Params& P, int d) {
  int nt[3];
  flux4_tile_counts(P, d, nt);
  return nt[0] * nt[1] * nt[2];
}

template <int DIR>
__device__ __forceinline__ void flux_tile4(const double* __restrict__ B, const Params& P,
                                           const double* __restrict__ qref, double dt, double* __restrict__ F,
                                           int lin) {
  static_assert(DIR != 1, "y faces use flux_tile");
  constexpr int D1 = (DIR + 1) % 3, D2 = (DIR + 2) % 3;
  constexpr int DO = DIR == 0 ? 1 : 2;  // the axis that is neither x nor t2: one row per block
  int fe[3], be[3], bo[3];
  face_extents(P, DIR, fe);
  b_extents(P, DIR, be, bo);
  int nt[3], tc[3];
  flux4_tile_counts(P, DIR, nt);
  tile_coords(lin, nt, D2, tc);  // t2 tiles adjacent: consecutive blocks share four staged rows
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  int f[3];
  f[0] = tc[0] * FLUX4_X + (lane & 15);
  f[D2] = tc[D2] * FLUX4_P + w;
  f[DO] = tc[DO];
  const int gpi = (lane >> 4) & 3;
  const int g1 = gpi >> 1, g2 = gpi & 1;
  const bool valid = f[0] < fe[0] && f[D2] < fe[D2];
  if (!valid) {  // keep the lane for the exchanges, on a real face
    f[0] = min(f[0], fe[0] - 1);
    f[D2] = min(f[D2], fe[D2] - 1);
  }

  // Staged rows: [quantity][row][face] of 16-byte entries, row r holding
  // t2 = first position - 2 + r (wrapped on a periodic axis; on a wall axis
  // clamped to the last ghost row, which only lanes past the grid's end
  // read).  Entry e = (q FLUX4_ROWS + r) FLUX4_X + face; thread tid copies
  // entries tid + 256 k, so each wave's copy lands in 64 consecutive entries.
  // Row and face of those entries do not depend on k and the quantity is
  // 2 k + tid / 128, so one lane address serves every copy: the k-th is 2 k
  // quantities (512 bytes) further.  The rows span -2 <= t <= 4 ceil(n/4) + 1,
  // within one period either side for every n >= 4.
  __shared__ double2 stage[B_COUNT][FLUX4_ROWS][FLUX4_X];
  constexpr int kEntries = B_COUNT * FLUX4_ROWS * FLUX4_X;
  {
    const int r = (tid >> 4) & (FLUX4_ROWS - 1), fi = tid & (FLUX4_X - 1);
    const int wu = __builtin_amdgcn_readfirstlane(w) & 3;  // LDS destinations in scalar registers
    int t = tc[D2] * FLUX4_P - 2 + r;
    if (P.bc[D2] == HGKS_BC_ISOTHERMAL_WALL) t = min(t, P.n[D2] + 1);
    else t = wrap1(t, P.n[D2]);
    int b[3];
    b[0] = min(tc[0] * FLUX4_X + fi, fe[0] - 1);
    b[D2] = t;
    b[DO] = f[DO];
    const HGKS_GLOBAL char* lane_src =
        reinterpret_cast<const HGKS_GLOBAL char*>(gmem(B)) +
        (b64_face(b[0] - bo[0], b[1] - bo[1], b[2] - bo[2], face_pitch(be[0]), be[1]) + (size_t)(tid >> 7) * 32) *
            sizeof(double);
#pragma unroll
    for (int k = 0; k < (kEntries + FLUX_THREADS - 1) / FLUX_THREADS; ++k)
      if (FLUX_THREADS * k + 64 * wu < kEntries)  // wave-uniform
        dma16_to_lds(lane_src + (size_t)(2 * k) * 32 * sizeof(double),
                     reinterpret_cast<double*>(&stage[0][0][0]) + 2 * (FLUX_THREADS * k + 64 * wu));
  }
  double sn = gmem(P.dface[DIR])[f[DIR]];
  double st1 = gmem(P.dgp[D1])[2 * f[D1] + g1];
  double st2 = gmem(P.dgp[D2])[2 * f[D2] + g2];
  const HGKS_GLOBAL double* qrg = gmem(qref);
  double rl[5];
  rl[0] = qrg[0];
  rl[1] = qrg[1 + DIR];
  rl[2] = qrg[1 + D1];
  rl[3] = qrg[1 + D2];
  rl[4] = qrg[4];
  wait_vmem();      // this wave's copies and loads have landed
  __syncthreads();  // and every wave's
  const double* const st = reinterpret_cast<const double*>(&stage[0][0][0]);
  const int base = (w * FLUX4_X + (lane & 15)) * 2 + g1;  // quantity 0, row w (stencil row 0), line g1
  auto begin = [&](int p) {
    // phase 1's quantities are read by then; their space takes the carried values
    if (p == 1) __syncthreads();
  };
  auto pair = [&](int qi0, double v[5]) {
#pragma unroll
    for (int j = 0; j < 5; ++j) v[j] = st[base + ((qi0 + g2) * FLUX4_ROWS + j) * FLUX4_X * 2];
  };
  auto plain = [&](int qi, double v[5]) {
#pragma unroll
    for (int j = 0; j < 5; ++j) v[j] = st[base + (qi * FLUX4_ROWS + j) * FLUX4_X * 2];
  };
  flux_lane<DIR, double, FLUX_THREADS, true>(begin, pair, plain, P, dt, F, f, valid, gpi, sn, st1, st2, rl,
                                             reinterpret_cast<double*>(&stage[0][0][0]));
}

// ---- FP64 flux tiles of y faces with the t2 stencils shared in LDS ---------
// For y faces t2 is x.  A flux block takes 16 faces along x at 4 consecutive
// z positions (t1; wave w holds position w); the t2 stencils of a row span its
// 20 faces x0 - 2 .. x0 + 17 (x wraps: it is never a wall axis).  At its start
// the block copies the 35 quantities of its 4 rows into LDS, 32 entries per
// row so that, as for the x and z faces, one lane address serves every copy
// (entries 20..31 repeat entry 19 and are never read).
constexpr int FLUX4Y_Z = 4, FLUX4Y_W = 32;
__host__ __device__ inline void flux4y_tile_counts(const Params& P, int nt[3]) {
  int fe[3];
  face_extents(P, 1, fe);
  nt[0] = (fe[0] + FLUX4_X - 1) / FLUX4_X;
  nt[1] = fe[1];
  nt[2] = (fe[2] + FLUX4Y_Z - 1) / FLUX4Y_Z;
}
__host__ __device__ inline int flux4y_tiles(const Params& P) {
  int nt[3];
  flux4y_tile_counts(P, nt);
  return nt[0] * nt[1] * nt[2];
}

__device__ __forceinline__ void flux_tile4y(const double* __restrict__ B, const Params& P,
                                            const double* __restrict__ qref, double dt, double* __restrict__ F,
                                            int lin) {
  constexpr int DIR = 1, D1 = 2, D2 = 0;
  int fe[3], be[3], bo[3];
  face_extents(P, DIR, fe);
  b_extents(P, DIR, be, bo);
  int nt[3], tc[3];
  flux4y_tile_counts(P, nt);
  tile_coords(lin, nt, 0, tc);  // x tiles adjacent: neighbours share their halo faces
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  int f[3];
  f[0] = tc[0] * FLUX4_X + (lane & 15);
  f[1] = tc[1];
  f[2] = tc[2] * FLUX4Y_Z + w;
  const int gpi = (lane >> 4) & 3;
  const int g1 = gpi >> 1, g2 = gpi & 1;
  const bool valid = f[0] < fe[0] && f[2] < fe[2];
  if (!valid) {  // keep the lane for the exchanges, on a real face
    f[0] = min(f[0], fe[0] - 1);
    f[2] = min(f[2], fe[2] - 1);
  }

  // Staged rows: [quantity][row][entry] of 16-byte entries (a face's two Gauss
  // lines), row r holding z = first position + r (clamped to the last face
  // for the rows past the grid, which only lanes past its end read) and entry
  // i the face x = x0 - 2 + min(i, 19).  Entry e = (q FLUX4Y_Z + r) FLUX4Y_W
  // + i; thread tid copies entries tid + 256 k: row and entry do not depend on
  // k and the quantity is 2 k + tid / 128.
  __shared__ double2 stage[B_COUNT][FLUX4Y_Z][FLUX4Y_W];
  constexpr int kEntries = B_COUNT * FLUX4Y_Z * FLUX4Y_W;
  {
    const int r = (tid >> 5) & (FLUX4Y_Z - 1), ei = tid & (FLUX4Y_W - 1);
    const int wu = __builtin_amdgcn_readfirstlane(w) & 3;  // LDS destinations in scalar registers
    // -2 <= x <= 16 ceil(n_x / 16) + 1: within one period either side for
    // n_x > 8; the few narrower grids take the division
    int x = tc[0] * FLUX4_X - 2 + min(ei, FLUX4_X + 3);
    if (P.n[0] > 8) x = wrap1(x, P.n[0]);
    else x = ((x % P.n[0]) + P.n[0]) % P.n[0];
    int b[3];
    b[0] = x;
    b[1] = f[1];
    b[2] = min(tc[2] * FLUX4Y_Z + r, fe[2] - 1);
    const HGKS_GLOBAL char* lane_src =
        reinterpret_cast<const HGKS_GLOBAL char*>(gmem(B)) +
        (b64_face(b[0] - bo[0], b[1] - bo[1], b[2] - bo[2], face_pitch(be[0]), be[1]) + (size_t)(tid >> 7) * 32) *
            sizeof(double);
#pragma unroll
    for (int k = 0; k < (kEntries + FLUX_THREADS - 1) / FLUX_THREADS; ++k)
      if (FLUX_THREADS * k + 64 * wu < kEntries)  // wave-uniform
        dma16_to_lds(lane_src + (size_t)(2 * k) * 32 * sizeof(double),
                     reinterpret_cast<double*>(&stage[0][0][0]) + 2 * (FLUX_THREADS * k + 64 * wu));
  }
  double sn = gmem(P.dface[DIR])[f[DIR]];
  double st1 = gmem(P.dgp[D1])[2 * f[D1] + g1];
  double st2 = gmem(P.dgp[D2])[2 * f[D2] + g2];
  const HGKS_GLOBAL double* qrg = gmem(qref);
  double rl[5];
  rl[0] = qrg[0];
  rl[1] = qrg[1 + DIR];
  rl[2] = qrg[1 + D1];
  rl[3] = qrg[1 + D2];
  rl[4] = qrg[4];
  wait_vmem();      // this wave's copies and loads have landed
  __syncthreads();  // and every wave's
  const double* const st = reinterpret_cast<const double*>(&stage[0][0][0]);
  const int base = (w * FLUX4Y_W + (lane & 15)) * 2 + g1;  // quantity 0, row w, stencil entry 0, line g1
  auto begin = [&](int p) {
    // phase 1's quantities are read by then; their space takes the carried values
    if (p == 1) __syncthreads();
  };
  auto pair = [&](int qi0, double v[5]) {
#pragma unroll
    for (int j = 0; j < 5; ++j) v[j] = st[base + ((qi0 + g2) * FLUX4Y_Z * FLUX4Y_W + j) * 2];
  };
  auto plain = [&](int qi, double v[5]) {
#pragma unroll
    for (int j = 0; j < 5; ++j) v[j] = st[base + (qi * FLUX4Y_Z * FLUX4Y_W + j) * 2];
  };
  static_assert(10 * FLUX4Y_Z * FLUX4Y_W * 2 >= 7 * FLUX_THREADS, "phase 1's quantities hold the carried values");
  flux_lane<DIR, double, FLUX_THREADS, true>(begin, pair, plain, P, dt, F, f, valid, gpi, sn, st1, st2, rl,
                                             reinterpret_cast<double*>(&stage[0][0][0]));
}

__global__ __launch_bounds__(FLUX_THREADS, FLUX_MIN_BLOCKS) void flux4y_kernel(const double* __restrict__ B, Params P,
                                                                              const double* __restrict__ qref,
                                                                              const Scalars* __restrict__ sc,
                                                                              int use_residual_dt,
                                                                              double* __restrict__ F) {
  const double dt = use_residual_dt ? sc->dt_residual : sc->dt;
  flux_tile4y(B, P, qref, dt, F, xcd_linear_block(flux4y_tiles(P)));
}

template <int DIR>
__global__ __launch_bounds__(FLUX_THREADS, FLUX_MIN_BLOCKS) void flux4_kernel(const double* __restrict__ B, Params P,
                                                                             const double* __restrict__ qref,
                                                                             const Scalars* __restrict__ sc,
                                                                             int use_residual_dt,
                                                                             double* __restrict__ F) {
  const double dt = use_residual_dt ? sc->dt_residual : sc->dt;
  flux_tile4<DIR>(B, P, qref, dt, F, xcd_linear_block(flux4_tiles(P, DIR)));
}

template <int DIR, class R>
__global__ __launch_bounds__(FLUX_THREADS, FLUX_MIN_BLOCKS) void flux_kernel(const R* __restrict__ B, Params P,
                                                            const double* __restrict__ qref,
                                                            const Scalars* __restrict__ sc, int use_residual_dt,
                                                            double* __restrict__ F) {
  const double dt = use_residual_dt ? sc->dt_residual : sc->dt;
  flux_tile<DIR, R, 16>(B, P, qref, dt, F, xcd_linear_block(flux_tiles<16>(P, DIR)));
}

// L and dL/dt of one cell from the six face fluxes, plus the body-force source
// S = (0, rho f, m . f) and its time derivative (0, f L_rho, f . L_m).
template <class S>
__device__ __forceinline__ void cell_residual(const S* __restrict__ qe, const double* __restrict__ F0,
                                              const double* __restrict__ F1, const double* __restrict__ F2,
                                              const Params& P, const double fb[3], int i, int j, int k, double L[5],
                                              double dL[5]) {
  const size_t n3 = cells(P);
  const size_t c = ((size_t)k * P.n[1] + j) * P.n[0] + i;
  const double vol = gmem(P.hcell[0])[i] * gmem(P.hcell[1])[j] * gmem(P.hcell[2])[k];
  const HGKS_GLOBAL double* Fd[3] = {gmem(F0), gmem(F1), gmem(F2)};
#pragma unroll
  for (int m = 0; m < 5; ++m) { L[m] = 0.0; dL[m] = 0.0; }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    int fe[3];
    face_extents(P, d, fe);
    const int fpitch = face_pitch(fe[0]);
    const size_t NF = (size_t)fpitch * fe[1] * fe[2];
    const size_t fm = ((size_t)k * fe[1] + j) * fpitch + i;
    const size_t step = d == 0 ? 1 : (d == 1 ? (size_t)fpitch : (size_t)fpitch * fe[1]);
    // right face; on a periodic normal axis the last cell's is face 0
    const int ci = d == 0 ? i : (d == 1 ? j : k);
    const size_t fp = fe[d] == P.n[d] && ci == P.n[d] - 1 ? fm - (size_t)ci * step : fm + step;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      L[m] -= (Fd[d][m * NF + fp] - Fd[d][m * NF + fm]) / vol;
      dL[m] -= (Fd[d][(5 + m) * NF + fp] - Fd[d][(5 + m) * NF + fm]) / vol;
    }
  }
  const HGKS_GLOBAL S* qg = gmem(qe);
  const double rho = qg[c], mx = qg[n3 + c], my = qg[2 * n3 + c], mz = qg[3 * n3 + c];
  const double lrho = L[0];
  L[1] += rho * fb[0];
  L[2] += rho * fb[1];
  L[3] += rho * fb[2];
  L[4] += mx * fb[0] + my * fb[1] + mz * fb[2];
  dL[1] += fb[0] * lrho;
  dL[2] += fb[1] * lrho;
  dL[3] += fb[2] * lrho;
  dL[4] += fb[0] * L[1] + fb[1] * L[2] + fb[2] * L[3];
}

// Wave speed max_d (|U_d| + c) / h_d of one cell.
__device__ __forceinline__ double cell_wave_rate(const double v[5], const Params& P, int i, int j, int k) {
  double ir = 1.0 / v[0];
  double U = v[1] * ir, V = v[2] * ir, W = v[3] * ir;
  double p = P.gm1 * (v[4] - 0.5 * v[0] * (U * U + V * V + W * W));
  double c = sqrt(P.gamma * p * ir);
  double r = (fabs(U) + c) / gmem(P.hcell[0])[i];
  r = fmax(r, (fabs(V) + c) / gmem(P.hcell[1])[j]);
  r = fmax(r, (fabs(W) + c) / gmem(P.hcell[2])[k]);
  return r;
}

// Block max of a non-negative double, then one atomic max on its bit pattern
// (non-negative doubles order like their unsigned 64-bit patterns).
__device__ __forceinline__ void block_max_atomic(double r, unsigned long long* dst) {
  __shared__ double red[16];
  for (int o = 32; o > 0; o >>= 1) r = fmax(r, __shfl_xor(r, o));
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) red[w] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) m = fmax(m, red[i]);
    atomicMax(dst, (unsigned long long)__double_as_longlong(m));
  }
  __syncthreads();  // red[] may be reused by the next call in this block
}

// Block sum in a fixed order (wave shuffles, then the waves in order), stored
// by thread 0: deterministic.
__device__ __forceinline__ void block_sum_store(double x, double* dst) {
  __shared__ double red[16];
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) red[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) t += red[i];
    *dst = t;
  }
  __syncthreads();  // red[] may be reused by the next call in this block
}

constexpr int CELL_THREADS = 256;

// S2O4 stage for cell block `blk` (CELL_THREADS cells) of one instance.
template <int STAGE, class S = double>
__device__ __forceinline__ void update_block(S* __restrict__ q, S* __restrict__ qs, S* __restrict__ acc,
                                             const double* __restrict__ F0, const double* __restrict__ F1,
                                             const double* __restrict__ F2, const Params& P, Scalars* __restrict__ sc,
                                             double* __restrict__ mpart, size_t blk) {
  const size_t n3 = cells(P);
  const size_t c = blk * CELL_THREADS + threadIdx.x;
  HGKS_GLOBAL S* qg = gmem(q);
  HGKS_GLOBAL S* qsg = gmem(qs);
  HGKS_GLOBAL S* accg = gmem(acc);
  const double fb[3] = {gmem(sc)->force_x, P.force[1], P.force[2]};
  double rate = 0.0, mflux = 0.0;
  if (c < n3) {
    const int i = (int)(c % P.n[0]);
    const int j = (int)((c / P.n[0]) % P.n[1]);
    const int k = (int)(c / ((size_t)P.n[0] * P.n[1]));
    const double dt = gmem(sc)->dt;
    double L[5], dL[5];
    if (STAGE == 1) {
      cell_residual(q, F0, F1, F2, P, fb, i, j, k, L, dL);
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        const double qn = qg[m * n3 + c];
        qsg[m * n3 + c] = S(qn + 0.5 * dt * L[m] + 0.125 * dt * dt * dL[m]);
        accg[m * n3 + c] = S(qn + dt * L[m] + dt * dt / 6.0 * dL[m]);
      }
    } else {
      cell_residual(qs, F0, F1, F2, P, fb, i, j, k, L, dL);
      double v[5];
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        v[m] = double(S(double(accg[m * n3 + c]) + dt * dt / 3.0 * dL[m]));
        qg[m * n3 + c] = S(v[m]);
      }
      rate = cell_wave_rate(v, P, i, j, k);
      if (P.flags & HGKS_FLAG_CONSTANT_MASS_FLUX)
        mflux = v[1] * gmem(P.hcell[0])[i] * gmem(P.hcell[1])[j] * gmem(P.hcell[2])[k];
    }
  }
  if (STAGE == 2) {
    block_max_atomic(rate, &sc->smax);
    if (P.flags & HGKS_FLAG_CONSTANT_MASS_FLUX) block_sum_store(mflux, &mpart[blk]);
  }
}

template <int STAGE, class S>
__global__ __launch_bounds__(CELL_THREADS) void update_kernel(S* __restrict__ q, S* __restrict__ qs,
                                                              S* __restrict__ acc, const double* __restrict__ F0,
                                                              const double* __restrict__ F1,
                                                              const double* __restrict__ F2, Params P,
                                                              Scalars* __restrict__ sc, double* __restrict__ mpart) {
  update_block<STAGE, S>(q, qs, acc, F0, F1, F2, P, sc, mpart, blockIdx.x);
}

__global__ __launch_bounds__(CELL_THREADS) void residual_kernel(const double* __restrict__ qe,
                                                                const double* __restrict__ F0,
                                                                const double* __restrict__ F1,
                                                                const double* __restrict__ F2, Params P,
                                                                const Scalars* __restrict__ sc,
                                                                double* __restrict__ Lo, double* __restrict__ dLo) {
  const size_t n3 = cells(P);
  const size_t c = (size_t)blockIdx.x * CELL_THREADS + threadIdx.x;
  if (c >= n3) return;
  const int i = (int)(c % P.n[0]);
  const int j = (int)((c / P.n[0]) % P.n[1]);
  const int k = (int)(c / ((size_t)P.n[0] * P.n[1]));
  double L[5], dL[5];
  const double fb[3] = {sc->force_x, P.force[1], P.force[2]};
  cell_residual(qe, F0, F1, F2, P, fb, i, j, k, L, dL);
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    Lo[m * n3 + c] = L[m];
    dLo[m * n3 + c] = dL[m];
  }
}

__global__ __launch_bounds__(CELL_THREADS) void wave_rate_kernel(const double* __restrict__ q, Params P,
                                                                 Scalars* __restrict__ sc) {
  const size_t n3 = cells(P);
  const size_t c = (size_t)blockIdx.x * CELL_THREADS + threadIdx.x;
  double rate = 0.0;
  if (c < n3) {
    const int i = (int)(c % P.n[0]);
    const int j = (int)((c / P.n[0]) % P.n[1]);
    const int k = (int)(c / ((size_t)P.n[0] * P.n[1]));
    double v[5];
#pragma unroll
    for (int m = 0; m < 5; ++m) v[m] = q[m * n3 + c];
    rate = cell_wave_rate(v, P, i, j, k);
  }
  block_max_atomic(rate, &sc->smax);
}

// Start of a step: choose dt (fixed, or CFL from the wave-speed maximum of
// the current state), advance the clock, clear the maximum for stage 2.
__global__ void begin_step_kernel(Scalars* sc, double cfl) {
  if (threadIdx.x != 0) return;
  const double smax = __longlong_as_double((long long)sc->smax);
  const double dt = sc->dt_fixed > 0.0 ? sc->dt_fixed : cfl / smax;
  sc->dt = dt;
  sc->t += dt;
  sc->steps += 1.0;
  sc->smax = 0ull;
}

__global__ void set_scalar_kernel(double* dst, double v) {
  if (threadIdx.x == 0) *dst = v;
}

// Element-wise precision conversion (the FP32 path's working copy of the state).
template <class A, class Bt>
__global__ __launch_bounds__(CELL_THREADS) void convert_kernel(const A* __restrict__ a, Bt* __restrict__ b, size_t n) {
  const size_t i = (size_t)blockIdx.x * CELL_THREADS + threadIdx.x;
  if (i < n) gmem(b)[i] = Bt(gmem(a)[i]);
}

// ---- statistics ----------------------------------------------------------
enum { ST_EK = 0, ST_ENS, ST_DIL, ST_TOT, ST_MAX = ST_TOT + 5, ST_MINP = ST_MAX + 5, ST_MINR, ST_BAD, ST_COUNT };

// Velocity U = m / rho of a padded-state cell (all three components from
// one load of the cell).
__device__ __forceinline__ void vel3(const double* __restrict__ q, const Params& P, int i, int j, int k,
                                     double u[3]) {
  double v[5];
  load_cell(q, P, i, j, k, v);
#pragma unroll
  for (int a = 0; a < 3; ++a) u[a] = v[1 + a] / v[0];
}

// Fourth-order central differences of the three velocity components along
// axis, in index space scaled by d(index)/dx at the cell centre: g[a] =
// dU_a / dx_axis.
__device__ __forceinline__ void dvel3(const double* __restrict__ q, const Params& P, int axis, int i, int j, int k,
                                      double g[3]) {
  int o[3] = {0, 0, 0};
  o[axis] = 1;
  double m2[3], m1[3], p1[3], p2[3];
  vel3(q, P, i - 2 * o[0], j - 2 * o[1], k - 2 * o[2], m2);
  vel3(q, P, i - o[0], j - o[1], k - o[2], m1);
  vel3(q, P, i + o[0], j + o[1], k + o[2], p1);
  vel3(q, P, i + 2 * o[0], j + 2 * o[1], k + 2 * o[2], p2);
  const int ia = axis == 0 ? i : (axis == 1 ? j : k);
  const double sc = P.dcen[axis][ia];
#pragma unroll
  for (int a = 0; a < 3; ++a) g[a] = (m2[a] - 8.0 * m1[a] + 8.0 * p1[a] - p2[a]) / 12.0 * sc;
}

__global__ __launch_bounds__(CELL_THREADS) void stats_partial_kernel(const double* __restrict__ q, Params P,
                                                                     double* __restrict__ part) {
  __shared__ double red[ST_COUNT][CELL_THREADS];
  const size_t n3 = cells(P);
  const size_t c = (size_t)blockIdx.x * CELL_THREADS + threadIdx.x;
  double s[ST_COUNT];
  for (int m = 0; m < ST_COUNT; ++m) s[m] = 0.0;
  s[ST_MINP] = INFINITY;
  s[ST_MINR] = INFINITY;
  if (c < n3) {
    const int i = (int)(c % P.n[0]);
    const int j = (int)((c / P.n[0]) % P.n[1]);
    const int k = (int)(c / ((size_t)P.n[0] * P.n[1]));
    double v[5];
    for (int m = 0; m < 5; ++m) v[m] = q[m * n3 + c];
    const double dv = P.hcell[0][i] * P.hcell[1][j] * P.hcell[2][k];
    const double ke = 0.5 * (v[1] * v[1] + v[2] * v[2] + v[3] * v[3]) / v[0];
    const double p = P.gm1 * (v[4] - ke);
    s[ST_EK] = ke * dv;
    double gr[3][3];  // gr[a][b] = dU_a / dx_b
    for (int b = 0; b < 3; ++b) {
      double g[3];
      dvel3(q, P, b, i, j, k, g);
#pragma unroll
      for (int a = 0; a < 3; ++a) gr[a][b] = g[a];
    }
    const double wx = gr[2][1] - gr[1][2], wy = gr[0][2] - gr[2][0], wz = gr[1][0] - gr[0][1];
    const double dv_ = gr[0][0] + gr[1][1] + gr[2][2];
    s[ST_ENS] = (wx * wx + wy * wy + wz * wz) * dv;
    s[ST_DIL] = dv_ * dv_ * dv;
    bool bad = false;
    for (int m = 0; m < 5; ++m) {
      s[ST_TOT + m] = v[m] * dv;
      s[ST_MAX + m] = fabs(v[m]);
      bad = bad || !isfinite(v[m]);
    }
    s[ST_MINP] = p;
    s[ST_MINR] = v[0];
    s[ST_BAD] = bad ? 1.0 : 0.0;
  }
  for (int m = 0; m < ST_COUNT; ++m) red[m][threadIdx.x] = s[m];
  __syncthreads();
  for (int w = CELL_THREADS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      for (int m = 0; m < ST_COUNT; ++m) {
        double a = red[m][threadIdx.x], b = red[m][threadIdx.x + w];
        if (m >= ST_MAX && m < ST_MAX + 5) red[m][threadIdx.x] = fmax(a, b);
        else if (m == ST_MINP || m == ST_MINR) red[m][threadIdx.x] = fmin(a, b);
        else if (m == ST_BAD) red[m][threadIdx.x] = fmax(a, b);
        else red[m][threadIdx.x] = a + b;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < ST_COUNT) part[(size_t)blockIdx.x * ST_COUNT + threadIdx.x] = red[threadIdx.x][0];
}

// Deterministic final reduction: block m reduces field m; thread t combines
// blocks t, t + 256, ... in order, then a fixed tree combines the threads.
__global__ __launch_bounds__(256) void stats_final_kernel(const double* __restrict__ part, int nblocks,
                                                          double* __restrict__ out) {
  __shared__ double red[256];
  const int m = blockIdx.x, t = threadIdx.x;
  const bool is_max = (m >= ST_MAX && m < ST_MAX + 5) || m == ST_BAD;
  const bool is_min = m == ST_MINP || m == ST_MINR;
  double a = is_min ? INFINITY : (is_max ? -INFINITY : 0.0);
  for (int b = t; b < nblocks; b += 256) {
    const double x = part[(size_t)b * ST_COUNT + m];
    a = is_max ? fmax(a, x) : (is_min ? fmin(a, x) : a + x);
  }
  red[t] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      const double x = red[t + w], y = red[t];
      red[t] = is_max ? fmax(y, x) : (is_min ? fmin(y, x) : y + x);
    }
    __syncthreads();
  }
  if (t == 0) out[m] = red[0];
}

// ---- batched ensemble ------------------------------------------------------
// Each instance has its own parameters, state, workspace and device scalars.
// Work lists (tiles or cell blocks) of all instances are concatenated; row r
// of the prefix table holds the instance offsets of list r.
struct BatchEntry {
  Params P;
  double* q;
  double* qs;
  double* acc;
  void* B;
  double* F[3];
  Scalars* sc;
  double* qref;
  double cfl;
  float* q32;         // whole-code FP32 members: the FP32 working copy of the state
  double* mpart;      // per-block sums of rho U dV (constant-mass-flux members)
  const double* mf;   // the controller's {rho_b, m_t}
  double inv_vol;     // 1 / domain volume
};
enum { PRE_RECON = 0, PRE_FLUX = 3, PRE_CELL = 9, PRE_ROWS = 10 };  // flux rows: TX 16, 32 x 3 directions
template <int TX> constexpr int flux_row(int d) { return PRE_FLUX + 3 * (TX == 16 ? 0 : 1) + d; }

struct BatchTable {
  const BatchEntry* E;
  const int* pre;     // [PRE_ROWS][n + 1]: prefix sums of the members' work items
  const int* coarse;  // per row: the member holding item k << BATCH_COARSE_SHIFT
  int coarse_off[PRE_ROWS];
  int n;
};
constexpr int BATCH_COARSE_SHIFT = 6;

// Member holding item t of work-list row `row`, and t's index within it: the
// coarse table gives the member of item (t >> 6) << 6, then a forward step
// over members that end before t (every member has at least one item).
__device__ __forceinline__ int find_instance(const BatchTable& T, int row, int t, int& local) {
  const int* pre = T.pre + row * (T.n + 1);
  int inst = T.coarse[T.coarse_off[row] + (t >> BATCH_COARSE_SHIFT)];
  while (t >= pre[inst + 1]) ++inst;
  local = t - pre[inst];
  return inst;
}

// The batched kernels run one block per work item of the slice [t0, t1) of
// the concatenated work list (all members, or a group of consecutive members);
// blocks are XCD-remapped so each XCD's L2 holds neighbouring tiles.
template <int DIR, class R, class ST>
__global__ __launch_bounds__(RECON_THREADS) void recon_batch_kernel(BatchTable T, int t0, int t1, int src_qs) {
  __shared__ R A[25][recon_lds_faces<DIR, R>()];
  const int t = t0 + xcd_linear_block(gridDim.x);
  if (t >= t1) return;
  int local;
  const BatchEntry& e = T.E[find_instance(T, PRE_RECON + DIR, t, local)];
  const ST* src;
  if constexpr (sizeof(ST) == 4) src = src_qs ? reinterpret_cast<const float*>(e.qs) : e.q32;
  else src = src_qs ? e.qs : e.q;
  recon_tile<DIR, R, ST>(src, e.P, e.qref, static_cast<R*>(e.B), local, A);
}

template <int DIR, class R, int TX>
__global__ __launch_bounds__(FLUX_THREADS, FLUX_MIN_BLOCKS) void flux_batch_kernel(BatchTable T, int t0, int t1) {
  const int t = t0 + xcd_linear_block(gridDim.x);
  if (t >= t1) return;
  int local;
  const BatchEntry& e = T.E[find_instance(T, flux_row<TX>(DIR), t, local)];
  if constexpr (sizeof(R) == 8 && DIR != 1)  // the tiles of a standalone run of the member
    flux_tile4<DIR>(static_cast<const double*>(e.B), e.P, e.qref, gmem(e.sc)->dt, e.F[DIR], local);
  else if constexpr (sizeof(R) == 8)
    flux_tile4y(static_cast<const double*>(e.B), e.P, e.qref, gmem(e.sc)->dt, e.F[DIR], local);
  else
    flux_tile<DIR, R, TX>(static_cast<const R*>(e.B), e.P, e.qref, gmem(e.sc)->dt, e.F[DIR], local);
}

template <int STAGE, class S>
__global__ __launch_bounds__(CELL_THREADS) void update_batch_kernel(BatchTable T, int t0, int t1) {
  const int t = t0 + xcd_linear_block(gridDim.x);
  if (t >= t1) return;
  int local;
  const BatchEntry& e = T.E[find_instance(T, PRE_CELL, t, local)];
  if constexpr (sizeof(S) == 4)
    update_block<STAGE, float>(e.q32, reinterpret_cast<float*>(e.qs), reinterpret_cast<float*>(e.acc), e.F[0],
                               e.F[1], e.F[2], e.P, e.sc, e.mpart, (size_t)local);
  else
    update_block<STAGE, double>(e.q, e.qs, e.acc, e.F[0], e.F[1], e.F[2], e.P, e.sc, e.mpart, (size_t)local);
}

// Start of a batched step: each instance takes its own CFL time step.
__global__ void begin_step_batch_kernel(BatchTable T) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T.n) return;
  Scalars* sc = T.E[i].sc;
  const double smax = __longlong_as_double((long long)sc->smax);
  const double dt = T.E[i].cfl / smax;
  sc->dt = dt;
  sc->t += dt;
  sc->steps += 1.0;
  sc->smax = 0ull;
}

// Each member's CFL time step from its current wave-speed maximum, nothing
// else changed (the autotuner's launches then work on real time steps).
__global__ void batch_cfl_dt_kernel(BatchTable T) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T.n) return;
  Scalars* sc = T.E[i].sc;
  sc->dt = T.E[i].cfl / __longlong_as_double((long long)sc->smax);
}

// Reference state of the FP32-reconstruction paths (mixed, FP32): the volume
// mean of Q, from the totals of the statistics reduction.  Reconstruction
// works on deviations from it.
__global__ void mean_state_kernel(const double* __restrict__ fin, double inv_vol, double* __restrict__ qref) {
  if (threadIdx.x < 5) qref[threadIdx.x] = fin[ST_TOT + threadIdx.x] * inv_vol;
}

// Constant streamwise mass flux (Sec. 4.2: the external force follows from a
// constant streamwise momentum flux).  At init: the target m_t and the mean
// density rho_b are the volume means of rho U and rho of the initial state.
// After each step, with e = m - m_t for the step's volume mean m of rho U,
// f <- f - (2 e^{n+1} - e^n) / (rho_b dt): the force that brings the error to
// zero over the next step if the wall drag stays what the last step showed.
// mf = {rho_b, m_t}.
__global__ void mass_flux_init_kernel(const double* __restrict__ fin, double inv_vol, double* __restrict__ mf,
                                      Scalars* __restrict__ sc) {
  if (threadIdx.x != 0) return;
  mf[0] = fin[ST_TOT + 0] * inv_vol;
  mf[1] = fin[ST_TOT + 1] * inv_vol;
  sc->m_prev = mf[1];
}

// One block of 256 threads: the volume mean of rho U from the stage-2 block
// sums (fixed order, so deterministic) and the force update.
__device__ __forceinline__ void mass_flux_update(const double* __restrict__ mpart, int nb, double inv_vol,
                                                 const double* __restrict__ mf, Scalars* __restrict__ sc) {
  __shared__ double red[256];
  double t = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) t += mpart[b];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double m = red[0] * inv_vol, mt = mf[1];
    const double e1 = m - mt, e0 = sc->m_prev - mt;
    sc->force_x -= (2.0 * e1 - e0) / (mf[0] * sc->dt);
    sc->m_prev = m;
  }
}
__global__ __launch_bounds__(256) void mass_flux_kernel(const double* __restrict__ mpart, int nb, double inv_vol,
                                                        const double* __restrict__ mf, Scalars* __restrict__ sc) {
  mass_flux_update(mpart, nb, inv_vol, mf, sc);
}
// The controller of every constant-mass-flux member of a batch: block i
// serves member i, the same reduction as a single instance's (the other
// members' blocks return at once).
__global__ __launch_bounds__(256) void mass_flux_batch_kernel(BatchTable T) {
  const BatchEntry& e = T.E[blockIdx.x];
  if (!(e.P.flags & HGKS_FLAG_CONSTANT_MASS_FLUX)) return;
  mass_flux_update(e.mpart, (int)((cells(e.P) + CELL_THREADS - 1) / CELL_THREADS), e.inv_vol, e.mf, e.sc);
}

// ---- device-side set-up (the entry point that takes no host buffers) ------
// Coordinate map of one axis: uniform, or the tanh stretching of Sec. 4.2,
// x(xi) = lo + (hi - lo) (1 + tanh(b (2 xi/n - 1)) / tanh b) / 2 for the
// continuous cell index xi in [0, n].
struct AxisMap {
  double lo, hi, b;
  int n, stretched;
};
__device__ __forceinline__ double map_coord(const AxisMap& m, double xi) {
  const double Lh = m.hi - m.lo;
  if (m.stretched) return m.lo + 0.5 * Lh * (1.0 + tanh(m.b * (2.0 * xi / m.n - 1.0)) / tanh(m.b));
  return m.lo + Lh * xi / m.n;
}
__device__ __forceinline__ double map_dcoord(const AxisMap& m, double xi) {
  const double Lh = m.hi - m.lo;
  if (m.stretched) {
    const double ch = cosh(m.b * (2.0 * xi / m.n - 1.0));
    return Lh * m.b / (m.n * tanh(m.b) * ch * ch);
  }
  return Lh / m.n;
}
// Metric arrays of one axis: cell widths h, and d(index)/dx at the faces
// (df, n + 1), the two Gauss points of each cell (dg) and the centres (dc).
__global__ __launch_bounds__(256) void geometry_kernel(AxisMap m, double* __restrict__ h, double* __restrict__ df,
                                                       double* __restrict__ dg, double* __restrict__ dc) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > m.n) return;
  const double hu = (m.hi - m.lo) / m.n;
  df[i] = m.stretched ? 1.0 / map_dcoord(m, double(i)) : 1.0 / hu;
  if (i == m.n) return;
  const double r3 = sqrt(3.0) / 6.0;
  h[i] = m.stretched ? map_coord(m, i + 1.0) - map_coord(m, double(i)) : hu;
  dg[2 * i] = m.stretched ? 1.0 / map_dcoord(m, i + 0.5 - r3) : 1.0 / hu;
  dg[2 * i + 1] = m.stretched ? 1.0 / map_dcoord(m, i + 0.5 + r3) : 1.0 / hu;
  dc[i] = m.stretched ? 1.0 / map_dcoord(m, i + 0.5) : 1.0 / hu;
}

// Device scalars of a residual evaluation: every field written (the memory
// keeps whatever an earlier call left there).
__global__ void residual_scalars_kernel(Scalars* sc, double dt, double force_x, double* __restrict__ qref) {
  if (threadIdx.x == 0) {
    Scalars s{};
    s.dt = dt;
    s.dt_residual = dt;
    s.force_x = force_x;
    *sc = s;
  }
  if (threadIdx.x < 5) qref[threadIdx.x] = 0.0;
}

}  // namespace hgks

// ===========================================================================
// Host side: context, workspace layout, launches, C ABI.
// ===========================================================================
using namespace hgks;

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t qs, acc, B, F[3], metric[3][4], scal, part, qref, mf, mpart, q32, total;
  size_t nb_elems;  // elements of B (per direction maximum)
  int stat_blocks;
};

// FP32 reconstruction and flux (the mixed and the FP32 paths).
bool precision_mixed(const hgks_config& c) { return c.precision == HGKS_MIXED || c.precision == HGKS_FP32; }
// The state, stage values and update in FP32 as well.
bool precision_fp32(const hgks_config& c) { return c.precision == HGKS_FP32; }

// Workspace carve of a configuration.  residual_only: just what L and dL/dt
// of a state need (face buffers, metric arrays, scalars, reduction partials,
// reference state), without the stage states and the controller's buffers.
Layout make_layout(const hgks_config& c, bool residual_only = false) {
  Params P{};
  for (int a = 0; a < 3; ++a) { P.n[a] = c.n[a]; P.bc[a] = c.bc[a]; }
  Layout L{};
  size_t off = 0;
  const size_t n3 = (size_t)c.n[0] * c.n[1] * c.n[2];
  auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  L.qs = residual_only ? 0 : take(5 * n3 * sizeof(double));
  L.acc = residual_only ? 0 : take(5 * n3 * sizeof(double));
  size_t nb = 0;
  for (int d = 0; d < 3; ++d) {
    int be[3], bo[3];
    b_extents(P, d, be, bo);
    nb = std::max(nb, (size_t)face_pitch(be[0]) * be[1] * be[2]);
  }
  L.nb_elems = (size_t)B_COUNT * 2 * nb;
  L.B = take(L.nb_elems * (precision_mixed(c) ? sizeof(float) : sizeof(double)));
  for (int d = 0; d < 3; ++d) {
    int fe[3];
    face_extents(P, d, fe);
    L.F[d] = take((size_t)10 * face_pitch(fe[0]) * fe[1] * fe[2] * sizeof(double));
  }
  for (int a = 0; a < 3; ++a) {
    L.metric[a][0] = take(c.n[a] * sizeof(double));            // hcell
    L.metric[a][1] = take((c.n[a] + 1) * sizeof(double));      // dface
    L.metric[a][2] = take(2 * c.n[a] * sizeof(double));        // dgp
    L.metric[a][3] = take(c.n[a] * sizeof(double));            // dcen
  }
  L.scal = take(sizeof(Scalars));
  L.stat_blocks = (int)((n3 + CELL_THREADS - 1) / CELL_THREADS);
  L.part = take(((size_t)L.stat_blocks + 1) * ST_COUNT * sizeof(double));
  L.qref = take(5 * sizeof(double));
  if (!residual_only) {
    L.mf = take(2 * sizeof(double));
    L.mpart = take(((n3 + CELL_THREADS - 1) / CELL_THREADS) * sizeof(double));
    L.q32 = precision_fp32(c) ? take(5 * n3 * sizeof(float)) : 0;  // FP32 path: working copy of the state
  }
  L.total = off;
  return L;
}

// Coordinate map of axis a: x(xi), xi in [0, n] the continuous cell index.
// Uniform, or (axis 1 with y_stretch = b > 0) the tanh map of Sec. 4.2:
// x = lo + (hi - lo) (1 + tanh(b (2 xi/n - 1)) / tanh b) / 2.
double coord(const hgks_config& c, int a, double xi) {
  const double Lh = c.hi[a] - c.lo[a];
  if (a == 1 && c.y_stretch > 0.0) {
    const double b = c.y_stretch;
    return c.lo[a] + 0.5 * Lh * (1.0 + std::tanh(b * (2.0 * xi / c.n[a] - 1.0)) / std::tanh(b));
  }
  return c.lo[a] + Lh * xi / c.n[a];
}
double dcoord(const hgks_config& c, int a, double xi) {
  const double Lh = c.hi[a] - c.lo[a];
  if (a == 1 && c.y_stretch > 0.0) {
    const double b = c.y_stretch;
    const double ch = std::cosh(b * (2.0 * xi / c.n[a] - 1.0));
    return Lh * b / (c.n[a] * std::tanh(b) * ch * ch);
  }
  return Lh / c.n[a];
}

// Kernel parameters of a configuration; the metric pointers are set by the
// caller once the metric arrays have a place.
Params make_params(const hgks_config& c) {
  Params P{};
  for (int a = 0; a < 3; ++a) {
    P.n[a] = c.n[a];
    P.bc[a] = c.bc[a];
    P.force[a] = c.body_force[a];
  }
  P.flags = c.flags;
  P.gamma = c.gamma;
  P.gm1 = c.gamma - 1.0;
  P.K = (5.0 - 3.0 * c.gamma) / (c.gamma - 1.0);
  P.mu_ref = c.mu_ref;
  P.T_ref = c.T_ref;
  P.mu_exp = c.mu_exp;
  P.pr_fix = 1.0 / c.prandtl - 1.0;
  P.T_wall = c.T_wall;
  P.iK3 = 1.0 / (P.K + 3.0);
  P.iT_ref = c.T_ref > 0.0 ? 1.0 / c.T_ref : 0.0;
  P.imu_ref = c.mu_ref > 0.0 ? 1.0 / c.mu_ref : 0.0;
  return P;
}

const char* kStatus[] = {"ok", "invalid argument", "out of memory", "device error", "non-finite state",
                         "non-positive density or pressure", "unsupported"};

}  // namespace

struct hgks_ctx_s {
  hgks_config cfg;
  hipStream_t stream;
  double* q;
  char* ws;
  size_t ws_bytes;
  Layout L;
  Params P;
  double* qs;
  double* acc;
  void* B;
  double* F[3];
  Scalars* sc;
  double* part;
  double* qref;
  float* q32;     // FP32 path: working copy of the state (Q* and the accumulator reuse qs, acc)
  double* mf;     // mass-flux controller: {rho_b, m_t}
  double* mpart;  // per-block sums of rho U dV (stage 2)
  hgks_status latched;
  double t0;
  std::string err;
  // profiling: event pairs per launch, in launch order
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_class;
  size_t ev_used = 0;
  // batched ensemble (hgks_batch_init): member contexts, device work table,
  // tuned launch shapes and the captured step
  std::vector<hgks_ctx> members;
  BatchTable table{};
  std::vector<int> pre;          // host copy of the prefix rows
  std::vector<int> group_first;  // member groups [group_first[g], group_first[g + 1])
  int tx = 16, group_mib = 0, tune_source = 0;
  bool mass_flux_members = false;  // a member runs the constant-mass-flux controller
  hipGraph_t graph = nullptr;      // batched step, or the single-instance step (hgks_step)
  hipGraphExec_t exec = nullptr;
  double dt_fixed = 0.0;           // last time-step rule written to the device scalars
  bool dt_fixed_known = false;
};

enum { PROF_RECON = 0, PROF_FLUX = 1, PROF_UPDATE = 2, PROF_OTHER = 3 };

// Record the start event of a launch of class cls (no-op unless profiling).
static hipError_t prof_begin(hgks_ctx ctx, int cls) {
  if (!ctx->prof) return hipSuccess;
  if (ctx->ev_used + 2 > ctx->ev_pool.size()) {
    for (int i = 0; i < 2; ++i) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      ctx->ev_pool.push_back(e);
    }
  }
  if (ctx->ev_class.size() < ctx->ev_pool.size() / 2) ctx->ev_class.resize(ctx->ev_pool.size() / 2);
  ctx->ev_class[ctx->ev_used / 2] = cls;
  return hipEventRecord(ctx->ev_pool[ctx->ev_used], ctx->stream);
}
static hipError_t prof_end(hgks_ctx ctx) {
  if (!ctx->prof) return hipSuccess;
  hipError_t r = hipEventRecord(ctx->ev_pool[ctx->ev_used + 1], ctx->stream);
  ctx->ev_used += 2;
  return r;
}

static hgks_status validate(const hgks_config* c, const char** why) {
  auto bad = [&](const char* m) { if (why) *why = m; return HGKS_E_INVALID; };
  if (!c) return bad("null config");
  if (c->abi_version != HGKS_ABI_VERSION) return bad("abi_version mismatch");
  for (int a = 0; a < 3; ++a) {
    if (c->n[a] < 4) return bad("each n must be >= 4");
    if (!(c->hi[a] > c->lo[a])) return bad("hi must exceed lo");
    if (c->bc[a] != HGKS_BC_PERIODIC && c->bc[a] != HGKS_BC_ISOTHERMAL_WALL) return bad("unknown bc");
    if (c->bc[a] == HGKS_BC_ISOTHERMAL_WALL && a != 1) return bad("walls are supported on the y axis only");
  }
  if ((size_t)c->n[0] * c->n[1] * c->n[2] > ((size_t)1 << 34)) return bad("grid too large");
  {
    // the flux kernel's 32-bit lane offsets into buffer B span one quantity
    // (both Gauss lines), the next quantity's offset and one z plane
    Params P{};
    for (int a = 0; a < 3; ++a) { P.n[a] = c->n[a]; P.bc[a] = c->bc[a]; }
    for (int d = 0; d < 3; ++d) {
      int be[3], bo[3];
      b_extents(P, d, be, bo);
      const size_t plane = (size_t)face_pitch(be[0]) * be[1];
      if (2 * sizeof(double) * plane * ((size_t)be[2] + 1) >= ((size_t)1 << 32)) return bad("grid too large");
    }
  }
  if (!(c->gamma > 1.0 && c->gamma <= 5.0 / 3.0)) return bad("gamma out of (1, 5/3]");
  if (!(c->prandtl > 0.0)) return bad("prandtl must be > 0");
  if (!(c->mu_ref >= 0.0)) return bad("mu_ref must be >= 0");
  if (c->mu_exp != 0.0 && !(c->T_ref > 0.0)) return bad("T_ref must be > 0 with a power-law viscosity");
  if (c->bc[1] == HGKS_BC_ISOTHERMAL_WALL && !(c->T_wall > 0.0)) return bad("T_wall must be > 0");
  if (!(c->y_stretch >= 0.0)) return bad("y_stretch must be >= 0");
  if (!(c->cfl > 0.0)) return bad("cfl must be > 0");
  if (!(c->rho_ref > 0.0)) return bad("rho_ref must be > 0");
  if (c->precision != HGKS_FP64 && c->precision != HGKS_MIXED && c->precision != HGKS_FP32)
    return bad("unknown precision");
  if ((c->flags & ~HGKS_FLAG_CONSTANT_MASS_FLUX) != 0) return bad("unknown flags");
  return HGKS_OK;
}

#define HIP_TRY(ctx, expr)                                                               \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess) {                                                              \
      (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(e_);                    \
      return HGKS_E_DEVICE;                                                              \
    }                                                                                    \
  } while (0)

// The flux launch of direction D: FP64 x and z faces in blocks of 16 faces at
// 4 t2 positions (flux4_kernel), the others in blocks of 64 faces of one t2
// position (flux_kernel).
template <int D, class R>
static void launch_flux(const Params& P, hipStream_t stream, const R* B, const double* qref, const Scalars* sc,
                        int use_residual_dt, double* F) {
  if constexpr (sizeof(R) == 8 && D != 1)
    hipLaunchKernelGGL((flux4_kernel<D>), dim3((unsigned)flux4_tiles(P, D)), dim3(FLUX_THREADS), 0, stream, B, P,
                       qref, sc, use_residual_dt, F);
  else if constexpr (sizeof(R) == 8)
    hipLaunchKernelGGL(flux4y_kernel, dim3((unsigned)flux4y_tiles(P)), dim3(FLUX_THREADS), 0, stream, B, P, qref, sc,
                       use_residual_dt, F);
  else
    hipLaunchKernelGGL((flux_kernel<D, R>), dim3((unsigned)flux_tiles<16>(P, D)), dim3(FLUX_THREADS), 0, stream, B,
                       P, qref, sc, use_residual_dt, F);
}

// Reconstruction and flux of the three directions of one stage on `stream`
// (faces of qin -> F[d]); hook(cls) / hook(-1) bracket each launch (the
// context's profiling events; a no-op elsewhere).
template <class R, class S, class Hook>
static hipError_t enqueue_fluxes(const Params& P, hipStream_t stream, const S* qin, R* B, double* const F[3],
                                 const Scalars* sc, const double* qref, int use_residual_dt, Hook&& hook) {
  auto recon_blocks = [&](int d) {
    return (unsigned)(d == 0 ? recon_tiles<0, R>(P) : (d == 1 ? recon_tiles<1, R>(P) : recon_tiles<2, R>(P)));
  };
  hipError_t e;
#define HGKS_DIRECTION(D)                                                                                    \
  if ((e = hook(PROF_RECON)) != hipSuccess) return e;                                                        \
  hipLaunchKernelGGL((recon_kernel<D, R, S>), dim3(recon_blocks(D)), dim3(RECON_THREADS), 0, stream, qin, P, \
                     qref, B);                                                                               \
  if ((e = hook(-1)) != hipSuccess) return e;                                                                \
  if ((e = hook(PROF_FLUX)) != hipSuccess) return e;                                                         \
  launch_flux<D, R>(P, stream, B, qref, sc, use_residual_dt, F[D]);                                          \
  if ((e = hook(-1)) != hipSuccess) return e;
  HGKS_DIRECTION(0)
  HGKS_DIRECTION(1)
  HGKS_DIRECTION(2)
#undef HGKS_DIRECTION
  return hipGetLastError();
}

template <class R, class S>
static hgks_status launch_fluxes(hgks_ctx ctx, const S* qin, int use_residual_dt) {
  auto hook = [ctx](int cls) { return cls >= 0 ? prof_begin(ctx, cls) : prof_end(ctx); };
  HIP_TRY(ctx, (enqueue_fluxes<R, S>(ctx->P, ctx->stream, qin, static_cast<R*>(ctx->B), ctx->F, ctx->sc,
                                     ctx->qref, use_residual_dt, hook)));
  return HGKS_OK;
}

static hgks_status launch_fluxes_any(hgks_ctx ctx, const double* qin, int use_residual_dt) {
  if (precision_mixed(ctx->cfg)) return launch_fluxes<float, double>(ctx, qin, use_residual_dt);
  return launch_fluxes<double, double>(ctx, qin, use_residual_dt);
}

// ---- the residual entry point that allocates nothing --------------------
// Its face buffers, metric arrays, scalars and reduction partials live in
// `scratch`, a static device array of HGKS_STATIC_SCRATCH_BYTES: each GPU the
// library runs on holds its own copy from module load to process exit.  In
// host code the array's name is a host-side stand-in, not a device address:
// host code uses only the address hipGetSymbolAddress returns, kept per device.
static __device__ __align__(256) unsigned char scratch[HGKS_STATIC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
thread_local char g_static_err[256] = "";

void static_error(const char* what, const char* detail) {
  std::snprintf(g_static_err, sizeof(g_static_err), "%s%s%s", what, detail[0] ? ": " : "", detail);
}

// The current device's copy of `scratch` (looked up once per device).
hipError_t scratch_on_current_device(char** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = static_cast<char*>(g_scratch_ptr[dev]);
  return hipSuccess;
}
}  // namespace

static unsigned cell_blocks(const Params& P) { return (unsigned)((cells(P) + CELL_THREADS - 1) / CELL_THREADS); }

// nsteps S2O4 steps on a state of type S (q, qs, acc: the state, Q*, the
// accumulator), R the reconstruction and flux type; the time step rule comes
// from the device scalars (dt_fixed).
template <class R, class S>
static hgks_status step_loop(hgks_ctx ctx, S* q, S* qs, S* acc, int32_t nsteps) {
  const Params& P = ctx->P;
  for (int s = 0; s < nsteps; ++s) {
    HIP_TRY(ctx, prof_begin(ctx, PROF_OTHER));
    hipLaunchKernelGGL(begin_step_kernel, dim3(1), dim3(64), 0, ctx->stream, ctx->sc, ctx->cfg.cfl);
    HIP_TRY(ctx, prof_end(ctx));
    hgks_status r = launch_fluxes<R, S>(ctx, q, 0);
    if (r != HGKS_OK) return r;
    HIP_TRY(ctx, prof_begin(ctx, PROF_UPDATE));
    hipLaunchKernelGGL((update_kernel<1, S>), dim3(cell_blocks(P)), dim3(CELL_THREADS), 0, ctx->stream, q, qs, acc,
                       ctx->F[0], ctx->F[1], ctx->F[2], P, ctx->sc, ctx->mpart);
    HIP_TRY(ctx, prof_end(ctx));
    r = launch_fluxes<R, S>(ctx, qs, 0);
    if (r != HGKS_OK) return r;
    HIP_TRY(ctx, prof_begin(ctx, PROF_UPDATE));
    hipLaunchKernelGGL((update_kernel<2, S>), dim3(cell_blocks(P)), dim3(CELL_THREADS), 0, ctx->stream, q, qs, acc,
                       ctx->F[0], ctx->F[1], ctx->F[2], P, ctx->sc, ctx->mpart);
    HIP_TRY(ctx, prof_end(ctx));
    if (P.flags & HGKS_FLAG_CONSTANT_MASS_FLUX) {
      double vol = 1.0;
      for (int a = 0; a < 3; ++a) vol *= ctx->cfg.hi[a] - ctx->cfg.lo[a];
      HIP_TRY(ctx, prof_begin(ctx, PROF_OTHER));
      hipLaunchKernelGGL(mass_flux_kernel, dim3(1), dim3(256), 0, ctx->stream, ctx->mpart, (int)cell_blocks(P),
                         1.0 / vol, ctx->mf, ctx->sc);
      HIP_TRY(ctx, prof_end(ctx));
    }
    HIP_TRY(ctx, hipGetLastError());
  }
  return HGKS_OK;
}


// ---- batched ensemble: host side ------------------------------------------

// Work-list prefix rows of a batch: per member, the reconstruction tiles of
// each direction, the flux tiles of each direction for tile widths 16 and 32,
// and the cell blocks.  Empty when a row's total does not fit an int.
static std::vector<int> batch_prefix(int n, const hgks_config* cfgs) {
  std::vector<int> pre((size_t)PRE_ROWS * (n + 1), 0);
  for (int i = 0; i < n; ++i) {
    Params P{};
    for (int a = 0; a < 3; ++a) { P.n[a] = cfgs[i].n[a]; P.bc[a] = cfgs[i].bc[a]; }
    long long items[PRE_ROWS];
    const bool f32 = cfgs[i].precision != HGKS_FP64;  // FP32 B: the wider reconstruction tiles
    items[PRE_RECON + 0] = f32 ? recon_tiles<0, float>(P) : recon_tiles<0, double>(P);
    items[PRE_RECON + 1] = f32 ? recon_tiles<1, float>(P) : recon_tiles<1, double>(P);
    items[PRE_RECON + 2] = f32 ? recon_tiles<2, float>(P) : recon_tiles<2, double>(P);
    for (int d = 0; d < 3; ++d) {
      // FP64: the staged 4-position tiles whatever the width
      const long long four = d == 1 ? flux4y_tiles(P) : flux4_tiles(P, d);
      items[flux_row<16>(d)] = f32 ? flux_tiles<16>(P, d) : four;
      items[flux_row<32>(d)] = f32 ? flux_tiles<32>(P, d) : four;
    }
    items[PRE_CELL] = (long long)((cells(P) + CELL_THREADS - 1) / CELL_THREADS);
    for (int r = 0; r < PRE_ROWS; ++r) {
      const long long v = (long long)pre[(size_t)r * (n + 1) + i] + items[r];
      if (v > INT32_MAX / 2) return {};
      pre[(size_t)r * (n + 1) + i + 1] = (int)v;
    }
  }
  return pre;
}

// Coarse member table of every row: entry k names the member holding item
// k << BATCH_COARSE_SHIFT; off[r] is where row r starts.
static std::vector<int> batch_coarse(int n, const std::vector<int>& pre, int off[PRE_ROWS]) {
  std::vector<int> c;
  for (int r = 0; r < PRE_ROWS; ++r) {
    off[r] = (int)c.size();
    const int* p = pre.data() + (size_t)r * (n + 1);
    int inst = 0;
    for (int t = 0; t < p[n]; t += 1 << BATCH_COARSE_SHIFT) {
      while (t >= p[inst + 1]) ++inst;
      c.push_back(inst);
    }
  }
  return c;
}

static size_t batch_table_bytes(int n, size_t coarse_entries) {
  return align256((size_t)n * sizeof(BatchEntry)) + align256((size_t)PRE_ROWS * (n + 1) * sizeof(int)) +
         align256(coarse_entries * sizeof(int));
}

// First item of member m in row r (m = n: the row's total).
static int batch_item(hgks_ctx b, int r, int m) { return b->pre[(size_t)r * (b->members.size() + 1) + m]; }

// Member groups for a budget of `mib` MiB of buffer B (0: one group): runs of
// consecutive members whose B fits the budget together, a member larger than
// the budget alone.  Reconstruction and flux of a direction run group by
// group, so a group's B can stay in the last-level cache between the two.
static void batch_set_groups(hgks_ctx b, int mib) {
  b->group_mib = mib;
  b->group_first.assign(1, 0);
  const int n = (int)b->members.size();
  const size_t budget = (size_t)mib << 20;
  size_t used = 0;
  for (int i = 0; i < n; ++i) {
    const size_t bytes = b->members[i]->L.nb_elems * (precision_mixed(b->cfg) ? sizeof(float) : sizeof(double));
    if (mib > 0 && i > b->group_first.back() && used + bytes > budget) {
      b->group_first.push_back(i);
      used = 0;
    }
    used += bytes;
  }
  b->group_first.push_back(n);
}

template <int DIR, class R, int TX, class ST>
static void enqueue_batch_direction(hgks_ctx b, int src_qs) {
  const BatchTable T = b->table;
  for (size_t g = 0; g + 1 < b->group_first.size(); ++g) {
    const int m0 = b->group_first[g], m1 = b->group_first[g + 1];
    const int r0 = batch_item(b, PRE_RECON + DIR, m0), r1 = batch_item(b, PRE_RECON + DIR, m1);
    hipLaunchKernelGGL((recon_batch_kernel<DIR, R, ST>), dim3(r1 - r0), dim3(RECON_THREADS), 0, b->stream, T, r0,
                       r1, src_qs);
    const int f0 = batch_item(b, flux_row<TX>(DIR), m0), f1 = batch_item(b, flux_row<TX>(DIR), m1);
    hipLaunchKernelGGL((flux_batch_kernel<DIR, R, TX>), dim3(f1 - f0), dim3(FLUX_THREADS), 0, b->stream, T, f0, f1);
  }
}
template <class R, int TX, class ST>
static void enqueue_batch_fluxes_tx(hgks_ctx b, int src_qs) {
  enqueue_batch_direction<0, R, TX, ST>(b, src_qs);
  enqueue_batch_direction<1, R, TX, ST>(b, src_qs);
  enqueue_batch_direction<2, R, TX, ST>(b, src_qs);
}
static void enqueue_batch_fluxes(hgks_ctx b, int src_qs) {
  if (precision_fp32(b->cfg)) {
    if (b->tx == 32) enqueue_batch_fluxes_tx<float, 32, float>(b, src_qs);
    else enqueue_batch_fluxes_tx<float, 16, float>(b, src_qs);
  } else if (precision_mixed(b->cfg)) {
    if (b->tx == 32) enqueue_batch_fluxes_tx<float, 32, double>(b, src_qs);
    else enqueue_batch_fluxes_tx<float, 16, double>(b, src_qs);
  } else {
    if (b->tx == 32) enqueue_batch_fluxes_tx<double, 32, double>(b, src_qs);
    else enqueue_batch_fluxes_tx<double, 16, double>(b, src_qs);
  }
}
// Whole-code FP32 members: the callers' FP64 states into the FP32 working
// copies (to_fp32) or back, as a single-instance hgks_step does around its
// steps.
static void batch_convert_states(hgks_ctx b, bool to_fp32) {
  for (hgks_ctx m : b->members) {
    const size_t n = 5 * cells(m->P);
    const unsigned g = (unsigned)((n + CELL_THREADS - 1) / CELL_THREADS);
    if (to_fp32)
      hipLaunchKernelGGL((convert_kernel<double, float>), dim3(g), dim3(CELL_THREADS), 0, b->stream, m->q, m->q32, n);
    else
      hipLaunchKernelGGL((convert_kernel<float, double>), dim3(g), dim3(CELL_THREADS), 0, b->stream, m->q32, m->q, n);
  }
}
// One full batched S2O4 step on the stream (also what the graph captures).
static void enqueue_batch_step(hgks_ctx b) {
  const BatchTable T = b->table;
  const int nc = batch_item(b, PRE_CELL, T.n);
  hipLaunchKernelGGL(begin_step_batch_kernel, dim3((T.n + 63) / 64), dim3(64), 0, b->stream, T);
  enqueue_batch_fluxes(b, 0);
  if (precision_fp32(b->cfg))
    hipLaunchKernelGGL((update_batch_kernel<1, float>), dim3(nc), dim3(CELL_THREADS), 0, b->stream, T, 0, nc);
  else
    hipLaunchKernelGGL((update_batch_kernel<1, double>), dim3(nc), dim3(CELL_THREADS), 0, b->stream, T, 0, nc);
  enqueue_batch_fluxes(b, 1);
  if (precision_fp32(b->cfg))
    hipLaunchKernelGGL((update_batch_kernel<2, float>), dim3(nc), dim3(CELL_THREADS), 0, b->stream, T, 0, nc);
  else
    hipLaunchKernelGGL((update_batch_kernel<2, double>), dim3(nc), dim3(CELL_THREADS), 0, b->stream, T, 0, nc);
  if (b->mass_flux_members)
    hipLaunchKernelGGL(mass_flux_batch_kernel, dim3(T.n), dim3(256), 0, b->stream, T);
}

// Milliseconds of `reps` runs of fn on the stream, timed with events.
template <class Fn>
static hgks_status time_on_stream(hgks_ctx b, Fn fn, int reps, float* ms) {
  hipEvent_t e0, e1;
  HIP_TRY(b, hipEventCreate(&e0));
  HIP_TRY(b, hipEventCreate(&e1));
  fn();  // warm
  HIP_TRY(b, hipEventRecord(e0, b->stream));
  for (int r = 0; r < reps; ++r) fn();
  HIP_TRY(b, hipEventRecord(e1, b->stream));
  HIP_TRY(b, hipEventSynchronize(e1));
  HIP_TRY(b, hipGetLastError());
  HIP_TRY(b, hipEventElapsedTime(ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return HGKS_OK;
}

static std::string tune_key(hgks_ctx b) {
  std::string k = "hgks-batch-v3 prec=" + std::to_string(b->cfg.precision) + " n=" + std::to_string(b->members.size());
  for (hgks_ctx m : b->members)
    k += " " + std::to_string(m->cfg.n[0]) + "x" + std::to_string(m->cfg.n[1]) + "x" + std::to_string(m->cfg.n[2]);
  return k;
}

// Launch-shape autotuner: the flux tile width (16 or 32 faces along x) and the
// member-group budget for buffer B (one group, or 256, 128, 64 MiB), timed on
// the ensemble's own state (reconstruction and flux write only workspace).
// Results are kept in the file named by HGKS_TUNE_CACHE when set.
static hgks_status batch_autotune(hgks_ctx b) {
  const char* path = std::getenv("HGKS_TUNE_CACHE");
  const std::string key = tune_key(b);
  if (path) {
    if (FILE* f = std::fopen(path, "r")) {
      char line[65536];
      while (std::fgets(line, sizeof(line), f)) {
        std::string l(line);
        const size_t tab = l.find('\t');
        if (tab == std::string::npos || l.substr(0, tab) != key) continue;
        int tx, mib;
        if (std::sscanf(l.c_str() + tab + 1, "%d %d", &tx, &mib) == 2 && (tx == 16 || tx == 32) && mib >= 0 &&
            mib <= (1 << 20)) {
          b->tx = tx;
          batch_set_groups(b, mib);
          b->tune_source = 2;
          std::fclose(f);
          return HGKS_OK;
        }
      }
      std::fclose(f);
    }
  }
  // the members' CFL time steps, so that the timed flux launches do the
  // work of a real step (the captured step sets them again every step)
  hipLaunchKernelGGL(batch_cfl_dt_kernel, dim3((b->table.n + 63) / 64), dim3(64), 0, b->stream, b->table);
  float best = 1e30f, ms = 0.0f;
  int best_tx = 16, best_mib = 0;
  for (int tx : {16, 32}) {
    for (int mib : {0, 256, 128, 64}) {
      b->tx = tx;
      batch_set_groups(b, mib);
      hgks_status st = time_on_stream(b, [&]() { enqueue_batch_fluxes(b, 0); }, 2, &ms);
      if (st != HGKS_OK) return st;
      if (ms < best) { best = ms; best_tx = tx; best_mib = mib; }
    }
  }
  b->tx = best_tx;
  batch_set_groups(b, best_mib);
  b->tune_source = 1;
  if (path) {
    if (FILE* f = std::fopen(path, "a")) {
      std::fprintf(f, "%s\t%d %d\n", key.c_str(), b->tx, b->group_mib);
      std::fclose(f);
    }
  }
  return HGKS_OK;
}

// Device half of hgks_init: workspace pointers, geometry upload, the first
// wave-speed reduction and the volume means some paths need.
static hgks_status init_device(hgks_ctx ctx) {
  const hgks_config* cfg = &ctx->cfg;
  const Layout& L = ctx->L;
  Params& P = ctx->P;
  ctx->qs = reinterpret_cast<double*>(ctx->ws + L.qs);
  ctx->acc = reinterpret_cast<double*>(ctx->ws + L.acc);
  ctx->B = ctx->ws + L.B;
  for (int d = 0; d < 3; ++d) ctx->F[d] = reinterpret_cast<double*>(ctx->ws + L.F[d]);
  ctx->sc = reinterpret_cast<Scalars*>(ctx->ws + L.scal);
  ctx->part = reinterpret_cast<double*>(ctx->ws + L.part);
  ctx->qref = reinterpret_cast<double*>(ctx->ws + L.qref);
  ctx->mf = reinterpret_cast<double*>(ctx->ws + L.mf);
  ctx->q32 = precision_fp32(*cfg) ? reinterpret_cast<float*>(ctx->ws + L.q32) : nullptr;
  ctx->mpart = reinterpret_cast<double*>(ctx->ws + L.mpart);

  // geometry: widths, d(index)/dx at faces, Gauss points and centres
  std::vector<double> host;
  std::vector<size_t> where;
  const double r3 = std::sqrt(3.0) / 6.0;
  for (int a = 0; a < 3; ++a) {
    const int n = cfg->n[a];
    const bool stretched = a == 1 && cfg->y_stretch > 0.0;
    const double hu = (cfg->hi[a] - cfg->lo[a]) / n;
    std::vector<double> h(n), df(n + 1), dg(2 * n), dc(n);
    for (int i = 0; i < n; ++i) {
      h[i] = stretched ? coord(*cfg, a, i + 1.0) - coord(*cfg, a, double(i)) : hu;
      dg[2 * i] = stretched ? 1.0 / dcoord(*cfg, a, i + 0.5 - r3) : 1.0 / hu;
      dg[2 * i + 1] = stretched ? 1.0 / dcoord(*cfg, a, i + 0.5 + r3) : 1.0 / hu;
      dc[i] = stretched ? 1.0 / dcoord(*cfg, a, i + 0.5) : 1.0 / hu;
    }
    for (int f = 0; f <= n; ++f) df[f] = stretched ? 1.0 / dcoord(*cfg, a, double(f)) : 1.0 / hu;
    const std::vector<double>* arr[4] = {&h, &df, &dg, &dc};
    for (int m = 0; m < 4; ++m) {
      double* dst = reinterpret_cast<double*>(ctx->ws + L.metric[a][m]);
      HIP_TRY(ctx, hipMemcpyAsync(dst, arr[m]->data(), arr[m]->size() * sizeof(double), hipMemcpyHostToDevice,
                                  ctx->stream));
      HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    }
    P.hcell[a] = reinterpret_cast<const double*>(ctx->ws + L.metric[a][0]);
    P.dface[a] = reinterpret_cast<const double*>(ctx->ws + L.metric[a][1]);
    P.dgp[a] = reinterpret_cast<const double*>(ctx->ws + L.metric[a][2]);
    P.dcen[a] = reinterpret_cast<const double*>(ctx->ws + L.metric[a][3]);
  }
  Scalars s0{};
  s0.t = ctx->t0;
  s0.force_x = cfg->body_force[0];
  double qref[5] = {0, 0, 0, 0, 0};
  HIP_TRY(ctx, hipMemcpyAsync(ctx->sc, &s0, sizeof(Scalars), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->qref, qref, sizeof(qref), hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  hipLaunchKernelGGL(wave_rate_kernel, dim3(cell_blocks(P)), dim3(CELL_THREADS), 0, ctx->stream, ctx->q, P, ctx->sc);
  if (precision_mixed(*cfg) || (cfg->flags & HGKS_FLAG_CONSTANT_MASS_FLUX)) {
    // volume means of the initial state: the mixed path's reference state,
    // the mass-flux controller's target and mean density
    const int nb = ctx->L.stat_blocks;
    double* fin = ctx->part + (size_t)nb * ST_COUNT;
    double vol = 1.0;
    for (int a = 0; a < 3; ++a) vol *= cfg->hi[a] - cfg->lo[a];
    hipLaunchKernelGGL(stats_partial_kernel, dim3(nb), dim3(CELL_THREADS), 0, ctx->stream, ctx->q, P, ctx->part);
    hipLaunchKernelGGL(stats_final_kernel, dim3(ST_COUNT), dim3(256), 0, ctx->stream, ctx->part, nb, fin);
    if (precision_mixed(*cfg))
      hipLaunchKernelGGL(mean_state_kernel, dim3(1), dim3(64), 0, ctx->stream, fin, 1.0 / vol, ctx->qref);
    if (cfg->flags & HGKS_FLAG_CONSTANT_MASS_FLUX)
      hipLaunchKernelGGL(mass_flux_init_kernel, dim3(1), dim3(64), 0, ctx->stream, fin, 1.0 / vol, ctx->mf, ctx->sc);
  }
  HIP_TRY(ctx, hipGetLastError());
  return HGKS_OK;
}

// Device half of hgks_batch_init: member contexts over slices of the
// workspace, the device work table, the tuned launch shapes and the captured
// step.  On failure the caller destroys b (and the members made so far).
static hgks_status batch_init_body(hgks_ctx b, int n, const hgks_config* cfgs, double* const* q_devs, void* ws_dev,
                                   void* hip_stream) {
  char* base = static_cast<char*>(ws_dev);
  size_t off = 0;
  std::vector<BatchEntry> host(n);
  for (int i = 0; i < n; ++i) {
    const size_t sz = align256(make_layout(cfgs[i]).total);
    hgks_ctx m = nullptr;
    hgks_status st = hgks_init(&cfgs[i], q_devs[i], base + off, sz, hip_stream, 0.0, &m);
    if (st != HGKS_OK) {
      b->err = "member " + std::to_string(i) + ": " + hgks_last_error(nullptr);
      return st;
    }
    b->members.push_back(m);
    off += sz;
    BatchEntry& e = host[i];
    e.P = m->P;
    e.q = m->q;
    e.qs = m->qs;
    e.acc = m->acc;
    e.B = m->B;
    for (int d = 0; d < 3; ++d) e.F[d] = m->F[d];
    e.sc = m->sc;
    e.qref = m->qref;
    e.cfl = cfgs[i].cfl;
    e.q32 = m->q32;
    e.mpart = m->mpart;
    e.mf = m->mf;
    double vol = 1.0;
    for (int a = 0; a < 3; ++a) vol *= cfgs[i].hi[a] - cfgs[i].lo[a];
    e.inv_vol = 1.0 / vol;
    if (cfgs[i].flags & HGKS_FLAG_CONSTANT_MASS_FLUX) b->mass_flux_members = true;
  }
  b->pre = batch_prefix(n, cfgs);
  const std::vector<int> coarse = batch_coarse(n, b->pre, b->table.coarse_off);
  BatchEntry* dE = reinterpret_cast<BatchEntry*>(base + off);
  off += align256((size_t)n * sizeof(BatchEntry));
  int* dpre = reinterpret_cast<int*>(base + off);
  off += align256(b->pre.size() * sizeof(int));
  int* dcoarse = reinterpret_cast<int*>(base + off);
  HIP_TRY(b, hipMemcpyAsync(dE, host.data(), (size_t)n * sizeof(BatchEntry), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(b, hipMemcpyAsync(dpre, b->pre.data(), b->pre.size() * sizeof(int), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(b, hipMemcpyAsync(dcoarse, coarse.data(), coarse.size() * sizeof(int), hipMemcpyHostToDevice, b->stream));
  HIP_TRY(b, hipStreamSynchronize(b->stream));
  b->table.E = dE;
  b->table.pre = dpre;
  b->table.coarse = dcoarse;
  b->table.n = n;
  // the autotuner's reconstructions read the FP32 members' working copies
  if (precision_fp32(b->cfg)) batch_convert_states(b, true);
  const hgks_status st = batch_autotune(b);
  if (st != HGKS_OK) return st;
  // capture one step
  HIP_TRY(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed));
  enqueue_batch_step(b);
  HIP_TRY(b, hipStreamEndCapture(b->stream, &b->graph));
  HIP_TRY(b, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  return HGKS_OK;
}

// FP64 FMA issue-rate probe: 8 independent chains of dependent FMAs per lane.
__global__ __launch_bounds__(256) void fma_probe_kernel(double* __restrict__ out, int iters) {
  double x[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) x[j] = 1.0 + 1e-3 * threadIdx.x + j;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = fma(x[j], 0.999999, 1e-7);
  }
  double sum = 0.0;
#pragma unroll
  for (int j = 0; j < 8; ++j) sum += x[j];
  out[(size_t)blockIdx.x * 256 + threadIdx.x] = sum;
}

extern "C" {

hgks_status hgks_workspace_size(const hgks_config* cfg, size_t* bytes) {
  if (!bytes) return HGKS_E_INVALID;
  hgks_status s = validate(cfg, nullptr);
  if (s != HGKS_OK) return s;
  *bytes = make_layout(*cfg).total;
  return HGKS_OK;
}

hgks_status hgks_init(const hgks_config* cfg, double* q_dev, void* ws_dev, size_t ws_bytes, void* hip_stream,
                      double t0, hgks_ctx* out) {
  if (!out) return HGKS_E_INVALID;
  *out = nullptr;
  hgks_status s = validate(cfg, nullptr);
  if (s != HGKS_OK) return s;
  if (!q_dev || !ws_dev) return HGKS_E_INVALID;
  if (((uintptr_t)ws_dev & 255u) != 0 || ((uintptr_t)q_dev & 7u) != 0) return HGKS_E_INVALID;
  Layout L = make_layout(*cfg);
  if (ws_bytes < L.total) return HGKS_E_INVALID;
  hgks_ctx ctx = new (std::nothrow) hgks_ctx_s();
  if (!ctx) return HGKS_E_NOMEM;
  ctx->cfg = *cfg;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  ctx->q = q_dev;
  ctx->ws = static_cast<char*>(ws_dev);
  ctx->ws_bytes = ws_bytes;
  ctx->L = L;
  ctx->latched = HGKS_OK;
  ctx->t0 = t0;
  ctx->P = make_params(*cfg);
  const hgks_status st = init_device(ctx);
  if (st != HGKS_OK) {
    // the context dies here: its error text goes to the thread's slot
    static_error("hgks_init", ctx->err.c_str());
    delete ctx;
    return st;
  }
  *out = ctx;
  return HGKS_OK;
}


hgks_status hgks_step(hgks_ctx ctx, int32_t nsteps, double dt_fixed) {
  if (!ctx || nsteps < 0 || !std::isfinite(dt_fixed) || !ctx->members.empty()) return HGKS_E_INVALID;
  if (ctx->latched != HGKS_OK) return ctx->latched;
  if (nsteps == 0) return HGKS_OK;
  // the time-step rule lives on the device, so one captured step serves any dt
  if (!ctx->dt_fixed_known || ctx->dt_fixed != dt_fixed) {
    hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(64), 0, ctx->stream, &ctx->sc->dt_fixed, dt_fixed);
    HIP_TRY(ctx, hipGetLastError());
    ctx->dt_fixed = dt_fixed;
    ctx->dt_fixed_known = true;
  }
  const bool fp32 = precision_fp32(ctx->cfg);
  const size_t n = 5 * cells(ctx->P);
  const unsigned g = (unsigned)((n + CELL_THREADS - 1) / CELL_THREADS);
  // FP32 path: the caller's FP64 state in (rounded on the first call, exact
  // afterwards since it then holds FP32 values), the steps on the FP32 working
  // copy, the result back to the caller's state.
  if (fp32)
    hipLaunchKernelGGL((convert_kernel<double, float>), dim3(g), dim3(CELL_THREADS), 0, ctx->stream, ctx->q, ctx->q32,
                       n);
  auto steps = [&](int32_t k) -> hgks_status {
    if (fp32)
      return step_loop<float, float>(ctx, ctx->q32, reinterpret_cast<float*>(ctx->qs),
                                     reinterpret_cast<float*>(ctx->acc), k);
    if (precision_mixed(ctx->cfg)) return step_loop<float, double>(ctx, ctx->q, ctx->qs, ctx->acc, k);
    return step_loop<double, double>(ctx, ctx->q, ctx->qs, ctx->acc, k);
  };
  hgks_status r = HGKS_OK;
  hipStreamCaptureStatus capturing = hipStreamCaptureStatusNone;
  if (ctx->stream) HIP_TRY(ctx, hipStreamIsCapturing(ctx->stream, &capturing));
  if (ctx->stream && !ctx->prof && capturing == hipStreamCaptureStatusNone) {
    // one S2O4 step captured once in a HIP graph and replayed: one launch per
    // step instead of 15 (a created stream only: the default stream cannot
    // be captured; profiling needs the events between plain launches; a
    // stream the caller is capturing gets plain launches, into its graph)
    if (!ctx->exec) {
      HIP_TRY(ctx, hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeRelaxed));
      r = steps(1);
      hipGraph_t graph = nullptr;
      const hipError_t e = hipStreamEndCapture(ctx->stream, &graph);
      if (r != HGKS_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return r;
      }
      HIP_TRY(ctx, e);
      ctx->graph = graph;
      HIP_TRY(ctx, hipGraphInstantiate(&ctx->exec, ctx->graph, nullptr, nullptr, 0));
    }
    for (int s = 0; s < nsteps; ++s) HIP_TRY(ctx, hipGraphLaunch(ctx->exec, ctx->stream));
  } else {
    r = steps(nsteps);
    if (r != HGKS_OK) return r;
  }
  if (fp32)
    hipLaunchKernelGGL((convert_kernel<float, double>), dim3(g), dim3(CELL_THREADS), 0, ctx->stream, ctx->q32, ctx->q,
                       n);
  HIP_TRY(ctx, hipGetLastError());
  return HGKS_OK;
}

hgks_status hgks_stats(hgks_ctx ctx, hgks_stats_t* out) {
  if (!ctx || !out || !ctx->members.empty()) return HGKS_E_INVALID;
  const Params& P = ctx->P;
  const int nb = ctx->L.stat_blocks;
  double* fin = ctx->part + (size_t)nb * ST_COUNT;
  hipLaunchKernelGGL(stats_partial_kernel, dim3(nb), dim3(CELL_THREADS), 0, ctx->stream, ctx->q, P, ctx->part);
  hipLaunchKernelGGL(stats_final_kernel, dim3(ST_COUNT), dim3(256), 0, ctx->stream, ctx->part, nb, fin);
  HIP_TRY(ctx, hipGetLastError());
  double h[ST_COUNT];
  Scalars sc;
  HIP_TRY(ctx, hipMemcpyAsync(h, fin, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipMemcpyAsync(&sc, ctx->sc, sizeof(sc), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  double vol = 1.0;
  for (int a = 0; a < 3; ++a) vol *= ctx->cfg.hi[a] - ctx->cfg.lo[a];
  const double rho0 = ctx->cfg.rho_ref, mu = ctx->cfg.mu_ref;
  std::memset(out, 0, sizeof(*out));
  out->t = sc.t;
  out->dt_last = sc.dt;
  out->steps = (int64_t)sc.steps;
  out->Ek = h[ST_EK] / (rho0 * vol);
  out->eps_sol = mu * h[ST_ENS] / (rho0 * vol);
  out->eps_dil = 4.0 / 3.0 * mu * h[ST_DIL] / (rho0 * vol);
  out->eps_com = out->eps_sol + out->eps_dil;
  for (int m = 0; m < 5; ++m) {
    out->total[m] = h[ST_TOT + m];
    out->max_abs[m] = h[ST_MAX + m];
  }
  out->min_p = h[ST_MINP];
  out->min_rho = h[ST_MINR];
  out->nonfinite = h[ST_BAD] != 0.0 ? 1 : 0;
  out->body_force_x = sc.force_x;
  if (out->nonfinite) ctx->latched = HGKS_E_NONFINITE;
  else if (!(out->min_p > 0.0) || !(out->min_rho > 0.0)) ctx->latched = HGKS_E_NEGATIVE_STATE;
  return HGKS_OK;
}

hgks_status hgks_dt(hgks_ctx ctx, double* dt_out) {
  if (!ctx || !dt_out || !ctx->members.empty()) return HGKS_E_INVALID;
  Scalars sc;
  HIP_TRY(ctx, hipMemcpyAsync(&sc, ctx->sc, sizeof(sc), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  const double smax = __builtin_bit_cast(double, sc.smax);
  *dt_out = ctx->cfg.cfl / smax;
  return HGKS_OK;
}

hgks_status hgks_residual(hgks_ctx ctx, const double* q_dev, double dt, double* L_dev, double* dL_dev) {
  if (!ctx || !q_dev || !L_dev || !dL_dev || !(dt > 0.0) || !ctx->members.empty()) return HGKS_E_INVALID;
  const Params& P = ctx->P;
  hipLaunchKernelGGL(set_scalar_kernel, dim3(1), dim3(64), 0, ctx->stream, &ctx->sc->dt_residual, dt);
  hgks_status r = launch_fluxes_any(ctx, q_dev, 1);
  if (r != HGKS_OK) return r;
  hipLaunchKernelGGL(residual_kernel, dim3(cell_blocks(P)), dim3(CELL_THREADS), 0, ctx->stream, q_dev, ctx->F[0],
                     ctx->F[1], ctx->F[2], P, ctx->sc, L_dev, dL_dev);
  HIP_TRY(ctx, hipGetLastError());
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return HGKS_OK;
}

hgks_status hgks_residual_static(const hgks_config* cfg, const double* q_dev, double dt, double* L_dev,
                                 double* dL_dev, void* hip_stream) {
  g_static_err[0] = '\0';
  const char* why = "";
  if (validate(cfg, &why) != HGKS_OK) {
    static_error("invalid configuration", why);
    return HGKS_E_INVALID;
  }
  if (!q_dev || !L_dev || !dL_dev || !(dt > 0.0) || !std::isfinite(dt) || ((uintptr_t)q_dev & 7u) != 0) {
    static_error("invalid argument", "null or misaligned pointer, or dt not positive and finite");
    return HGKS_E_INVALID;
  }
  const Layout L = make_layout(*cfg, true);
  if (L.total > (size_t)HGKS_STATIC_SCRATCH_BYTES) {
    char detail[160];
    std::snprintf(detail, sizeof(detail), "the grid needs %zu bytes of face buffers, more than the %zu of the static array",
                  L.total, (size_t)HGKS_STATIC_SCRATCH_BYTES);
    static_error("grid too large for hgks_residual_static", detail);
    return HGKS_E_UNSUPPORTED;
  }
  char* base = nullptr;
  hipError_t e = scratch_on_current_device(&base);
  if (e != hipSuccess) {
    static_error("hipGetSymbolAddress(scratch)", hipGetErrorString(e));
    return HGKS_E_DEVICE;
  }
  const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
  Params P = make_params(*cfg);
  for (int a = 0; a < 3; ++a) {
    double* h = reinterpret_cast<double*>(base + L.metric[a][0]);
    double* df = reinterpret_cast<double*>(base + L.metric[a][1]);
    double* dg = reinterpret_cast<double*>(base + L.metric[a][2]);
    double* dc = reinterpret_cast<double*>(base + L.metric[a][3]);
    const AxisMap m{cfg->lo[a], cfg->hi[a], cfg->y_stretch, cfg->n[a], a == 1 && cfg->y_stretch > 0.0};
    hipLaunchKernelGGL(geometry_kernel, dim3((cfg->n[a] + 256) / 256), dim3(256), 0, stream, m, h, df, dg, dc);
    P.hcell[a] = h;
    P.dface[a] = df;
    P.dgp[a] = dg;
    P.dcen[a] = dc;
  }
  Scalars* sc = reinterpret_cast<Scalars*>(base + L.scal);
  double* qref = reinterpret_cast<double*>(base + L.qref);
  double* F[3];
  for (int d = 0; d < 3; ++d) F[d] = reinterpret_cast<double*>(base + L.F[d]);
  hipLaunchKernelGGL(residual_scalars_kernel, dim3(1), dim3(64), 0, stream, sc, dt, cfg->body_force[0], qref);
  auto no_hook = [](int) { return hipSuccess; };
  if (precision_mixed(*cfg)) {
    // reference state of the FP32 reconstruction: the volume mean of q_dev
    double* part = reinterpret_cast<double*>(base + L.part);
    double* fin = part + (size_t)L.stat_blocks * ST_COUNT;
    double vol = 1.0;
    for (int a = 0; a < 3; ++a) vol *= cfg->hi[a] - cfg->lo[a];
    hipLaunchKernelGGL(stats_partial_kernel, dim3(L.stat_blocks), dim3(CELL_THREADS), 0, stream, q_dev, P, part);
    hipLaunchKernelGGL(stats_final_kernel, dim3(ST_COUNT), dim3(256), 0, stream, part, L.stat_blocks, fin);
    hipLaunchKernelGGL(mean_state_kernel, dim3(1), dim3(64), 0, stream, fin, 1.0 / vol, qref);
    e = enqueue_fluxes<float, double>(P, stream, q_dev, reinterpret_cast<float*>(base + L.B), F, sc, qref, 1, no_hook);
  } else {
    e = enqueue_fluxes<double, double>(P, stream, q_dev, reinterpret_cast<double*>(base + L.B), F, sc, qref, 1,
                                       no_hook);
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(residual_kernel, dim3(cell_blocks(P)), dim3(CELL_THREADS), 0, stream, q_dev, F[0], F[1], F[2],
                       P, sc, L_dev, dL_dev);
    e = hipGetLastError();
  }
  if (e != hipSuccess) {
    static_error("kernel launch", hipGetErrorString(e));
    return HGKS_E_DEVICE;
  }
  return HGKS_OK;
}

hgks_status hgks_profile(hgks_ctx ctx, int32_t enable) {
  if (!ctx) return HGKS_E_INVALID;
  ctx->prof = enable != 0;
  return HGKS_OK;
}

hgks_status hgks_profile_read(hgks_ctx ctx, double ms[HGKS_PROFILE_CLASSES], int64_t launches[HGKS_PROFILE_CLASSES]) {
  if (!ctx || !ms || !launches) return HGKS_E_INVALID;
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  for (int c = 0; c < HGKS_PROFILE_CLASSES; ++c) { ms[c] = 0.0; launches[c] = 0; }
  for (size_t i = 0; i + 1 < ctx->ev_used; i += 2) {
    float t = 0.0f;
    HIP_TRY(ctx, hipEventElapsedTime(&t, ctx->ev_pool[i], ctx->ev_pool[i + 1]));
    const int c = ctx->ev_class[i / 2];
    ms[c] += t;
    launches[c] += 1;
  }
  ctx->ev_used = 0;
  return HGKS_OK;
}

hgks_status hgks_fma_probe(double* out_dev, int32_t blocks, int32_t iters, void* hip_stream) {
  if (!out_dev || blocks <= 0 || iters <= 0) return HGKS_E_INVALID;
  hipLaunchKernelGGL(fma_probe_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)hip_stream, out_dev, iters);
  return hipGetLastError() == hipSuccess ? HGKS_OK : HGKS_E_DEVICE;
}

hgks_status hgks_destroy(hgks_ctx ctx) {
  if (!ctx) return HGKS_E_INVALID;
  for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
  if (ctx->exec) (void)hipGraphExecDestroy(ctx->exec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  for (hgks_ctx m : ctx->members) hgks_destroy(m);
  delete ctx;
  return HGKS_OK;
}

const char* hgks_status_string(hgks_status s) {
  int i = (int)s;
  if (i < 0 || i > 6) return "unknown status";
  return kStatus[i];
}

const char* hgks_last_error(hgks_ctx ctx) {
  if (ctx) return ctx->err.c_str();
  return g_static_err[0] ? g_static_err : "null context";
}

hgks_status hgks_batch_workspace_size(int32_t n, const hgks_config* cfgs, size_t* bytes) {
  if (n <= 0 || !cfgs || !bytes) return HGKS_E_INVALID;
  size_t total = 0;
  for (int i = 0; i < n; ++i) {
    if (validate(&cfgs[i], nullptr) != HGKS_OK) return HGKS_E_INVALID;
    if (cfgs[i].precision != cfgs[0].precision) return HGKS_E_INVALID;
    total += align256(make_layout(cfgs[i]).total);
  }
  const std::vector<int> pre = batch_prefix(n, cfgs);
  if (pre.empty()) return HGKS_E_INVALID;
  int off[PRE_ROWS];
  *bytes = total + batch_table_bytes(n, batch_coarse(n, pre, off).size());
  return HGKS_OK;
}

hgks_status hgks_batch_init(int32_t n, const hgks_config* cfgs, double* const* q_devs, void* ws_dev, size_t ws_bytes,
                            void* hip_stream, hgks_ctx* out) {
  if (!out) return HGKS_E_INVALID;
  *out = nullptr;
  size_t need = 0;
  const hgks_status sz = hgks_batch_workspace_size(n, cfgs, &need);
  if (sz != HGKS_OK) return sz;
  if (!q_devs || !ws_dev || ws_bytes < need || ((uintptr_t)ws_dev & 255u) != 0) return HGKS_E_INVALID;
  if (!hip_stream) return HGKS_E_INVALID;  // graph capture needs a created (non-default) stream
  for (int i = 0; i < n; ++i)
    if (!q_devs[i]) return HGKS_E_INVALID;
  hgks_ctx b = new (std::nothrow) hgks_ctx_s();
  if (!b) return HGKS_E_NOMEM;
  b->cfg = cfgs[0];
  b->stream = static_cast<hipStream_t>(hip_stream);
  b->ws = static_cast<char*>(ws_dev);
  b->ws_bytes = ws_bytes;
  b->latched = HGKS_OK;
  const hgks_status st = batch_init_body(b, n, cfgs, q_devs, ws_dev, hip_stream);
  if (st != HGKS_OK) {
    static_error("hgks_batch_init", b->err.c_str());
    hgks_destroy(b);
    return st;
  }
  *out = b;
  return HGKS_OK;
}

hgks_status hgks_batch_step(hgks_ctx ctx, int32_t nsteps) {
  if (!ctx || nsteps < 0 || ctx->members.empty() || !ctx->exec) return HGKS_E_INVALID;
  for (hgks_ctx m : ctx->members)
    if (m->latched != HGKS_OK) return m->latched;
  if (nsteps == 0) return HGKS_OK;
  const bool fp32 = precision_fp32(ctx->cfg);
  if (fp32) batch_convert_states(ctx, true);
  for (int s = 0; s < nsteps; ++s) HIP_TRY(ctx, hipGraphLaunch(ctx->exec, ctx->stream));
  if (fp32) batch_convert_states(ctx, false);
  HIP_TRY(ctx, hipGetLastError());
  return HGKS_OK;
}

hgks_status hgks_batch_stats(hgks_ctx ctx, int32_t i, hgks_stats_t* out) {
  if (!ctx || !out || i < 0 || i >= (int32_t)ctx->members.size()) return HGKS_E_INVALID;
  hgks_ctx m = ctx->members[i];
  const hgks_status st = hgks_stats(m, out);
  if (st != HGKS_OK) ctx->err = m->err;
  return st;
}

hgks_status hgks_batch_info(hgks_ctx ctx, int64_t info[8]) {
  if (!ctx || !info || ctx->members.empty()) return HGKS_E_INVALID;
  const int n = (int)ctx->members.size();
  const int fr = ctx->tx == 32 ? flux_row<32>(0) : flux_row<16>(0);
  info[0] = n;
  info[1] = ctx->tx;
  info[2] = ctx->group_mib;
  info[3] = (int64_t)ctx->group_first.size() - 1;
  info[4] = (int64_t)batch_item(ctx, fr, n) + batch_item(ctx, fr + 1, n) + batch_item(ctx, fr + 2, n);
  info[5] = ctx->tune_source;
  info[6] = (int64_t)batch_item(ctx, PRE_RECON, n) + batch_item(ctx, PRE_RECON + 1, n) + batch_item(ctx, PRE_RECON + 2, n);
  info[7] = batch_item(ctx, PRE_CELL, n);
  return HGKS_OK;
}

}  // extern "C"
