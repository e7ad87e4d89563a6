// Learned surrogate of the ReaxFF energy: atom-centred descriptors, an
// ensemble of per-element networks on BF16 matrix cores, forces, training,
// and the disagreement gate with the plain FP64 evaluation as fallback.
//
// Model (per atom, neighbours within r_c = 5 A; Behler-Parrinello radial
// functions and a power-spectrum angular part):
//   radial   G[16 b + k] = sum_{j of element b} R_k(r_ij)
//   angular  G[64 + 16 p + 8 (l - 1) + n]
//            = sum_{j of b, k of c} A_n(r_ij) A_n(r_ik) cos^l theta_jik
//   computed here in factorised form from per-element moments
//   M1_b,n = sum_j A_n(r_ij) u_ij and M2_b,n = sum_j A_n(r_ij) u_ij u_ij^T:
//   the l = 1 sum is M1_b . M1_c and the l = 2 sum is M2_b : M2_c.
//   Network of member m, centre element e: x = (G - shift) * scale,
//   Z1 = x W1 + b1, H1 = silu(Z1), Z2 = H1 W2 + b2, H2 = silu(Z2),
//   E_a = H2 . w3 + b3.  Matrix products on v_mfma_f32_16x16x32_bf16 with
//   BF16 operands and FP32 accumulation; everything else FP32.
//
// Layouts.  Atoms are processed in the cell-sorted order of a 5 A
// neighbour list (an internal library context).  Network rows are the
// atoms grouped by element, each group padded to a multiple of 64, so a
// 64-row tile belongs to one element network.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

using namespace rx;

namespace rx {
namespace sur {

constexpr int NR = 16, NA = 8, NPAIR = 10, ND = 224, HID = 128;
constexpr int NPAR = ND * HID + HID + HID * HID + HID + HID + 1;
constexpr int OFF_W1 = 0, OFF_B1 = ND * HID, OFF_W2 = OFF_B1 + HID, OFF_B2 = OFF_W2 + HID * HID,
              OFF_W3 = OFF_B2 + HID, OFF_B3 = OFF_W3 + HID;
constexpr int TILE = 64;
constexpr float RC = 5.0f;
constexpr float ETA_R = 0.5f / (0.3f * 0.3f);
constexpr float ETA_A = 0.5f / (0.5f * 0.5f);
constexpr float PIF = 3.14159265358979f;
constexpr int NM = 72;   // moment floats per (atom, element): M1 8x3, M2 8x6 (xx yy zz xy xz yz)

__device__ __forceinline__ float mu_r(int k) { return 0.5f + 0.3f * (float)k; }
__device__ __forceinline__ float mu_a(int n) { return 1.0f + 0.5f * (float)n; }
// unordered element pair (b <= c) -> index in (0,0) (0,1) (0,2) (0,3) (1,1) ... (3,3)
__device__ __forceinline__ int pidx(int b, int c) {
  if (b > c) { const int t = b; b = c; c = t; }
  return b * 4 - (b * (b - 1)) / 2 + (c - b);
}

__device__ __forceinline__ float sigm(float z) { return 1.0f / (1.0f + __expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigm(z); }
__device__ __forceinline__ float dsilu(float z) { const float s = sigm(z); return s * (1.0f + z * (1.0f - s)); }
__device__ __forceinline__ float d2silu(float z) {
  const float s = sigm(z);
  return s * (1.0f - s) * (2.0f + z * (1.0f - 2.0f * s));
}

// float -> bfloat16 bits, round to nearest, ties to even
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8 ld8(const uint16_t* p) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  return __builtin_bit_cast(bf16x8, v);
}
// eight values p[0], p[s], ..., p[7 s] (a fragment read across rows of an LDS tile)
__device__ __forceinline__ bf16x8 ld8s(const uint16_t* p, int s) {
  uint16_t t[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) t[i] = p[i * s];
  uint4 v;
  v.x = (uint32_t)t[0] | ((uint32_t)t[1] << 16);
  v.y = (uint32_t)t[2] | ((uint32_t)t[3] << 16);
  v.z = (uint32_t)t[4] | ((uint32_t)t[5] << 16);
  v.w = (uint32_t)t[6] | ((uint32_t)t[7] << 16);
  return __builtin_bit_cast(bf16x8, v);
}
__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// C[64 x N] = A[64 x K] * B for a 64-row tile: A row-major in LDS (leading
// dimension lda, K contiguous), B given transposed in global memory as
// Bt[N][K].  Wave w owns column tiles w, w + 4, ...; acc[rt][c] holds the
// 16 x 16 block (row tile rt, column tile w + 4 c).  Lane l holds rows
// 16 rt + 4 (l >> 4) + i, column 16 ct + (l & 15).  All of the wave's B
// fragments are loaded before the first product, so the weights cost one
// memory round trip per product rather than one per 32-wide K step.
template <int N, int K, int CT>
__device__ __forceinline__ void gemm_tile(const uint16_t* __restrict__ A, int lda,
                                          const uint16_t* __restrict__ Bt, f32x4 (&acc)[4][CT]) {
  static_assert(K % 32 == 0, "K in steps of 32");
  constexpr int KB = K / 32;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[rt][c] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kl = (lane >> 4) * 8, rl = lane & 15;
  bf16x8 bf[KB][CT];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb)
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const int ct = w + 4 * c;
      bf[kb][c] = ct * 16 < N ? ld8(Bt + (int64_t)(ct * 16 + rl) * K + kb * 32 + kl) : bf16x8{};
    }
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    bf16x8 a[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) a[rt] = ld8(A + (rt * 16 + rl) * lda + kb * 32 + kl);
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const int ct = w + 4 * c;
      if (ct * 16 < N) {
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) acc[rt][c] = mfma(a[rt], bf[kb][c], acc[rt][c]);
      }
    }
  }
}

// C[M x N] += sum over the 64 tile rows t of A[t][m] B[t][n] (both LDS, row-major
// in t), accumulated into global memory with atomic adds: a weight gradient.
template <int M, int N>
__device__ __forceinline__ void gemm_tn_atomic(const uint16_t* __restrict__ A, int lda,
                                               const uint16_t* __restrict__ B, int ldb,
                                               float* __restrict__ C) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int kl = (lane >> 4) * 8, rl = lane & 15;
  constexpr int MT = M / 16, NTL = N / 16;
  for (int tIdx = w; tIdx < MT * NTL; tIdx += 4) {
    const int mt = tIdx / NTL, nt = tIdx % NTL;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < TILE; kb += 32) {
      const bf16x8 a = ld8s(A + (kb + kl) * lda + mt * 16 + rl, lda);
      const bf16x8 b = ld8s(B + (kb + kl) * ldb + nt * 16 + rl, ldb);
      acc = mfma(a, b, acc);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = mt * 16 + 4 * (lane >> 4) + i, n = nt * 16 + rl;
      if (acc[i] != 0.f) atomicAdd(&C[m * N + n], acc[i]);
    }
  }
}

// ---------------------------------------------------------------------------
// network rows: atoms grouped by element, groups padded to 64
// ---------------------------------------------------------------------------
struct Rows {
  int32_t* flag;      // [n + 1] scratch for the per-element scans
  int32_t* pre;       // [4][n + 1] exclusive scans
  int32_t* base;      // [8]: padded group starts (4) and counts (4)
  int32_t* rowof;     // [n] sorted atom -> row
  int32_t* rowatom;   // [rows] row -> sorted atom or -1
  int32_t* tile_elem; // [tiles] element of each 64-row tile or -1
  int64_t cap_rows = 0, cap_n = 0;
};

__global__ void k_elem_flag(int64_t n, const int32_t* __restrict__ type_s, int e, int32_t* __restrict__ flag) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s < n) flag[s] = type_s[s] == e;
  if (s == n) flag[s] = 0;
}

// padded group starts from the four scan totals; clears the row map
__global__ void k_row_bases(int64_t n, const int32_t* __restrict__ pre, int32_t* __restrict__ base) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    int start = 0;
    for (int e = 0; e < 4; ++e) {
      const int cnt = pre[e * (n + 1) + n];
      base[e] = start;
      base[4 + e] = cnt;
      start += (cnt + TILE - 1) / TILE * TILE;
    }
  }
}

// clears the row map and labels every 64-row tile with its element (-1: unused)
__global__ void k_row_assign(int64_t rows, const int32_t* __restrict__ base, int32_t* __restrict__ rowatom,
                             int32_t* __restrict__ tile_elem) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s < rows) rowatom[s] = -1;
  if (s < rows / TILE) {
    int e = -1;
    const int r = (int)s * TILE;
    for (int k = 0; k < 4; ++k) {
      const int lo = base[k], hi = base[k] + (base[4 + k] + TILE - 1) / TILE * TILE;
      if (r >= lo && r < hi) e = k;
    }
    tile_elem[s] = e;
  }
}

__global__ void k_row_fill(int64_t n, const int32_t* __restrict__ type_s, const int32_t* __restrict__ pre,
                           const int32_t* __restrict__ base, int32_t* __restrict__ rowof,
                           int32_t* __restrict__ rowatom) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int e = type_s[s];
  const int r = base[e] + pre[e * (n + 1) + s];
  rowof[s] = r;
  rowatom[r] = (int)s;
}

// ---------------------------------------------------------------------------
// descriptors (JVP = false) and their directional derivative along a
// per-atom field v (JVP = true).  One thread per (atom, neighbour element
// b), 32 atoms per 128-thread block; moments meet in LDS for the angular
// contractions.  Outputs, in network rows: xq = bf16((G - shift) scale)
// (or bf16(u scale) for the JVP); optionally G in FP32, sorted order.
// ---------------------------------------------------------------------------
struct DescArgs {
  Grid g;
  int64_t n;
  const double4* xs;
  const int32_t* far_cnt;
  const int32_t* far_j;
  int32_t far_w;
  const int32_t* rowof;
  const float* shift;
  const float* scale;
  const float* v;        // JVP field [n][3], sorted order
  uint16_t* xq;          // [rows][ND]
  float* G;              // optional [n][ND]
  float* mom;            // optional [n][4][NM] moments (forward pass only)
  const int32_t* seg;    // [n][4] element segment starts of the rows, or null (unsorted rows)
};

template <bool JVP>
__global__ __launch_bounds__(128) void k_desc(DescArgs a) {
  __shared__ float sm[32][4][NM];
  __shared__ float sd[JVP ? 32 : 1][4][NM];
  const int al = threadIdx.x >> 2, b = threadIdx.x & 3;
  const int64_t i = (int64_t)blockIdx.x * 32 + al;
  float gr[NR], m[NM], dm[JVP ? NM : 1];
#pragma unroll
  for (int k = 0; k < NR; ++k) gr[k] = 0.f;
#pragma unroll
  for (int k = 0; k < NM; ++k) m[k] = 0.f;
  if (JVP) {
#pragma unroll
    for (int k = 0; k < NM; ++k) dm[k] = 0.f;
  }
  int row = -1;
  if (i < a.n) {
    row = a.rowof[i];
    const double4 xi = a.xs[i];
    float vix = 0.f, viy = 0.f, viz = 0.f;
    if (JVP) { vix = a.v[3 * i]; viy = a.v[3 * i + 1]; viz = a.v[3 * i + 2]; }
    const int cnt = a.far_cnt[i];
    const int32_t* __restrict__ rowp = a.far_j + i * (int64_t)a.far_w;
    int k0 = 0, k1 = cnt;
    if (a.seg) {
      k0 = a.seg[i * 4 + b];
      k1 = b < 3 ? a.seg[i * 4 + b + 1] : cnt;
    }
    for (int k = k0; k < k1; ++k) {
      const int j = rowp[k];
      const double4 xj = a.xs[j];
      if ((int)xj.w != b) continue;
      double dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
      if (a.g.periodic) {
        dx = min_image(dx, a.g.L[0], a.g.invL[0]);
        dy = min_image(dy, a.g.L[1], a.g.invL[1]);
        dz = min_image(dz, a.g.L[2], a.g.invL[2]);
      }
      const double r2d = dx * dx + dy * dy + dz * dz;
      if (!(r2d < (double)(RC * RC))) continue;
      const float r = (float)sqrt(r2d);
      const float ir = 1.0f / r;
      const float ux = (float)dx * ir, uy = (float)dy * ir, uz = (float)dz * ir;
      const float fc = 0.5f * (__cosf(PIF * r / RC) + 1.0f);
      const float dfc = -0.5f * (PIF / RC) * __sinf(PIF * r / RC);
      float s = 0.f, px = 0.f, py = 0.f, pz = 0.f;   // v_j - v_i along u, and its normal part / r
      if (JVP) {
        const float ex = a.v[3 * j] - vix, ey = a.v[3 * j + 1] - viy, ez = a.v[3 * j + 2] - viz;
        s = ex * ux + ey * uy + ez * uz;
        px = (ex - s * ux) * ir;
        py = (ey - s * uy) * ir;
        pz = (ez - s * uz) * ir;
      }
#pragma unroll
      for (int k = 0; k < NR; ++k) {
        const float t = r - mu_r(k);
        const float e = __expf(-ETA_R * t * t);
        if (JVP) gr[k] += (e * (-2.0f * ETA_R * t) * fc + e * dfc) * s;
        else gr[k] += e * fc;
      }
      const float uu[6] = {ux * ux, uy * uy, uz * uz, ux * uy, ux * uz, uy * uz};
#pragma unroll
      for (int nn = 0; nn < NA; ++nn) {
        const float t = r - mu_a(nn);
        const float e = __expf(-ETA_A * t * t);
        const float A = e * fc;
        m[nn * 3 + 0] += A * ux;
        m[nn * 3 + 1] += A * uy;
        m[nn * 3 + 2] += A * uz;
#pragma unroll
        for (int q = 0; q < 6; ++q) m[24 + nn * 6 + q] += A * uu[q];
        if (JVP) {
          const float dA = (e * (-2.0f * ETA_A * t) * fc + e * dfc) * s;
          // d(A u) = dA u + A p ;  d(A u u^T) = dA u u^T + A (p u^T + u p^T)
          dm[nn * 3 + 0] += dA * ux + A * px;
          dm[nn * 3 + 1] += dA * uy + A * py;
          dm[nn * 3 + 2] += dA * uz + A * pz;
          dm[24 + nn * 6 + 0] += dA * uu[0] + A * 2.0f * px * ux;
          dm[24 + nn * 6 + 1] += dA * uu[1] + A * 2.0f * py * uy;
          dm[24 + nn * 6 + 2] += dA * uu[2] + A * 2.0f * pz * uz;
          dm[24 + nn * 6 + 3] += dA * uu[3] + A * (px * uy + ux * py);
          dm[24 + nn * 6 + 4] += dA * uu[4] + A * (px * uz + ux * pz);
          dm[24 + nn * 6 + 5] += dA * uu[5] + A * (py * uz + uy * pz);
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NM; ++k) sm[al][b][k] = m[k];
  if (!JVP && a.mom && i < a.n) {
#pragma unroll
    for (int k = 0; k < NM; ++k) a.mom[(i * 4 + b) * NM + k] = m[k];
  }
  if (JVP) {
#pragma unroll
    for (int k = 0; k < NM; ++k) sd[al][b][k] = dm[k];
  }
  if (row >= 0) {
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      const int f = b * NR + k;
      const float val = JVP ? gr[k] * a.scale[f] : (gr[k] - a.shift[f]) * a.scale[f];
      a.xq[(int64_t)row * ND + f] = f2bf(val);
      if (a.G) a.G[i * ND + f] = gr[k];
    }
  }
  __syncthreads();
  if (row < 0) return;
  // 160 angular features of atom i, features b, b + 4, ... for this thread
  for (int f = b; f < NPAIR * 16; f += 4) {
    const int p = f >> 4, l = (f >> 3) & 1, nn = f & 7;
    // pair p -> (pb, pc)
    int pb = 0, pc = 0, cnt = 0;
    for (int x = 0; x < 4; ++x)
      for (int y = x; y < 4; ++y) {
        if (cnt == p) { pb = x; pc = y; }
        ++cnt;
      }
    const float* M1b = &sm[al][pb][nn * 3];
    const float* M1c = &sm[al][pc][nn * 3];
    const float* M2b = &sm[al][pb][24 + nn * 6];
    const float* M2c = &sm[al][pc][24 + nn * 6];
    float val;
    if (!JVP) {
      val = l == 0 ? M1b[0] * M1c[0] + M1b[1] * M1c[1] + M1b[2] * M1c[2]
                   : M2b[0] * M2c[0] + M2b[1] * M2c[1] + M2b[2] * M2c[2] +
                         2.0f * (M2b[3] * M2c[3] + M2b[4] * M2c[4] + M2b[5] * M2c[5]);
    } else {
      const float* D1b = &sd[al][pb][nn * 3];
      const float* D1c = &sd[al][pc][nn * 3];
      const float* D2b = &sd[al][pb][24 + nn * 6];
      const float* D2c = &sd[al][pc][24 + nn * 6];
      if (l == 0) {
        val = D1b[0] * M1c[0] + D1b[1] * M1c[1] + D1b[2] * M1c[2] + M1b[0] * D1c[0] + M1b[1] * D1c[1] +
              M1b[2] * D1c[2];
      } else {
        val = D2b[0] * M2c[0] + D2b[1] * M2c[1] + D2b[2] * M2c[2] +
              2.0f * (D2b[3] * M2c[3] + D2b[4] * M2c[4] + D2b[5] * M2c[5]) + M2b[0] * D2c[0] +
              M2b[1] * D2c[1] + M2b[2] * D2c[2] + 2.0f * (M2b[3] * D2c[3] + M2b[4] * D2c[4] + M2b[5] * D2c[5]);
      }
    }
    const int fi = 4 * NR + f;
    const float xv = JVP ? val * a.scale[fi] : (val - a.shift[fi]) * a.scale[fi];
    a.xq[(int64_t)row * ND + fi] = f2bf(xv);
    if (a.G) a.G[i * ND + fi] = val;
  }
}

// ---------------------------------------------------------------------------
// network forward and input-gradient backward on one 64-row tile, member
// blockIdx.y: per-row energies and dE_a/dG_a (already times scale)
// ---------------------------------------------------------------------------
struct NetArgs {
  const float* theta;          // [M][4][NPAR] FP32 master
  const uint16_t* W1;          // [M*4][ND][HID]  bf16 (= Bt of x W1^T products)
  const uint16_t* Wt1;         // [M*4][HID][ND]
  const uint16_t* W2;          // [M*4][HID][HID]
  const uint16_t* Wt2;         // [M*4][HID][HID]
  const float* scale;          // [ND]
  const int32_t* tile_elem;
  const int32_t* rowatom;
  const uint16_t* xq;          // [rows][ND]
  int64_t rows;
  float* Erow;                 // [M][rows]
  float* gG;                   // [M][rows][ND]
};

constexpr int LDX = ND + 8, LDH = HID + 8;   // padded LDS leading dimensions

__global__ __launch_bounds__(256) void k_net_infer(NetArgs a) {
  __shared__ __align__(16) uint16_t sx[TILE * LDX];
  __shared__ __align__(16) uint16_t sa[TILE * LDH];
  __shared__ __align__(16) uint16_t sb[TILE * LDH];
  __shared__ float se[TILE];
  const int tile = blockIdx.x, mem = blockIdx.y;
  const int e = a.tile_elem[tile];
  if (e < 0) return;
  const int net = mem * 4 + e;
  const float* th = a.theta + (int64_t)net * NPAR;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, rl = lane & 15, rq = lane >> 4;
  const int64_t r0 = (int64_t)tile * TILE;
  // x tile -> LDS (16-byte chunks)
  for (int c = threadIdx.x; c < TILE * (ND / 8); c += 256) {
    const int rr = c / (ND / 8), kk = (c % (ND / 8)) * 8;
    *reinterpret_cast<uint4*>(&sx[rr * LDX + kk]) =
        *reinterpret_cast<const uint4*>(&a.xq[(r0 + rr) * ND + kk]);
  }
  if (threadIdx.x < TILE) se[threadIdx.x] = 0.f;
  __syncthreads();
  // layer 1
  f32x4 acc[4][2];
  gemm_tile<HID, ND, 2>(sx, LDX, a.Wt1 + (int64_t)net * HID * ND, acc);
  float s1[4][2][4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int col = (w + 4 * c) * 16 + rl;
      const float bb = th[OFF_B1 + col];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rr = rt * 16 + 4 * rq + i;
        const float z = acc[rt][c][i] + bb;
        s1[rt][c][i] = dsilu(z);
        sa[rr * LDH + col] = f2bf(silu(z));
      }
    }
  __syncthreads();
  // layer 2, energy, and dE/dZ2
  gemm_tile<HID, HID, 2>(sa, LDH, a.Wt2 + (int64_t)net * HID * HID, acc);
#pragma unroll
  for (int rt = 0; rt < 4; ++rt) {
    float ep[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int col = (w + 4 * c) * 16 + rl;
      const float bb = th[OFF_B2 + col], w3 = th[OFF_W3 + col];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rr = rt * 16 + 4 * rq + i;
        const float z = acc[rt][c][i] + bb;
        ep[i] += silu(z) * w3;
        sb[rr * LDH + col] = f2bf(w3 * dsilu(z));
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float v = ep[i];
      for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (rl == 0) atomicAdd(&se[rt * 16 + 4 * rq + i], v);
    }
  }
  __syncthreads();
  // dE/dH1 = d2 W2^T, times silu'(Z1)
  gemm_tile<HID, HID, 2>(sb, LDH, a.W2 + (int64_t)net * HID * HID, acc);
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int col = (w + 4 * c) * 16 + rl;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rr = rt * 16 + 4 * rq + i;
        sa[rr * LDH + col] = f2bf(acc[rt][c][i] * s1[rt][c][i]);
      }
    }
  __syncthreads();
  // dE/dx = d1 W1^T  (N = 224: 14 column tiles over 4 waves)
  f32x4 acc2[4][4];
  gemm_tile<ND, HID, 4>(sa, LDH, a.W1 + (int64_t)net * ND * HID, acc2);
  float* __restrict__ gout = a.gG + ((int64_t)mem * a.rows + r0) * ND;
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int ct = w + 4 * c;
      if (ct * 16 >= ND) continue;
      const int col = ct * 16 + rl;
      const float sc = a.scale[col];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rr = rt * 16 + 4 * rq + i;
        gout[rr * ND + col] = acc2[rt][c][i] * sc;
      }
    }
  if (threadIdx.x < TILE) a.Erow[(int64_t)mem * a.rows + r0 + threadIdx.x] = se[threadIdx.x] + th[OFF_B3];
}

// ---------------------------------------------------------------------------
// forces of every member, without atomics.  Pass 1, one thread per (atom i,
// neighbour element b): the adjoints of atom i's features give dE_i/dd_ij
// for each neighbour j of element b, written to j's slot of i's neighbour
// row (w[m][i * far_w + k]).  Pass 2, one thread per atom: with the mirror
// slot of each pair, F_i = sum_k (w_ik - w_{j_k, i}) (d_ij = x_j - x_i, so
// dE/dx_i = -sum_k w_ik + sum_k w_{j_k, i}).
// ---------------------------------------------------------------------------
struct ForceArgs {
  Grid g;
  int64_t n, rows, slots;
  int32_t members;
  const double4* xs;
  const int32_t* far_cnt;
  const int32_t* far_j;
  int32_t far_w;
  const int32_t* rowof;
  const float* gG;   // [M][rows][ND]
  const float* mom;  // [n][4][NM] moments of the descriptor pass
  const int32_t* mir;  // [n * far_w] mirror slots
  float4* w;         // [M/4][slots][3]: for j = row_i[k], dE_i/dd_ij of the 4 members
                     // of a chunk packed in 12 floats (read by j)
  float* Fown;       // [M][n][3]: sum over i's own pairs
};

// Neighbour rows in increasing index order (rank sort in LDS, one wavefront
// per row of at most SORT_MAX entries), so that mirror slots can be found by
// binary search.  The order of a row is free: every kernel reading it indexes
// its per-pair data by slot.
constexpr int SORT_MAX = 256;
constexpr int KEY_SHIFT = 27;   // sort key (element << 27) | index; atoms < 2^27

__global__ __launch_bounds__(256) void k_far_sort(int64_t n, const int32_t* __restrict__ far_cnt,
                                                  int32_t* __restrict__ far_j, int32_t far_w,
                                                  const int32_t* __restrict__ type_s, int32_t* __restrict__ seg) {
  __shared__ int32_t buf[4][SORT_MAX];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + wv;
  if (i >= n) return;
  const int cnt = far_cnt[i];
  int32_t* __restrict__ row = far_j + i * (int64_t)far_w;
  int c0 = 0, c1 = 0, c2 = 0;
  for (int k = lane; k < cnt; k += 64) {
    const int j = row[k];
    const int t = type_s[j];
    buf[wv][k] = (t << KEY_SHIFT) | j;
    c0 += t < 1;
    c1 += t < 2;
    c2 += t < 3;
  }
  for (int off = 32; off > 0; off >>= 1) {
    c0 += __shfl_down(c0, off, 64);
    c1 += __shfl_down(c1, off, 64);
    c2 += __shfl_down(c2, off, 64);
  }
  if (lane == 0) {
    seg[i * 4 + 0] = 0;
    seg[i * 4 + 1] = c0;
    seg[i * 4 + 2] = c1;
    seg[i * 4 + 3] = c2;
  }
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  for (int k = lane; k < cnt; k += 64) {
    const int key = buf[wv][k];
    int rank = 0;
    for (int t = 0; t < cnt; ++t) rank += buf[wv][t] < key;
    row[rank] = key & ((1 << KEY_SHIFT) - 1);
  }
}

// mirror slot of every neighbour-row entry: mir[i * far_w + k] = slot of i in
// row j_k (sorted by element, then index), by binary search; -1 if absent
__global__ __launch_bounds__(256) void k_far_mirror(int64_t n, const int32_t* __restrict__ far_cnt,
                                                    const int32_t* __restrict__ far_j, int32_t far_w,
                                                    const int32_t* __restrict__ type_s,
                                                    const int32_t* __restrict__ seg, int32_t* __restrict__ mir) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const int cnt = far_cnt[i];
  const int ti = type_s[i];
  const int32_t* __restrict__ row = far_j + i * (int64_t)far_w;
  for (int k = lane; k < cnt; k += 64) {
    const int j = row[k];
    const int32_t* __restrict__ rj = far_j + (int64_t)j * far_w;
    const int cj = far_cnt[j];
    int lo = seg[(int64_t)j * 4 + ti];
    int hi = ti < 3 ? seg[(int64_t)j * 4 + ti + 1] : cj;
    const int end = hi;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (rj[mid] < (int)i) lo = mid + 1;
      else hi = mid;
    }
    mir[i * (int64_t)far_w + k] = (lo < end && rj[lo] == (int)i) ? lo : -1;
  }
}

// linear-search variant for rows longer than SORT_MAX (unsorted rows)
__global__ __launch_bounds__(256) void k_far_mirror_scan(int64_t n, const int32_t* __restrict__ far_cnt,
                                                         const int32_t* __restrict__ far_j, int32_t far_w,
                                                         int32_t* __restrict__ mir) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const int cnt = far_cnt[i];
  const int32_t* __restrict__ row = far_j + i * (int64_t)far_w;
  for (int k = 0; k < cnt; ++k) {
    const int j = row[k];
    const int cj = far_cnt[j];
    const int32_t* __restrict__ rj = far_j + (int64_t)j * far_w;
    int m = -1;
    for (int t0 = 0; t0 < cj && m < 0; t0 += 64) {
      const int t = t0 + lane;
      const unsigned long long hit = ballot(t < cj && rj[t] == (int)i);
      if (hit) m = t0 + __ffsll((long long)hit) - 1;
    }
    if (lane == 0) mir[i * (int64_t)far_w + k] = m;
  }
}

// Pair contributions, one wavefront per atom i, one neighbour slot per lane.
// The wavefront first builds, for a chunk of up to 4 members, the adjoints of
// atom i's features seen from each neighbour element b (in LDS):
//   radial  gR_b,k = dE_i/dG[16 b + k]
//   M1      g1_b,n = sum_c (2 if c = b else 1) dE_i/dA1_(bc),n  M1_c,n
//   M2      g2_b,n = sum_c (2 if c = b else 1) dE_i/dA2_(bc),n  M2_c,n
// (M from the descriptor pass); then each lane forms dE_i/dd_ij for its
// neighbour j from the radial and angular basis of r_ij.
constexpr int GAM = NR + NA * 3 + NA * 6;   // 88 adjoint floats per element
constexpr int MCH = 4;                      // members per chunk
static_assert(MCH == 4, "pair records pack exactly four members");

__global__ __launch_bounds__(256) void k_sur_pairw(ForceArgs a) {
  __shared__ float sg[4][MCH][4][GAM];
  __shared__ float smm[4][4][NM];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + wv;
  if (i >= a.n) return;                       // wave-uniform; no block barriers below
  for (int k = lane; k < 4 * NM; k += 64) smm[wv][k / NM][k % NM] = a.mom[i * 4 * NM + k];
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  const double4 xi = a.xs[i];
  const int cnt = a.far_cnt[i];
  const int32_t* __restrict__ rowp = a.far_j + i * (int64_t)a.far_w;
  const int row = a.rowof[i];
  for (int m0 = 0; m0 < a.members; m0 += MCH) {
    const int mc = a.members - m0 < MCH ? a.members - m0 : MCH;
    // adjoints of each member of the chunk: lane l takes member half l / 32
    // of a member pair, neighbour element b = (l / 8) mod 4 and angular
    // channel n = l mod 8, and forms all nine (M1, M2) components of that
    // (b, n) from dE/dG read straight from memory; the radial part is a copy.
    const int hb = (lane >> 3) & 3, hn = lane & 7;
#pragma unroll
    for (int mm = 0; mm < MCH; ++mm)
      if (mm < mc) {
        const float* __restrict__ g = a.gG + ((int64_t)(m0 + mm) * a.rows + row) * ND;
        sg[wv][mm][lane / NR][lane % NR] = g[lane];     // 4 NR = 64 radial values
      }
#pragma unroll
    for (int mp = 0; mp < MCH; mp += 2) {
      const int mm = mp + (lane >> 5);
      if (mm < mc) {
        const float* __restrict__ g = a.gG + ((int64_t)(m0 + mm) * a.rows + row) * ND;
        float g1[3] = {0.f, 0.f, 0.f}, g2[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const float w = c == hb ? 2.0f : 1.0f;
          const float a1 = w * g[4 * NR + pidx(hb, c) * 16 + hn];
          const float a2 = w * g[4 * NR + pidx(hb, c) * 16 + 8 + hn];
#pragma unroll
          for (int comp = 0; comp < 3; ++comp) g1[comp] += a1 * smm[wv][c][hn * 3 + comp];
#pragma unroll
          for (int comp = 0; comp < 6; ++comp) g2[comp] += a2 * smm[wv][c][24 + hn * 6 + comp];
        }
#pragma unroll
        for (int comp = 0; comp < 3; ++comp) sg[wv][mm][hb][NR + hn * 3 + comp] = g1[comp];
#pragma unroll
        for (int comp = 0; comp < 6; ++comp) sg[wv][mm][hb][NR + NA * 3 + hn * 6 + comp] = g2[comp];
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    float fo[MCH][3];
#pragma unroll
    for (int mm = 0; mm < MCH; ++mm) fo[mm][0] = fo[mm][1] = fo[mm][2] = 0.f;
    for (int k = lane; k < cnt; k += 64) {
      const int j = rowp[k];
      const double4 xj = a.xs[j];
      const int b = (int)xj.w;
      double dx = xj.x - xi.x, dy = xj.y - xi.y, dz = xj.z - xi.z;
      if (a.g.periodic) {
        dx = min_image(dx, a.g.L[0], a.g.invL[0]);
        dy = min_image(dy, a.g.L[1], a.g.invL[1]);
        dz = min_image(dz, a.g.L[2], a.g.invL[2]);
      }
      const double r2d = dx * dx + dy * dy + dz * dz;
      const bool in = r2d < (double)(RC * RC);
      const float r = in ? (float)sqrt(r2d) : RC, ir = 1.0f / r;
      const float ux = (float)dx * ir, uy = (float)dy * ir, uz = (float)dz * ir;
      const float fc = 0.5f * (__cosf(PIF * r / RC) + 1.0f);
      const float dfc = -0.5f * (PIF / RC) * __sinf(PIF * r / RC);
      float dR[NR], A[NA], dA[NA];
#pragma unroll
      for (int k2 = 0; k2 < NR; ++k2) {
        const float t = r - mu_r(k2);
        const float e = __expf(-ETA_R * t * t);
        dR[k2] = e * (-2.0f * ETA_R * t) * fc + e * dfc;
      }
#pragma unroll
      for (int nn = 0; nn < NA; ++nn) {
        const float t = r - mu_a(nn);
        const float e = __expf(-ETA_A * t * t);
        A[nn] = e * fc;
        dA[nn] = e * (-2.0f * ETA_A * t) * fc + e * dfc;
      }
      float ww[MCH][3];
#pragma unroll
      for (int mm = 0; mm < MCH; ++mm) {
        ww[mm][0] = ww[mm][1] = ww[mm][2] = 0.f;
        if (mm >= mc) continue;
        const float* __restrict__ G = sg[wv][mm][b];
        float sr = 0.f;
#pragma unroll
        for (int k2 = 0; k2 < NR; ++k2) sr += G[k2] * dR[k2];
        float wx = sr * ux, wy = sr * uy, wz = sr * uz;
#pragma unroll
        for (int nn = 0; nn < NA; ++nn) {
          const float* g1 = G + NR + nn * 3;
          const float* g2 = G + NR + NA * 3 + nn * 6;
          // M1: d/dd of A(r) (g1 . u) = dA (g1.u) u + (A / r)(g1 - (g1.u) u)
          const float gu = g1[0] * ux + g1[1] * uy + g1[2] * uz;
          // M2: symmetric Gamma (xx yy zz xy xz yz): u^T Gamma u and Gamma u
          const float Gx = g2[0] * ux + g2[3] * uy + g2[4] * uz;
          const float Gy = g2[3] * ux + g2[1] * uy + g2[5] * uz;
          const float Gz = g2[4] * ux + g2[5] * uy + g2[2] * uz;
          const float uGu = ux * Gx + uy * Gy + uz * Gz;
          const float cu = dA[nn] * (gu + uGu) - A[nn] * ir * (gu + 2.0f * uGu);
          wx += cu * ux + A[nn] * ir * (g1[0] + 2.0f * Gx);
          wy += cu * uy + A[nn] * ir * (g1[1] + 2.0f * Gy);
          wz += cu * uz + A[nn] * ir * (g1[2] + 2.0f * Gz);
        }
        if (!in) { wx = 0.f; wy = 0.f; wz = 0.f; }
        fo[mm][0] += wx;
        fo[mm][1] += wy;
        fo[mm][2] += wz;
        ww[mm][0] = wx;
        ww[mm][1] = wy;
        ww[mm][2] = wz;
      }
      // own side: F_i += w; the neighbour's side, all members of the chunk in
      // one 48-byte record, stays in i's own slot k (coalesced) and is pulled
      // by j through the mirror index
      float4* __restrict__ wp = a.w + ((int64_t)(m0 / MCH) * a.slots + i * (int64_t)a.far_w + k) * 3;
      wp[0] = make_float4(ww[0][0], ww[0][1], ww[0][2], ww[1][0]);
      wp[1] = make_float4(ww[1][1], ww[1][2], ww[2][0], ww[2][1]);
      wp[2] = make_float4(ww[2][2], ww[3][0], ww[3][1], ww[3][2]);
    }
    for (int mm = 0; mm < mc; ++mm) {
      float fx = fo[mm][0], fy = fo[mm][1], fz = fo[mm][2];
      for (int off = 32; off > 0; off >>= 1) {
        fx += __shfl_down(fx, off, 64);
        fy += __shfl_down(fy, off, 64);
        fz += __shfl_down(fz, off, 64);
      }
      if (lane == 0) {
        float* f = a.Fown + ((int64_t)(m0 + mm) * a.n + i) * 3;
        f[0] = fx;
        f[1] = fy;
        f[2] = fz;
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  }
}

// F[m][j] = Fown[m][j] - sum_k w[m][i, slot of j in row i] over the neighbours
// i = row_j[k] (the slot is mir[j, k]), sorted order; one wavefront per atom,
// one neighbour per lane, one 48-byte record per neighbour for each chunk of
// 4 members
__global__ __launch_bounds__(256) void k_sur_gather(int64_t n, int32_t members, int64_t slots,
                                                    const int32_t* __restrict__ far_cnt,
                                                    const int32_t* __restrict__ far_j, int32_t far_w,
                                                    const int32_t* __restrict__ mir,
                                                    const float4* __restrict__ w, const float* __restrict__ Fown,
                                                    float* __restrict__ F) {
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const int cnt = far_cnt[i];
  const int64_t base = i * (int64_t)far_w;
  for (int m0 = 0; m0 < members; m0 += 4) {
    const float4* __restrict__ wc = w + (int64_t)(m0 / 4) * slots * 3;
    float f[12];
#pragma unroll
    for (int q = 0; q < 12; ++q) f[q] = 0.f;
    for (int k = lane; k < cnt; k += 64) {
      const int mk = mir[base + k];
      if (mk < 0) continue;
      const float4* __restrict__ p = wc + ((int64_t)far_j[base + k] * far_w + mk) * 3;
      const float4 p0 = p[0], p1 = p[1], p2 = p[2];
      f[0] += p0.x; f[1] += p0.y; f[2] += p0.z; f[3] += p0.w;
      f[4] += p1.x; f[5] += p1.y; f[6] += p1.z; f[7] += p1.w;
      f[8] += p2.x; f[9] += p2.y; f[10] += p2.z; f[11] += p2.w;
    }
#pragma unroll
    for (int q = 0; q < 12; ++q)
      for (int off = 32; off > 0; off >>= 1) f[q] += __shfl_down(f[q], off, 64);
    if (lane == 0) {
      for (int mm = 0; mm < 4 && m0 + mm < members; ++mm) {
        const int64_t o = ((int64_t)(m0 + mm) * n + i) * 3;
        F[o] = Fown[o] - f[3 * mm];
        F[o + 1] = Fown[o + 1] - f[3 * mm + 1];
        F[o + 2] = Fown[o + 2] - f[3 * mm + 2];
      }
    }
  }
}

// descriptor rows from sorted to caller order
__global__ void k_unsort_rows(int64_t n, const int32_t* __restrict__ perm, const float* __restrict__ Gs,
                              float* __restrict__ G) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n * ND) return;
  const int64_t s = k / ND;
  G[(int64_t)perm[s] * ND + k % ND] = Gs[k];
}

// sum of valid per-row energies of every member (FP64); a small grid strides
// over the rows, so each member's total takes one atomic add per workgroup
__global__ void k_sur_energy(int64_t rows, int32_t members, const int32_t* __restrict__ rowatom,
                             const float* __restrict__ Erow, double* __restrict__ E) {
  for (int m = 0; m < members; ++m) {
    double v = 0.0;
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows;
         r += (int64_t)gridDim.x * blockDim.x)
      if (rowatom[r] >= 0) v += (double)Erow[(int64_t)m * rows + r];
    block_add<256>(v, E + m);
  }
}

// per-atom energies in caller order
__global__ void k_sur_eatom(int64_t n, int64_t rows, int32_t members, const int32_t* __restrict__ perm,
                            const int32_t* __restrict__ rowof, const float* __restrict__ Erow,
                            float* __restrict__ out) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  for (int m = 0; m < members; ++m) out[(int64_t)m * n + perm[s]] = Erow[(int64_t)m * rows + rowof[s]];
}

// members' forces to caller order, their mean (FP64), the spread
// sigma_i = sqrt(mean_m |F_i^m - Fbar_i|^2) and the gate mask sigma_i > thr
__global__ void k_sur_ensemble(int64_t n, int32_t members, const int32_t* __restrict__ perm,
                               const float* __restrict__ F, float* __restrict__ Fout,
                               double* __restrict__ Fbar, float* __restrict__ sigma, uint8_t* __restrict__ mask,
                               double thr, unsigned long long* __restrict__ nflag) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  unsigned long long c = 0;
  if (s < n) {
    const int o = perm[s];
    double mx = 0, my = 0, mz = 0;
    for (int m = 0; m < members; ++m) {
      const float* f = F + ((int64_t)m * n + s) * 3;
      mx += f[0]; my += f[1]; mz += f[2];
      if (Fout) {
        float* d = Fout + ((int64_t)m * n + o) * 3;
        d[0] = f[0]; d[1] = f[1]; d[2] = f[2];
      }
    }
    mx /= members; my /= members; mz /= members;
    double v = 0.0;
    for (int m = 0; m < members; ++m) {
      const float* f = F + ((int64_t)m * n + s) * 3;
      v += (f[0] - mx) * (f[0] - mx) + (f[1] - my) * (f[1] - my) + (f[2] - mz) * (f[2] - mz);
    }
    const double sg = sqrt(v / members);
    if (Fbar) { Fbar[3 * (int64_t)o] = mx; Fbar[3 * (int64_t)o + 1] = my; Fbar[3 * (int64_t)o + 2] = mz; }
    if (sigma) sigma[o] = (float)sg;
    const bool f = sg > thr;
    if (mask) mask[o] = f;
    c = f;
  }
  // one count per workgroup (256 threads)
  __shared__ int rc[4];
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
  if ((threadIdx.x & 63) == 0) rc[threadIdx.x >> 6] = (int)c;
  __syncthreads();
  if (threadIdx.x == 0 && nflag) {
    const int t = rc[0] + rc[1] + rc[2] + rc[3];
    if (t) atomicAdd(nflag, (unsigned long long)t);
  }
}

// gated forces: exact ReaxFF where the mask is set, the ensemble mean elsewhere
__global__ void k_sur_merge(int64_t n, const uint8_t* __restrict__ mask, const double* __restrict__ Fr,
                            double* __restrict__ F) {
  const int64_t o = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (o < n && mask[o]) {
    F[3 * o] = Fr[3 * o];
    F[3 * o + 1] = Fr[3 * o + 1];
    F[3 * o + 2] = Fr[3 * o + 2];
  }
}

// ---------------------------------------------------------------------------
// training
// ---------------------------------------------------------------------------
// force residual of one member, sorted order, and its sum of squares
__global__ void k_sur_residual(int64_t n, const int32_t* __restrict__ perm, const float* __restrict__ F,
                               const double* __restrict__ Fref, float* __restrict__ res, double* __restrict__ ss) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  double v = 0.0;
  if (s < n) {
    const int o = perm[s];
    for (int k = 0; k < 3; ++k) {
      const float d = (float)((double)F[3 * s + k] - Fref[3 * (int64_t)o + k]);
      res[3 * s + k] = d;
      v += (double)d * d;
    }
  }
  block_add<256>(v, ss);
}

struct TrainArgs {
  const float* theta;          // member's [4][NPAR]
  const uint16_t* W1;          // member's [4][ND][HID]
  const uint16_t* Wt1;
  const uint16_t* W2;
  const uint16_t* Wt2;
  const int32_t* tile_elem;
  const int32_t* rowatom;
  const uint16_t* xq;          // [rows][ND]
  const uint16_t* uq;          // [rows][ND]
  const double* Etot;          // member's total energy
  double eref, wE, natoms;
  float cF;
  float* grad;                 // member's [4][NPAR], accumulated with atomic adds
};

// Per 64-row tile: primal and tangent (along u) passes, then the reverse of
// (E, dE/du) with seeds (cE, cF) to the parameters.
__global__ __launch_bounds__(256) void k_net_train(TrainArgs a) {
  __shared__ __align__(16) uint16_t sx[TILE * LDX];
  __shared__ __align__(16) uint16_t su[TILE * LDX];
  __shared__ __align__(16) uint16_t sa[TILE * LDH];   // H1 -> later bZ1
  __shared__ __align__(16) uint16_t sc[TILE * LDH];   // dH1 -> later bdZ1
  __shared__ __align__(16) uint16_t sd[TILE * LDH];   // bZ2
  __shared__ __align__(16) uint16_t sg[TILE * LDH];   // bdZ2
  __shared__ float sw3[HID], sb2[HID], sb1[HID];
  const int tile = blockIdx.x;
  const int e = a.tile_elem[tile];
  if (e < 0) return;
  const float* th = a.theta + (int64_t)e * NPAR;
  float* gr = a.grad + (int64_t)e * NPAR;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, rl = lane & 15, rq = lane >> 4;
  const int64_t r0 = (int64_t)tile * TILE;
  const float cE = (float)(2.0 * a.wE * (a.Etot[0] - a.eref) / (a.natoms * a.natoms));
  const float cF = a.cF;
  for (int c = threadIdx.x; c < TILE * (ND / 8); c += 256) {
    const int rr = c / (ND / 8), kk = (c % (ND / 8)) * 8;
    *reinterpret_cast<uint4*>(&sx[rr * LDX + kk]) = *reinterpret_cast<const uint4*>(&a.xq[(r0 + rr) * ND + kk]);
    *reinterpret_cast<uint4*>(&su[rr * LDX + kk]) = *reinterpret_cast<const uint4*>(&a.uq[(r0 + rr) * ND + kk]);
  }
  if (threadIdx.x < HID) sw3[threadIdx.x] = sb2[threadIdx.x] = sb1[threadIdx.x] = 0.f;
  // valid rows of this tile (padding rows contribute nothing)
  bool valid[4][4];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) valid[rt][i] = a.rowatom[r0 + rt * 16 + 4 * rq + i] >= 0;
  __syncthreads();
  const int W1o = e * ND * HID, W2o = e * HID * HID;
  f32x4 acc[4][2], acd[4][2];
  // layer 1: primal and tangent
  gemm_tile<HID, ND, 2>(sx, LDX, a.Wt1 + W1o, acc);
  gemm_tile<HID, ND, 2>(su, LDX, a.Wt1 + W1o, acd);
  float s1[4][2][4], q1[4][2][4], t1[4][2][4];   // silu'(Z1), silu''(Z1), dZ1
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int col = (w + 4 * c) * 16 + rl;
      const float bb = th[OFF_B1 + col];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rr = rt * 16 + 4 * rq + i;
        const float z = acc[rt][c][i] + bb;
        s1[rt][c][i] = dsilu(z);
        q1[rt][c][i] = d2silu(z);
        t1[rt][c][i] = acd[rt][c][i];
        sa[rr * LDH + col] = f2bf(silu(z));
        sc[rr * LDH + col] = f2bf(s1[rt][c][i] * acd[rt][c][i]);
      }
    }
  __syncthreads();
  // layer 2: primal and tangent, output seeds
  gemm_tile<HID, HID, 2>(sa, LDH, a.Wt2 + W2o, acc);
  gemm_tile<HID, HID, 2>(sc, LDH, a.Wt2 + W2o, acd);
  float nvalid = 0.f;
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int i = 0; i < 4; ++i) nvalid += valid[rt][i] ? 1.f : 0.f;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int col = (w + 4 * c) * 16 + rl;
    const float bb = th[OFF_B2 + col], w3 = th[OFF_W3 + col];
    float gw3 = 0.f, gb2 = 0.f;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rr = rt * 16 + 4 * rq + i;
        const float z = acc[rt][c][i] + bb;
        const float s2 = dsilu(z), dz2 = acd[rt][c][i];
        float bz2 = cE * w3 * s2 + cF * w3 * d2silu(z) * dz2;
        float bdz2 = cF * w3 * s2;
        if (!valid[rt][i]) { bz2 = 0.f; bdz2 = 0.f; }
        else gw3 += cE * silu(z) + cF * s2 * dz2;
        gb2 += bz2;
        sd[rr * LDH + col] = f2bf(bz2);
        sg[rr * LDH + col] = f2bf(bdz2);
      }
    // columns are shared by the 4 row groups of the wave (lanes rl, rl+16, ...)
    gw3 += __shfl_xor(gw3, 16, 64);
    gw3 += __shfl_xor(gw3, 32, 64);
    gb2 += __shfl_xor(gb2, 16, 64);
    gb2 += __shfl_xor(gb2, 32, 64);
    if (rq == 0) {
      sw3[col] += gw3;
      sb2[col] += gb2;
    }
  }
  // b3: cE per valid row; a lane's rows depend only on its 16-lane group, so
  // the tile's count is the sum over the four groups of one wave
  {
    float nv = nvalid;
    nv += __shfl_xor(nv, 16, 64);
    nv += __shfl_xor(nv, 32, 64);
    if (threadIdx.x == 0) atomicAdd(&gr[OFF_B3], cE * nv);
  }
  __syncthreads();
  // W2 gradient: H1^T bZ2 + dH1^T bdZ2
  gemm_tn_atomic<HID, HID>(sa, LDH, sd, LDH, gr + OFF_W2);
  gemm_tn_atomic<HID, HID>(sc, LDH, sg, LDH, gr + OFF_W2);
  // back to layer 1: bH1 = bZ2 W2^T, bdH1 = bdZ2 W2^T
  gemm_tile<HID, HID, 2>(sd, LDH, a.W2 + W2o, acc);
  gemm_tile<HID, HID, 2>(sg, LDH, a.W2 + W2o, acd);
  __syncthreads();   // sa, sc are read by the W2 gradient above
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int col = (w + 4 * c) * 16 + rl;
    float gb1 = 0.f;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rr = rt * 16 + 4 * rq + i;
        const float bz1 = acc[rt][c][i] * s1[rt][c][i] + acd[rt][c][i] * q1[rt][c][i] * t1[rt][c][i];
        const float bdz1 = acd[rt][c][i] * s1[rt][c][i];
        gb1 += bz1;
        sa[rr * LDH + col] = f2bf(bz1);
        sc[rr * LDH + col] = f2bf(bdz1);
      }
    gb1 += __shfl_xor(gb1, 16, 64);
    gb1 += __shfl_xor(gb1, 32, 64);
    if (rq == 0) sb1[col] += gb1;
  }
  __syncthreads();
  // W1 gradient: x^T bZ1 + u^T bdZ1
  gemm_tn_atomic<ND, HID>(sx, LDX, sa, LDH, gr + OFF_W1);
  gemm_tn_atomic<ND, HID>(su, LDX, sc, LDH, gr + OFF_W1);
  if (threadIdx.x < HID) {
    atomicAdd(&gr[OFF_W3 + threadIdx.x], sw3[threadIdx.x]);
    atomicAdd(&gr[OFF_B2 + threadIdx.x], sb2[threadIdx.x]);
    atomicAdd(&gr[OFF_B1 + threadIdx.x], sb1[threadIdx.x]);
  }
}

// Adam over every parameter; bias corrections c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t)
__global__ void k_adam(int64_t np, float* __restrict__ theta, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= np) return;
  const float gk = g[k];
  const float mk = b1 * m[k] + (1.0f - b1) * gk;
  const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  theta[k] -= lr * (mk * c1) / (sqrtf(vk * c2) + eps);
}

// bf16 copies of W1, W1^T, W2, W2^T of every network
__global__ void k_wconvert(int32_t nnets, const float* __restrict__ theta, uint16_t* __restrict__ W1,
                           uint16_t* __restrict__ Wt1, uint16_t* __restrict__ W2, uint16_t* __restrict__ Wt2) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t per = (int64_t)ND * HID + (int64_t)HID * HID;
  if (k >= per * nnets) return;
  const int net = (int)(k / per);
  const int64_t o = k % per;
  const float* th = theta + (int64_t)net * NPAR;
  if (o < ND * HID) {
    const int d = (int)(o / HID), j = (int)(o % HID);
    const uint16_t b = f2bf(th[OFF_W1 + o]);
    W1[(int64_t)net * ND * HID + d * HID + j] = b;
    Wt1[(int64_t)net * ND * HID + j * ND + d] = b;
  } else {
    const int64_t o2 = o - ND * HID;
    const int j1 = (int)(o2 / HID), j2 = (int)(o2 % HID);
    const uint16_t b = f2bf(th[OFF_W2 + o2]);
    W2[(int64_t)net * HID * HID + j1 * HID + j2] = b;
    Wt2[(int64_t)net * HID * HID + j2 * HID + j1] = b;
  }
}

// loss of every member: wE ((E - Eref) / N)^2 + wF / (3N) sum |res|^2
__global__ void k_sur_loss(int32_t members, const double* __restrict__ E, const double* __restrict__ ss, double eref,
                           double wE, double wF, double natoms, double* __restrict__ loss) {
  const int m = threadIdx.x;
  if (m < members) {
    const double de = (E[m] - eref) / natoms;
    loss[m] = wE * de * de + wF / (3.0 * natoms) * ss[m];
  }
}

}  // namespace sur
}  // namespace rx

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
using namespace rx::sur;

namespace rx {
// Normalisation statistics of descriptor rows G (rows x ND, FP32): per
// feature the mean, then the mean square deviation from it (two passes, FP64
// sums), one thread per feature over a block of 256 rows.
__global__ __launch_bounds__(256) void k_col_stats(int64_t rows, const float* __restrict__ G,
                                                   const double* __restrict__ mean, double* __restrict__ acc) {
  const int c = threadIdx.x;
  if (c >= ND) return;
  const int64_t r0 = (int64_t)blockIdx.x * 256, r1 = r0 + 256 < rows ? r0 + 256 : rows;
  double v = 0.0;
  for (int64_t r = r0; r < r1; ++r) {
    const double x = (double)G[r * ND + c];
    if (mean) {
      const double d = x - mean[c];
      v += d * d;
    } else {
      v += x;
    }
  }
  if (v != 0.0) atomicAdd(&acc[c], v);
}

// sums -> mean (in place) or shift = mean, scale = 1 / max(std, floor)
__global__ void k_col_final(int64_t rows, double* __restrict__ sum, const double* __restrict__ sq,
                            double floor_, float* __restrict__ shift, float* __restrict__ scale) {
  const int c = threadIdx.x;
  if (c >= ND) return;
  if (!sq) {
    sum[c] /= (double)rows;
    return;
  }
  const double sd = sqrt(sq[c] / (double)rows);
  shift[c] = (float)sum[c];
  scale[c] = (float)(1.0 / (sd > floor_ ? sd : floor_));
}
}  // namespace rx

struct reaxff_surrogate {
  reaxff_ctx* nb = nullptr;      // internal context: 5 A neighbour list
  int device = 0;
  int32_t members = 0;
  int64_t nparams = 0;           // members * 4 * NPAR
  float* theta = nullptr;        // device FP32 master
  float* grad = nullptr;
  float* adam_m = nullptr;
  float* adam_v = nullptr;
  int64_t adam_t = 0;
  uint16_t *W1 = nullptr, *Wt1 = nullptr, *W2 = nullptr, *Wt2 = nullptr;
  float* shift = nullptr;        // [ND]
  float* scale = nullptr;
  // per-frame buffers
  Rows R{};
  uint16_t* xq = nullptr;        // [rows][ND]
  uint16_t* uq = nullptr;
  float* Erow = nullptr;         // [M][rows]
  float* gG = nullptr;           // [M][rows][ND]
  float* F = nullptr;            // [M][n][3]
  float4* w = nullptr;           // [M][n * far_w] per-pair force contributions received
  float* Fown = nullptr;         // [M][n][3]
  int32_t* mir = nullptr;        // [n * far_w] mirror slots of the neighbour rows
  float* mom = nullptr;          // [n][4][NM] descriptor moments
  int32_t* seg = nullptr;        // [n][4] element segment starts of the sorted rows
  bool sorted_rows = false;
  int64_t cap_slots = 0;
  float* res = nullptr;          // [n][3]
  float* G = nullptr;            // [n][ND] (descriptor output for callers)
  double* Etot = nullptr;        // [M]
  double* ss = nullptr;          // [M]
  unsigned long long* nflag = nullptr;
  unsigned long long* nflag_host = nullptr;
  double* Fbar = nullptr;        // [n][3] (gated path)
  double* Freax = nullptr;       // [n][3]
  double* Ereax = nullptr;       // [NTERMS]
  int64_t cap_n = 0, cap_rows = 0;
  int64_t n = 0, rows = 0;
  std::string err;
};

namespace {

int sfail(reaxff_surrogate* s, int code, const std::string& msg) {
  if (s) s->err = msg;
  return code;
}

#define SHIP(s, expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return sfail(s, REAXFF_ERR_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

template <class T>
int salloc(reaxff_surrogate* s, T*& p, int64_t count) {
  if (p) (void)hipFree(p);
  p = nullptr;
  hipError_t e = hipMalloc(&p, sizeof(T) * std::max<int64_t>(count, 1));
  if (e != hipSuccess) return sfail(s, REAXFF_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  return 0;
}

unsigned nb(int64_t n, int bs) { return (unsigned)std::max<int64_t>((n + bs - 1) / bs, 1); }

// lists, rows and buffers for n atoms
int prepare(reaxff_surrogate* s, int64_t n, const double* pos, const int32_t* type, const double* box,
            hipStream_t st) {
  int rc = reaxff_build_lists(s->nb, n, pos, type, box, st);
  if (rc) return sfail(s, rc, std::string("neighbour list: ") + reaxff_last_error(s->nb));
  const int64_t rows = (n + 4 * (TILE - 1) + TILE - 1) / TILE * TILE;
  if (n > s->cap_n || rows > s->cap_rows) {
    const int64_t cn = std::max<int64_t>(n + n / 8, 64), cr = (cn + 4 * TILE + TILE - 1) / TILE * TILE;
    const int M = s->members;
    if ((rc = salloc(s, s->R.flag, cn + 1)) || (rc = salloc(s, s->R.pre, 4 * (cn + 1))) ||
        (rc = salloc(s, s->R.base, 8)) || (rc = salloc(s, s->R.rowof, cn)) ||
        (rc = salloc(s, s->R.rowatom, cr)) || (rc = salloc(s, s->R.tile_elem, cr / TILE)) ||
        (rc = salloc(s, s->xq, cr * ND)) || (rc = salloc(s, s->uq, cr * ND)) ||
        (rc = salloc(s, s->Erow, (int64_t)M * cr)) || (rc = salloc(s, s->gG, (int64_t)M * cr * ND)) ||
        (rc = salloc(s, s->F, (int64_t)M * cn * 3)) || (rc = salloc(s, s->res, cn * 3)) ||
        (rc = salloc(s, s->Fbar, cn * 3)) || (rc = salloc(s, s->Freax, cn * 3)) ||
        (rc = salloc(s, s->mom, cn * 4 * NM)) || (rc = salloc(s, s->seg, cn * 4)) ||
        (rc = salloc(s, s->Fown, (int64_t)M * cn * 3)))
      return rc;
    s->cap_n = cn;
    s->cap_rows = cr;
  }
  s->n = n;
  s->rows = rows;
  if (n == 0) return 0;
  const rx::Lists& L = s->nb->L;
  const int64_t slots = n * (int64_t)L.far_w;
  if (slots > s->cap_slots) {
    const int64_t cs = slots + slots / 8;
    if ((rc = salloc(s, s->w, (int64_t)3 * ((s->members + 3) / 4) * cs)) || (rc = salloc(s, s->mir, cs))) return rc;
    s->cap_slots = cs;
  }
  s->sorted_rows = L.far_w <= SORT_MAX && n < (1 << KEY_SHIFT);
  if (s->sorted_rows) {
    hipLaunchKernelGGL(k_far_sort, dim3(nb(n, 4)), dim3(256), 0, st, n, L.far_cnt, L.far_j, L.far_w, L.type_s,
                       s->seg);
    s->nb->prof.begin(KID_SUR_MIRROR, st);
    hipLaunchKernelGGL(k_far_mirror, dim3(nb(n, 4)), dim3(256), 0, st, n, L.far_cnt, L.far_j, L.far_w, L.type_s,
                       s->seg, s->mir);
    s->nb->prof.end(st);
  } else {
    hipLaunchKernelGGL(k_far_mirror_scan, dim3(nb(n, 4)), dim3(256), 0, st, n, L.far_cnt, L.far_j, L.far_w,
                       s->mir);
  }
  // rows: stable partition of the sorted atoms by element, groups padded to 64
  for (int e = 0; e < 4; ++e) {
    hipLaunchKernelGGL(k_elem_flag, dim3(nb(n + 1, 256)), dim3(256), 0, st, n, L.type_s, e, s->R.flag);
    if ((rc = rx::scan_i32(s->R.flag, s->R.pre + e * (n + 1), n + 1, s->nb->sc, st)))
      return sfail(s, REAXFF_ERR_HIP, "row scan failed");
  }
  hipLaunchKernelGGL(k_row_bases, dim3(1), dim3(64), 0, st, n, s->R.pre, s->R.base);
  hipLaunchKernelGGL(k_row_assign, dim3(nb(rows, 256)), dim3(256), 0, st, rows, s->R.base, s->R.rowatom,
                     s->R.tile_elem);
  hipLaunchKernelGGL(k_row_fill, dim3(nb(n, 256)), dim3(256), 0, st, n, L.type_s, s->R.pre, s->R.base, s->R.rowof,
                     s->R.rowatom);
  // padding rows of the network inputs are zero
  SHIP(s, hipMemsetAsync(s->xq, 0, sizeof(uint16_t) * rows * ND, st));
  SHIP(s, hipMemsetAsync(s->uq, 0, sizeof(uint16_t) * rows * ND, st));
  return hipGetLastError() == hipSuccess ? 0 : sfail(s, REAXFF_ERR_HIP, "row kernels");
}

DescArgs desc_args(reaxff_surrogate* s, const float* v, uint16_t* out, float* G) {
  const rx::Lists& L = s->nb->L;
  DescArgs a{};
  a.g = s->nb->grid;
  a.n = s->n;
  a.xs = L.xs;
  a.far_cnt = L.far_cnt;
  a.far_j = L.far_j;
  a.far_w = L.far_w;
  a.rowof = s->R.rowof;
  a.shift = s->shift;
  a.scale = s->scale;
  a.v = v;
  a.xq = out;
  a.G = G;
  a.seg = s->sorted_rows ? s->seg : nullptr;
  return a;
}

// descriptors, networks, energies and member forces (sorted order) of the prepared frame
int evaluate_frame(reaxff_surrogate* s, hipStream_t st) {
  const int64_t n = s->n, rows = s->rows;
  const int M = s->members;
  SHIP(s, hipMemsetAsync(s->Etot, 0, sizeof(double) * M, st));
  if (n == 0) return 0;
  {
    DescArgs da = desc_args(s, nullptr, s->xq, nullptr);
    da.mom = s->mom;
    s->nb->prof.begin(KID_SUR_DESC, st);
    hipLaunchKernelGGL(k_desc<false>, dim3(nb(n, 32)), dim3(128), 0, st, da);
    s->nb->prof.end(st);
  }
  NetArgs na{};
  na.theta = s->theta;
  na.W1 = s->W1;
  na.Wt1 = s->Wt1;
  na.W2 = s->W2;
  na.Wt2 = s->Wt2;
  na.scale = s->scale;
  na.tile_elem = s->R.tile_elem;
  na.rowatom = s->R.rowatom;
  na.xq = s->xq;
  na.rows = rows;
  na.Erow = s->Erow;
  na.gG = s->gG;
  s->nb->prof.begin(KID_SUR_NET, st);
  hipLaunchKernelGGL(k_net_infer, dim3((unsigned)(rows / TILE), M), dim3(256), 0, st, na);
  s->nb->prof.end(st);
  hipLaunchKernelGGL(k_sur_energy, dim3(std::min<int64_t>(std::max<int64_t>(nb(rows, 256), 1), 128)), dim3(256), 0,
                     st, rows, M, s->R.rowatom, s->Erow, s->Etot);
  const rx::Lists& L = s->nb->L;
  ForceArgs fa{};
  fa.g = s->nb->grid;
  fa.n = n;
  fa.rows = rows;
  fa.slots = s->cap_slots;
  fa.members = M;
  fa.xs = L.xs;
  fa.far_cnt = L.far_cnt;
  fa.far_j = L.far_j;
  fa.far_w = L.far_w;
  fa.rowof = s->R.rowof;
  fa.gG = s->gG;
  fa.mom = s->mom;
  fa.mir = s->mir;
  fa.w = s->w;
  fa.Fown = s->Fown;
  s->nb->prof.begin(KID_SUR_PAIRW, st);
  hipLaunchKernelGGL(k_sur_pairw, dim3(nb(n, 4)), dim3(256), 0, st, fa);
  s->nb->prof.end(st);
  s->nb->prof.begin(KID_SUR_GATHER, st);
  hipLaunchKernelGGL(k_sur_gather, dim3(nb(n, 4)), dim3(256), 0, st, n, M, s->cap_slots, L.far_cnt, L.far_j,
                     L.far_w, s->mir, s->w, s->Fown, s->F);
  s->nb->prof.end(st);
  return hipGetLastError() == hipSuccess ? 0 : sfail(s, REAXFF_ERR_HIP, "surrogate kernels");
}

int convert_weights(reaxff_surrogate* s, hipStream_t st) {
  const int64_t per = (int64_t)ND * HID + (int64_t)HID * HID;
  const int nets = 4 * s->members;
  hipLaunchKernelGGL(k_wconvert, dim3(nb(per * nets, 256)), dim3(256), 0, st, nets, s->theta, s->W1, s->Wt1, s->W2,
                     s->Wt2);
  return hipGetLastError() == hipSuccess ? 0 : sfail(s, REAXFF_ERR_HIP, "weight conversion");
}

bool dev_ok(const void* p) { return p != nullptr; }

}  // namespace

extern "C" {

int64_t reaxff_surrogate_param_count(void) { return NPAR; }

int reaxff_surrogate_create(reaxff_ctx* ctx, int32_t members, reaxff_surrogate** out) {
  if (!ctx || !out || members < 1 || members > 16) {
    if (ctx) ctx->err = "reaxff_surrogate_create: bad arguments (members 1..16)";
    return REAXFF_ERR_ARG;
  }
  *out = nullptr;
  reaxff_surrogate* s = new reaxff_surrogate();
  s->device = ctx->device;
  s->members = members;
  s->nparams = (int64_t)members * 4 * NPAR;
  reaxff_cutoffs c = ctx->cut;
  // only the 5 A neighbour rows of this context are used: bond and H-bond
  // lists are kept empty (sub-bond-length cutoffs)
  c.r_nonb = 5.0;
  c.r_bond = 0.1;
  c.r_hb = 0.1;
  int rc = reaxff_create(&ctx->hp, &c, ctx->device, &s->nb);
  auto bail = [&](int code) {
    if (ctx) ctx->err = s->err.empty() ? (s->nb ? reaxff_last_error(s->nb) : "reaxff_surrogate_create") : s->err;
    reaxff_surrogate_destroy(s);
    return code;
  };
  if (rc) return bail(rc);
  // the descriptor kernels address neighbours by sorted index
  s->nb->L.far_slots = 0;
  const int64_t wsz = (int64_t)members * 4 * ND * HID, w2sz = (int64_t)members * 4 * HID * HID;
  if ((rc = salloc(s, s->theta, s->nparams)) || (rc = salloc(s, s->grad, s->nparams)) ||
      (rc = salloc(s, s->adam_m, s->nparams)) || (rc = salloc(s, s->adam_v, s->nparams)) ||
      (rc = salloc(s, s->W1, wsz)) || (rc = salloc(s, s->Wt1, wsz)) || (rc = salloc(s, s->W2, w2sz)) ||
      (rc = salloc(s, s->Wt2, w2sz)) || (rc = salloc(s, s->shift, ND)) || (rc = salloc(s, s->scale, ND)) ||
      (rc = salloc(s, s->Etot, members)) || (rc = salloc(s, s->ss, members)) || (rc = salloc(s, s->nflag, 1)) ||
      (rc = salloc(s, s->Ereax, NTERMS)))
    return bail(rc);
  if (hipHostMalloc(&s->nflag_host, sizeof(unsigned long long)) != hipSuccess) return bail(REAXFF_ERR_HIP);
  (void)hipMemset(s->theta, 0, sizeof(float) * s->nparams);
  (void)hipMemset(s->adam_m, 0, sizeof(float) * s->nparams);
  (void)hipMemset(s->adam_v, 0, sizeof(float) * s->nparams);
  (void)hipMemset(s->shift, 0, sizeof(float) * ND);
  std::vector<float> one(ND, 1.0f);
  (void)hipMemcpy(s->scale, one.data(), sizeof(float) * ND, hipMemcpyHostToDevice);
  if ((rc = convert_weights(s, nullptr))) return bail(rc);
  if (hipDeviceSynchronize() != hipSuccess) return bail(REAXFF_ERR_HIP);
  *out = s;
  return REAXFF_OK;
}

void reaxff_surrogate_destroy(reaxff_surrogate* s) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  (void)hipDeviceSynchronize();
  for (void* p : {(void*)s->theta, (void*)s->grad, (void*)s->adam_m, (void*)s->adam_v, (void*)s->W1, (void*)s->Wt1,
                  (void*)s->W2, (void*)s->Wt2, (void*)s->shift, (void*)s->scale, (void*)s->R.flag,
                  (void*)s->R.pre, (void*)s->R.base, (void*)s->R.rowof, (void*)s->R.rowatom,
                  (void*)s->R.tile_elem, (void*)s->xq, (void*)s->uq, (void*)s->Erow, (void*)s->gG, (void*)s->F,
                  (void*)s->res, (void*)s->G, (void*)s->w, (void*)s->mir, (void*)s->mom, (void*)s->seg, (void*)s->Fown, (void*)s->Etot, (void*)s->ss, (void*)s->nflag, (void*)s->Fbar,
                  (void*)s->Freax, (void*)s->Ereax})
    if (p) (void)hipFree(p);
  if (s->nflag_host) (void)hipHostFree(s->nflag_host);
  if (s->nb) reaxff_destroy(s->nb);
  delete s;
}

const char* reaxff_surrogate_last_error(const reaxff_surrogate* s) { return s ? s->err.c_str() : "null surrogate"; }

int reaxff_surrogate_set_params(reaxff_surrogate* s, const float* theta, const float* shift, const float* scale) {
  if (!s) return REAXFF_ERR_ARG;
  SHIP(s, hipSetDevice(s->device));
  if (theta) SHIP(s, hipMemcpy(s->theta, theta, sizeof(float) * s->nparams, hipMemcpyHostToDevice));
  if (shift) SHIP(s, hipMemcpy(s->shift, shift, sizeof(float) * ND, hipMemcpyHostToDevice));
  if (scale) SHIP(s, hipMemcpy(s->scale, scale, sizeof(float) * ND, hipMemcpyHostToDevice));
  if (theta) {
    (void)hipMemset(s->adam_m, 0, sizeof(float) * s->nparams);
    (void)hipMemset(s->adam_v, 0, sizeof(float) * s->nparams);
    s->adam_t = 0;
    int rc = convert_weights(s, nullptr);
    if (rc) return rc;
  }
  SHIP(s, hipDeviceSynchronize());
  return REAXFF_OK;
}

int reaxff_surrogate_get_params(reaxff_surrogate* s, float* theta, float* shift, float* scale) {
  if (!s) return REAXFF_ERR_ARG;
  SHIP(s, hipSetDevice(s->device));
  SHIP(s, hipDeviceSynchronize());
  if (theta) SHIP(s, hipMemcpy(theta, s->theta, sizeof(float) * s->nparams, hipMemcpyDeviceToHost));
  if (shift) SHIP(s, hipMemcpy(shift, s->shift, sizeof(float) * ND, hipMemcpyDeviceToHost));
  if (scale) SHIP(s, hipMemcpy(scale, s->scale, sizeof(float) * ND, hipMemcpyDeviceToHost));
  return REAXFF_OK;
}

int reaxff_surrogate_descriptors(reaxff_surrogate* s, int64_t n, const double* pos, const int32_t* type,
                                 const double* box, float* G, hipStream_t stream) {
  if (!s || n < 0 || (n > 0 && (!pos || !type || !G))) return sfail(s, REAXFF_ERR_ARG, "descriptors: bad argument");
  SHIP(s, hipSetDevice(s->device));
  int rc = prepare(s, n, pos, type, box, stream);
  if (rc || n == 0) return rc;
  if ((rc = salloc(s, s->G, n * ND))) return rc;
  hipLaunchKernelGGL(k_desc<false>, dim3(nb(n, 32)), dim3(128), 0, stream, desc_args(s, nullptr, s->xq, s->G));
  hipLaunchKernelGGL(k_unsort_rows, dim3(nb(n * ND, 256)), dim3(256), 0, stream, n, s->nb->L.perm, s->G, G);
  SHIP(s, hipGetLastError());
  return REAXFF_OK;
}

int reaxff_surrogate_evaluate(reaxff_surrogate* s, int64_t n, const double* pos, const int32_t* type,
                              const double* box, double* energies, float* eatom, float* forces, double* fmean,
                              float* sigma, hipStream_t stream) {
  if (!s || n < 0 || (n > 0 && (!pos || !type)) || !energies)
    return sfail(s, REAXFF_ERR_ARG, "evaluate: bad argument");
  SHIP(s, hipSetDevice(s->device));
  int rc = prepare(s, n, pos, type, box, stream);
  if (rc) return rc;
  if ((rc = evaluate_frame(s, stream))) return rc;
  const int M = s->members;
  if (n > 0) {
    if (eatom)
      hipLaunchKernelGGL(k_sur_eatom, dim3(nb(n, 256)), dim3(256), 0, stream, n, s->rows, M, s->nb->L.perm,
                         s->R.rowof, s->Erow, eatom);
    hipLaunchKernelGGL(k_sur_ensemble, dim3(nb(n, 256)), dim3(256), 0, stream, n, M, s->nb->L.perm, s->F, forces,
                       fmean, sigma, (uint8_t*)nullptr, 0.0, (unsigned long long*)nullptr);
  }
  SHIP(s, hipMemcpyAsync(energies, s->Etot, sizeof(double) * M, hipMemcpyDeviceToDevice, stream));
  return hipGetLastError() == hipSuccess ? 0 : sfail(s, REAXFF_ERR_HIP, "evaluate");
}

int reaxff_surrogate_train_step(reaxff_surrogate* s, int64_t n, const double* pos, const int32_t* type,
                                const double* box, double eref, const double* fref, double wE, double wF, double lr,
                                double* loss, hipStream_t stream) {
  if (!s || n <= 0 || !pos || !type || !fref || !loss) return sfail(s, REAXFF_ERR_ARG, "train_step: bad argument");
  SHIP(s, hipSetDevice(s->device));
  int rc = prepare(s, n, pos, type, box, stream);
  if (rc) return rc;
  if ((rc = evaluate_frame(s, stream))) return rc;
  const int M = s->members;
  SHIP(s, hipMemsetAsync(s->ss, 0, sizeof(double) * M, stream));
  SHIP(s, hipMemsetAsync(s->grad, 0, sizeof(float) * s->nparams, stream));
  for (int m = 0; m < M; ++m) {
    hipLaunchKernelGGL(k_sur_residual, dim3(nb(n, 256)), dim3(256), 0, stream, n, s->nb->L.perm, s->F + (int64_t)m * n * 3,
                       fref, s->res, s->ss + m);
    hipLaunchKernelGGL(k_desc<true>, dim3(nb(n, 32)), dim3(128), 0, stream, desc_args(s, s->res, s->uq, nullptr));
    TrainArgs ta{};
    ta.theta = s->theta + (int64_t)m * 4 * NPAR;
    ta.W1 = s->W1 + (int64_t)m * 4 * ND * HID;
    ta.Wt1 = s->Wt1 + (int64_t)m * 4 * ND * HID;
    ta.W2 = s->W2 + (int64_t)m * 4 * HID * HID;
    ta.Wt2 = s->Wt2 + (int64_t)m * 4 * HID * HID;
    ta.tile_elem = s->R.tile_elem;
    ta.rowatom = s->R.rowatom;
    ta.xq = s->xq;
    ta.uq = s->uq;
    ta.Etot = s->Etot + m;
    ta.eref = eref;
    ta.wE = wE;
    ta.natoms = (double)n;
    ta.cF = (float)(-2.0 * wF / (3.0 * (double)n));
    ta.grad = s->grad + (int64_t)m * 4 * NPAR;
    hipLaunchKernelGGL(k_net_train, dim3((unsigned)(s->rows / TILE)), dim3(256), 0, stream, ta);
  }
  hipLaunchKernelGGL(k_sur_loss, dim3(1), dim3(64), 0, stream, M, s->Etot, s->ss, eref, wE, wF, (double)n, loss);
  if (lr > 0.0) {
    s->adam_t += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 / (1.0 - std::pow(b1, (double)s->adam_t)));
    const float c2 = (float)(1.0 / (1.0 - std::pow(b2, (double)s->adam_t)));
    hipLaunchKernelGGL(k_adam, dim3(nb(s->nparams, 256)), dim3(256), 0, stream, s->nparams, s->theta, s->grad,
                       s->adam_m, s->adam_v, (float)lr, (float)b1, (float)b2, 1e-8f, c1, c2);
    if ((rc = convert_weights(s, stream))) return rc;
  }
  return hipGetLastError() == hipSuccess ? 0 : sfail(s, REAXFF_ERR_HIP, "train_step");
}

reaxff_ctx* reaxff_surrogate_context(reaxff_surrogate* s) { return s ? s->nb : nullptr; }

int reaxff_surrogate_normaliser(reaxff_surrogate* s, int64_t rows, const float* G, double std_floor, float* shift,
                                float* scale, hipStream_t stream) {
  if (!s || rows < 1 || !G || !shift || !scale || !(std_floor > 0.0))
    return sfail(s, REAXFF_ERR_ARG, "normaliser: bad argument");
  SHIP(s, hipSetDevice(s->device));
  double* acc = nullptr;
  float* out = nullptr;
  SHIP(s, hipMalloc(&acc, sizeof(double) * 2 * ND));
  const hipError_t ea = hipMalloc(&out, sizeof(float) * 2 * ND);
  if (ea != hipSuccess) {
    (void)hipFree(acc);
    return sfail(s, REAXFF_ERR_HIP, std::string("hipMalloc: ") + hipGetErrorString(ea));
  }
  const unsigned blocks = nb(rows, 256);
  hipError_t e = hipMemsetAsync(acc, 0, sizeof(double) * 2 * ND, stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_col_stats, dim3(blocks), dim3(256), 0, stream, rows, G, (const double*)nullptr, acc);
    hipLaunchKernelGGL(k_col_final, dim3(1), dim3(256), 0, stream, rows, acc, (const double*)nullptr, std_floor,
                       out, out + ND);
    hipLaunchKernelGGL(k_col_stats, dim3(blocks), dim3(256), 0, stream, rows, G, acc, acc + ND);
    hipLaunchKernelGGL(k_col_final, dim3(1), dim3(256), 0, stream, rows, acc, acc + ND, std_floor, out, out + ND);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(shift, out, sizeof(float) * ND, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipMemcpyAsync(scale, out + ND, sizeof(float) * ND, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  (void)hipFree(acc);
  (void)hipFree(out);
  if (e != hipSuccess) return sfail(s, REAXFF_ERR_HIP, std::string("normaliser: ") + hipGetErrorString(e));
  return REAXFF_OK;
}

int reaxff_surrogate_get_grad(reaxff_surrogate* s, float* grad) {
  if (!s || !grad) return REAXFF_ERR_ARG;
  SHIP(s, hipSetDevice(s->device));
  SHIP(s, hipDeviceSynchronize());
  SHIP(s, hipMemcpy(grad, s->grad, sizeof(float) * s->nparams, hipMemcpyDeviceToHost));
  return REAXFF_OK;
}

int reaxff_surrogate_gated_forces(reaxff_surrogate* s, reaxff_ctx* plain, int64_t n, const double* pos,
                                  const int32_t* type, const double* q, const double* box, double threshold,
                                  double* forces, uint8_t* mask, double* energies, int64_t* nflagged,
                                  int64_t* nsub, hipStream_t stream) {
  if (!s || !plain || n < 0 || (n > 0 && (!pos || !type || !q || !forces || !mask)) || !energies)
    return sfail(s, REAXFF_ERR_ARG, "gated_forces: bad argument");
  SHIP(s, hipSetDevice(s->device));
  int rc = prepare(s, n, pos, type, box, stream);
  if (rc) return rc;
  if ((rc = evaluate_frame(s, stream))) return rc;
  const int M = s->members;
  SHIP(s, hipMemsetAsync(s->nflag, 0, sizeof(unsigned long long), stream));
  if (n > 0)
    hipLaunchKernelGGL(k_sur_ensemble, dim3(nb(n, 256)), dim3(256), 0, stream, n, M, s->nb->L.perm, s->F,
                       (float*)nullptr, forces, (float*)nullptr, mask, threshold, s->nflag);
  SHIP(s, hipMemcpyAsync(energies, s->Etot, sizeof(double) * M, hipMemcpyDeviceToDevice, stream));
  SHIP(s, hipMemcpyAsync(s->nflag_host, s->nflag, sizeof(unsigned long long), hipMemcpyDeviceToHost, stream));
  SHIP(s, hipStreamSynchronize(stream));
  const int64_t nf = (int64_t)*s->nflag_host;
  if (nflagged) *nflagged = nf;
  if (nsub) *nsub = 0;
  if (nf > 0) {
    // fallback: exact plain FP64 forces on the flagged atoms, from the plain
    // evaluation of the atoms their forces depend on (reaxff_forces_masked)
    if ((rc = reaxff_forces_masked(plain, n, pos, type, q, box, mask, forces, nsub, stream)))
      return sfail(s, rc, std::string("fallback forces: ") + reaxff_last_error(plain));
  }
  return hipGetLastError() == hipSuccess ? 0 : sfail(s, REAXFF_ERR_HIP, "gated_forces");
}

}  // extern "C"
