// Complex64 dense transforms on fp16 matrix cores with a two-term split.
//
// Every FP32 operand value a is carried as a pair of fp16 numbers
//     hi = fp16(a s),  lo = fp16(a s - hi),
// with s a power of two that puts the largest magnitude of its group in
// [2^12, 2^13).  fp16 keeps 11 significant bits, so hi + lo holds a s to about
// 2^-22 of that largest magnitude (values too small for lo lose only what lies
// below 2^-26 of it, subnormal handling aside).  A product of table T and data
// X then takes three fp16 matrix products with FP32 accumulation,
//     T X ~ (Th Xh + Th Xl + Tl Xh) / (s_T s_X),
// dropping Tl Xl (2^-22 of the result scale).  fp16 x fp16 products are exact
// in FP32, so the accuracy is that of an FP32 product of the rounded operands:
// the complex64 solve converges under FP64-residual refinement as it does with
// FP32 transforms, at the fp16 matrix rate (16x the FP32 one on gfx950).
// Table scales are fixed per table on the host; data scales per panel, from the
// largest magnitude a workgroup loads.
//
// A workgroup owns a panel of 16 CT columns: x lines (contiguous), or columns
// of one y plane (strided).  It loads all of K for them, splits them into LDS,
// and computes every output row before writing, so panels are independent and
// the y transform runs in place.  Complex tables act through their real
// embedding (K = 2 n_in, columns = vectors); real tables act on real and
// imaginary parts alike (K = n_in, columns = (vector, component) pairs).
//
// v_mfma_f32_16x16x32_f16: operand A (16 x 32) at lane l holds row l % 16,
// k = 8 (l / 16) + j (j < 8); operand B (32 x 16) holds k = 8 (l / 16) + j,
// column l % 16; result D holds row 4 (l / 16) + i, column l % 16 (i < 4).
// Here A = table rows (outputs), B = panel columns.  Table fragment (mt, ks)
// is 64 lanes x 8 halves of hi followed by the same of lo: element
// (16 mt + l % 16, 32 ks + 8 (l / 16) + j).
// LDS holds the panel as hi[c][k] and lo[c][k], rows of LK halves (K padded to
// a multiple of 64), with the 8-half groups of row c permuted as g -> g ^ (c % 8)
// so the 16-byte operand reads of 8 consecutive rows fall in distinct banks;
// the largest panel (K = 512) takes exactly 64 KiB.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace hs {

namespace {

typedef _Float16 h8_t __attribute__((ext_vector_type(8)));
typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
typedef float f4_t __attribute__((ext_vector_type(4)));

constexpr int H3_THREADS = 512;
constexpr int H3_WAVES = H3_THREADS / 64;
constexpr int H3_RED = 32;   // LDS bytes of the maxima in front of the panel
constexpr int H3_PPW = 1;   // panels per workgroup: the loads of the next overlap the products of the current

// Panel width: 16 CT columns.  CT = 4 where the panel rows are at most 256
// halves (LDS 64 KiB), CT = 2 up to 512.
constexpr int h3_ct(int K) { return ((K + 63) & ~63) <= 256 ? 4 : 2; }

__device__ __forceinline__ f4_t mma16(h8_t a, h8_t b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

// Power-of-two scale exponent e for a group whose largest magnitude is m:
// m 2^e lies in [2^12, 2^13) (e = 0 for m = 0 or non-finite m).
__device__ __forceinline__ int panel_exp(float m) {
  if (!(m > 0.f) || !(m <= 3.0e38f)) return 0;
  int ex;
  (void)frexpf(m, &ex);                 // m = f 2^ex, f in [0.5, 1)
  return max(-100, min(100, 13 - ex));
}

// LDS index of element (c, k) of a panel with row length LK
__device__ __forceinline__ int swz(int c, int k, int LK) { return c * LK + ((((k >> 3) ^ (c & 7))) << 3) + (k & 7); }

__device__ __forceinline__ void split(float a, _Float16& h, _Float16& lo) {
  h = (_Float16)a;
  lo = (_Float16)(a - (float)h);        // a - h is exact in FP32
}

// Largest value of m over the workgroup.  red: H3_WAVES floats of LDS of its
// own; the barrier also orders every earlier LDS read of the workgroup before
// what follows.
__device__ __forceinline__ float wg_max(float m, float* red) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = m;
  __syncthreads();
  float r = red[0];
#pragma unroll
  for (int i = 1; i < H3_WAVES; ++i) r = fmaxf(r, red[i]);
  return r;
}

// NO output tiles (rows 16 (w + 8 j)) of one wave against the CT column tiles
// of the panel, all of K.  The table fragments of step ks + 1 load while step
// ks multiplies: two register sets in turn (no copies between them, so no
// wait lands right after a load), each load group fenced from the products by
// a scheduling barrier so it is issued before them.
template <int NO, int CT, bool SYNC, typename Epi>
__device__ __forceinline__ void h3_tiles(const h8_t* __restrict__ ft, const _Float16* hi, const _Float16* lo,
                                         int LK, int KS, int w, int l, Epi&& epi) {
  const h8_t* fa[NO];
#pragma unroll
  for (int j = 0; j < NO; ++j) fa[j] = ft + (int64_t)(w + H3_WAVES * j) * KS * 128 + l;
  f4_t acc[NO][CT];
#pragma unroll
  for (int j = 0; j < NO; ++j)
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[j][c] = f4_t{0, 0, 0, 0};
  const int rowb = (l & 15) * LK, xv = l & 7;   // column 16 c + l % 16 has (l % 16) % 8 = l % 8
  auto fetch = [&](int ks, h8_t (&h)[NO], h8_t (&lw)[NO]) {
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      h[j] = fa[j][ks * 128];
      lw[j] = fa[j][ks * 128 + 64];
    }
  };
  auto step = [&](int ks, const h8_t (&h)[NO], const h8_t (&lw)[NO]) {
#pragma unroll
    for (int c = 0; c < CT; ++c) {
      const int o = c * 16 * LK + rowb + (((4 * ks + (l >> 4)) ^ xv) << 3);
      const h8_t bh = *reinterpret_cast<const h8_t*>(hi + o);
      const h8_t bl = *reinterpret_cast<const h8_t*>(lo + o);
#pragma unroll
      for (int j = 0; j < NO; ++j) {
        acc[j][c] = mma16(lw[j], bh, acc[j][c]);
        acc[j][c] = mma16(h[j], bl, acc[j][c]);
        acc[j][c] = mma16(h[j], bh, acc[j][c]);
      }
    }
  };
  h8_t h0[NO], l0[NO], h1[NO], l1[NO];
  fetch(0, h0, l0);
  for (int ks = 0; ks < KS; ks += 2) {   // KS is even
    fetch(ks + 1, h1, l1);
    __builtin_amdgcn_sched_barrier(0);
    step(ks, h0, l0);
    fetch(ks + 2 < KS ? ks + 2 : ks + 1, h0, l0);
    __builtin_amdgcn_sched_barrier(0);
    step(ks + 1, h1, l1);
  }
  if (SYNC) __syncthreads();   // every wave is done with the panel before results replace it
#pragma unroll
  for (int j = 0; j < NO; ++j)
#pragma unroll
    for (int c = 0; c < CT; ++c) epi(w + H3_WAVES * j, c, acc[j][c]);
}

// The wave's output tiles w, w + 8, ... below MT (a wave-uniform count; at
// most 4 for K <= 512, 2 for K <= 256).  SYNC: one workgroup barrier between
// the products and the results (in every wave, with or without tiles).
template <int CT, bool SYNC, typename Epi>
__device__ __forceinline__ void h3_dispatch(int MT, const h8_t* ft, const _Float16* hi, const _Float16* lo, int LK,
                                            int KS, int w, int l, Epi&& epi) {
  constexpr int NOMAX = CT == 4 ? 2 : 4;
  const int ntw = MT > w ? (MT - w + H3_WAVES - 1) / H3_WAVES : 0;
  switch (ntw < NOMAX ? ntw : NOMAX) {
    case 1: h3_tiles<1, CT, SYNC>(ft, hi, lo, LK, KS, w, l, epi); break;
    case 2: h3_tiles<2, CT, SYNC>(ft, hi, lo, LK, KS, w, l, epi); break;
    case 3: if constexpr (NOMAX >= 3) h3_tiles<3, CT, SYNC>(ft, hi, lo, LK, KS, w, l, epi); break;
    case 4: if constexpr (NOMAX >= 4) h3_tiles<4, CT, SYNC>(ft, hi, lo, LK, KS, w, l, epi); break;
    default: if (SYNC) __syncthreads(); break;
  }
}

template <typename CI>
__device__ __forceinline__ float2 ld_f2(const CI* p) {
  const CI v = *p;
  return make_float2(float(v.x), float(v.y));
}

// Real-table results: lane pairs (2c, 2c + 1) hold the real and imaginary
// parts of rows b..b+3 of one vector; after the exchange the even lane holds
// complex rows b, b+1 and the odd lane rows b+2, b+3.
__device__ __forceinline__ void pair_exchange(const f4_t& a, int odd, float2& z0, float2& z1) {
  const float s0 = odd ? a[0] : a[2];
  const float s1 = odd ? a[1] : a[3];
  const float t0 = __shfl_xor(s0, 1);
  const float t1 = __shfl_xor(s1, 1);
  if (odd) {
    z0 = make_float2(t0, a[2]);
    z1 = make_float2(t1, a[3]);
  } else {
    z0 = make_float2(a[0], t0);
    z1 = make_float2(a[1], t1);
  }
}

template <typename CO, bool ACC>
__device__ __forceinline__ void st_c(CO* p, float2 v) {
  using RO = decltype(p->x);
  if (ACC) {
    CO o = *p;
    o.x = RO(o.x + RO(v.x));
    o.y = RO(o.y + RO(v.y));
    *p = o;
  } else {
    CO o;
    o.x = RO(v.x);
    o.y = RO(v.y);
    *p = o;
  }
}

// Split a loaded value pair into LDS: EMB stores the complex value as the two
// consecutive rows 2 i, 2 i + 1 of column c; !EMB stores its parts as row i of
// columns 2 c and 2 c + 1.
template <bool EMB>
__device__ __forceinline__ void put_split(_Float16* hi, _Float16* lo, int LK, int c, int i, float2 v, float s) {
  _Float16 h0, l0, h1, l1;
  split(v.x * s, h0, l0);
  split(v.y * s, h1, l1);
  if (EMB) {
    const int o = swz(c, 2 * i, LK);
    *reinterpret_cast<h2_t*>(hi + o) = h2_t{h0, h1};
    *reinterpret_cast<h2_t*>(lo + o) = h2_t{l0, l1};
  } else {
    const int o0 = swz(2 * c, i, LK), o1 = swz(2 * c + 1, i, LK);
    hi[o0] = h0;
    hi[o1] = h1;
    lo[o0] = l0;
    lo[o1] = l1;
  }
}

// ------------------------------------------------------------------ x lines
// EMB: panel columns are lines (16 CT of them), K = 2 n_in.
// !EMB: panel columns are (line, component) pairs (8 CT lines), K = n_in.
// A workgroup takes H3_PPW consecutive panels of one descriptor.
template <bool EMB, int CT, typename CI, typename CO, bool ACC>
__global__ __launch_bounds__(H3_THREADS, 4) void k_xform_lines_h3(const XformDesc* __restrict__ descs,
                                                              const h8_t* __restrict__ htab,
                                                              const CI* __restrict__ src, CO* __restrict__ dst) {
  extern __shared__ unsigned char smem_raw[];
  constexpr int C = 16 * CT;
  constexpr int VL = EMB ? C : C / 2;            // lines per panel
  constexpr int LPW = VL / H3_WAVES;             // lines loaded per wave
  constexpr int IT = (EMB ? 8 : 16) / CT;        // complex per lane and line: 64 IT >= padded K / (EMB ? 2 : 1)
  const XformDesc d = descs[blockIdx.y];
  const int r = blockIdx.z;
  const int64_t lines = (int64_t)d.P * d.Q;
  const int64_t np = (lines + VL - 1) / VL;
  const int64_t pb = (int64_t)blockIdx.x * H3_PPW;
  if (pb >= np) return;
  const int pe = int(min((int64_t)H3_PPW, np - pb));
  const int K = EMB ? 2 * d.n_in : d.n_in;
  const int Kp = (K + 63) & ~63;                // K padded to an even number of 32-wide steps
  const int LK = Kp;                            // LDS row length (halves)
  const int NCP = EMB ? Kp / 2 : Kp;            // complex slots per line, padding included
  const int N = EMB ? 2 * d.n_out : d.n_out;
  const int MT = (N + 15) / 16, KS = Kp / 32;
  float* red = reinterpret_cast<float*>(smem_raw);   // H3_WAVES partial maxima, then the panel
  _Float16* hi = reinterpret_cast<_Float16*>(smem_raw + H3_RED);
  _Float16* lo = hi + C * LK;
  const int tid = threadIdx.x, l = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const h8_t* ft = htab + d.htab;
  const int odd = l & 1;

  // panel lines w + 8 a, complex elements l + 64 i
  float2 v[LPW][IT];
  auto load = [&](int64_t L0) {
#pragma unroll
    for (int a = 0; a < LPW; ++a) {
      const int64_t L = L0 + w + H3_WAVES * a;
      const bool ok = L < lines;
      const unsigned Lc = unsigned(ok ? L : lines - 1), Qu = unsigned(d.Q);
      const int p = int(Lc / Qu), q = int(Lc % Qu);
      const CI* sl = src + d.src + (int64_t)r * d.src_r + (int64_t)p * d.src_p + (int64_t)q * d.src_q;
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int i = l + 64 * it;
        v[a][it] = (ok && i < d.n_in) ? ld_f2(sl + i) : make_float2(0.f, 0.f);
      }
    }
  };
  load(pb * VL);
  for (int pi = 0; pi < pe; ++pi) {
    const int64_t L0 = (pb + pi) * VL;
    float m = 0.f;
#pragma unroll
    for (int a = 0; a < LPW; ++a)
#pragma unroll
      for (int it = 0; it < IT; ++it) m = fmaxf(m, fmaxf(fabsf(v[a][it].x), fabsf(v[a][it].y)));
    const int ex = panel_exp(wg_max(m, red));   // also: the previous panel's products are done
    const float s = ldexpf(1.f, ex);
#pragma unroll
    for (int a = 0; a < LPW; ++a)
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int i = l + 64 * it;
        if (i < NCP) put_split<EMB>(hi, lo, LK, w + H3_WAVES * a, i, v[a][it], s);
      }
    __syncthreads();
    if (pi + 1 < pe) load(L0 + VL);

    // results go through LDS (line-major, odd row stride) so each wave then
    // writes (or accumulates into) whole lines with contiguous accesses
    const float oscale = ldexpf(d.hsinv, -ex);
    float2* stg = reinterpret_cast<float2*>(smem_raw + H3_RED);
    const int SO = d.n_out | 1;
    h3_dispatch<CT, true>(MT, ft, hi, lo, LK, KS, w, l, [&](int mt, int ct, const f4_t& a) {
      const int c = 16 * ct + (l & 15);
      float2 z0, z1;
      int b, line;
      if (EMB) {
        b = 8 * mt + 2 * (l >> 4);
        line = c;
        z0 = make_float2(a[0], a[1]);
        z1 = make_float2(a[2], a[3]);
      } else {
        pair_exchange(a, odd, z0, z1);
        b = 16 * mt + 4 * (l >> 4) + 2 * odd;
        line = c >> 1;
      }
      if (b < d.n_out) stg[line * SO + b] = make_float2(z0.x * oscale, z0.y * oscale);
      if (b + 1 < d.n_out) stg[line * SO + b + 1] = make_float2(z1.x * oscale, z1.y * oscale);
    });
    __syncthreads();
    constexpr int OT = (EMB ? 8 : 16) / CT;   // 64 OT >= n_out
    CO* dls[LPW];
    CO old[LPW][OT];
#pragma unroll
    for (int a = 0; a < LPW; ++a) {
      const int64_t L = L0 + w + H3_WAVES * a;
      const unsigned Lc = unsigned(L < lines ? L : lines - 1), Qu = unsigned(d.Q);
      const int p = int(Lc / Qu), q = int(Lc % Qu);
      dls[a] = dst + d.dst + (int64_t)r * d.dst_r + (int64_t)p * d.dst_p + (int64_t)q * d.dst_q;
      if (ACC) {
#pragma unroll
        for (int it = 0; it < OT; ++it) {
          const int i = l + 64 * it;
          if (L < lines && i < d.n_out) old[a][it] = dls[a][i];
        }
      }
    }
#pragma unroll
    for (int a = 0; a < LPW; ++a) {
      const int c = w + H3_WAVES * a;
      if (L0 + c >= lines) continue;
#pragma unroll
      for (int it = 0; it < OT; ++it) {
        const int i = l + 64 * it;
        if (i < d.n_out) {
          const float2 v2 = stg[c * SO + i];
          using RO = decltype(old[0][0].x);
          CO o;
          if (ACC) {
            o.x = RO(old[a][it].x + RO(v2.x));
            o.y = RO(old[a][it].y + RO(v2.y));
          } else {
            o.x = RO(v2.x);
            o.y = RO(v2.y);
          }
          dls[a][i] = o;
        }
      }
    }
  }
}

// ------------------------------------------------------------------ y planes
// In place on complex64 data: EMB panels are 16 CT columns of one plane,
// !EMB panels 8 CT columns as (column, component) pairs.  A workgroup takes
// H3_PPW consecutive panels of one descriptor (column blocks, then planes).
template <bool EMB, int CT>
__global__ __launch_bounds__(H3_THREADS, 4) void k_xform_y_h3(const XformYDesc* __restrict__ descs,
                                                          const h8_t* __restrict__ htab, float2* __restrict__ ws) {
  extern __shared__ unsigned char smem_raw[];
  constexpr int C = 16 * CT;
  constexpr int VC = EMB ? C : C / 2;             // data columns per panel
  constexpr int RPW = 64 / VC;                    // rows per wave and step
  constexpr int RPS = RPW * H3_WAVES;             // rows per workgroup step
  constexpr int IT = (EMB ? 512 : 1024) / CT / RPS;   // steps: padded K / (EMB ? 2 : 1) rows at most
  const XformYDesc d = descs[blockIdx.y];
  const int r = blockIdx.z;
  const int cblocks = (d.ncols + VC - 1) / VC;
  const int64_t np = (int64_t)cblocks * d.P;
  const int64_t pb = (int64_t)blockIdx.x * H3_PPW;
  if (pb >= np) return;
  const int pe = int(min((int64_t)H3_PPW, np - pb));
  const int n = d.n;
  const int K = EMB ? 2 * n : n;
  const int Kp = (K + 63) & ~63;
  const int LK = Kp;
  const int NCP = EMB ? Kp / 2 : Kp;             // rows of the panel, padding included
  const int MT = (K + 15) / 16, KS = Kp / 32;
  float* red = reinterpret_cast<float*>(smem_raw);   // H3_WAVES partial maxima, then the panel
  _Float16* hi = reinterpret_cast<_Float16*>(smem_raw + H3_RED);
  _Float16* lo = hi + C * LK;
  const int tid = threadIdx.x, l = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int col = l % VC;
  const h8_t* ft = htab + d.htab;
  const int odd = l & 1;

  float2 v[IT];
  auto load = [&](int64_t pan) {
    const int p = int(pan / cblocks), x = int(pan % cblocks) * VC + col;
    const float2* bp = ws + d.data + (int64_t)r * d.s_r + (int64_t)p * d.s_p;
    const bool xok = x < d.ncols;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int i = RPS * it + RPW * w + l / VC;
      v[it] = (xok && i < n) ? bp[(int64_t)i * d.s_k + x] : make_float2(0.f, 0.f);
    }
  };
  load(pb);
  for (int pi = 0; pi < pe; ++pi) {
    const int64_t pan = pb + pi;
    const int p = int(pan / cblocks), x0 = int(pan % cblocks) * VC;
    float2* base = ws + d.data + (int64_t)r * d.s_r + (int64_t)p * d.s_p;
    float m = 0.f;
#pragma unroll
    for (int it = 0; it < IT; ++it) m = fmaxf(m, fmaxf(fabsf(v[it].x), fabsf(v[it].y)));
    const int ex = panel_exp(wg_max(m, red));   // also: the previous panel's products are done
    const float s = ldexpf(1.f, ex);
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int i = RPS * it + RPW * w + l / VC;
      if (i < NCP) put_split<EMB>(hi, lo, LK, col, i, v[it], s);
    }
    __syncthreads();   // every read of this panel's columns is done
    if (pi + 1 < pe) load(pan + 1);

    const float oscale = ldexpf(d.hsinv, -ex);
    h3_dispatch<CT, false>(MT, ft, hi, lo, LK, KS, w, l, [&](int mt, int ct, const f4_t& a) {
      const int c = 16 * ct + (l & 15);
      const int xo = x0 + (EMB ? c : c >> 1);
      float2 z0, z1;
      int b;
      if (EMB) {
        b = 8 * mt + 2 * (l >> 4);
        z0 = make_float2(a[0], a[1]);
        z1 = make_float2(a[2], a[3]);
      } else {
        pair_exchange(a, odd, z0, z1);
        b = 16 * mt + 4 * (l >> 4) + 2 * odd;
      }
      if (xo >= d.ncols) return;
      if (b < n) base[(int64_t)b * d.s_k + xo] = make_float2(z0.x * oscale, z0.y * oscale);
      if (b + 1 < n) base[(int64_t)(b + 1) * d.s_k + xo] = make_float2(z1.x * oscale, z1.y * oscale);
    });
  }
}

size_t h3_lds_bytes(int K, int CT) {
  const int LK = (K + 63) & ~63;
  return H3_RED + size_t(2) * 16 * CT * LK * sizeof(_Float16);
}

// x lines also stage their results: lines per panel x (n_out | 1) complex64
size_t h3_lines_lds_bytes(int K, int n_out_max, int CT, bool real) {
  const size_t stage = H3_RED + size_t(real ? 8 : 16) * CT * size_t(n_out_max | 1) * sizeof(float2);
  return std::max(h3_lds_bytes(K, CT), stage);
}

}  // namespace

// ------------------------------------------------------------------ host side
bool h3_fits(int n, bool real) { return real ? n <= 512 : n <= 256; }

int64_t h3_table_frags(int n_out, int n_in, bool real) {
  const int N = real ? n_out : 2 * n_out, K = real ? n_in : 2 * n_in;
  return int64_t((N + 15) / 16) * ((K + 63) / 64) * 2 * 128;   // 16-byte units; an even number of k-steps
}

float h3_table_build(const std::complex<double>* T, int n_out, int n_in, bool real, _Float16* out) {
  const int N = real ? n_out : 2 * n_out, K = real ? n_in : 2 * n_in;
  const int MT = (N + 15) / 16, KS = (K + 63) / 64 * 2;
  auto elem = [&](int o, int k) -> double {
    if (o >= N || k >= K) return 0.0;
    if (real) return T[(size_t)o * n_in + k].real();
    const std::complex<double> t = T[(size_t)(o / 2) * n_in + (k / 2)];
    const int c = o % 2, cp = k % 2;
    return (c == cp) ? t.real() : (c == 0 ? -t.imag() : t.imag());
  };
  double m = 0;
  for (int o = 0; o < N; ++o)
    for (int k = 0; k < K; ++k) m = std::max(m, std::fabs(elem(o, k)));
  int ex = 0;
  if (m > 0) {
    (void)std::frexp(m, &ex);
    ex = 13 - ex;
  }
  const double st = std::ldexp(1.0, ex);
  for (int mt = 0; mt < MT; ++mt)
    for (int ks = 0; ks < KS; ++ks)
      for (int l = 0; l < 64; ++l)
        for (int j = 0; j < 8; ++j) {
          const double a = elem(mt * 16 + l % 16, ks * 32 + 8 * (l / 16) + j) * st;
          const _Float16 h = (_Float16)a;
          const _Float16 lw = (_Float16)(a - (double)h);
          const size_t f = ((size_t)mt * KS + ks) * 128;
          out[(f + l) * 8 + j] = h;
          out[(f + 64 + l) * 8 + j] = lw;
        }
  return float(std::ldexp(1.0, -ex));
}

static int desc_k(const XformDesc& d) { return d.real_tab ? d.n_in : 2 * d.n_in; }
static int desc_k(const XformYDesc& d) { return d.real_tab ? d.n : 2 * d.n; }
int h3_width(const XformDesc& d) { return h3_ct(desc_k(d)); }
int h3_width(const XformYDesc& d) { return h3_ct(desc_k(d)); }

static int h3_lines_tiles(const XformDesc& d, int ct) {
  const int64_t lines = (int64_t)d.P * d.Q;
  const int vl = (d.real_tab ? 8 : 16) * ct;
  const int64_t panels = (lines + vl - 1) / vl;
  return int((panels + H3_PPW - 1) / H3_PPW);
}

static int h3_y_tiles(const XformYDesc& d, int ct) {
  const int vc = (d.real_tab ? 8 : 16) * ct;
  const int64_t panels = (int64_t)((d.ncols + vc - 1) / vc) * d.P;
  return int((panels + H3_PPW - 1) / H3_PPW);
}

template <bool EMB, int CT, typename CI, typename CO, bool ACC>
static void launch_h3(const XformDesc* d, int ndesc, int tiles, size_t lds, const void* htab, const void* src,
                      void* dst, int nrhs, hipStream_t st) {
  hipLaunchKernelGGL((k_xform_lines_h3<EMB, CT, CI, CO, ACC>), dim3(tiles, ndesc, nrhs), dim3(H3_THREADS), lds, st,
                     d, (const h8_t*)htab, (const CI*)src, (CO*)dst);
}

template <bool EMB, int CT>
static void lines_h3_io(int in64, int out64, int acc, const XformDesc* d, int ndesc, int tiles, size_t lds,
                        const void* htab, const void* src, void* dst, int nrhs, hipStream_t st) {
  if (!in64 && !out64)
    launch_h3<EMB, CT, float2, float2, false>(d, ndesc, tiles, lds, htab, src, dst, nrhs, st);
  else if (in64 && !out64)
    launch_h3<EMB, CT, double2, float2, false>(d, ndesc, tiles, lds, htab, src, dst, nrhs, st);
  else if (!in64 && out64 && acc)
    launch_h3<EMB, CT, float2, double2, true>(d, ndesc, tiles, lds, htab, src, dst, nrhs, st);
  else if (!in64 && out64)
    launch_h3<EMB, CT, float2, double2, false>(d, ndesc, tiles, lds, htab, src, dst, nrhs, st);
  else
    launch_h3<EMB, CT, double2, double2, false>(d, ndesc, tiles, lds, htab, src, dst, nrhs, st);
}

// One launch per list; the narrowest panel any descriptor needs is used for all.
void xform_lines_h3(int in64, int out64, int acc, const XformDesc* dev, const XformDesc* host, int ndesc,
                    const void* htab, const void* src, void* dst, int nrhs, hipStream_t st) {
  if (ndesc == 0 || nrhs == 0) return;
  int ct = 4, kmax = 0;
  for (int i = 0; i < ndesc; ++i) {
    ct = std::min(ct, h3_width(host[i]));
    kmax = std::max(kmax, desc_k(host[i]));
  }
  int tiles = 0, nomax = 0;
  for (int i = 0; i < ndesc; ++i) {
    tiles = std::max(tiles, h3_lines_tiles(host[i], ct));
    nomax = std::max(nomax, host[i].n_out);
  }
  if (tiles == 0) return;
  const bool real = host[0].real_tab != 0;
  const size_t lds = h3_lines_lds_bytes(kmax, nomax, ct, real);
  if (real && ct == 4)
    lines_h3_io<false, 4>(in64, out64, acc, dev, ndesc, tiles, lds, htab, src, dst, nrhs, st);
  else if (real)
    lines_h3_io<false, 2>(in64, out64, acc, dev, ndesc, tiles, lds, htab, src, dst, nrhs, st);
  else if (ct == 4)
    lines_h3_io<true, 4>(in64, out64, acc, dev, ndesc, tiles, lds, htab, src, dst, nrhs, st);
  else
    lines_h3_io<true, 2>(in64, out64, acc, dev, ndesc, tiles, lds, htab, src, dst, nrhs, st);
}

void xform_y_h3(const XformYDesc* dev, const XformYDesc* host, int ndesc, const void* htab, void* ws, int nrhs,
                hipStream_t st) {
  if (ndesc == 0 || nrhs == 0) return;
  int ct = 4, kmax = 0;
  for (int i = 0; i < ndesc; ++i) {
    ct = std::min(ct, h3_width(host[i]));
    kmax = std::max(kmax, desc_k(host[i]));
  }
  int tiles = 0;
  for (int i = 0; i < ndesc; ++i) tiles = std::max(tiles, h3_y_tiles(host[i], ct));
  if (tiles == 0) return;
  const size_t lds = h3_lds_bytes(kmax, ct);
  const dim3 grid(tiles, ndesc, nrhs);
  const bool real = host[0].real_tab != 0;
  if (real && ct == 4)
    hipLaunchKernelGGL((k_xform_y_h3<false, 4>), grid, dim3(H3_THREADS), lds, st, dev, (const h8_t*)htab, (float2*)ws);
  else if (real)
    hipLaunchKernelGGL((k_xform_y_h3<false, 2>), grid, dim3(H3_THREADS), lds, st, dev, (const h8_t*)htab, (float2*)ws);
  else if (ct == 4)
    hipLaunchKernelGGL((k_xform_y_h3<true, 4>), grid, dim3(H3_THREADS), lds, st, dev, (const h8_t*)htab, (float2*)ws);
  else
    hipLaunchKernelGGL((k_xform_y_h3<true, 2>), grid, dim3(H3_THREADS), lds, st, dev, (const h8_t*)htab, (float2*)ws);
}

}  // namespace hs
