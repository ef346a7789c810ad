// Dense transforms on matrix cores (gfx950 MFMA), used for the generalized
// eigenvector tables of non-uniform axes (and of uniform axes whose length
// has no power-of-two sine transform), and for face / interface lines.
//
// A complex n_out x n_in table T acts on interleaved complex data as a real
// matrix E of size 2 n_out x 2 n_in:
//     E[2o+c][2i+c'] = [[Re T, -Im T], [Im T, Re T]][c][c'] (o, i)
// so that (E v)[2o+c] is component c of (T v)[o] for interleaved v.  E is
// stored once per table, zero-padded to multiples of 16 in both dimensions
// and pre-arranged in 16 x 4 MFMA operand fragments: fragment (mt, ks) holds
// E[16 mt + l % 16][4 ks + l / 16] at lane l, so a fragment load is one
// contiguous 64-value read.
//
// x lines (contiguous): C[line][n] = sum_k X[line][k] E[n][k]  (data = A operand,
//   staged in LDS; table = B operand read as fragments).
// y planes (in place): C[m][x] = sum_k E[m][k] X[k][x] with X[2i+c][x] the
//   component c of element (i, x); a workgroup owns 16 columns of one plane,
//   holds all of K for them in LDS and computes every output row before
//   writing, so no other workgroup touches its columns.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"

#include <algorithm>
#include <vector>

namespace hs {

namespace {

typedef double f64x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

template <typename R> struct mfma;
template <> struct mfma<double> {
  using acc = f64x4_t;
  static __device__ __forceinline__ acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // row of the 16 x 16 result held in element i of lane l (column l % 16)
  static __device__ __forceinline__ int row(int l, int i) { return 4 * i + (l >> 4); }
};
template <> struct mfma<float> {
  using acc = f32x4_t;
  static __device__ __forceinline__ acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int i) { return 4 * (l >> 4) + i; }
};

template <typename T> struct comp_of;
template <> struct comp_of<double2> { using type = double; };
template <> struct comp_of<float2> { using type = float; };

template <typename CI>
__device__ __forceinline__ typename comp_of<CI>::type comp(const CI& v, int c) {
  return c ? v.y : v.x;
}

// ------------------------------------------------------------------ x lines
constexpr int XM_BM = 64;   // lines per workgroup
constexpr int XM_BN = 64;   // real outputs per workgroup (32 complex)
constexpr int XM_KC = 16;   // reals per K chunk (8 complex inputs)
constexpr int XM_LD = XM_KC + 1;   // LDS row stride (odd: rows fall in distinct banks)

template <typename R, typename CI, typename CO, bool ACC>
__global__ __launch_bounds__(256) void k_xform_lines_mfma(const XformDesc* __restrict__ descs,
                                                         const cplx<R>* __restrict__ tab,
                                                         const CI* __restrict__ src, CO* __restrict__ dst) {
  using M = mfma<R>;
  using acc_t = typename M::acc;
  __shared__ R As[2][XM_BM * XM_LD];
  const XformDesc d = descs[blockIdx.y];
  const int r = blockIdx.z;
  const int64_t lines = (int64_t)d.P * d.Q;
  const int ntiles = (2 * d.n_out + XM_BN - 1) / XM_BN;
  const int64_t lt = blockIdx.x / ntiles;
  const int nt = int(blockIdx.x % ntiles);
  if (lt * XM_BM >= lines) return;
  const int K2 = 2 * d.n_in;
  const int nchunk = (K2 + XM_KC - 1) / XM_KC;
  const int KS = nchunk * 4;               // k-steps of 4 in the fragment table
  const int MT = (2 * d.n_out + 15) / 16;  // 16-row fragment tiles of the table
  const R* ft = reinterpret_cast<const R*>(tab + d.ftab);

  const int tid = threadIdx.x, l = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform
  const int wm = w >> 1, wn = w & 1;       // wave tile: 32 lines x 32 outputs

  // global -> LDS: thread loads complex elements 2*(tid%4), +1 of line tid/4
  const int ld_line = tid >> 2, ld_c = (tid & 3) * 2;
  const int64_t Lld = lt * XM_BM + ld_line;
  const bool ld_ok = Lld < lines;
  const CI* sline;
  {
    const int64_t Lc = ld_ok ? Lld : lines - 1;
    const int p = int(Lc / d.Q), q = int(Lc % d.Q);
    sline = src + d.src + (int64_t)r * d.src_r + (int64_t)p * d.src_p + (int64_t)q * d.src_q;
  }
  auto load_chunk = [&](int ch, R (&v)[4]) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int i = ch * (XM_KC / 2) + ld_c + e;   // complex input index
      const CI x = sline[i < d.n_in ? i : d.n_in - 1];
      const bool ok = ld_ok && i < d.n_in;
      v[2 * e] = ok ? R(x.x) : R(0);
      v[2 * e + 1] = ok ? R(x.y) : R(0);
    }
  };
  auto store_chunk = [&](int buf, const R (&v)[4]) {
#pragma unroll
    for (int e = 0; e < 4; ++e) As[buf][ld_line * XM_LD + 2 * ld_c + e] = v[e];
  };

  acc_t c[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) c[i][j] = acc_t{0, 0, 0, 0};

  // table fragment tiles of this wave (16 real outputs each)
  int mt[2];
  bool mt_ok[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    mt[j] = nt * (XM_BN / 16) + wn * 2 + j;
    mt_ok[j] = mt[j] < MT;
  }

  // table fragments of a chunk: 4 k-steps x 2 tiles, fetched one chunk ahead
  // (tiles past MT read tile MT - 1 and are zeroed)
  const R* fj[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) fj[j] = ft + (int64_t)min(mt[j], MT - 1) * KS * 64 + l;
  auto load_frags = [&](int ch, R (&b)[4][2]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int j = 0; j < 2; ++j) b[s][j] = fj[j][(ch * 4 + s) * 64];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        if (!mt_ok[j]) b[s][j] = R(0);
  };
  R v[4];
  R bfr[4][2], bnx[4][2];
  load_frags(0, bfr);
  load_chunk(0, v);
  store_chunk(0, v);
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nchunk) {
      load_chunk(ch + 1, v);
      load_frags(ch + 1, bnx);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      R afr[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) afr[i] = As[buf][(wm * 32 + i * 16 + (l & 15)) * XM_LD + s * 4 + (l >> 4)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) c[i][j] = M::mma(afr[i], bfr[s][j], c[i][j]);
    }
    if (ch + 1 < nchunk) {
      store_chunk(buf ^ 1, v);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int j = 0; j < 2; ++j) bfr[s][j] = bnx[s][j];
    }
    __syncthreads();
  }

  // results: row = line, column = real output index (interleaved complex)
  using RO = typename comp_of<CO>::type;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t L = lt * XM_BM + wm * 32 + i * 16 + M::row(l, e);
      if (L >= lines) continue;
      const int p = int(L / d.Q), q = int(L % d.Q);
      RO* dline = reinterpret_cast<RO*>(dst + d.dst + (int64_t)r * d.dst_r + (int64_t)p * d.dst_p +
                                        (int64_t)q * d.dst_q);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int n = nt * XM_BN + wn * 32 + j * 16 + (l & 15);
        if (n < 2 * d.n_out) {
          if (ACC)
            dline[n] = RO(dline[n] + RO(c[i][j][e]));
          else
            dline[n] = RO(c[i][j][e]);
        }
      }
    }
  }
}

// ------------------------------------------------------------------ y planes
constexpr int YM_NC = 16;    // complex columns per workgroup
constexpr int YM_THREADS = 512;
constexpr int YM_WAVES = YM_THREADS / 64;

// NT output tiles (rows 16 (w + ws j), j < NT) of one wave over all of K; the
// table fragments of 4 k-steps are fetched one group ahead.
template <typename R, int NT>
__device__ __forceinline__ void y_tiles(const R* __restrict__ ft, const R* Bs, int KS, int K2, int w, int ws, int l,
                                        cplx<R>* base, int64_t s_k, int x, bool xok) {
  using M = mfma<R>;
  using acc_t = typename M::acc;
  const R* fj[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) fj[j] = ft + (int64_t)(w + ws * j) * KS * 64 + l;
  R acur[4][NT], anx[4][NT];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int j = 0; j < NT; ++j) acur[s][j] = fj[j][s * 64];
  acc_t c[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) c[j] = acc_t{0, 0, 0, 0};
  const int ngroups = KS / 4;
  for (int g = 0; g < ngroups; ++g) {
    const int gn = g + 1 < ngroups ? g + 1 : g;   // last group re-reads itself
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int j = 0; j < NT; ++j) anx[s][j] = fj[j][(gn * 4 + s) * 64];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const R b = Bs[((g * 4 + s) * 4 + (l >> 4)) * YM_NC + (l & 15)];
#pragma unroll
      for (int j = 0; j < NT; ++j) c[j] = M::mma(acur[s][j], b, c[j]);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int j = 0; j < NT; ++j) acur[s][j] = anx[s][j];
  }
  // every read of this workgroup's columns is done (all of K sits in LDS)
  if (xok) {
#pragma unroll
    for (int j = 0; j < NT; ++j) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = (w + ws * j) * 16 + M::row(l, e);
        if (m < K2) {
          R* o = reinterpret_cast<R*>(base + (int64_t)(m >> 1) * s_k + x);
          o[m & 1] = c[j][e];
        }
      }
    }
  }
}

// G panels (16 columns of one plane each) per workgroup: with G > 1 the
// waves split into G teams of 8 / G, team g takes panel blockIdx.x * G + g
// (short axes have fewer output tiles than a workgroup has waves).
template <typename R, int TPW, int G>   // TPW: most 16-row output tiles per wave
__global__ __launch_bounds__(YM_THREADS) void k_xform_y_mfma(const XformYDesc* __restrict__ descs,
                                                            const cplx<R>* __restrict__ tab,
                                                            cplx<R>* __restrict__ ws) {
  static_assert(G == 1 || G == 2 || G == 4, "panels per workgroup");
  constexpr int TW = YM_WAVES / G;   // waves per panel
  extern __shared__ unsigned char smem_raw[];
  const XformYDesc d = descs[blockIdx.y];
  const int r = blockIdx.z;
  const int cblocks = (d.ncols + YM_NC - 1) / YM_NC;
  const int64_t npan = (int64_t)cblocks * d.P;
  const int64_t pan0 = (int64_t)blockIdx.x * G;
  if (pan0 >= npan) return;
  const int n = d.n;
  const int K2 = 2 * n;
  const int KS = ((K2 + 15) / 16) * 4;     // a multiple of 4
  const int MT = (K2 + 15) / 16;
  const int PS = KS * 4 * YM_NC;           // LDS reals of one panel
  R* Bs0 = reinterpret_cast<R*>(smem_raw);   // [G][KS*4][YM_NC]
  const R* ft = reinterpret_cast<const R*>(tab + d.ftab);
  const int tid = threadIdx.x, l = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform

  // the whole K extent of each panel's 16 columns into LDS (rows past 2n and
  // panels past the last are zero)
  for (int e = tid; e < G * KS * 2 * YM_NC; e += YM_THREADS) {
    const int g = e / (KS * 2 * YM_NC), e2 = e % (KS * 2 * YM_NC);
    const int i = e2 / YM_NC, col = e2 % YM_NC;
    const int64_t pan = pan0 + g;
    cplx<R> v = mk<R>(0, 0);
    if (pan < npan) {
      const int p = int(pan / cblocks), x = int(pan % cblocks) * YM_NC + col;
      if (i < n && x < d.ncols) v = ws[d.data + (int64_t)r * d.s_r + (int64_t)p * d.s_p + (int64_t)i * d.s_k + x];
    }
    Bs0[g * PS + (2 * i) * YM_NC + col] = v.x;
    Bs0[g * PS + (2 * i + 1) * YM_NC + col] = v.y;
  }

  __syncthreads();
  // this wave's panel and output tiles t, t + TW, ... below MT (wave-uniform)
  const int g = w / TW, t = w % TW;
  const int64_t pan = pan0 + g;
  if (pan >= npan) return;
  const int p = int(pan / cblocks), x0 = int(pan % cblocks) * YM_NC;
  cplx<R>* base = ws + d.data + (int64_t)r * d.s_r + (int64_t)p * d.s_p;
  const int ntw = MT > t ? (MT - t + TW - 1) / TW : 0;
  const int x = x0 + (l & 15);
  const R* Bs = Bs0 + g * PS;
  switch (ntw < TPW ? ntw : TPW) {
    case 0: break;
#define HS_YCASE(N) \
    case N: if constexpr (N <= TPW) y_tiles<R, N>(ft, Bs, KS, K2, t, TW, l, base, d.s_k, x, x < d.ncols); break;
    HS_YCASE(1) HS_YCASE(2) HS_YCASE(3) HS_YCASE(4) HS_YCASE(5) HS_YCASE(6) HS_YCASE(7) HS_YCASE(8)
#undef HS_YCASE
    default: break;
  }
}

// ------------------------------------------------------------------ real tables
// A real table T (the sine matrix of a uniform axis whose length has no
// power-of-two sine transform) acts on the real and imaginary parts alike, so
// the product needs no embedding: its fragments hold T itself (fragment
// (mt, ks) holds T[16 mt + l % 16][4 ks + l / 16] at lane l), and
//   x lines: rows are (line, component) pairs, K = n_in;
//   y planes: columns are (column, component) pairs, 2 x 16 per workgroup.
// Half the products of the embedded form.

template <typename R, typename CI, typename CO, bool ACC>
__global__ __launch_bounds__(256) void k_xform_lines_mfma_real(const XformDesc* __restrict__ descs,
                                                              const cplx<R>* __restrict__ tab,
                                                              const CI* __restrict__ src, CO* __restrict__ dst) {
  using M = mfma<R>;
  using acc_t = typename M::acc;
  constexpr int BL = XM_BM / 2;            // 32 lines = 64 (line, component) rows
  __shared__ R As[2][XM_BM * XM_LD];       // [row = 2 line + c][k]
  const XformDesc d = descs[blockIdx.y];
  const int r = blockIdx.z;
  const int64_t lines = (int64_t)d.P * d.Q;
  const int ntiles = (d.n_out + XM_BN - 1) / XM_BN;
  const int64_t lt = blockIdx.x / ntiles;
  const int nt = int(blockIdx.x % ntiles);
  if (lt * BL >= lines) return;
  const int nchunk = (d.n_in + XM_KC - 1) / XM_KC;
  const int KS = nchunk * 4;
  const int MT = (d.n_out + 15) / 16;
  const R* ft = reinterpret_cast<const R*>(tab + d.ftab);
  const int tid = threadIdx.x, l = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = w >> 1, wn = w & 1;

  // global -> LDS: thread loads complex inputs 2*(tid%8), +1 of line tid/8
  const int ld_line = tid >> 3, ld_c = (tid & 7) * 2;
  const int64_t Lld = lt * BL + ld_line;
  const bool ld_ok = Lld < lines;
  const CI* sline;
  {
    const int64_t Lc = ld_ok ? Lld : lines - 1;
    const int p = int(Lc / d.Q), q = int(Lc % d.Q);
    sline = src + d.src + (int64_t)r * d.src_r + (int64_t)p * d.src_p + (int64_t)q * d.src_q;
  }
  auto load_chunk = [&](int ch, R (&v)[4]) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int i = ch * XM_KC + ld_c + e;
      const CI x = sline[i < d.n_in ? i : d.n_in - 1];
      const bool ok = ld_ok && i < d.n_in;
      v[2 * e] = ok ? R(x.x) : R(0);
      v[2 * e + 1] = ok ? R(x.y) : R(0);
    }
  };
  auto store_chunk = [&](int buf, const R (&v)[4]) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      As[buf][(2 * ld_line) * XM_LD + ld_c + e] = v[2 * e];
      As[buf][(2 * ld_line + 1) * XM_LD + ld_c + e] = v[2 * e + 1];
    }
  };
  int mt[2];
  bool mt_ok[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    mt[j] = nt * (XM_BN / 16) + wn * 2 + j;
    mt_ok[j] = mt[j] < MT;
  }
  const R* fj[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) fj[j] = ft + (int64_t)min(mt[j], MT - 1) * KS * 64 + l;
  auto load_frags = [&](int ch, R (&b)[4][2]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int j = 0; j < 2; ++j) b[s][j] = fj[j][(ch * 4 + s) * 64];
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        if (!mt_ok[j]) b[s][j] = R(0);
  };
  acc_t c[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) c[i][j] = acc_t{0, 0, 0, 0};
  R v[4];
  R bfr[4][2], bnx[4][2];
  load_frags(0, bfr);
  load_chunk(0, v);
  store_chunk(0, v);
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nchunk) {
      load_chunk(ch + 1, v);
      load_frags(ch + 1, bnx);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      R afr[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) afr[i] = As[buf][(wm * 32 + i * 16 + (l & 15)) * XM_LD + s * 4 + (l >> 4)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) c[i][j] = M::mma(afr[i], bfr[s][j], c[i][j]);
    }
    if (ch + 1 < nchunk) {
      store_chunk(buf ^ 1, v);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int j = 0; j < 2; ++j) bfr[s][j] = bnx[s][j];
    }
    __syncthreads();
  }
  using RO = typename comp_of<CO>::type;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int row = wm * 32 + i * 16 + M::row(l, e);   // (line, component) row
      const int64_t L = lt * BL + (row >> 1);
      if (L >= lines) continue;
      const int cc = row & 1;
      const int p = int(L / d.Q), q = int(L % d.Q);
      RO* dline = reinterpret_cast<RO*>(dst + d.dst + (int64_t)r * d.dst_r + (int64_t)p * d.dst_p +
                                        (int64_t)q * d.dst_q);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int o = nt * XM_BN + wn * 32 + j * 16 + (l & 15);
        if (o < d.n_out) {
          if (ACC)
            dline[2 * o + cc] = RO(dline[2 * o + cc] + RO(c[i][j][e]));
          else
            dline[2 * o + cc] = RO(c[i][j][e]);
        }
      }
    }
  }
}

// NT row tiles x 2 column tiles (32 real columns) of one wave for a real table.
template <typename R, int NT>
__device__ __forceinline__ void y_tiles_real(const R* __restrict__ ft, const R* Bs, int KS, int n, int w, int l,
                                             cplx<R>* base, int64_t s_k, int x0, int ncols) {
  using M = mfma<R>;
  using acc_t = typename M::acc;
  const R* fj[NT];
#pragma unroll
  for (int j = 0; j < NT; ++j) fj[j] = ft + (int64_t)(w + YM_WAVES * j) * KS * 64 + l;
  R acur[4][NT], anx[4][NT];
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int j = 0; j < NT; ++j) acur[s][j] = fj[j][s * 64];
  acc_t c[NT][2];
#pragma unroll
  for (int j = 0; j < NT; ++j) c[j][0] = c[j][1] = acc_t{0, 0, 0, 0};
  const int ngroups = KS / 4;
  for (int g = 0; g < ngroups; ++g) {
    const int gn = g + 1 < ngroups ? g + 1 : g;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int j = 0; j < NT; ++j) anx[s][j] = fj[j][(gn * 4 + s) * 64];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = (g * 4 + s) * 4 + (l >> 4);
      const R b0 = Bs[k * (2 * YM_NC) + (l & 15)];
      const R b1 = Bs[k * (2 * YM_NC) + 16 + (l & 15)];
#pragma unroll
      for (int j = 0; j < NT; ++j) {
        c[j][0] = M::mma(acur[s][j], b0, c[j][0]);
        c[j][1] = M::mma(acur[s][j], b1, c[j][1]);
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int j = 0; j < NT; ++j) acur[s][j] = anx[s][j];
  }
#pragma unroll
  for (int j = 0; j < NT; ++j) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int col = h * 16 + (l & 15);   // (column, component) index
      const int x = x0 + (col >> 1);
      if (x >= ncols) continue;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int o = (w + YM_WAVES * j) * 16 + M::row(l, e);
        if (o < n) {
          R* out = reinterpret_cast<R*>(base + (int64_t)o * s_k + x);
          out[col & 1] = c[j][h][e];
        }
      }
    }
  }
}

template <typename R, int TPW>
__global__ __launch_bounds__(YM_THREADS) void k_xform_y_mfma_real(const XformYDesc* __restrict__ descs,
                                                                 const cplx<R>* __restrict__ tab,
                                                                 cplx<R>* __restrict__ ws) {
  extern __shared__ unsigned char smem_raw[];
  R* Bs = reinterpret_cast<R*>(smem_raw);   // [KS*4][2*YM_NC]: row k = element k of 16 complex columns
  const XformYDesc d = descs[blockIdx.y];
  const int r = blockIdx.z;
  const int cblocks = (d.ncols + YM_NC - 1) / YM_NC;
  const int p = blockIdx.x / cblocks, cb = blockIdx.x % cblocks;
  if (p >= d.P) return;
  const int n = d.n;
  const int KS = ((n + 15) / 16) * 4;
  const int MT = (n + 15) / 16;
  const R* ft = reinterpret_cast<const R*>(tab + d.ftab);
  cplx<R>* base = ws + d.data + (int64_t)r * d.s_r + (int64_t)p * d.s_p;
  const int x0 = cb * YM_NC;
  const int tid = threadIdx.x, l = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int e = tid; e < KS * 4 * YM_NC; e += YM_THREADS) {
    const int i = e / YM_NC, col = e % YM_NC;
    const int x = x0 + col;
    cplx<R> v = mk<R>(0, 0);
    if (i < n && x < d.ncols) v = base[(int64_t)i * d.s_k + x];
    Bs[i * (2 * YM_NC) + 2 * col] = v.x;
    Bs[i * (2 * YM_NC) + 2 * col + 1] = v.y;
  }
  __syncthreads();
  const int ntw = MT > w ? (MT - w + YM_WAVES - 1) / YM_WAVES : 0;
  switch (ntw < TPW ? ntw : TPW) {
    case 0: break;
#define HS_YCASE(N) \
    case N: if constexpr (N <= TPW) y_tiles_real<R, N>(ft, Bs, KS, n, w, l, base, d.s_k, x0, d.ncols); break;
    HS_YCASE(1) HS_YCASE(2) HS_YCASE(3) HS_YCASE(4)
#undef HS_YCASE
    default: break;
  }
}

// ------------------------------------------------------------------ small line sets
// Few or short lines (interface and face lines, narrow PML blocks): complex
// FMA on 16 x 16 output tiles, K staged through LDS in steps of 32; more
// workgroups than the matrix-core tiling would give for such sizes.  The next
// step's data and table values are loaded into registers while the current
// step is multiplied, so a workgroup waits for memory once, not once per step.
template <typename CO, typename CI>
__device__ __forceinline__ CO cvt(CI v) {
  CO o;
  o.x = (decltype(o.x))v.x;
  o.y = (decltype(o.y))v.y;
  return o;
}

constexpr int XL_T = 16;
constexpr int XL_K = 32;

// TM x TM outputs per thread: a workgroup owns 16 TM lines x 16 TM outputs.
template <typename R, typename CI, typename CO, bool ACC, int TM>
__global__ __launch_bounds__(256) void k_xform_lines_small(const XformDesc* __restrict__ descs,
                                                     const cplx<R>* __restrict__ tab,
                                                     const CI* __restrict__ src, CO* __restrict__ dst) {
  using C = cplx<R>;
  constexpr int TT = XL_T * TM;                 // tile edge
  constexpr int NE = TT * XL_K / 256;           // elements of each array per thread and step
  static_assert(NE * 256 == TT * XL_K, "whole steps per thread");
  const XformDesc d = descs[blockIdx.y];
  const int r = blockIdx.z;
  const int lines = d.P * d.Q;
  const int ntl = (lines + TT - 1) / TT;
  const int nto = (d.n_out + TT - 1) / TT;
  const int tile = blockIdx.x;
  if (tile >= ntl * nto) return;
  const int tl = tile % ntl, to = tile / ntl;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  __shared__ C sA[TT][XL_K + 1];
  __shared__ C sT[TT][XL_K + 1];
  C acc[TM][TM];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TM; ++j) acc[i][j] = mk<R>(0, 0);
  const CI* s0 = src + d.src + (int64_t)r * d.src_r;
  const C* T = tab + d.tab;
  // element e = threadIdx.x + 256 i of a step: row e / XL_K, column e % XL_K;
  // the line and table-row offsets of this thread's rows do not change
  int64_t aoff[NE], toff[NE];
  bool aok[NE], tok[NE];
#pragma unroll
  for (int i = 0; i < NE; ++i) {
    const int li = (threadIdx.x + 256 * i) / XL_K;
    const int L = tl * TT + li, O = to * TT + li;
    aok[i] = L < lines;
    const int Lc = aok[i] ? L : 0;
    aoff[i] = (int64_t)(Lc / d.Q) * d.src_p + (int64_t)(Lc % d.Q) * d.src_q;
    tok[i] = O < d.n_out;
    toff[i] = (int64_t)(tok[i] ? O : 0) * d.n_in;
  }
  C ra[NE], rt[NE];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int k = k0 + (threadIdx.x + 256 * i) % XL_K;
      const bool kin = k < d.n_in;
      ra[i] = (aok[i] && kin) ? cvt<C>(s0[aoff[i] + k]) : mk<R>(0, 0);
      rt[i] = (tok[i] && kin) ? T[toff[i] + k] : mk<R>(0, 0);
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < d.n_in; k0 += XL_K) {
#pragma unroll
    for (int i = 0; i < NE; ++i) {
      const int e = threadIdx.x + 256 * i;
      sA[e / XL_K][e % XL_K] = ra[i];
      sT[e / XL_K][e % XL_K] = rt[i];
    }
    __syncthreads();
    if (k0 + XL_K < d.n_in) fetch(k0 + XL_K);
#pragma unroll 4
    for (int kk = 0; kk < XL_K; ++kk) {
      C a[TM], t[TM];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        a[i] = sA[ty + XL_T * i][kk];
        t[i] = sT[tx + XL_T * i][kk];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TM; ++j) acc[i][j] = cfma(a[i], t[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < TM; ++i) {
    const int L = tl * TT + ty + XL_T * i;
    if (L >= lines) continue;
    const int p = L / d.Q, q = L % d.Q;
    CO* out = dst + d.dst + (int64_t)r * d.dst_r + (int64_t)p * d.dst_p + (int64_t)q * d.dst_q;
#pragma unroll
    for (int j = 0; j < TM; ++j) {
      const int o = to * TT + tx + XL_T * j;
      if (o >= d.n_out) continue;
      if (ACC) {
        CO prev = out[o];
        prev.x += acc[i][j].x;
        prev.y += acc[i][j].y;
        out[o] = prev;
      } else {
        out[o] = cvt<CO>(acc[i][j]);
      }
    }
  }
}

}  // namespace

// ------------------------------------------------------------------ host side
int64_t mfma_rtable_reals(int n_out, int n_in) {
  return int64_t((n_out + 15) / 16) * 16 * (((n_in + 15) / 16) * 16);
}

void mfma_rtable_build(const std::complex<double>* T, int n_out, int n_in, double* out) {
  const int MT = (n_out + 15) / 16;
  const int KS = ((n_in + 15) / 16) * 4;
  for (int mt = 0; mt < MT; ++mt)
    for (int ks = 0; ks < KS; ++ks)
      for (int l = 0; l < 64; ++l) {
        const int m = mt * 16 + (l % 16), k = ks * 4 + (l / 16);
        out[((size_t)mt * KS + ks) * 64 + l] = (m < n_out && k < n_in) ? T[(size_t)m * n_in + k].real() : 0.0;
      }
}

int64_t mfma_table_reals(int n_out, int n_in) {
  const int64_t rows = ((2 * n_out + 15) / 16) * 16;
  const int64_t cols = ((2 * n_in + 15) / 16) * 16;
  return rows * cols;
}

void mfma_table_build(const std::complex<double>* T, int n_out, int n_in, double* out) {
  const int MT = (2 * n_out + 15) / 16;
  const int KS = ((2 * n_in + 15) / 16) * 4;
  for (int mt = 0; mt < MT; ++mt)
    for (int ks = 0; ks < KS; ++ks)
      for (int l = 0; l < 64; ++l) {
        const int m = mt * 16 + (l % 16), k = ks * 4 + (l / 16);
        double v = 0;
        if (m < 2 * n_out && k < 2 * n_in) {
          const std::complex<double> t = T[(size_t)(m / 2) * n_in + (k / 2)];
          const int c = m % 2, cp = k % 2;
          v = (c == cp) ? t.real() : (c == 0 ? -t.imag() : t.imag());
        }
        out[((size_t)mt * KS + ks) * 64 + l] = v;
      }
}

bool xform_lines_use_mfma(const XformDesc& d) {
  // matrix cores for long lines in numbers that fill the chip (per right-hand
  // side, so a block takes the same kernel alone and in a batch; 512 lines
  // are the two faces of a block over 256 planes)
  return std::max(d.n_in, d.n_out) >= 24 && (int64_t)d.P * d.Q >= 512;
}

LinesLaunch xform_lines_launch(const XformDesc* d, int ndesc, bool mfma, bool real) {
  LinesLaunch L;
  L.mfma = mfma;
  L.real = real;
  int64_t m = 0;
  for (int i = 0; i < ndesc; ++i) {
    const int64_t lines = (int64_t)d[i].P * d[i].Q;
    int64_t t;
    if (mfma && real)
      t = ((lines + XM_BM / 2 - 1) / (XM_BM / 2)) * ((d[i].n_out + XM_BN - 1) / XM_BN);
    else if (mfma)
      t = ((lines + XM_BM - 1) / XM_BM) * ((2 * d[i].n_out + XM_BN - 1) / XM_BN);
    else
      t = ((lines + XL_T - 1) / XL_T) * ((d[i].n_out + XL_T - 1) / XL_T);
    m = std::max(m, t);
  }
  L.tiles = int(m);
  if (!mfma) {
    // 32 x 32 tiles (2 x 2 outputs per thread: half the table and data
    // re-reads per output) where every descriptor has more than 16 outputs and
    // they still give each CU a workgroup
    int64_t m2 = 0, sum2 = 0;
    bool wide = ndesc > 0;
    for (int i = 0; i < ndesc; ++i) {
      const int64_t lines = (int64_t)d[i].P * d[i].Q;
      const int64_t t = ((lines + 2 * XL_T - 1) / (2 * XL_T)) * ((d[i].n_out + 2 * XL_T - 1) / (2 * XL_T));
      wide = wide && d[i].n_out > XL_T;
      m2 = std::max(m2, t);
      sum2 += t;
    }
    if (wide && sum2 >= 256) {
      L.tm = 2;
      L.tiles = int(m2);
    }
  }
  return L;
}

template <typename R, typename CI, typename CO, bool ACC>
static void launch_lines(const XformDesc* d, int ndesc, const LinesLaunch& L, const void* tab, const void* src,
                         void* dst, int nrhs, hipStream_t st) {
  const dim3 grid(L.tiles, ndesc, nrhs);
  if (L.mfma && L.real)
    hipLaunchKernelGGL((k_xform_lines_mfma_real<R, CI, CO, ACC>), grid, dim3(256), 0, st, d, (const cplx<R>*)tab,
                       (const CI*)src, (CO*)dst);
  else if (L.mfma)
    hipLaunchKernelGGL((k_xform_lines_mfma<R, CI, CO, ACC>), grid, dim3(256), 0, st, d, (const cplx<R>*)tab,
                       (const CI*)src, (CO*)dst);
  else if (L.tm == 2)
    hipLaunchKernelGGL((k_xform_lines_small<R, CI, CO, ACC, 2>), grid, dim3(256), 0, st, d, (const cplx<R>*)tab,
                       (const CI*)src, (CO*)dst);
  else
    hipLaunchKernelGGL((k_xform_lines_small<R, CI, CO, ACC, 1>), grid, dim3(256), 0, st, d, (const cplx<R>*)tab,
                       (const CI*)src, (CO*)dst);
}

void xform_lines(int prec, int in64, int out64, int acc, const XformDesc* d, int ndesc, const LinesLaunch& L,
                 const void* tab, const void* src, void* dst, int nrhs, hipStream_t st) {
  if (ndesc == 0 || L.tiles == 0 || nrhs == 0) return;
  if (prec == 0) {
    if (acc)
      launch_lines<double, double2, double2, true>(d, ndesc, L, tab, src, dst, nrhs, st);
    else
      launch_lines<double, double2, double2, false>(d, ndesc, L, tab, src, dst, nrhs, st);
    return;
  }
  // complex64 compute; boundary passes may read or write complex128
  if (!in64 && !out64) {
    launch_lines<float, float2, float2, false>(d, ndesc, L, tab, src, dst, nrhs, st);
  } else if (in64 && !out64) {
    launch_lines<float, double2, float2, false>(d, ndesc, L, tab, src, dst, nrhs, st);
  } else if (!in64 && out64) {
    if (acc)
      launch_lines<float, float2, double2, true>(d, ndesc, L, tab, src, dst, nrhs, st);
    else
      launch_lines<float, float2, double2, false>(d, ndesc, L, tab, src, dst, nrhs, st);
  } else {
    launch_lines<float, double2, double2, false>(d, ndesc, L, tab, src, dst, nrhs, st);
  }
}

bool xform_y_use_mfma(int prec, int n) { return n >= 16 && n <= (prec == 0 ? 256 : 512); }

int xform_y_mfma_tiles(const XformYDesc& d) { return ((d.ncols + YM_NC - 1) / YM_NC) * d.P; }

void xform_y_mfma(int prec, const XformYDesc* d, int ndesc, int max_n, int max_tiles, const void* tab, void* ws,
                  int nrhs, hipStream_t st, bool real) {
  if (ndesc == 0 || nrhs == 0 || max_tiles == 0) return;
  if (real) {
    // rows of n reals x 32 real columns; at most 4 row tiles per wave
    const size_t rows = size_t((max_n + 15) / 16) * 16;
    const dim3 grid(max_tiles, ndesc, nrhs);
    if (prec == 0)
      hipLaunchKernelGGL((k_xform_y_mfma_real<double, 4>), grid, dim3(YM_THREADS), rows * 2 * YM_NC * sizeof(double),
                         st, d, (const double2*)tab, (double2*)ws);
    else
      hipLaunchKernelGGL((k_xform_y_mfma_real<float, 4>), grid, dim3(YM_THREADS), rows * 2 * YM_NC * sizeof(float),
                         st, d, (const float2*)tab, (float2*)ws);
    return;
  }
  // output tiles per wave: ceil(2 max_n / 16 / 8) <= 4 (n <= 256) or 8 (n <= 512);
  // axes of at most 2 (4) output tiles put 4 (2) panels in a workgroup
  const size_t rows = size_t((2 * max_n + 15) / 16) * 16;
  const int mt = (2 * max_n + 15) / 16;
  const int G = mt <= 2 ? 4 : mt <= 4 ? 2 : 1;
  const dim3 grid((max_tiles + G - 1) / G, ndesc, nrhs);
  const size_t csz = prec == 0 ? sizeof(double) : sizeof(float);
  const size_t lds = G * rows * YM_NC * csz;
  if (prec == 0) {
    if (G == 4)
      hipLaunchKernelGGL((k_xform_y_mfma<double, 1, 4>), grid, dim3(YM_THREADS), lds, st, d, (const double2*)tab,
                         (double2*)ws);
    else if (G == 2)
      hipLaunchKernelGGL((k_xform_y_mfma<double, 1, 2>), grid, dim3(YM_THREADS), lds, st, d, (const double2*)tab,
                         (double2*)ws);
    else
      hipLaunchKernelGGL((k_xform_y_mfma<double, 4, 1>), grid, dim3(YM_THREADS), lds, st, d, (const double2*)tab,
                         (double2*)ws);
  } else {
    if (G == 4)
      hipLaunchKernelGGL((k_xform_y_mfma<float, 1, 4>), grid, dim3(YM_THREADS), lds, st, d, (const float2*)tab,
                         (float2*)ws);
    else if (G == 2)
      hipLaunchKernelGGL((k_xform_y_mfma<float, 1, 2>), grid, dim3(YM_THREADS), lds, st, d, (const float2*)tab,
                         (float2*)ws);
    else if (max_n <= 256)
      hipLaunchKernelGGL((k_xform_y_mfma<float, 4, 1>), grid, dim3(YM_THREADS), lds, st, d, (const float2*)tab,
                         (float2*)ws);
    else
      hipLaunchKernelGGL((k_xform_y_mfma<float, 8, 1>), grid, dim3(YM_THREADS), lds, st, d, (const float2*)tab,
                         (float2*)ws);
  }
}

// group of a descriptor: 0..3 split-fp16 matrix cores (complex64 path):
// real table wide / narrow panels, embedded table wide / narrow; 4 / 5 matrix
// cores in the compute precision with a real / embedded table; 6 complex FMA
// tiles
static int lines_group(const XformDesc& d) {
  if (!xform_lines_use_mfma(d)) return 6;
  if (d.htab >= 0) return (d.real_tab ? 0 : 2) + (h3_width(d) == 4 ? 0 : 1);
  return d.real_tab ? 4 : 5;
}
static int y_group(int prec, const XformYDesc& d) {
  if (!xform_y_use_mfma(prec, d.n)) return 6;
  // short embedded axes (at most 3 output tiles) go to the compute-precision
  // kernel, which puts several panels in a workgroup (measured: faster at 23
  // nodes, slower than the split-fp16 kernel at 31)
  if (d.htab >= 0 && (d.real_tab || d.n > 24)) return (d.real_tab ? 0 : 2) + (h3_width(d) == 4 ? 0 : 1);
  return d.real_tab ? 4 : 5;
}

int partition_lines(std::vector<XformDesc>& v) {
  std::stable_sort(v.begin(), v.end(),
                   [](const XformDesc& a, const XformDesc& b) { return lines_group(a) < lines_group(b); });
  return int(std::count_if(v.begin(), v.end(), [](const XformDesc& d) { return lines_group(d) < 6; }));
}

int partition_y(int prec, std::vector<XformYDesc>& v) {
  std::stable_sort(v.begin(), v.end(),
                   [prec](const XformYDesc& a, const XformYDesc& b) { return y_group(prec, a) < y_group(prec, b); });
  return int(std::count_if(v.begin(), v.end(), [prec](const XformYDesc& d) { return y_group(prec, d) < 6; }));
}

void run_lines_list(int prec, int in64, int out64, int acc, const XformDesc* dev, const std::vector<XformDesc>& host,
                    const void* tab, const void* htab, const void* src, void* dst, int nrhs, hipStream_t st) {
  const int n = int(host.size());
  for (int b = 0; b < n;) {
    const int g = lines_group(host[b]);
    int e = b;
    while (e < n && lines_group(host[e]) == g) ++e;
    if (g < 4)
      xform_lines_h3(in64, out64, acc, dev + b, host.data() + b, e - b, htab, src, dst, nrhs, st);
    else
      xform_lines(prec, in64, out64, acc, dev + b, e - b, xform_lines_launch(host.data() + b, e - b, g < 6, g == 4),
                  tab, src, dst, nrhs, st);
    b = e;
  }
}

void run_y_list(int prec, const XformYDesc* dev, const std::vector<XformYDesc>& host, const void* tab,
                const void* htab, void* ws, int nrhs, hipStream_t st) {
  const int n = int(host.size());
  for (int b = 0; b < n;) {
    const int g = y_group(prec, host[b]);
    int e = b;
    int max_n = 0, t16 = 0, t8 = 0;
    while (e < n && y_group(prec, host[e]) == g) max_n = std::max(max_n, host[e].n), ++e;
    // the small-tile kernel takes several planes per workgroup (as many as its
    // launch will use for the group's longest axis)
    const int pw16 = g >= 6 ? xform_y_ppw(prec, max_n, 16) : 1, pw8 = g >= 6 ? xform_y_ppw(prec, max_n, 8) : 1;
    for (int i = b; i < e; ++i) {
      t16 = std::max(t16, xform_y_tiles(host[i], 16, pw16));
      t8 = std::max(t8, xform_y_tiles(host[i], 8, pw8));
    }
    if (g < 4)
      xform_y_h3(dev + b, host.data() + b, e - b, htab, ws, nrhs, st);
    else if (g < 6)
      xform_y_mfma(prec, dev + b, e - b, max_n, t16, tab, ws, nrhs, st, g == 4);   // 16-column tiles
    else
      xform_y(prec, dev + b, e - b, max_n, t16, t8, tab, ws, nrhs, st);
    b = e;
  }
}

}  // namespace hs
