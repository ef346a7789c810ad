// HIP kernels of the separable Helmholtz block solver (gfx950).
//
// Every stage kernel is batched over blocks: blockIdx.y selects a descriptor
// (one block, face set or interface line set), blockIdx.z the right-hand side,
// blockIdx.x a tile.  Descriptors hold element offsets relative to base
// pointers given at launch, so one descriptor table serves every solve.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "kernels.hpp"

#include <algorithm>
#include <functional>
#include <vector>
#include <mutex>
#include <string>

namespace hs {

namespace {

// Streaming store of a complex value (written once, not re-read by this
// kernel): marked non-temporal so that it does not displace reused lines.
__device__ __forceinline__ void st_stream(double2* p, double2 v) {
  typedef double v2d __attribute__((ext_vector_type(2)));
  __builtin_nontemporal_store(v2d{v.x, v.y}, reinterpret_cast<v2d*>(p));
}
__device__ __forceinline__ void st_stream(float2* p, float2 v) {
  typedef float v2f __attribute__((ext_vector_type(2)));
  __builtin_nontemporal_store(v2f{v.x, v.y}, reinterpret_cast<v2f*>(p));
}

template <typename T> struct real_of;
template <> struct real_of<double2> { using type = double; };
template <> struct real_of<float2> { using type = float; };

template <typename CO, typename CI>
__device__ __forceinline__ CO cvt(CI v) {
  CO o;
  o.x = (decltype(o.x))v.x;
  o.y = (decltype(o.y))v.y;
  return o;
}

// ---------------------------------------------------------------------------
// Dense transform along a strided axis, in place: for planes p0 .. p0 + ppw - 1
// and columns [c0, c0 + CT), data[o][c] = sum_k T[o][k] data[k][c].  Every
// column panel of the workgroup is staged in LDS before any output is
// written; several planes per workgroup keep short axes (a few tens of rows)
// from running as many tiny workgroups.
// ---------------------------------------------------------------------------
template <typename R, int CT>
__global__ __launch_bounds__(256) void k_xform_y(const XformYDesc* __restrict__ descs,
                                                 const cplx<R>* __restrict__ tab,
                                                 cplx<R>* __restrict__ ws, int ppw) {
  using C = cplx<R>;
  extern __shared__ unsigned char smem_raw[];
  C* panel = reinterpret_cast<C*>(smem_raw);   // [ppw][n][CT]
  const XformYDesc d = descs[blockIdx.y];
  const int r = blockIdx.z;
  const int ntc = (d.ncols + CT - 1) / CT;
  const int npg = (d.P + ppw - 1) / ppw;
  const int tile = blockIdx.x;
  if (tile >= ntc * npg) return;
  const int p0 = (tile / ntc) * ppw, c0 = (tile % ntc) * CT;
  const int np = min(ppw, d.P - p0);
  C* base = ws + d.data + (int64_t)r * d.s_r + (int64_t)p0 * d.s_p;
  const int n = d.n;
  const int pe = n * CT;   // elements of one plane's panel
  for (int e = threadIdx.x; e < np * pe; e += 256) {
    const int pp = e / pe, k = (e % pe) / CT, c = e % CT;
    panel[e] = (c0 + c < d.ncols) ? base[(int64_t)pp * d.s_p + (int64_t)k * d.s_k + c0 + c] : mk<R>(0, 0);
  }
  __syncthreads();
  const C* T = tab + d.tab;
  constexpr int RG = 256 / CT;  // output rows handled in parallel
  const int c = threadIdx.x % CT, og = threadIdx.x / CT;
  if (c0 + c >= d.ncols) return;
  for (int q = og; q < np * n; q += RG) {
    const int pp = q / n, o = q % n;
    C acc = mk<R>(0, 0);
    const C* Trow = T + (int64_t)o * n;
    const C* pc = panel + pp * pe + c;
    for (int k = 0; k < n; ++k) acc = cfma(Trow[k], pc[k * CT], acc);
    base[(int64_t)pp * d.s_p + (int64_t)o * d.s_k + c0 + c] = acc;
  }
}

// ---------------------------------------------------------------------------
// Orthonormal DST-I of lines of n = N - 1 points (N = 16 V a power of two,
// 16 <= N <= 512) by one complex FFT of length N.  With x_0 = x_N = 0,
//   y_j = sin(pi j / N) (x_j + x_{N-j}) + (x_j - x_{N-j}) / 2,   Z = FFT_N(y),
// the sums S_k = sum_j x_j sin(pi j k / N) are
//   S_{2m}   = i (Z_m - Z_{N-m}) / 2                           m = 1 .. N/2-1
//   S_{2m+1} = Z_0 / 2 + sum_{m' = 1 .. m} (Z_m' + Z_{N-m'}) / 2   m = 0 .. N/2-1
// (the part of y symmetric about N/2 carries the odd sums, the antisymmetric
// part the even ones; complex x by linearity), and the transform is
// sqrt(2 / N) S_k.  The FFT is split 16 x V: each of 16 lanes per line runs a
// V-point FFT in registers over y[t + 16 v], applies the twiddles W_N^{t k2},
// exchanges through a padded LDS row and finishes with 16-point FFTs over t.
// Lane t then forms the terms of N/32 consecutive m (running sums within the
// lane, the totals of the lanes before it through LDS) and writes S into the
// LDS slots it alone read; the lines are stored from there.  A workgroup
// stages whole lines, so the same kernel serves contiguous x lines and
// strided y lines, in place.
// ---------------------------------------------------------------------------
constexpr int TW_N = 1024;   // tw[k] = exp(-2 pi i k / 1024)

__host__ __device__ constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }
__host__ __device__ constexpr int bitrevc(int i, int lg) {
  int r = 0;
  for (int b = 0; b < lg; ++b) r |= ((i >> b) & 1) << (lg - 1 - b);
  return r;
}

// In-place radix-2 decimation-in-time FFT of V register values (natural order in and out).
template <typename C, int V>
__device__ __forceinline__ void fft_reg(C (&a)[V], const C* __restrict__ tw) {
  constexpr int LG = ilog2c(V);
#pragma unroll
  for (int i = 0; i < V; ++i) {
    const int j = bitrevc(i, LG);
    if (j > i) {
      C t = a[i];
      a[i] = a[j];
      a[j] = t;
    }
  }
#pragma unroll
  for (int len = 2; len <= V; len <<= 1) {
#pragma unroll
    for (int i = 0; i < V; i += len) {
#pragma unroll
      for (int k = 0; k < len / 2; ++k) {
        const C u = a[i + k];
        const C v = a[i + k + len / 2];
        C t;
        if (k == 0) {
          t = v;
        } else if (4 * k == len) {  // multiply by -i
          t.x = v.y;
          t.y = -v.x;
        } else {
          t = cmul(v, tw[k * (TW_N / len)]);
        }
        a[i + k] = cadd(u, t);
        a[i + k + len / 2] = csub(u, t);
      }
    }
  }
}

template <typename R, typename CI, typename CO, bool ACC, int V, int LT>
__global__ __launch_bounds__(16 * LT) void k_dst(const DstDesc* __restrict__ descs, const cplx<R>* __restrict__ tw,
                                                 const CI* __restrict__ src, CO* __restrict__ dst) {
  using C = cplx<R>;
  constexpr int N = 16 * V;
  constexpr int n = N - 1;
  constexpr int XS = 17 * V + 1;               // LDS row of a line: entry (k2, k1) at slot 17 k2 + k1
  constexpr int MPL = N >= 32 ? N / 32 : 1;    // terms m per lane in the sums
  constexpr int PL = (N / 2) / MPL;            // lanes holding terms (16; 8 for N = 16)
  extern __shared__ unsigned char dst_smem[];   // row[LT * XS], then tot[LT * 16]
  C* row = reinterpret_cast<C*>(dst_smem);
  C* tot = row + LT * XS;
  const DstDesc d = descs[blockIdx.y];
  const int lines = d.P * d.Q;
  const int l0 = blockIdx.x * LT;
  if (l0 >= lines) return;
  const int r = blockIdx.z;
  // lanes run along a line for contiguous lines (x) and across lines for
  // strided ones (y), so that each group of lanes touches consecutive addresses
  const bool along = d.src_i == 1;
  const int li = along ? int(threadIdx.x >> 4) : int(threadIdx.x % LT);
  const int t = along ? int(threadIdx.x & 15) : int(threadIdx.x / LT);
  const int g = l0 + li;
  const bool ok = g < lines;
  const int gc = ok ? g : lines - 1;   // a valid line for lanes past the end
  const int p = gc / d.Q, q = gc % d.Q;
  const CI* sl = src + d.src + (int64_t)r * d.src_r + (int64_t)p * d.src_p + (int64_t)q * d.src_q;
  // y_j, j = t + 16 v, from x_j (element j - 1) and x_{N-j} (element N - j - 1);
  // j = 0 loads element 0 (unused).  Contiguous lines (a line's lanes in one
  // wave) with V <= 16 load each element once and stage it in the line's LDS
  // row at slot e + e / 16, where the lane of j reads x_{N-j}.  Other lines
  // load x_{N-j} as well: in FP64 after every x_j load is issued (these
  // workgroups are held to two waves per SIMD by their LDS, so the registers
  // that takes cost no occupancy), in FP32 pair by pair (measured faster
  // there).  `along` is uniform over the workgroup.
  C* crow = row + li * XS;
  C a[V];
  auto combine = [&](int v, const C& x1, const C& x2) {
    const int j = t + 16 * v;
    const R sn = -tw[j * (TW_N / (2 * N))].y;   // sin(pi j / N)
    const R on = (ok && j >= 1) ? R(1) : R(0);
    a[v].x = on * fma(sn, x1.x + x2.x, R(0.5) * (x1.x - x2.x));
    a[v].y = on * fma(sn, x1.y + x2.y, R(0.5) * (x1.y - x2.y));
  };
  auto e1_of = [&](int v) { const int j = t + 16 * v; return j >= 1 ? j - 1 : 0; };
  auto e2_of = [&](int v) { const int j = t + 16 * v; return j >= 1 ? N - j - 1 : 0; };
  auto staged = [&]() {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int j = t + 16 * v;
      if (j >= 1) crow[(j - 1) + (j - 1) / 16] = a[v];
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const int e2 = e2_of(v);
      combine(v, a[v], crow[e2 + e2 / 16]);
    }
    __syncthreads();   // every read of the staged line is done before the row is reused
  };
  if constexpr (sizeof(R) == 8) {
#pragma unroll
    for (int v = 0; v < V; ++v) a[v] = cvt<C>(sl[(int64_t)e1_of(v) * d.src_i]);
    if (V <= 16 && along) {
      staged();
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) combine(v, a[v], cvt<C>(sl[(int64_t)e2_of(v) * d.src_i]));
    }
  } else {
    if (V <= 16 && along) {
#pragma unroll
      for (int v = 0; v < V; ++v) a[v] = cvt<C>(sl[(int64_t)e1_of(v) * d.src_i]);
      staged();
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const C x1 = cvt<C>(sl[(int64_t)e1_of(v) * d.src_i]);
        const C x2 = cvt<C>(sl[(int64_t)e2_of(v) * d.src_i]);
        combine(v, x1, x2);
      }
    }
  }
  fft_reg<C, V>(a, tw);
#pragma unroll
  for (int k2 = 1; k2 < V; ++k2) a[k2] = cmul(a[k2], tw[((t * k2) % N) * (TW_N / N)]);
#pragma unroll
  for (int k2 = 0; k2 < V; ++k2) crow[k2 * 17 + t] = a[k2];
  __syncthreads();
  // 16-point FFTs over t; Z_{k2 + V k1} goes back to the slots just read
  constexpr int G = V >= 16 ? V / 16 : 1;
#pragma unroll
  for (int gg = 0; gg < G; ++gg) {
    const int k2 = t + 16 * gg;
    if (k2 < V) {
      C b[16];
#pragma unroll
      for (int k1 = 0; k1 < 16; ++k1) b[k1] = crow[k2 * 17 + k1];
      fft_reg<C, 16>(b, tw);
#pragma unroll
      for (int k1 = 0; k1 < 16; ++k1) crow[k2 * 17 + k1] = b[k1];
    }
  }
  __syncthreads();
  auto zslot = [](int m) { return (m % V) * 17 + m / V; };
  // terms of m = t MPL .. t MPL + MPL - 1: running sums of the odd outputs;
  // the even outputs S_{2m} go straight to the slot of Z_{N-m} (read by this
  // lane only)
  C cs[MPL];
  C run = mk<R>(0, 0);
  if (t < PL) {
#pragma unroll
    for (int i = 0; i < MPL; ++i) {
      const int m = t * MPL + i;
      const C zm = crow[zslot(m)];
      C c;
      if (m == 0) {
        c.x = R(0.5) * zm.x;
        c.y = R(0.5) * zm.y;
      } else {
        const C zn = crow[zslot(N - m)];
        c.x = R(0.5) * (zm.x + zn.x);
        c.y = R(0.5) * (zm.y + zn.y);
        C e;
        e.x = R(0.5) * (zn.y - zm.y);
        e.y = R(0.5) * (zm.x - zn.x);
        crow[zslot(N - m)] = e;
      }
      run = cadd(run, c);
      cs[i] = run;
    }
  }
  tot[li * 16 + t] = t < PL ? run : mk<R>(0, 0);
  __syncthreads();
  if (t < PL) {
    C off = mk<R>(0, 0);
    for (int u = 0; u < t; ++u) off = cadd(off, tot[li * 16 + u]);
#pragma unroll
    for (int i = 0; i < MPL; ++i) crow[zslot(t * MPL + i)] = cadd(cs[i], off);
  }
  __syncthreads();
  if (!ok) return;
  const R sc = R(sqrt(2.0 / double(N)));
  CO* dl = dst + d.dst + (int64_t)r * d.dst_r + (int64_t)p * d.dst_p + (int64_t)q * d.dst_q;
#pragma unroll
  for (int c = 0; c < V; ++c) {
    const int k = t + 16 * c;
    if (k >= 1 && k <= n) {
      const C v = crow[(k & 1) ? zslot(k >> 1) : zslot(N - (k >> 1))];
      C o;
      o.x = sc * v.x;
      o.y = sc * v.y;
      CO* ptr = dl + (int64_t)(k - 1) * d.dst_i;
      if (ACC) {
        CO pv = *ptr;
        pv.x += o.x;
        pv.y += o.y;
        *ptr = pv;
      } else {
        *ptr = cvt<CO>(o);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Batched z solves: for every (a, b) mode of a block one tridiagonal system
// (Dz - diag k^2 + (lam_a + mu_b) I) x = rhs in z (eq. (5)), solved by
// Gaussian elimination without pivoting.
//
// Partitioned form, everything in registers: a workgroup takes MW modes and
// splits each mode's z line into P chunks, one lane per (mode, chunk).
//  1. Each chunk eliminates its own rows top-down and bottom-up, which gives
//     the chunk's response at its first and last row to its right-hand side
//     (y) and to unit values of the neighbouring unknowns above (v) and
//     below (w):  x_k = y_k - lo_{k0} v_k x_{k0-1} - up_{k1} w_k x_{k1+1}.
//  2. One lane per mode solves the reduced system on the chunk ends
//     (first F_j, last L_j), a block recurrence of 2 x 2 structure.
//  3. Each chunk re-solves its rows with the now known x_{k0-1}, x_{k1+1}.
// Reads the right-hand side once and writes the solution once.
// ---------------------------------------------------------------------------
template <typename R> struct quad_of;
template <> struct quad_of<double> { using type = double4; };
template <> struct quad_of<float> { using type = float4; };

template <typename C>
__device__ __forceinline__ C shfl_xor_c(C v, int mask, int width) {
  C o;
  o.x = __shfl_xor(v.x, mask, width);
  o.y = __shfl_xor(v.y, mask, width);
  return o;
}

// 1/z for pivots (|z| bounded away from 0 and infinity by the plan's pivot
// scan): hardware reciprocal of |z|^2 refined by Newton steps.
__device__ __forceinline__ double rcp_refined(double n) {
  double r = __builtin_amdgcn_rcp(n);
  double e = fma(-n, r, 1.0);
  r = fma(r, e, r);
  e = fma(-n, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float rcp_refined(float n) {
  float r = __builtin_amdgcn_rcpf(n);
  const float e = fmaf(-n, r, 1.0f);
  return fmaf(r, e, r);
}
template <typename C>
__device__ __forceinline__ C crcp_fast(C z) {
  const auto inv = rcp_refined(z.x * z.x + z.y * z.y);
  C r;
  r.x = z.x * inv;
  r.y = -z.y * inv;
  return r;
}

constexpr int PS_LMAX = 16;   // most rows per chunk held in registers
// Register rows L of a kernel instance: 8 where the chunks are that short (half
// the registers, twice the resident waves), else PS_LMAX.
__host__ __device__ __forceinline__ int psweep_regrows(int lc) { return lc <= 8 ? 8 : PS_LMAX; }

// Rows of a chunk: every chunk of a line has the same length, so that loop
// bounds are uniform across the workgroup; the line is padded past nz.
__host__ __device__ __forceinline__ int psweep_rows(int nz, int chunks) {
  const int l = (nz + chunks - 1) / chunks;
  return l < 2 ? 2 : l;
}

// Padded rows past the end of a line have zero couplings and a large real
// diagonal: they never influence real rows, and their (finite) values are
// discarded.
constexpr double kPadDiag = 1099511627776.0;   // 2^40

// Workgroups of a launch are dealt to the 8 XCDs in turn (each XCD has its own
// L2). xcd_linear renumbers workgroup i of n so that every XCD takes one
// contiguous range of the new numbers (a permutation of 0..n-1).
__host__ __device__ __forceinline__ int xcd_linear(int i, int n) {
  const int q = n >> 3, rm = n & 7, x = i & 7;
  return x * q + (x < rm ? x : rm) + (i >> 3);
}

// Modes of a workgroup. A solve whose right-hand side is only low-rank terms
// (no dense input) on rows of at least MW modes: tile t covers modes
// a0 .. a0 + MW - 1 of one row b (t = column band * nb + b), and the tiles are
// renumbered so that an XCD takes whole column bands, whose y-type low-rank
// lines then stay in its L2 while it walks the rows. Otherwise MW consecutive
// modes of the plane: workgroups in flight then read one contiguous stretch
// of a dense input, which HBM serves better than scattered rows.
struct SweepTile {
  bool two_d;      // one row of the plane
  int64_t m0;      // first mode
  int a0, b;       // first column and row (tiles)
};
__host__ __device__ __forceinline__ bool psweep_two_d(const SweepDesc& d, int mw) {
  return !d.dense_in && d.na >= mw;
}
__host__ __device__ __forceinline__ int64_t psweep_tiles(const SweepDesc& d, int mw) {
  return psweep_two_d(d, mw) ? (int64_t)d.nb * ((d.na + mw - 1) / mw) : ((int64_t)d.rs * d.nb + mw - 1) / mw;
}
// tile of workgroup wg < tiles
__host__ __device__ __forceinline__ SweepTile psweep_tile(const SweepDesc& d, int mw, int tiles, int wg) {
  const int nb = d.nb, na = d.na;
  SweepTile st;
  st.two_d = psweep_two_d(d, mw);
  if (st.two_d) {
    const int t = xcd_linear(wg, tiles);
    st.a0 = (t / nb) * mw;
    st.b = t % nb;
    st.m0 = (int64_t)st.b * d.rs + st.a0;
  } else {
    st.m0 = (int64_t)wg * mw;
    st.a0 = 0;
    st.b = 0;
  }
  return st;
}
// mode ml (< mw) of a tile, numbered m = b*rs + a (its offset in a plane):
// false past the row (tiles), in a row's padding or past the plane
__host__ __device__ __forceinline__ bool psweep_mode(const SweepDesc& d, const SweepTile& t, int ml, int64_t& m) {
  const int64_t mm = t.m0 + ml;
  const bool on = t.two_d ? t.a0 + ml < d.na : mm < (int64_t)d.rs * d.nb && int(mm % d.rs) < d.na;
  m = on ? mm : 0;
  return on;
}

// RS: storage precision of the workspace arrays; R: arithmetic precision and
// precision of the tables `tab`.
//
// One workgroup solves MW modes; each mode's z line is cut into P chunks of
// Lc rows, one lane per chunk:
//  1. per chunk, a top-down elimination (keeping the reciprocal pivots) gives
//     the local solution, the response to a unit value in the first row and
//     the response to a unit value in the last row, at the last row; a
//     bottom-up elimination gives the same three at the first row;
//  2. one lane per mode solves the reduced system on the chunk end values;
//  3. every chunk is solved again with its neighbours' end values moved to the
//     right-hand side, with the stored pivots (no divisions).
// FULL: every chunk has exactly L rows (known at compile time, so the row
// loops have no bounds to test and the scheduler can overlap the rows'
// independent work); otherwise Lc <= L rows from nz.
template <typename RS, typename R, int P, int MW, int L, bool FULL>
__device__ __forceinline__ void psweep_body(const SweepDesc& d, const cplx<R>* __restrict__ tab,
                                            cplx<RS>* __restrict__ ws, unsigned char* smem_raw, int xcap,
                                            const SweepTile& tile) {
  using C = cplx<R>;
  using CS = cplx<RS>;
  using Q = typename quad_of<R>::type;
  const int na = d.na, nb = d.nb, nz = d.nz;
  const int64_t plane = d.plane;
  const int Lc = FULL ? L : psweep_rows(nz, P);
  const int nzp = P * Lc;
  Q* zt = reinterpret_cast<Q*>(smem_raw);   // (dg.x, dg.y, lo, up) per z, padded to nzp rows
  R* zs = reinterpret_cast<R*>(smem_raw + size_t(nzp) * sizeof(Q));   // sigma per z (scales the shift)
  C* xch = reinterpret_cast<C*>(smem_raw + ((size_t(nzp) * (sizeof(Q) + sizeof(R)) + 255) / 256) * 256);   // [P][6][MW]
  C* gxs = xch + 6 * P * MW;                 // x-type term lines [t][2 rows b][nzp]
  for (int k = threadIdx.x; k < nzp; k += 256) {
    Q q;
    if (k < nz) {
      const C dg = tab[d.zdiag + k];
      q.x = dg.x;
      q.y = dg.y;
      q.z = tab[d.zlo + k].x;
      q.w = k + 1 < nz ? tab[d.zup + k].x : R(0);
    } else {
      q.x = R(kPadDiag);
      q.y = R(0);
      q.z = R(0);
      q.w = R(0);
    }
    zt[k] = q;
    zs[k] = k < nz ? tab[d.zsig + k].x : R(0);
  }
  // The x-type low-rank terms G_t(b, z) are shared by every mode of a row b;
  // consecutive modes lie on at most two rows when na >= MW, whose lines are
  // staged in LDS once (rows past the line hold the last row). Staging pays
  // where a dense right-hand side is read as well (its loads overlap); without
  // one the extra round trip costs more than it saves.
  const int r = blockIdx.z;
  const int b_lo = int(tile.m0 / d.rs);
  const bool xstage = d.dense_in && d.nxt > 0 && na >= MW && 2 * d.nxt * nzp <= xcap;
  if (xstage) {
#pragma unroll
    for (int t = 0; t < kMaxTerms; ++t) {
      if (t < d.nxt) {
        const CS* g = ws + d.gx[t] + (int64_t)r * d.gx_r;
        for (int i = threadIdx.x; i < 2 * nzp; i += 256) {
          const int br = min(b_lo + i / nzp, nb - 1), k = min(i % nzp, nz - 1);
          gxs[t * 2 * nzp + i] = cvt<C>(g[br + (int64_t)k * d.gx_z]);
        }
      }
    }
  }
  const int ml = threadIdx.x % MW, j = threadIdx.x / MW;
  int64_t m;
  const bool mact = psweep_mode(d, tile, ml, m);
  const int k0 = j * Lc;
  // rows addressed in memory: kb .. kb + nv - 1 (clamped into the line)
  const int kb = k0 < nz ? k0 : nz - 1;
  const int nv = k0 < nz ? min(nz - k0, Lc) : 1;
  const int a = int(m % d.rs), b = int(m / d.rs);
  const C s = mact ? cadd(tab[d.lam_x + a], tab[d.lam_y + b]) : mk<R>(1, 0);
  auto X = [&](int f, int jj) -> C& { return xch[(jj * 6 + f) * MW + ml]; };

  // right-hand side of the chunk. Every register row is loaded, rows past the
  // chunk or the line from the last valid row: their values only reach rows
  // that are never used or padded rows. Row offsets fit in 32 bits (at most
  // 15 planes past the chunk's first row; plans hold at most 2^28 modes per
  // plane).
  C rb[L];
  auto row_off = [&](int kk, uint32_t stride) -> uint32_t {
    return kk < nv ? uint32_t(kk) * stride : uint32_t(nv - 1) * stride;
  };
  if (d.dense_in) {
    const CS* src = ws + d.data + (int64_t)r * d.data_r + m + (int64_t)kb * plane;
#pragma unroll
    for (int kk = 0; kk < L; ++kk) rb[kk] = cvt<C>(src[row_off(kk, uint32_t(plane))]);
  } else {
#pragma unroll
    for (int kk = 0; kk < L; ++kk) rb[kk] = mk<R>(0, 0);
  }
  // low-rank terms: coefficient of the mode times a line shared by a row of
  // modes; staged x-type lines are added after the barrier
#pragma unroll
  for (int i = 0; i < 2 * kMaxTerms; ++i) {
    const bool isx = i < kMaxTerms;
    const int t = isx ? i : i - kMaxTerms;
    if (t < (isx ? d.nxt : d.nyt) && !(isx && xstage)) {
      const C c = isx ? tab[d.colx[t] + (int64_t)a * d.colx_stride[t]]
                      : tab[d.coly[t] + (int64_t)b * d.coly_stride[t]];
      const int64_t gz = isx ? d.gx_z : d.gy_z;
      const CS* g = (isx ? ws + d.gx[t] + (int64_t)r * d.gx_r + b : ws + d.gy[t] + (int64_t)r * d.gy_r + a) +
                    (int64_t)kb * gz;
#pragma unroll
      for (int kk = 0; kk < L; ++kk) rb[kk] = cfma(c, cvt<C>(g[row_off(kk, uint32_t(gz))]), rb[kk]);
    }
  }
  __syncthreads();
  if (xstage) {
    const int brow = mact ? b - b_lo : 0;
#pragma unroll
    for (int t = 0; t < kMaxTerms; ++t) {
      if (t < d.nxt) {
        const C c = tab[d.colx[t] + (int64_t)a * d.colx_stride[t]];
        const C* gl = gxs + (t * 2 + brow) * nzp;
#pragma unroll
        for (int kk = 0; kk < L; ++kk) rb[kk] = cfma(c, gl[min(k0 + kk, nzp - 1)], rb[kk]);
      }
    }
  }

  // 1. local eliminations: y (local solution), v (unit value in the first
  // row), w (unit value in the last row) at the chunk's last row (top-down)
  // and first row (bottom-up)
  C ip[L];
  C yl = mk<R>(0, 0), vl = mk<R>(0, 0), wl = mk<R>(0, 0);
  C yf = mk<R>(0, 0), vf = mk<R>(0, 0), wf = mk<R>(0, 0);
  {
    C cp = mk<R>(0, 0);
#pragma unroll
    for (int kk = 0; kk < L; ++kk) {
      if (kk < Lc) {
        const Q q = zt[k0 + kk];
        const R sg = zs[k0 + kk];
        C piv;
        piv.x = fma(sg, s.x, q.x) - q.z * cp.x;
        piv.y = fma(sg, s.y, q.y) - q.z * cp.y;
        const C ipk = crcp_fast(piv);
        ip[kk] = ipk;
        C t;
        t.x = rb[kk].x - q.z * yl.x;
        t.y = rb[kk].y - q.z * yl.y;
        yl = cmul(t, ipk);
        t.x = (kk == 0 ? R(1) : R(0)) - q.z * vl.x;
        t.y = -q.z * vl.y;
        vl = cmul(t, ipk);
        cp.x = q.w * ipk.x;
        cp.y = q.w * ipk.y;
        wl = ipk;
      }
    }
    C cn = mk<R>(0, 0);
#pragma unroll
    for (int kk = L - 1; kk >= 0; --kk) {
      if (kk < Lc) {
        const Q q = zt[k0 + kk];
        const R sg = zs[k0 + kk];
        C piv;
        piv.x = fma(sg, s.x, q.x) - q.w * cn.x;
        piv.y = fma(sg, s.y, q.y) - q.w * cn.y;
        const C ipk = crcp_fast(piv);
        C t;
        t.x = rb[kk].x - q.w * yf.x;
        t.y = rb[kk].y - q.w * yf.y;
        yf = cmul(t, ipk);
        t.x = (kk == Lc - 1 ? R(1) : R(0)) - q.w * wf.x;
        t.y = -q.w * wf.y;
        wf = cmul(t, ipk);
        cn.x = q.z * ipk.x;
        cn.y = q.z * ipk.y;
        vf = ipk;
      }
    }
  }

  // 2. reduced system on the chunk end values F_j (first) and L_j (last):
  //   F_j = yf_j - al_j vf_j L_{j-1} - be_j wf_j F_{j+1}
  //   L_j = yl_j - al_j vl_j L_{j-1} - be_j wl_j F_{j+1}
  // (al_j: coupling of the chunk's first row to the row before, be_j: of its
  // last row to the row after). Forward elimination gives L_j = p_j + q_j F_{j+1}
  // with q_j = (A_j q_{j-1} + B_j) / (C_j q_{j-1} + 1), a Moebius map carried in
  // homogeneous form (n, d) so that its chain has no divisions; then
  // p_j = alpha_j + beta_j p_{j-1} and F_j = g_j + h_j F_{j+1} are affine
  // chains. The chains run on one lane per mode; every division in between
  // runs on the chunk's own lane.
  const R al = zt[k0].z, be = zt[k0 + Lc - 1].w;
  {
    C Am = csub(cmul(vl, wf), cmul(wl, vf));
    Am.x *= al * be;
    Am.y *= al * be;
    X(0, j) = Am;
    X(1, j) = mk<R>(-be * wl.x, -be * wl.y);
    X(2, j) = mk<R>(al * vf.x, al * vf.y);
  }
  __syncthreads();
  if (j == 0) {
    C n = mk<R>(0, 0), dd = mk<R>(1, 0);
#pragma unroll
    for (int jj = 0; jj < P; ++jj) {
      const C Am = X(0, jj), Bm = X(1, jj), Cm = X(2, jj);
      C n2 = cfma(Bm, dd, cmul(Am, n));
      C d2 = cfma(Cm, n, dd);
      if ((jj & 3) == 3) {
        // rescale by a power of two (the pair is only defined up to a factor)
        const R mag = fabs(n2.x) + fabs(n2.y) + fabs(d2.x) + fabs(d2.y);
        const R sc = mag > R(0) ? ldexp(R(1), -ilogb(mag)) : R(1);
        n2.x *= sc; n2.y *= sc; d2.x *= sc; d2.y *= sc;
      }
      n = n2;
      dd = d2;
      X(3, jj) = n;
      X(4, jj) = dd;
    }
  }
  __syncthreads();
  C qm = mk<R>(0, 0);   // q_{j-1}
  if (j > 0) qm = cmul(X(3, j - 1), crcp_fast(X(4, j - 1)));
  C gy, gp, hj;
  {
    C D = mk<R>(al * vf.x, al * vf.y);
    D = cfma(D, qm, mk<R>(1, 0));                 // 1 + al vf q_{j-1}
    const C iD = crcp_fast(D);
    gy = cmul(yf, iD);
    gp = cmul(vf, iD);
    gp.x *= -al;
    gp.y *= -al;
    hj = cmul(wf, iD);
    hj.x *= -be;
    hj.y *= -be;
    const C alv = mk<R>(-al * vl.x, -al * vl.y);   // -al vl
    X(0, j) = cfma(alv, cmul(qm, gy), yl);          // alpha = yl - al vl q gy
    X(1, j) = cmul(alv, cfma(qm, gp, mk<R>(1, 0)));  // beta = -al vl (1 + q gp)
  }
  __syncthreads();
  if (j == 0) {
    C pp = mk<R>(0, 0);
#pragma unroll
    for (int jj = 0; jj < P; ++jj) {
      pp = cfma(X(1, jj), pp, X(0, jj));
      X(2, jj) = pp;
    }
  }
  __syncthreads();
  const C pm = j > 0 ? X(2, j - 1) : mk<R>(0, 0);   // p_{j-1}
  X(3, j) = cfma(gp, pm, gy);                        // g_j
  X(4, j) = hj;
  __syncthreads();
  if (j == 0) {
    C F = mk<R>(0, 0);
#pragma unroll
    for (int jj = P - 1; jj >= 0; --jj) {
      F = cfma(X(4, jj), F, X(3, jj));
      X(5, jj) = F;
    }
  }
  __syncthreads();

  // 3. re-solve each chunk with its neighbours' end values, reusing the pivots
  {
    const C Fj = X(5, j);
    const C XL = j > 0 ? cfma(qm, Fj, pm) : mk<R>(0, 0);   // L_{j-1} = p_{j-1} + q_{j-1} F_j
    const C XR = j + 1 < P ? X(5, j + 1) : mk<R>(0, 0);   // F_{j+1}
    C dp = mk<R>(0, 0);
#pragma unroll
    for (int kk = 0; kk < L; ++kk) {
      if (kk < Lc) {
        const Q q = zt[k0 + kk];
        C rhs = rb[kk];
        if (kk == 0) rhs = cfms(mk<R>(q.z, 0), XL, rhs);
        if (kk == Lc - 1) rhs = cfms(mk<R>(q.w, 0), XR, rhs);
        C t;
        t.x = rhs.x - q.z * dp.x;
        t.y = rhs.y - q.z * dp.y;
        dp = cmul(t, ip[kk]);
        rb[kk] = dp;
      }
    }
    C xn = mk<R>(0, 0);
#pragma unroll
    for (int kk = L - 1; kk >= 0; --kk) {
      if (kk < Lc) {
        const R up = zt[k0 + kk].w;
        C c;
        c.x = up * ip[kk].x;
        c.y = up * ip[kk].y;
        rb[kk] = cfms(c, xn, rb[kk]);
        xn = rb[kk];
      }
    }
    if (mact) {
      CS* dst = ws + d.out + (int64_t)r * d.out_r + m + (int64_t)k0 * plane;
#pragma unroll
      for (int kk = 0; kk < L; ++kk)
        if (kk < Lc && k0 + kk < nz) {
          // complex128 block solves: the output streams past the reused
          // low-rank lines (non-temporal stores measured faster there only)
          if (sizeof(RS) == 8 && d.dense_in)
            st_stream(dst + (int64_t)kk * plane, cvt<CS>(rb[kk]));
          else
            dst[(int64_t)kk * plane] = cvt<CS>(rb[kk]);
        }
    }
  }
}

// complex128: every workgroup runs the FP64 body. complex64 storage: a
// workgroup holding a mode near resonance (small Re(lam_x + lam_y)) runs its z
// solves in FP64 from the FP64 tables.  The host lists those workgroups once
// per k^2 and chunking (SweepSel): FP64SEL = true launches run exactly the
// listed (descriptor, workgroup) pairs, FP64SEL = false launches skip the
// workgroups whose bit is set and solve the others in FP32.  Every workgroup
// thus runs in exactly one of them, and each kernel gets its own register
// allocation.
template <typename R, int P, int MW, int L, bool FP64SEL, bool FULL>
__global__ __launch_bounds__(256) void k_psweep(const SweepDesc* __restrict__ descs,
                                                const cplx<R>* __restrict__ tab,
                                                const double2* __restrict__ tab64,
                                                cplx<R>* __restrict__ ws, int xcap, SweepSel sel) {
  static_assert(P * MW == 256, "256 lanes per workgroup");
  extern __shared__ unsigned char smem_raw[];
  int di = int(blockIdx.y), wg = int(blockIdx.x);
  if constexpr (FP64SEL) {
    const int2 e = sel.list[blockIdx.x];
    di = e.x;
    wg = e.y;
  } else if (sel.bits && ((sel.bits[(int64_t)di * sel.words + (wg >> 5)] >> (wg & 31)) & 1u)) {
    return;
  }
  const SweepDesc d = descs[di];
  const int64_t tiles = psweep_tiles(d, MW);
  if ((int64_t)wg >= tiles) return;
  const SweepTile tile = psweep_tile(d, MW, int(tiles), wg);
  if constexpr (sizeof(R) == 8 || !FP64SEL)
    psweep_body<R, R, P, MW, L, FULL>(d, tab, ws, smem_raw, xcap, tile);
  else
    psweep_body<R, double, P, MW, L, FULL>(d, tab64, ws, smem_raw, xcap, tile);
}


// v from the lane that DPP control CTRL names (quad permutes, row mirrors,
// row broadcasts); rows outside ROWS get zero.
template <int CTRL, int ROWS, typename R>
__device__ __forceinline__ R dpp_take(R v) {
  return __builtin_amdgcn_update_dpp(R(0), v, CTRL, ROWS, 0xf, false);
}
// Sum of v over aligned groups of L lanes (L a power of two, at most 64; a
// wave-uniform value): pairs, quads, half-rows and rows of 16 by lane
// permutations (every lane of a group of up to 16 then holds its sum), then
// the broadcasts of lane 15 into the next row and of lane 31 into rows 2 and
// 3.  The sum is in the group's last lane in every case.
template <typename C>
__device__ __forceinline__ C group_sum_dpp(C v, int L) {
  if (L > 1) { v.x += dpp_take<0xB1, 0xf>(v.x); v.y += dpp_take<0xB1, 0xf>(v.y); }     // lane ^ 1
  if (L > 2) { v.x += dpp_take<0x4E, 0xf>(v.x); v.y += dpp_take<0x4E, 0xf>(v.y); }     // lane ^ 2
  if (L > 4) { v.x += dpp_take<0x141, 0xf>(v.x); v.y += dpp_take<0x141, 0xf>(v.y); }   // 7 - lane in 8
  if (L > 8) { v.x += dpp_take<0x140, 0xf>(v.x); v.y += dpp_take<0x140, 0xf>(v.y); }   // 15 - lane in 16
  if (L > 16) { v.x += dpp_take<0x142, 0xa>(v.x); v.y += dpp_take<0x142, 0xa>(v.y); }  // lane 15 -> next row
  if (L > 32) { v.x += dpp_take<0x143, 0xc>(v.x); v.y += dpp_take<0x143, 0xc>(v.y); }  // lane 31 -> rows 2, 3
  return v;
}

// Fused contraction over both axes of a plane X(r,z,b,a) (a contiguous): one
// workgroup reads the rows b of one slab of one z plane once and forms
//   out_x,t(b) = sum_a cx_t[a] X(b,a)   (complete in the workgroup)
//   out_y,t(a) = sum_b cy_t[b] X(b,a)   (over the slab's rows)
// A row is spread over L = min(64, pow2 >= na) lanes of a wave, each lane
// holding SMAX >= ceil(na / L) columns; a wave holds 64 / L rows at a time.
// Coefficients are staged in LDS, zero past na, so every lane loads from a
// valid (clamped) column and all loads of U rows are in flight together.
// The x sums of a row reduce over its L lanes by DPP moves (VALU latency,
// where shuffles through the LDS crossbar would each wait a round trip).
// Without prefetching, full-wave rows are first exchanged across 32 and 16
// lanes (transposed: each exchange keeps half of the rows), which spends
// fewer VALU cycles on several terms than one DPP chain per row.
template <typename R, int SMAX, int NT, bool PF>
__global__ __launch_bounds__(256) void k_contract(const ContractDesc* __restrict__ descs, int max_slab, int max_cs,
                                                  const cplx<R>* __restrict__ tab, cplx<R>* __restrict__ ws) {
  using C = cplx<R>;
  constexpr int U = SMAX <= 2 ? 4 : 2;
  constexpr int SW = SMAX * 64;   // LDS stride of one x term
  static_assert(NT <= kMaxContractTerms, "term count");
  extern __shared__ unsigned char smem_raw[];
  const ContractDesc d = descs[blockIdx.y];
  const int z = blockIdx.x / (max_slab * max_cs);
  const int cs = (blockIdx.x / max_slab) % max_cs, slab = blockIdx.x % max_slab;
  if (z >= d.nz || slab >= d.nslab || cs >= d.ncs) return;
  const int r = blockIdx.z;
  const int c0 = cs * d.cols;                      // first column of this column slab
  const int na = min(d.na, c0 + d.cols) - c0;      // its columns
  int L = 1;
  while (L < na && L < 64) L <<= 1;
  const int G = 64 / L;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int la = lane & (L - 1), rg = w * G + lane / L, RG = 4 * G;
  const int b0 = slab * d.rows, nrow = min(d.nb, b0 + d.rows) - b0;
  C* cxs = reinterpret_cast<C*>(smem_raw);   // [nxt][SMAX*64], zero past na
  C* cys = cxs + d.nxt * SW;                 // [nyt][rows]
  C* yb = cys + d.nyt * d.rows;              // [3][NT][64]
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    if (t < d.nxt)
      for (int i = threadIdx.x; i < SW; i += 256)
        cxs[t * SW + i] = i < na ? tab[d.cx[t] + (int64_t)(c0 + i) * d.cx_stride[t]] : mk<R>(0, 0);
    if (t < d.nyt)
      for (int i = threadIdx.x; i < nrow; i += 256) cys[t * d.rows + i] = tab[d.cy[t] + (int64_t)(b0 + i) * d.cy_stride[t]];
  }
  __syncthreads();

  C yacc[SMAX][NT];
#pragma unroll
  for (int s = 0; s < SMAX; ++s)
#pragma unroll
    for (int t = 0; t < NT; ++t) yacc[s][t] = mk<R>(0, 0);
  const C* xp = ws + d.src + (int64_t)r * d.src_r + (int64_t)z * d.plane + (int64_t)b0 * d.rs + c0;
  int col[SMAX];
#pragma unroll
  for (int s = 0; s < SMAX; ++s) col[s] = min(la + s * L, na - 1);
  // x sums of this column slab: final, or a partial added by the second pass
  auto xout = [&](int t) -> int64_t {
    return d.ncs > 1 ? d.xpart + (int64_t)r * d.xpart_r + (int64_t)cs * d.xpart_s + t * d.xpart_t +
                           (int64_t)z * d.xpart_z
                     : d.dx + t * d.dx_t + (int64_t)r * d.dx_r + (int64_t)z * d.dx_z;
  };
  // PF: the rows of the next group load while this group's sums are formed
  C xn[PF ? U : 1][SMAX];
  auto load_rows = [&](int i0, C (&x)[U][SMAX]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t row = (int64_t)min(i0 + u * RG, nrow - 1) * d.rs;
#pragma unroll
      for (int s = 0; s < SMAX; ++s) x[u][s] = xp[row + col[s]];
    }
  };
  if constexpr (PF)
    if (rg < nrow) load_rows(rg, xn);
  for (int i0 = rg; i0 < nrow; i0 += U * RG) {
    C xv[U][SMAX];
    if constexpr (PF) {
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int s = 0; s < SMAX; ++s) xv[u][s] = xn[u][s];
      if (i0 + U * RG < nrow) load_rows(i0 + U * RG, xn);
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t row = (int64_t)min(i0 + u * RG, nrow - 1) * d.rs;
#pragma unroll
        for (int s = 0; s < SMAX; ++s) xv[u][s] = xp[row + col[s]];
      }
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (t < d.nyt) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int bi = i0 + u * RG;
          const C cv = cys[t * d.rows + min(bi, nrow - 1)];
          const C c = bi < nrow ? cv : mk<R>(0, 0);
#pragma unroll
          for (int s = 0; s < SMAX; ++s) yacc[s][t] = cfma(c, xv[u][s], yacc[s][t]);
        }
      }
      if (t < d.nxt) {
        C p[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          p[u] = mk<R>(0, 0);
#pragma unroll
          for (int s = 0; s < SMAX; ++s) p[u] = cfma(cxs[t * SW + la + s * L], xv[u][s], p[u]);
        }
        if (!PF && L == 64) {
          // full-wave rows, reduced together: the exchanges across 32 and 16
          // lanes each keep half of the rows (transposed), then DPP within
          // the rows of 16 lanes
          C v;
          int ur;
          const bool hi5 = (lane & 32) != 0, hi4 = (lane & 16) != 0;
          if constexpr (U == 4) {
            // rows {0,1} stay in the low half-wave, rows {2,3} in the high one
            const C q0 = cadd(hi5 ? p[2] : p[0], shfl_xor_c(hi5 ? p[0] : p[2], 32, 64));
            const C q1 = cadd(hi5 ? p[3] : p[1], shfl_xor_c(hi5 ? p[1] : p[3], 32, 64));
            // row (hi5 ? 2 : 0) + (hi4 ? 1 : 0) stays
            v = cadd(hi4 ? q1 : q0, shfl_xor_c(hi4 ? q0 : q1, 16, 64));
            ur = (hi5 ? 2 : 0) + (hi4 ? 1 : 0);
          } else {
            // row 0 stays in the low half-wave, row 1 in the high one
            v = cadd(hi5 ? p[1] : p[0], shfl_xor_c(hi5 ? p[0] : p[1], 32, 64));
            v = cadd(v, shfl_xor_c(v, 16, 64));
            ur = hi5 ? 1 : 0;
          }
          v = group_sum_dpp(v, 16);
          const int bi = i0 + ur * RG;
          const bool wr = U == 4 ? (lane & 15) == 15 : (lane & 31) == 31;
          if (wr && bi < nrow) ws[xout(t) + b0 + bi] = v;
        } else {
          // each row's sum over its L lanes by DPP moves, in the group's last lane
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const C v = group_sum_dpp(p[u], L);
            const int bi = i0 + u * RG;
            if (la == L - 1 && bi < nrow) ws[xout(t) + b0 + bi] = v;
          }
        }
      }
    }
  }
  // y sums: over the row groups of a wave, then over the four waves (fixed order)
  const int S = (na + L - 1) / L;
#pragma unroll
  for (int m = 1; m < 64; m <<= 1) {
    if (m >= L) {
#pragma unroll
      for (int s = 0; s < SMAX; ++s)
#pragma unroll
        for (int t = 0; t < NT; ++t)
          if (t < d.nyt) yacc[s][t] = cadd(yacc[s][t], shfl_xor_c(yacc[s][t], m, 64));
    }
  }
  const bool split = d.nslab > 1;
#pragma unroll
  for (int s = 0; s < SMAX; ++s) {
    if (s < S && d.nyt > 0) {
      if (w > 0 && lane < L)
#pragma unroll
        for (int t = 0; t < NT; ++t)
          if (t < d.nyt) yb[((w - 1) * NT + t) * 64 + lane] = yacc[s][t];
      __syncthreads();
      const int al = la + s * L;
      const int a = c0 + al;
      if (w == 0 && lane < L && al < na) {
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          if (t < d.nyt) {
            C v = cadd(yacc[s][t], yb[(0 * NT + t) * 64 + lane]);
            v = cadd(v, yb[(1 * NT + t) * 64 + lane]);
            v = cadd(v, yb[(2 * NT + t) * 64 + lane]);
            const int64_t o = split ? d.part + (int64_t)r * d.part_r + (int64_t)slab * d.part_s + t * d.part_t +
                                          (int64_t)z * d.part_z + a
                                    : d.dy + t * d.dy_t + (int64_t)r * d.dy_r + (int64_t)z * d.dy_z + a;
            ws[o] = v;
          }
        }
      }
      __syncthreads();
    }
  }
}

// Slab sums of split planes, added in slab order: y sums over row slabs
// (elements [0, nyt*nz*na)), then x sums over column slabs (the next
// nxt*nz*nb elements).
template <typename R>
__global__ __launch_bounds__(256) void k_contract_fin(const ContractDesc* __restrict__ descs,
                                                      cplx<R>* __restrict__ ws) {
  using C = cplx<R>;
  const ContractDesc d = descs[blockIdx.y];
  const int r = blockIdx.z;
  const int64_t ny_el = d.nslab > 1 ? (int64_t)d.nyt * d.nz * d.na : 0;
  const int64_t nx_el = d.ncs > 1 ? (int64_t)d.nxt * d.nz * d.nb : 0;
  int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < ny_el) {
    const int64_t per_t = (int64_t)d.nz * d.na;
    const int t = int(e / per_t), z = int((e % per_t) / d.na), a = int(e % d.na);
    const C* p = ws + d.part + (int64_t)r * d.part_r + t * d.part_t + (int64_t)z * d.part_z + a;
    C v = p[0];
    for (int s = 1; s < d.nslab; ++s) v = cadd(v, p[(int64_t)s * d.part_s]);
    ws[d.dy + t * d.dy_t + (int64_t)r * d.dy_r + (int64_t)z * d.dy_z + a] = v;
    return;
  }
  e -= ny_el;
  if (e < nx_el) {
    const int64_t per_t = (int64_t)d.nz * d.nb;
    const int t = int(e / per_t), z = int((e % per_t) / d.nb), b = int(e % d.nb);
    const C* p = ws + d.xpart + (int64_t)r * d.xpart_r + t * d.xpart_t + (int64_t)z * d.xpart_z + b;
    C v = p[0];
    for (int c = 1; c < d.ncs; ++c) v = cadd(v, p[(int64_t)c * d.xpart_s]);
    ws[d.dx + t * d.dx_t + (int64_t)r * d.dx_r + (int64_t)z * d.dx_z + b] = v;
  }
}

// Dense spectral right-hand side of the global solve (ExpandDesc): a
// workgroup owns 64 columns a of one z plane and walks its rows b in tiles
// of 16, one row in four per wave.  Terms are taken 16 at a time; the
// per-column factors (cx_i[a], gy_j(a)) and the per-row factors (gx_i(b),
// cy_j[b]) of a chunk are staged in LDS, zero past the term counts.  A
// later chunk adds to what the same thread stored for the element before.
template <typename R>
__global__ __launch_bounds__(256) void k_expand(ExpandDesc e, const cplx<R>* __restrict__ tab,
                                                cplx<R>* __restrict__ ws) {
  using C = cplx<R>;
  constexpr int TC = 16, TB = 16;
  __shared__ C colf[2][TC][64];
  __shared__ C rowf[2][TC][TB];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int a0 = blockIdx.x * 64, z = blockIdx.y, r = blockIdx.z;
  const int a = min(a0 + lane, e.na - 1);
  const bool aok = a0 + lane < e.na;
  const C* gx = ws + e.gx + (int64_t)r * e.gx_r + (int64_t)z * e.gx_z;
  const C* gy = ws + e.gy + (int64_t)r * e.gy_r + (int64_t)z * e.gy_z;
  C* out = ws + e.out + (int64_t)r * e.out_r + (int64_t)z * e.plane;
  const int nch = (max(e.nxt, e.nyt) + TC - 1) / TC;
  for (int ch = 0; ch < nch; ++ch) {
    const int t0 = ch * TC;
    const int nx = min(max(e.nxt - t0, 0), TC), ny = min(max(e.nyt - t0, 0), TC);
    const int nt = max(nx, ny);
    __syncthreads();
    for (int i = threadIdx.x; i < TC * 64; i += 256) {
      const int t = i / 64, l = i % 64;
      const int aa = min(a0 + l, e.na - 1);
      colf[0][t][l] = t < nx ? tab[e.cx + (int64_t)(t0 + t) * e.na + aa] : mk<R>(0, 0);
      colf[1][t][l] = t < ny ? gy[(int64_t)(t0 + t) * e.gy_t + aa] : mk<R>(0, 0);
    }
    for (int b0 = 0; b0 < e.nb; b0 += TB) {
      __syncthreads();
      for (int i = threadIdx.x; i < 2 * TC * TB; i += 256) {
        const int sd = i / (TC * TB), t = (i / TB) % TC, q = i % TB;
        const int bb = min(b0 + q, e.nb - 1);
        C v = mk<R>(0, 0);
        if (sd == 0 && t < nx) v = gx[(int64_t)(t0 + t) * e.gx_t + bb];
        if (sd == 1 && t < ny) v = tab[e.cy + (int64_t)(t0 + t) * e.nb + bb];
        rowf[sd][t][q] = v;
      }
      __syncthreads();
      C acc[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int b = b0 + w * 4 + q;
        acc[q] = ch > 0 && aok && b < e.nb ? out[(int64_t)b * e.rs + a] : mk<R>(0, 0);
      }
      for (int t = 0; t < nt; ++t) {
        const C cxv = colf[0][t][lane], gyv = colf[1][t][lane];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          acc[q] = cfma(cxv, rowf[0][t][w * 4 + q], acc[q]);
          acc[q] = cfma(rowf[1][t][w * 4 + q], gyv, acc[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int b = b0 + w * 4 + q;
        if (aok && b < e.nb) out[(int64_t)b * e.rs + a] = acc[q];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Nested partitions (step 5 solved by a coarser plan): the residual on the
// separator lines scattered onto a zeroed grid array F(r,z,y,x) (crossings
// from the x lines, whose residual holds them), and the coarser plan's
// solution W read back onto the lines.
// ---------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_ml_zero(cplx<R>* __restrict__ F, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) F[i] = mk<R>(0, 0);
}

template <typename R>
__global__ __launch_bounds__(256) void k_ml_scatter(SigmaGeom g, const cplx<R>* __restrict__ ws,
                                                    cplx<R>* __restrict__ F) {
  const int r = blockIdx.z;
  const int64_t nline_x = (int64_t)g.nsx * g.nz * g.NY;
  const int64_t nline_y = (int64_t)g.nsy * g.nz * g.NX;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  cplx<R>* Fr = F + (int64_t)r * g.f_r;
  if (e < nline_x) {
    const int y = int(e % g.NY);
    const int z = int((e / g.NY) % g.nz);
    const int si = int(e / ((int64_t)g.NY * g.nz));
    Fr[((int64_t)z * g.NY + y) * g.NX + g.sep_x[si]] = ws[g.rx + (((int64_t)r * g.nsx + si) * g.nz + z) * g.NY + y];
  } else if (e < nline_x + nline_y) {
    const int64_t e2 = e - nline_x;
    const int x = int(e2 % g.NX);
    if (g.xblk[x] < 0) return;
    const int z = int((e2 / g.NX) % g.nz);
    const int ti = int(e2 / ((int64_t)g.NX * g.nz));
    Fr[((int64_t)z * g.NY + g.sep_y[ti]) * g.NX + x] = ws[g.ry + (((int64_t)r * g.nsy + ti) * g.nz + z) * g.NX + x];
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_ml_gather(SigmaGeom g, const double2* __restrict__ W,
                                                   cplx<R>* __restrict__ ws) {
  const int r = blockIdx.z;
  const int64_t nline_x = (int64_t)g.nsx * g.nz * g.NY;
  const int64_t nline_y = (int64_t)g.nsy * g.nz * g.NX;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const double2* Wr = W + (int64_t)r * g.f_r;
  if (e < nline_x) {
    const int y = int(e % g.NY);
    const int z = int((e / g.NY) % g.nz);
    const int si = int(e / ((int64_t)g.NY * g.nz));
    ws[g.wx + (((int64_t)r * g.nsx + si) * g.nz + z) * g.NY + y] =
        cvt<cplx<R>>(Wr[((int64_t)z * g.NY + y) * g.NX + g.sep_x[si]]);
  } else if (e < nline_x + nline_y) {
    const int64_t e2 = e - nline_x;
    const int x = int(e2 % g.NX);
    const int z = int((e2 / g.NX) % g.nz);
    const int ti = int(e2 / ((int64_t)g.NX * g.nz));
    ws[g.wy + (((int64_t)r * g.nsy + ti) * g.nz + z) * g.NX + x] =
        cvt<cplx<R>>(Wr[((int64_t)z * g.NY + g.sep_y[ti]) * g.NX + x]);
  }
}

// ---------------------------------------------------------------------------
// Interface kernels (steps 3-6 of the two-level reduction)
// ---------------------------------------------------------------------------

// Step 4: residual on the separator lines.
//  rx(s, y, z) = f(s,y,z) + cl_s v(s-1,y,z) + cr_s v(s+1,y,z)   (y not a separator; else f)
//  ry(t, x, z) = f(x,t,z) + cb_t v(x,t-1,z) + ct_t v(x,t+1,z)   (x not a separator; else 0)
// v next to a separator is read from the face arrays of the neighbouring blocks.
template <typename R, typename CI>
__global__ __launch_bounds__(256) void k_sigma_resid(SigmaGeom g, const CI* __restrict__ f,
                                                     cplx<R>* __restrict__ ws) {
  using C = cplx<R>;
  const int r = blockIdx.z;
  const int64_t nline_x = (int64_t)g.nsx * g.nz * g.NY;
  const int64_t nline_y = (int64_t)g.nsy * g.nz * g.NX;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const CI* fr = f + (int64_t)r * g.f_r;
  const C* coef = reinterpret_cast<const C*>(g.coef);
  if (e < nline_x) {
    const int y = int(e % g.NY);
    const int z = int((e / g.NY) % g.nz);
    const int si = int(e / ((int64_t)g.NY * g.nz));
    const int s = g.sep_x[si];
    C v = cvt<C>(fr[((int64_t)z * g.NY + y) * g.NX + s]);
    const int jb = g.yblk[y];
    if (jb >= 0) {
      const int yl = g.yloc[y];
      // left neighbour block (column si), its right face; right block (si+1), left face
      const int bl = jb * g.nbx_blocks + si;
      const int br = jb * g.nbx_blocks + si + 1;
      const C vl = ws[g.face + (((int64_t)bl * g.rmax + r) * 4 + 1) * g.face_f + (int64_t)z * g.NF + yl];
      const C vr = ws[g.face + (((int64_t)br * g.rmax + r) * 4 + 0) * g.face_f + (int64_t)z * g.NF + yl];
      const R sg = coef[g.zsig + z].x;
      v = cfma(cscale(coef[g.cx_lo + si], sg), vl, v);
      v = cfma(cscale(coef[g.cx_hi + si], sg), vr, v);
    }
    ws[g.rx + (((int64_t)r * g.nsx + si) * g.nz + z) * g.NY + y] = v;
  } else if (e < nline_x + nline_y) {
    const int64_t e2 = e - nline_x;
    const int x = int(e2 % g.NX);
    const int z = int((e2 / g.NX) % g.nz);
    const int ti = int(e2 / ((int64_t)g.NX * g.nz));
    const int t = g.sep_y[ti];
    C v = mk<R>(0, 0);
    const int ib = g.xblk[x];
    if (ib >= 0) {
      v = cvt<C>(fr[((int64_t)z * g.NY + t) * g.NX + x]);
      const int xl = g.xloc[x];
      const int bb = ti * g.nbx_blocks + ib;        // block below (row ti), its top face
      const int bt = (ti + 1) * g.nbx_blocks + ib;  // block above, its bottom face
      const C vb = ws[g.face + (((int64_t)bb * g.rmax + r) * 4 + 3) * g.face_f + (int64_t)z * g.NF + xl];
      const C vt = ws[g.face + (((int64_t)bt * g.rmax + r) * 4 + 2) * g.face_f + (int64_t)z * g.NF + xl];
      const R sg = coef[g.zsig + z].x;
      v = cfma(cscale(coef[g.cy_lo + ti], sg), vb, v);
      v = cfma(cscale(coef[g.cy_hi + ti], sg), vt, v);
    }
    ws[g.ry + (((int64_t)r * g.nsy + ti) * g.nz + z) * g.NX + x] = v;
  }
}

// Step 6 (lift): the Dirichlet data w on the separators enter the first and
// last interior lines of each block as g = -A_{I,Sigma} w_Sigma.
// face order: 0 = low x (left), 1 = high x (right), 2 = low y, 3 = high y.
template <typename R>
__global__ __launch_bounds__(256) void k_lift(SigmaGeom g, const LiftBlock* __restrict__ lb,
                                              cplx<R>* __restrict__ ws) {
  using C = cplx<R>;
  // B's two-entry arrays are read through selects below: a run-time index
  // into them would place B in scratch memory
  const LiftBlock B = lb[blockIdx.y];
  const int r = blockIdx.z;
  const int64_t per_face = (int64_t)g.nz * g.NF;
  const C* coef = reinterpret_cast<const C*>(g.coef);
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < 4 * per_face; e += (int64_t)gridDim.x * 256) {
    const int face = int(e / per_face);
    const int z = int((e % per_face) / g.NF);
    const int i = int(e % g.NF);
    C v = mk<R>(0, 0);
    const R sg = coef[g.zsig + z].x;   // sigma of the plane scales the x / y couplings
    if (face < 2) {
      const int si = face == 0 ? B.sep_lo_x : B.sep_hi_x;
      if (si >= 0 && i < B.nby)
        v = cmul(cscale(coef[face == 0 ? B.cfx[0] : B.cfx[1]], sg),
                 ws[g.wx + (((int64_t)r * g.nsx + si) * g.nz + z) * g.NY + B.y0 + i]);
    } else {
      const int ti = face == 2 ? B.sep_lo_y : B.sep_hi_y;
      if (ti >= 0 && i < B.nbx)
        v = cmul(cscale(coef[face == 2 ? B.cfy[0] : B.cfy[1]], sg),
                 ws[g.wy + (((int64_t)r * g.nsy + ti) * g.nz + z) * g.NX + B.x0 + i]);
    }
    ws[g.gface + (((int64_t)blockIdx.y * g.rmax + r) * 4 + face) * g.face_f + (int64_t)z * g.NF + i] = v;
  }
}

// Step 7 on the separators: u = w there (crossings from the x lines).
template <typename R, typename CO, bool ACC>
__global__ __launch_bounds__(256) void k_sigma_scatter(SigmaGeom g, const cplx<R>* __restrict__ ws,
                                                       CO* __restrict__ u) {
  const int r = blockIdx.z;
  const int64_t nline_x = (int64_t)g.nsx * g.nz * g.NY;
  const int64_t nline_y = (int64_t)g.nsy * g.nz * g.NX;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  CO* ur = u + (int64_t)r * g.f_r;
  int64_t dst;
  cplx<R> v;
  if (e < nline_x) {
    const int y = int(e % g.NY);
    const int z = int((e / g.NY) % g.nz);
    const int si = int(e / ((int64_t)g.NY * g.nz));
    dst = ((int64_t)z * g.NY + y) * g.NX + g.sep_x[si];
    v = ws[g.wx + (((int64_t)r * g.nsx + si) * g.nz + z) * g.NY + y];
  } else if (e < nline_x + nline_y) {
    const int64_t e2 = e - nline_x;
    const int x = int(e2 % g.NX);
    if (g.xblk[x] < 0) return;
    const int z = int((e2 / g.NX) % g.nz);
    const int ti = int(e2 / ((int64_t)g.NX * g.nz));
    dst = ((int64_t)z * g.NY + g.sep_y[ti]) * g.NX + x;
    v = ws[g.wy + (((int64_t)r * g.nsy + ti) * g.nz + z) * g.NX + x];
  } else {
    return;
  }
  if (ACC) {
    CO p = ur[dst];
    p.x += v.x;
    p.y += v.y;
    ur[dst] = p;
  } else {
    ur[dst] = cvt<CO>(v);
  }
}

// ---------------------------------------------------------------------------
// FP64 residual r = f - A u with the 7-point stencil of eq. (2) (D-form).
// ---------------------------------------------------------------------------
// Residual r = f - A u (or A u) of the 7-point operator in FP64.  A
// workgroup owns a 64 (x) x 4 (y) tile of columns and marches along a chunk
// of z: u at z - 1 and z stay in registers, u at z + 1 is the one new HBM
// read per point, and the x / y neighbours of plane z come through L1 (the
// tile reads them itself).  No barriers, so the unrolled march keeps several
// planes of loads in flight.  Outside the grid u counts as zero (Dirichlet),
// which drops the boundary terms; the terms are summed in the order centre,
// x-1, x+1, y-1, y+1, z-1, z+1.
constexpr int RZ_TX = 64, RZ_TY = 4, RZ_ZC = 32;

// p[0] where c holds, else zero.  Returned by value: a conditional between
// the load and a named zero would be an lvalue, which clang lowers to one
// flat load from a select of the global address and a stack slot.
__device__ __forceinline__ double2 load_or_zero(bool c, const double2* p) {
  double2 v = mk<double>(0, 0);
  if (c) v = *p;
  return v;
}

// part (may be NULL): per workgroup, the sums of |r|^2, |f|^2 and |u|^2 over
// its points (three doubles at part + 3 * workgroup index, workgroups
// numbered x fastest, then z chunk, then right-hand side); write_out = 0
// evaluates those sums without storing r.
// Workgroup (bx, by, bz) of a grid (gx, gy, nrhs): column tile bx, z chunk by,
// right-hand side bz.
template <typename CO>
__device__ __forceinline__ void residual_body(const StencilGeom& g, const double2* __restrict__ f,
                                              const double2* __restrict__ u, CO* __restrict__ out, int negate_f,
                                              double* __restrict__ part, int write_out, int bx, int by, int bz,
                                              int gx, int gy) {
  const int tx = threadIdx.x & (RZ_TX - 1), ty = threadIdx.x / RZ_TX;
  const int xt = (g.nx + RZ_TX - 1) / RZ_TX;
  const int x = (bx % xt) * RZ_TX + tx, y = (bx / xt) * RZ_TY + ty;
  double rr = 0, ff = 0, uu = 0;
  if (x < g.nx && y < g.ny) {
    const int z0 = by * RZ_ZC, z1 = min(g.nz, z0 + RZ_ZC);
    const int64_t sy = g.nx, sz = (int64_t)g.nx * g.ny;
    const double2* uc0 = u + (int64_t)bz * sz * g.nz + (int64_t)y * sy + x;   // column (x, y)
    const int64_t col = uc0 - u;
    const double2 cxd = g.xd[x], cyd = g.yd[y];
    const double2 cxl = g.xl[x], cxu = g.xu[x], cyl = g.yl[y], cyu = g.yu[y];
    const bool hx0 = x > 0, hx1 = x + 1 < g.nx, hy0 = y > 0, hy1 = y + 1 < g.ny;
    double2 um = load_or_zero(z0 > 0, uc0 + (int64_t)(z0 - 1) * sz);
    double2 uc = uc0[(int64_t)z0 * sz];
    const double2 cxy = cadd(cxd, cyd);
#pragma unroll 4
    for (int z = z0; z < z1; ++z) {
      const double2* pz = uc0 + (int64_t)z * sz;
      const double2 up = load_or_zero(z + 1 < g.nz, pz + sz);
      const double2 vxl = load_or_zero(hx0, pz - 1), vxu = load_or_zero(hx1, pz + 1);
      const double2 vyl = load_or_zero(hy0, pz - sy), vyu = load_or_zero(hy1, pz + sy);
      // sigma of the plane scales its x and y terms (exact when it is 1)
      const double sg = g.sg[z].x;
      double2 au = cmul(cadd(cscale(cxy, sg), g.zd[z]), uc);
      au = cfma(cscale(cxl, sg), vxl, au);
      au = cfma(cscale(cxu, sg), vxu, au);
      au = cfma(cscale(cyl, sg), vyl, au);
      au = cfma(cscale(cyu, sg), vyu, au);
      au = cfma(g.zl[z], um, au);
      au = cfma(g.zu[z], up, au);
      const int64_t e = col + (int64_t)z * sz;
      if (negate_f) {
        if (write_out) out[e] = cvt<CO>(au);
      } else {
        const double2 fe = f[e];
        const double2 r = csub(fe, au);
        if (write_out) out[e] = cvt<CO>(r);
        if (part) {
          rr = fma(r.x, r.x, fma(r.y, r.y, rr));
          ff = fma(fe.x, fe.x, fma(fe.y, fe.y, ff));
          uu = fma(uc.x, uc.x, fma(uc.y, uc.y, uu));
        }
      }
      um = uc;
      uc = up;
    }
  }
  if (!part) return;
  // workgroup sums in a fixed order: butterfly within each wave, then the
  // four wave sums in order
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    rr += __shfl_xor(rr, m, 64);
    ff += __shfl_xor(ff, m, 64);
    uu += __shfl_xor(uu, m, 64);
  }
  __shared__ double red[3][RZ_TX * RZ_TY / 64];
  const int wave = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) {
    red[0][wave] = rr;
    red[1][wave] = ff;
    red[2][wave] = uu;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double s = 0;
    for (int w = 0; w < RZ_TX * RZ_TY / 64; ++w) s += red[threadIdx.x][w];
    const int64_t wg = ((int64_t)bz * gy + by) * gx + bx;
    part[3 * wg + threadIdx.x] = s;
  }
}

template <typename CO>
__global__ __launch_bounds__(RZ_TX * RZ_TY) void k_residual(StencilGeom g, const double2* __restrict__ f,
                                                            const double2* __restrict__ u, CO* __restrict__ out,
                                                            int negate_f, double* __restrict__ part,
                                                            int write_out) {
  residual_body<CO>(g, f, u, out, negate_f, part, write_out, int(blockIdx.x), int(blockIdx.y), int(blockIdx.z),
                    int(gridDim.x), int(gridDim.y));
}

// Residuals r = f - A u (complex64 output) of many plans in one launch: the
// workgroups of plan i (its column tiles x z chunks x right-hand sides) are
// the contiguous range [l[i].wg0, l[i + 1].wg0) of a flat grid, found by a
// binary search over the list.
__global__ __launch_bounds__(RZ_TX * RZ_TY) void k_residual_list(const ResidualItem* __restrict__ l, int n,
                                                                 const double2* __restrict__ f0,
                                                                 const double2* __restrict__ u0,
                                                                 float2* __restrict__ r0) {
  const int64_t wg = blockIdx.x;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (l[mid].wg0 <= wg) lo = mid; else hi = mid - 1;
  }
  const ResidualItem& it = l[lo];
  const int64_t loc = wg - it.wg0;
  const int bx = int(loc % it.gx), by = int((loc / it.gx) % it.gy), bz = int(loc / ((int64_t)it.gx * it.gy));
  residual_body<float2>(it.g, f0 + it.f, u0 + it.u, r0 + it.r, 0, nullptr, 1, bx, by, bz, it.gx, it.gy);
}

// Per right-hand side r, the sums of the residual kernel's workgroup partials
// (nwg of them per right-hand side) in a fixed order: out[3 r + {0, 1, 2}] =
// |r|^2, |f|^2, |u|^2.
__global__ __launch_bounds__(256) void k_norm_finish(const double* __restrict__ part, int64_t nwg,
                                                     double* __restrict__ out) {
  const int r = blockIdx.x;
  const double* p = part + 3 * (int64_t)r * nwg;
  double acc[3] = {0, 0, 0};
  for (int64_t i = threadIdx.x; i < nwg; i += 256)
    for (int c = 0; c < 3; ++c) acc[c] += p[3 * i + c];
  __shared__ double red[3][256];
  for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x < 3) out[3 * r + threadIdx.x] = red[threadIdx.x][0];
}

// Adjoint pre/post scaling with the mass matrix M = Mx (x) My (x) Mz of eq. (3):
// pre  out = M^{-1} conj(in),  post  out = conj(M in).
__global__ __launch_bounds__(256) void k_conj_mass(StencilGeom g, const double2* __restrict__ in,
                                                   double2* __restrict__ out, int inverse) {
  const int r = blockIdx.z;
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= n) return;
  const int x = int(e % g.nx);
  const int y = int((e / g.nx) % g.ny);
  const int z = int(e / ((int64_t)g.nx * g.ny));
  const double2 w = cmul(cmul(g.mx[x], g.my[y]), g.mz[z]);
  const double2 v = in[r * n + e];
  // inverse: M^{-1} conj(in)   forward: conj(M in)
  out[r * n + e] = inverse ? cmul(crcp(w), cconj(v)) : cconj(cmul(w, v));
}

// Layer gradient: partial sums of a * conj(u) over slices of each z plane,
// then per-layer sums of the partials.  Workgroup (z, s) of right-hand side r
// sums slice s of plane z (elements [s*chunk, (s+1)*chunk)) into
// part[(r * nz + z) * S + s]; the slices of a plane and the tree within a
// workgroup are summed in a fixed order, so results repeat bit for bit.
__global__ __launch_bounds__(256) void k_plane_dot(int64_t plane, int nz, int S, const double2* __restrict__ a,
                                                   const double2* __restrict__ u, double2* __restrict__ part) {
  const int z = blockIdx.x / S, sl = blockIdx.x % S, r = blockIdx.z;
  const int64_t chunk = (plane + S - 1) / S;
  const int64_t i0 = (int64_t)sl * chunk, i1 = min(plane, i0 + chunk);
  const double2* ap = a + ((int64_t)r * nz + z) * plane;
  const double2* up = u + ((int64_t)r * nz + z) * plane;
  double2 acc = mk<double>(0, 0);
  for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) acc = cfma(ap[i], cconj(up[i]), acc);
  __shared__ double2 red[256];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] = cadd(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[((int64_t)r * nz + z) * S + sl] = red[0];
}

__global__ __launch_bounds__(64) void k_layer_sum(int nz, int S, int nlayers, const int* __restrict__ layer_of_z,
                                                  const double2* __restrict__ part, double2* __restrict__ grad) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.z;
  if (l >= nlayers) return;
  double2 acc = mk<double>(0, 0);
  for (int z = 0; z < nz; ++z)
    if (layer_of_z[z] == l)
      for (int sl = 0; sl < S; ++sl) acc = cadd(acc, part[((int64_t)r * nz + z) * S + sl]);
  grad[(int64_t)r * nlayers + l] = acc;
}

inline unsigned grid1(int64_t n) { return unsigned((n + 255) / 256); }

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------- sine transform
// Kernels whose dynamic LDS exceeds 64 KiB ask for it once (gfx950 has 160 KiB
// per workgroup).
static void allow_lds(const void* fn, size_t bytes) {
  static std::mutex mu;
  static std::vector<std::pair<const void*, size_t>> done;
  std::lock_guard<std::mutex> lock(mu);
  for (auto& e : done)
    if (e.first == fn && e.second >= bytes) return;
  (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
  done.push_back({fn, bytes});
}

// LDS of one workgroup of lt lines (rows of 17 V + 1 complex values and the
// lanes' partial sums)
static size_t dst_lds_bytes(int prec, int V, int lt) {
  const size_t csz = prec == 0 ? 16 : 8;
  return size_t(lt) * (17 * V + 1 + 16) * csz;
}

int dst_lines_per_wg(int prec, int V) {
  int lt = 16;
  while (lt > 4 && dst_lds_bytes(prec, V, lt) > 40960) lt /= 2;
  return lt;
}

bool dst_lt_ok(int prec, int V, int lt) {
  return (lt == 4 || lt == 8 || lt == 16) && dst_lds_bytes(prec, V, lt) <= kMaxLdsBytes;
}

template <typename R, typename CI, typename CO, bool ACC>
static void launch_dst_t(int V, const DstDesc* d, int ndesc, int max_lines, const void* tw, const void* src,
                         void* dst, int nrhs, hipStream_t st, int lt) {
  const int prec = sizeof(R) == 8 ? 0 : 1;
  if (!dst_lt_ok(prec, V, lt)) lt = dst_lines_per_wg(prec, V);
  const dim3 grid((max_lines + lt - 1) / lt, ndesc, nrhs);
  const cplx<R>* T = (const cplx<R>*)tw;
  const size_t lds = dst_lds_bytes(prec, V, lt);
#define HS_DST_CASE(VV, LL)                                                                                    \
  if (V == VV && lt == LL) {                                                                                   \
    auto kfn = k_dst<R, CI, CO, ACC, VV, LL>;                                                                  \
    if (lds > 65536) allow_lds(reinterpret_cast<const void*>(kfn), lds);                                       \
    hipLaunchKernelGGL(kfn, grid, dim3(16 * LL), lds, st, d, T, (const CI*)src, (CO*)dst);                     \
    return;                                                                                                    \
  }
  HS_DST_CASE(1, 16)
  HS_DST_CASE(1, 8)
  HS_DST_CASE(1, 4)
  HS_DST_CASE(2, 16)
  HS_DST_CASE(2, 8)
  HS_DST_CASE(2, 4)
  HS_DST_CASE(4, 16)
  HS_DST_CASE(4, 8)
  HS_DST_CASE(4, 4)
  HS_DST_CASE(8, 16)
  HS_DST_CASE(8, 8)
  HS_DST_CASE(8, 4)
  HS_DST_CASE(16, 16)
  HS_DST_CASE(16, 8)
  HS_DST_CASE(16, 4)
  HS_DST_CASE(32, 16)
  HS_DST_CASE(32, 8)
  HS_DST_CASE(32, 4)
#undef HS_DST_CASE
}

void dst_lines(int prec, int in64, int out64, int acc, int V, const DstDesc* d, int ndesc, int max_lines,
               const void* tw, const void* src, void* dst, int nrhs, hipStream_t st, int lt) {
  if (ndesc == 0 || max_lines == 0 || nrhs == 0) return;
  if (prec == 0) {
    launch_dst_t<double, double2, double2, false>(V, d, ndesc, max_lines, tw, src, dst, nrhs, st, lt);
  } else if (!in64 && !out64) {
    launch_dst_t<float, float2, float2, false>(V, d, ndesc, max_lines, tw, src, dst, nrhs, st, lt);
  } else if (in64 && !out64) {
    launch_dst_t<float, double2, float2, false>(V, d, ndesc, max_lines, tw, src, dst, nrhs, st, lt);
  } else if (!in64 && out64) {
    if (acc)
      launch_dst_t<float, float2, double2, true>(V, d, ndesc, max_lines, tw, src, dst, nrhs, st, lt);
    else
      launch_dst_t<float, float2, double2, false>(V, d, ndesc, max_lines, tw, src, dst, nrhs, st, lt);
  } else {
    launch_dst_t<float, double2, double2, false>(V, d, ndesc, max_lines, tw, src, dst, nrhs, st, lt);
  }
}

// planes per workgroup of the strided dense transform: panels of at most
// 24 KiB in all (one plane where a panel alone is that large)
int xform_y_ppw(int prec, int max_n, int ct) {
  const size_t esz = prec == 0 ? sizeof(double2) : sizeof(float2);
  const size_t one = size_t(std::max(max_n, 1)) * ct * esz;
  return int(std::max<size_t>(1, std::min<size_t>(16, 24576 / one)));
}

void xform_y(int prec, const XformYDesc* d, int ndesc, int max_n, int max_tiles16, int max_tiles8,
             const void* tab, void* ws, int nrhs, hipStream_t st) {
  if (ndesc == 0 || nrhs == 0) return;
  const bool wide = max_n <= 256;
  const int CT = wide ? 16 : 8;
  const size_t esz = prec == 0 ? sizeof(double2) : sizeof(float2);
  const int ppw = xform_y_ppw(prec, max_n, CT);
  const size_t lds = size_t(ppw) * max_n * CT * esz;
  const int tiles = wide ? max_tiles16 : max_tiles8;
  if (prec == 0) {
    if (wide)
      hipLaunchKernelGGL((k_xform_y<double, 16>), dim3(tiles, ndesc, nrhs), dim3(256), lds, st, d,
                         (const double2*)tab, (double2*)ws, ppw);
    else
      hipLaunchKernelGGL((k_xform_y<double, 8>), dim3(tiles, ndesc, nrhs), dim3(256), lds, st, d,
                         (const double2*)tab, (double2*)ws, ppw);
  } else {
    if (wide)
      hipLaunchKernelGGL((k_xform_y<float, 16>), dim3(tiles, ndesc, nrhs), dim3(256), lds, st, d,
                         (const float2*)tab, (float2*)ws, ppw);
    else
      hipLaunchKernelGGL((k_xform_y<float, 8>), dim3(tiles, ndesc, nrhs), dim3(256), lds, st, d,
                         (const float2*)tab, (float2*)ws, ppw);
  }
}

int xform_y_tiles(const XformYDesc& d, int ct, int ppw) {
  return ((d.ncols + ct - 1) / ct) * ((d.P + ppw - 1) / ppw);
}

// Staged x-type term lines: at most this many bytes of LDS.
constexpr size_t kSweepStageBytes = 32768;

int sweep_stage_cap(int nz, int chunks, int max_xterms) {
  const int64_t need = 2LL * max_xterms * chunks * psweep_rows(nz, chunks);
  return need > 0 && need * int64_t(sizeof(double2)) <= int64_t(kSweepStageBytes) ? int(need) : 0;
}

size_t sweep_lds_bytes(int arith_bytes, int nz, int chunks, int max_xterms) {
  // arith_bytes: 8 for FP64 arithmetic, 4 for FP32
  const size_t rows = size_t(chunks) * psweep_rows(nz, chunks);
  const size_t cs = 2 * size_t(arith_bytes);   // one complex value
  return (rows * (2 * cs + size_t(arith_bytes)) + 255) / 256 * 256 + 6 * 256 * cs +
         size_t(sweep_stage_cap(nz, chunks, max_xterms)) * cs;
}

bool sweep_rows_fixed(int chunks, int nz) {
  if (!sweep_chunks_ok(chunks, nz)) return false;
  const int rows = psweep_rows(nz, chunks);
  return rows == psweep_regrows(rows);
}

int sweep_default_chunks(int nz) { return nz > 16 * PS_LMAX ? 32 : 16; }

bool sweep_chunks_ok(int chunks, int nz) {
  return (chunks == 8 || chunks == 16 || chunks == 32) && nz <= chunks * PS_LMAX;
}

bool side_stream_create(SideStream& s) {
  if (hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking) != hipSuccess) return false;
  if (hipEventCreateWithFlags(&s.fork, hipEventDisableTiming) != hipSuccess) return false;
  if (hipEventCreateWithFlags(&s.join, hipEventDisableTiming) != hipSuccess) return false;
  return true;
}

void side_stream_destroy(SideStream& s) {
  if (s.fork) (void)hipEventDestroy(s.fork);
  if (s.join) (void)hipEventDestroy(s.join);
  if (s.st) (void)hipStreamDestroy(s.st);
  s = SideStream{};
}

int sweep_effective_chunks(int chunks, int max_nz) {
  return sweep_chunks_ok(chunks, max_nz) ? chunks : sweep_default_chunks(max_nz);
}

// max_modes: largest nb * (na rounded up to 32) over the descriptors, which
// covers the tiles of either mode packing; a multiple of 8 workgroups along x
// keeps workgroup i of every descriptor on XCD i mod 8
int sweep_grid_x(int64_t max_modes, int chunks) {
  const int mw = 256 / chunks;
  const int64_t tiles = (max_modes + mw - 1) / mw;
  return int((tiles + 7) / 8 * 8);
}

void sweep_select(const SweepDesc* d, int ndesc, int64_t max_modes, int chunks,
                  const std::function<double(int64_t)>& lam_re, SweepSelHost& out) {
  const int mw = 256 / chunks;
  out.words = (sweep_grid_x(max_modes, chunks) + 31) / 32;
  out.list.clear();
  out.bits.assign(size_t(ndesc) * out.words, 0u);
  for (int di = 0; di < ndesc; ++di) {
    const SweepDesc& s = d[di];
    const int64_t tiles = psweep_tiles(s, mw);
    for (int wg = 0; wg < tiles; ++wg) {
      const SweepTile t = psweep_tile(s, mw, int(tiles), wg);
      bool low = false;
      for (int ml = 0; ml < mw && !low; ++ml) {
        int64_t m;
        if (!psweep_mode(s, t, ml, m)) continue;
        const int a = int(m % s.rs), b = int(m / s.rs);
        low = lam_re(s.lam_x + a) + lam_re(s.lam_y + b) <= s.fp64_below;
      }
      if (low) {
        out.list.push_back(make_int2(di, wg));
        out.bits[size_t(di) * out.words + (wg >> 5)] |= 1u << (wg & 31);
      }
    }
  }
}

void sweep(int prec, const SweepDesc* d, int ndesc, int64_t max_modes, int max_nz, int max_xterms, const void* tab,
           const void* tab64, void* ws, int nrhs, hipStream_t st, int chunks, const SweepSel* sel,
           const SideStream* side, int full_nz) {
  if (ndesc == 0 || nrhs == 0 || max_modes == 0) return;
  chunks = sweep_effective_chunks(chunks, max_nz);
  size_t lds = sweep_lds_bytes(prec == 0 ? 8 : 4, max_nz, chunks, max_xterms);
  const int xcap = sweep_stage_cap(max_nz, chunks, max_xterms);
  const dim3 grid(unsigned(sweep_grid_x(max_modes, chunks)), ndesc, nrhs);
  // complex64: the selection made for this chunking (one per chunk count)
  SweepSel sc{};
  if (prec != 0 && sel) sc = sel[chunks == 8 ? 0 : chunks == 16 ? 1 : 2];
  if (sc.n == 0) sc.bits = nullptr;   // nothing selected: no bit to test
  const int rows = psweep_rows(max_nz, chunks);
  const bool short_rows = psweep_regrows(rows) == 8;
  // full chunks: every descriptor's z line fills its chunks' register rows
  const bool full = full_nz == max_nz && rows == psweep_regrows(rows);
#define HS_PSWEEP_L(RR, CC, PP, MM, LL, SEL, STREAM, LDS, GRID)                                          \
  do {                                                                                                     \
    if (full)                                                                                              \
      hipLaunchKernelGGL((k_psweep<RR, PP, MM, LL, SEL, true>), GRID, dim3(256), LDS, STREAM, d,           \
                         (const CC*)tab, (const double2*)tab64, (CC*)ws, xcap, sc);                        \
    else                                                                                                   \
      hipLaunchKernelGGL((k_psweep<RR, PP, MM, LL, SEL, false>), GRID, dim3(256), LDS, STREAM, d,          \
                         (const CC*)tab, (const double2*)tab64, (CC*)ws, xcap, sc);                        \
  } while (0)
#define HS_PSWEEP(RR, CC, PP, MM, SEL, STREAM, LDS, GRID)                                                 \
  do {                                                                                                     \
    if (short_rows)                                                                                        \
      HS_PSWEEP_L(RR, CC, PP, MM, 8, SEL, STREAM, LDS, GRID);                                              \
    else                                                                                                   \
      HS_PSWEEP_L(RR, CC, PP, MM, PS_LMAX, SEL, STREAM, LDS, GRID);                                        \
  } while (0)
  if (prec == 0) {
    if (chunks == 32) HS_PSWEEP(double, double2, 32, 8, false, st, lds, grid);
    else if (chunks == 16) HS_PSWEEP(double, double2, 16, 16, false, st, lds, grid);
    else HS_PSWEEP(double, double2, 8, 32, false, st, lds, grid);
  } else {
    const size_t lds64 = sweep_lds_bytes(8, max_nz, chunks, max_xterms);
    const bool fp64_modes = sc.n > 0;
    const dim3 grid64(unsigned(sc.n), 1, nrhs);
    const bool fork = fp64_modes && side && side->st;
    hipStream_t s64 = fork ? side->st : st;
    if (fork) {
      (void)hipEventRecord(side->fork, st);
      (void)hipStreamWaitEvent(s64, side->fork, 0);
    }
    if (fp64_modes) {
      if (chunks == 32) HS_PSWEEP(float, float2, 32, 8, true, s64, lds64, grid64);
      else if (chunks == 16) HS_PSWEEP(float, float2, 16, 16, true, s64, lds64, grid64);
      else HS_PSWEEP(float, float2, 8, 32, true, s64, lds64, grid64);
    }
    if (chunks == 32) HS_PSWEEP(float, float2, 32, 8, false, st, lds, grid);
    else if (chunks == 16) HS_PSWEEP(float, float2, 16, 16, false, st, lds, grid);
    else HS_PSWEEP(float, float2, 8, 32, false, st, lds, grid);
    if (fork) {
      (void)hipEventRecord(side->join, s64);
      (void)hipStreamWaitEvent(st, side->join, 0);
    }
  }
#undef HS_PSWEEP
#undef HS_PSWEEP_L
}

void contract_split(ContractDesc& d, int terms) {
  // at most 256 columns per workgroup (4 per lane, which keeps the kernel at
  // three waves per SIMD), 128 with more than 4 terms (their accumulators);
  // about 16K elements per workgroup: whole planes for blocks, row slabs for
  // the global plane so that there are enough workgroups to fill the chip
  const int nt = std::max(terms, std::max(d.nxt, d.nyt));
  const int cmax = nt > kMaxTerms ? 128 : 256;
  d.ncs = (d.na + cmax - 1) / cmax;
  d.cols = (d.na + d.ncs - 1) / d.ncs;
  const int64_t elems = (int64_t)d.cols * d.nb;
  int nslab = int(std::max<int64_t>(1, std::min<int64_t>(d.nb, (elems + 16383) / 16384)));
  d.rows = (d.nb + nslab - 1) / nslab;
  d.nslab = d.rows > 0 ? (d.nb + d.rows - 1) / d.rows : 1;
}

static int contract_lanes(int na) {
  int L = 1;
  while (L < na && L < 64) L <<= 1;
  return L;
}

ContractLaunch contract_launch(const ContractDesc* d, int ndesc, int prec) {
  ContractLaunch L;
  L.ndesc = ndesc;
  size_t lds_elems = 0, lds_x = 0;
  for (int i = 0; i < ndesc; ++i) {
    const int ln = contract_lanes(d[i].cols);
    const int S = (d[i].cols + ln - 1) / ln;
    L.max_slab = std::max(L.max_slab, d[i].nslab);
    L.max_cs = std::max(L.max_cs, d[i].ncs);
    L.smax = std::max(L.smax, S);
    L.max_nz = std::max(L.max_nz, d[i].nz);
    const int64_t fin = (d[i].nslab > 1 ? (int64_t)d[i].nyt * d[i].nz * d[i].na : 0) +
                        (d[i].ncs > 1 ? (int64_t)d[i].nxt * d[i].nz * d[i].nb : 0);
    L.fin_units = std::max<int64_t>(L.fin_units, fin);
    lds_elems = std::max<size_t>(lds_elems, size_t(d[i].nyt) * d[i].rows + 3 * kMaxContractTerms * 64);
    lds_x = std::max<size_t>(lds_x, size_t(d[i].nxt));
    L.max_terms = std::max(L.max_terms, std::max(d[i].nxt, d[i].nyt));
  }
  L.smax = L.smax <= 1 ? 1 : L.smax <= 2 ? 2 : L.smax <= 4 ? 4 : L.smax <= 6 ? 6 : 8;
  L.lds = (lds_elems + lds_x * L.smax * 64) * (prec == 0 ? 16 : 8);
  return L;
}

template <typename R, int SMAX, int NT>
static void launch_contract(const ContractDesc* d, const ContractLaunch& L, const void* tab, void* ws, int nrhs,
                            hipStream_t st) {
  using C = cplx<R>;
  const dim3 grid(unsigned(L.max_nz * L.max_slab * L.max_cs), unsigned(L.ndesc), unsigned(nrhs));
  hipLaunchKernelGGL((k_contract<R, SMAX, NT, NT == 2 && SMAX <= 4>), grid, dim3(256), L.lds, st, d, L.max_slab, L.max_cs, (const C*)tab,
                     (C*)ws);
  if (L.fin_units > 0)
    hipLaunchKernelGGL((k_contract_fin<R>), dim3(unsigned((L.fin_units + 255) / 256), L.ndesc, nrhs), dim3(256), 0,
                       st, d, (C*)ws);
}

template <typename R, int NT>
static void contract_nt(const ContractDesc* d, const ContractLaunch& L, const void* tab, void* ws, int nrhs,
                        hipStream_t st) {
  if constexpr (NT > kMaxTerms) {
    // descriptors of more than kMaxTerms terms hold at most 128 columns
    if (L.smax <= 1)
      launch_contract<R, 1, NT>(d, L, tab, ws, nrhs, st);
    else
      launch_contract<R, 2, NT>(d, L, tab, ws, nrhs, st);
  } else {
    if (L.smax <= 1)
      launch_contract<R, 1, NT>(d, L, tab, ws, nrhs, st);
    else if (L.smax <= 2)
      launch_contract<R, 2, NT>(d, L, tab, ws, nrhs, st);
    else if (L.smax <= 4)
      launch_contract<R, 4, NT>(d, L, tab, ws, nrhs, st);
    else if (L.smax <= 6)
      launch_contract<R, 6, NT>(d, L, tab, ws, nrhs, st);
    else
      launch_contract<R, 8, NT>(d, L, tab, ws, nrhs, st);
  }
}

// two-term sums (the four faces of a block) get their own, smaller kernels;
// more than kMaxTerms terms (interface contractions of many separators) take
// narrow column slabs
template <typename R>
static void contract_r(const ContractDesc* d, const ContractLaunch& L, const void* tab, void* ws, int nrhs,
                       hipStream_t st) {
  if (L.max_terms <= 2)
    contract_nt<R, 2>(d, L, tab, ws, nrhs, st);
  else if (L.max_terms <= kMaxTerms)
    contract_nt<R, kMaxTerms>(d, L, tab, ws, nrhs, st);
  else
    contract_nt<R, kMaxContractTerms>(d, L, tab, ws, nrhs, st);
}

void contract(int prec, const ContractDesc* d, const ContractLaunch& L, const void* tab, void* ws, int nrhs,
              hipStream_t st) {
  if (L.ndesc == 0 || nrhs == 0 || L.max_nz == 0) return;
  if (prec == 0)
    contract_r<double>(d, L, tab, ws, nrhs, st);
  else
    contract_r<float>(d, L, tab, ws, nrhs, st);
}

void expand(int prec, const ExpandDesc& e, const void* tab, void* ws, int nrhs, hipStream_t st) {
  if (nrhs == 0 || e.na == 0 || e.nb == 0 || e.nz == 0) return;
  const dim3 grid(unsigned((e.na + 63) / 64), unsigned(e.nz), unsigned(nrhs));
  if (prec == 0)
    hipLaunchKernelGGL((k_expand<double>), grid, dim3(256), 0, st, e, (const double2*)tab, (double2*)ws);
  else
    hipLaunchKernelGGL((k_expand<float>), grid, dim3(256), 0, st, e, (const float2*)tab, (float2*)ws);
}

void sigma_resid(int prec, int in64, const SigmaGeom& g, const void* f, void* ws, int nrhs, hipStream_t st) {
  const int64_t n = (int64_t)g.nsx * g.nz * g.NY + (int64_t)g.nsy * g.nz * g.NX;
  if (n == 0 || nrhs == 0) return;
  if (prec == 0)
    hipLaunchKernelGGL((k_sigma_resid<double, double2>), dim3(grid1(n), 1, nrhs), dim3(256), 0, st, g,
                       (const double2*)f, (double2*)ws);
  else if (in64)
    hipLaunchKernelGGL((k_sigma_resid<float, double2>), dim3(grid1(n), 1, nrhs), dim3(256), 0, st, g,
                       (const double2*)f, (float2*)ws);
  else
    hipLaunchKernelGGL((k_sigma_resid<float, float2>), dim3(grid1(n), 1, nrhs), dim3(256), 0, st, g,
                       (const float2*)f, (float2*)ws);
}

void lift(int prec, const SigmaGeom& g, const LiftBlock* lb, int nblocks, void* ws, int nrhs,
          hipStream_t st) {
  if (nblocks == 0 || nrhs == 0) return;
  const int64_t n = 4LL * g.nz * g.NF;
  unsigned gx = unsigned(std::min<int64_t>((n + 255) / 256, 1024));
  if (prec == 0)
    hipLaunchKernelGGL((k_lift<double>), dim3(gx, nblocks, nrhs), dim3(256), 0, st, g, lb, (double2*)ws);
  else
    hipLaunchKernelGGL((k_lift<float>), dim3(gx, nblocks, nrhs), dim3(256), 0, st, g, lb, (float2*)ws);
}

void sigma_scatter(int prec, int acc, const SigmaGeom& g, const void* ws, void* u, int nrhs, hipStream_t st) {
  const int64_t n = (int64_t)g.nsx * g.nz * g.NY + (int64_t)g.nsy * g.nz * g.NX;
  if (n == 0 || nrhs == 0) return;
  if (prec == 0)
    hipLaunchKernelGGL((k_sigma_scatter<double, double2, false>), dim3(grid1(n), 1, nrhs), dim3(256), 0, st,
                       g, (const double2*)ws, (double2*)u);
  else if (acc)
    hipLaunchKernelGGL((k_sigma_scatter<float, double2, true>), dim3(grid1(n), 1, nrhs), dim3(256), 0, st, g,
                       (const float2*)ws, (double2*)u);
  else
    hipLaunchKernelGGL((k_sigma_scatter<float, double2, false>), dim3(grid1(n), 1, nrhs), dim3(256), 0, st,
                       g, (const float2*)ws, (double2*)u);
}

void ml_scatter(int prec, const SigmaGeom& g, void* ws, int64_t f_off, int nrhs, hipStream_t st) {
  const int64_t n = (int64_t)g.nsx * g.nz * g.NY + (int64_t)g.nsy * g.nz * g.NX;
  if (nrhs == 0) return;
  const int64_t total = (int64_t)nrhs * g.f_r;
  const unsigned zb = unsigned(std::min<int64_t>((total + 255) / 256, 65536));
  if (prec == 0) {
    double2* F = (double2*)ws + f_off;
    hipLaunchKernelGGL((k_ml_zero<double>), dim3(zb), dim3(256), 0, st, F, total);
    if (n > 0)
      hipLaunchKernelGGL((k_ml_scatter<double>), dim3(grid1(n), 1, nrhs), dim3(256), 0, st, g, (const double2*)ws, F);
  } else {
    float2* F = (float2*)ws + f_off;
    hipLaunchKernelGGL((k_ml_zero<float>), dim3(zb), dim3(256), 0, st, F, total);
    if (n > 0)
      hipLaunchKernelGGL((k_ml_scatter<float>), dim3(grid1(n), 1, nrhs), dim3(256), 0, st, g, (const float2*)ws, F);
  }
}

void ml_gather(int prec, const SigmaGeom& g, const void* W, void* ws, int nrhs, hipStream_t st) {
  const int64_t n = (int64_t)g.nsx * g.nz * g.NY + (int64_t)g.nsy * g.nz * g.NX;
  if (n == 0 || nrhs == 0) return;
  if (prec == 0)
    hipLaunchKernelGGL((k_ml_gather<double>), dim3(grid1(n), 1, nrhs), dim3(256), 0, st, g, (const double2*)W,
                       (double2*)ws);
  else
    hipLaunchKernelGGL((k_ml_gather<float>), dim3(grid1(n), 1, nrhs), dim3(256), 0, st, g, (const double2*)W,
                       (float2*)ws);
}

static dim3 residual_grid(const StencilGeom& g, int nrhs) {
  return dim3(unsigned(((g.nx + RZ_TX - 1) / RZ_TX) * ((g.ny + RZ_TY - 1) / RZ_TY)),
              unsigned((g.nz + RZ_ZC - 1) / RZ_ZC), unsigned(nrhs));
}

int64_t residual_workgroups(const StencilGeom& g) {
  const dim3 gr = residual_grid(g, 1);
  return (int64_t)gr.x * gr.y;
}

int64_t residual_list_items(std::vector<ResidualItem>& items) {
  int64_t wg = 0;
  for (auto& it : items) {
    const dim3 gr = residual_grid(it.g, it.nrhs);
    it.gx = int(gr.x);
    it.gy = int(gr.y);
    it.wg0 = wg;
    wg += (int64_t)gr.x * gr.y * gr.z;
  }
  return wg;
}

void residual_list(const ResidualItem* dev, int n, int64_t total_wg, const void* f0, const void* u0, void* r0,
                   hipStream_t st) {
  if (n == 0 || total_wg == 0) return;
  hipLaunchKernelGGL(k_residual_list, dim3(unsigned(total_wg)), dim3(RZ_TX * RZ_TY), 0, st, dev, n,
                     (const double2*)f0, (const double2*)u0, (float2*)r0);
}

void residual(const StencilGeom& g, const void* f, const void* u, void* out, int out64, int apply_only,
              int nrhs, hipStream_t st, double* part, double* norms, int write_out) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  if (n == 0 || nrhs == 0) return;
  if (apply_only) part = nullptr;
  const dim3 grid = residual_grid(g, nrhs);
  if (out64)
    hipLaunchKernelGGL((k_residual<double2>), grid, dim3(RZ_TX * RZ_TY), 0, st, g, (const double2*)f,
                       (const double2*)u, (double2*)out, apply_only, part, write_out);
  else
    hipLaunchKernelGGL((k_residual<float2>), grid, dim3(RZ_TX * RZ_TY), 0, st, g, (const double2*)f,
                       (const double2*)u, (float2*)out, apply_only, part, write_out);
  if (part && norms)
    hipLaunchKernelGGL(k_norm_finish, dim3(unsigned(nrhs)), dim3(256), 0, st, (const double*)part,
                       (int64_t)grid.x * grid.y, norms);
}

void conj_mass(const StencilGeom& g, const void* in, void* out, int inverse, int nrhs, hipStream_t st) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  if (n == 0 || nrhs == 0) return;
  hipLaunchKernelGGL(k_conj_mass, dim3(grid1(n), 1, nrhs), dim3(256), 0, st, g, (const double2*)in,
                     (double2*)out, inverse);
}

// Static scratch of the allocation-free gradient entry point: the slice
// partials of one call (kGradScratchElems complex128 values, 1 MiB per device,
// held until the process ends).  In host code `scratch` only names the
// symbol: kernels take the device address that grad_scratch_init looked up.
__device__ __align__(256) double2 scratch[kGradScratchElems];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

bool grad_scratch_init(int device, std::string& err) {
  if (device < 0 || device >= kMaxDevices) {
    err = "device index beyond the static scratch table";
    return false;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return true;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    err = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
    return false;
  }
  g_scratch_ptr[device] = ptr;
  return true;
}

void* grad_scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

int grad_slices(int64_t plane, int nz, int nrhs) {
  // about 2048 workgroups in all, each summing at least 2048 elements
  int64_t S = 2048 / std::max<int64_t>(1, (int64_t)nz * nrhs);
  S = std::min<int64_t>(S, std::max<int64_t>(1, plane / 2048));
  return int(std::max<int64_t>(1, std::min<int64_t>(S, 64)));
}

int64_t grad_partials(int64_t plane, int nz, int nrhs) {
  return (int64_t)nrhs * nz * grad_slices(plane, nz, nrhs);
}

void grad_layers(int64_t plane, int nz, int nlayers, const int* layer_of_z, const void* a, const void* u,
                 void* part, void* grad, int nrhs, hipStream_t st) {
  if (nz == 0 || nrhs == 0) return;
  const int S = grad_slices(plane, nz, nrhs);
  hipLaunchKernelGGL(k_plane_dot, dim3(unsigned(nz * S), 1, nrhs), dim3(256), 0, st, plane, nz, S,
                     (const double2*)a, (const double2*)u, (double2*)part);
  hipLaunchKernelGGL(k_layer_sum, dim3((nlayers + 63) / 64, 1, nrhs), dim3(64), 0, st, nz, S, nlayers,
                     layer_of_z, (const double2*)part, (double2*)grad);
}

}  // namespace hs
