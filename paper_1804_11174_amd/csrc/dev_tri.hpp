#pragma once
// Device pieces of the first-order (triangular) shape of adjustable width:
// the standard-PIC weighting function with its half-width chosen by the CV
// objective (Sec. I, first-order weighting; Sec. IV, the comparison of
// shapes and costs).
//
//   T_h(d)    = max(0, 1 - |d|/h) / h,                 0 < h <= L/2,
//   Tbar_h(d) = (B(d/h) + B((L - d)/h)) / h,            d in [0, L/2],
//   B(u)      = (max(0, 2 - u)^3 - 4 max(0, 1 - u)^3) / 6,  u >= 0,
//
// Tbar is the two-fold convolution (the triangle is a box convolved with
// itself, so Tbar is the cubic B-spline); the second B term is the
// periodic image, which only widths h > L/4 can reach. No transcendental
// is needed anywhere: the pair sums are plain ALU work, and the support is
// compact, so tile pairs farther apart than 2 h_max are skipped whole and,
// within a pair of tiles, a wave stops at the first width (widest first)
// for which every pair of the wave lies outside the support.
//
// Pair distances are periodic and in fractions of the period: from the
// wrapped position / L in double, or from the 32-bit fixed-point phase in
// float (the phase difference in wrapping integer arithmetic is the exact
// periodic separation). Partial sums are raw: sum of B(u) * 6 and sum of
// max(0, 1 - u); the finalize divides by 6 h and h.
#include "dev_cv.hpp"
#include "dev_density.hpp"

namespace kde {

// Per-width constants of the pair kernel. scale[b] turns a periodic
// distance in the packed unit into u = d / h_b; `period` is the period in
// that unit (1 or 2^32); hfrac2[b] = 2 h_b / L is the distance (in
// fractions of the period) from which width b contributes nothing;
// `reach` is the largest of them; image bit b is set when h_b > L/4.
template <typename T>
struct TriConsts {
  int B;
  uint64_t image;
  double reach;
  T period;
  T scale[KDE_MAX_KAPPAS];
  double hfrac2[KDE_MAX_KAPPAS];
};

template <typename T>
inline TriConsts<T> make_tri_consts(const double* widths, int B, double L) {
  TriConsts<T> K{};
  K.B = B;
  const double unit = std::is_same<T, float>::value ? 1.0 / 4294967296.0 : 1.0;  // packed unit in periods
  K.period = T(1.0 / unit);
  double hmax = 0.0;
  for (int b = 0; b < B; ++b) {
    K.scale[b] = T(unit * L / widths[b]);
    K.hfrac2[b] = 2.0 * widths[b] / L;
    if (widths[b] > 0.25 * L) K.image |= (uint64_t(1) << b);
    hmax = widths[b] > hmax ? widths[b] : hmax;
  }
  K.reach = 2.0 * hmax / L;
  return K;
}

// Periodic distance of two packed particles in the packed unit.
__device__ __forceinline__ double tri_dist(FracPos a, FracPos b) {
  const double r = fabs(a.f - b.f);
  return fmin(r, 1.0 - r);
}
__device__ __forceinline__ float tri_dist(uint32_t a, uint32_t b) {
  const int32_t dd = int32_t(a - b);
  const uint32_t m = dd < 0 ? uint32_t(-int64_t(dd)) : uint32_t(dd);
  return float(m);
}

// Cubic B-spline times 6 and the triangle's raw value at u >= 0.
template <typename T>
__device__ __forceinline__ void tri_terms(T u, T& kb6, T& k1) {
  const T a = fmax(T(0), T(2) - u);
  const T c = fmax(T(0), T(1) - u);
  kb6 = a * a * a - T(4) * (c * c * c);
  k1 = c;
}

template <typename T, int BC>
struct TriSmem {
  typename TriPacked<T>::type tj[kCvTile];
  double red[kBlock / 64][2 * BC];
  double unit_acc[2 * KDE_MAX_KAPPAS];
  int bstart;
};

// The passes of one tile pair over widths [b_start, B), widest first; per
// j the wave stops at the first width whose support no lane reaches (the
// narrower ones are zero as well). LIVE_ALL: every (i, j) of the pair is
// counted (an off-diagonal pair of full tiles), so no per-term mask.
template <typename T, int BC, bool LIVE_ALL>
__device__ __forceinline__ void tri_passes(typename TriPacked<T>::type pi, bool valid_i, bool diag, int nj,
                                           int b_start, const TriConsts<T>& K, TriSmem<T, BC>& sm) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  for (int b_hi = K.B; b_hi > b_start; b_hi -= BC) {
    const int b_lo = max(b_start, b_hi - BC);
    Acc<T> s1[BC], s2[BC];
#pragma unroll
    for (int bb = 0; bb < BC; ++bb) {
      s1[bb].zero();
      s2[bb].zero();
    }
    for (int jj = 0; jj < nj; ++jj) {
      const bool live = LIVE_ALL || (valid_i && (!diag || jj > tid));
      const T r = tri_dist(pi, sm.tj[jj]);
      bool go = true;  // uniform across the wave
#pragma unroll
      for (int bb = BC - 1; bb >= 0; --bb) {
        const int b = b_lo + bb;
        if (b < b_hi && go) {
          const T u = r * K.scale[b];
          const bool img = (K.image >> b) & 1;
          go = img || !__all(!live || u >= T(2));
          if (go) {
            T kb6, k1;
            tri_terms(u, kb6, k1);
            if (img) {
              T kb6i, k1i;
              tri_terms((K.period - r) * K.scale[b], kb6i, k1i);
              kb6 += kb6i;
            }
            if (LIVE_ALL) {
              s1[bb].add(kb6);
              s2[bb].add(k1);
            } else {
              s1[bb].add(live ? kb6 : T(0));
              s2[bb].add(live ? k1 : T(0));
            }
          }
        }
      }
      if ((jj & (kRun - 1)) == kRun - 1) fold_all(s1, s2);
    }
    fold_all(s1, s2);
#pragma unroll
    for (int bb = 0; bb < BC; ++bb) {
      const double v1 = wave_sum(s1[bb].value());
      const double v2 = wave_sum(s2[bb].value());
      if (lane == 0) {
        sm.red[wave][bb] = v1;
        sm.red[wave][BC + bb] = v2;
      }
    }
    __syncthreads();
    if (tid < 2 * BC) {
      const int bb = tid % BC, which = tid / BC;
      if (b_lo + bb < b_hi) {
        double v = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) v += sm.red[w][tid];
        sm.unit_acc[which * K.B + b_lo + bb] += v;
      }
    }
    __syncthreads();
  }
}

// One tile pair (I, J) of the triangle pair sums; adds its 2B raw sums
// [Tbar sums x 6 h | T sums x h] into the slot's running sums sm.unit_acc.
// `cells` is the cell count of the sort that ordered the packed particles,
// which bounds the distance between the two tiles from below by `gap`
// (tile_gap); widths with 2 h <= gap L contribute nothing to the pair, and
// a pair farther apart than every support is skipped whole.
// Ends with a barrier.
template <typename T, int BC>
__device__ __forceinline__ void tri_tile_pair(const typename TriPacked<T>::type* __restrict__ packed, int64_t n,
                                              int cells, int I, int J, const TriConsts<T>& K, TriSmem<T, BC>& sm) {
  using P = typename TriPacked<T>::type;
  const int tid = threadIdx.x;
  const int64_t i0 = int64_t(I) * kCvTile, j0 = int64_t(J) * kCvTile;
  const int ni = int(min(int64_t(kCvTile), n - i0));
  const int nj = int(min(int64_t(kCvTile), n - j0));
  if (tid == 0) {
    const double gap = tile_gap(packed, i0, ni, j0, nj, cells, 0.0);
    int bs = 0;
    if (I != J) {
      if (gap >= K.reach) {
        bs = K.B;
      } else {
        while (bs < K.B && K.hfrac2[bs] <= gap) ++bs;
      }
    }
    sm.bstart = bs;
  }
  __syncthreads();
  const int b_start = sm.bstart;
  if (b_start >= K.B) {
    __syncthreads();
    return;
  }
  for (int k = tid; k < nj; k += kBlock) sm.tj[k] = packed[j0 + k];
  const bool valid_i = tid < ni;
  const P pi = valid_i ? packed[i0 + tid] : P{};
  const bool diag = (I == J);
  __syncthreads();
  if (!diag && ni == kCvTile)
    tri_passes<T, BC, true>(pi, valid_i, diag, nj, b_start, K, sm);
  else
    tri_passes<T, BC, false>(pi, valid_i, diag, nj, b_start, K, sm);
}

// One slot of the triangle pair sums: the tile pairs slot, slot + nslots,
// ... of the list of pair_decode (as cv_slot), all widths; writes the
// slot's 2B raw sums to `out`. Ends with a barrier.
template <typename T, int BC>
__device__ __forceinline__ void tri_slot(const typename TriPacked<T>::type* __restrict__ packed, int64_t n, int cells,
                                         int64_t slot, int64_t nslots, const TriConsts<T>& K, double* __restrict__ out,
                                         TriSmem<T, BC>& sm) {
  const int tid = threadIdx.x;
  for (int k = tid; k < 2 * K.B; k += kBlock) sm.unit_acc[k] = 0.0;
  const int ntiles = int((n + kCvTile - 1) / kCvTile);
  const int64_t items = int64_t(ntiles) * (ntiles + 1) / 2;
  for (int64_t k = slot; k < items; k += nslots) {
    int I, J;
    pair_decode(k, ntiles, I, J);
    tri_tile_pair<T, BC>(packed, n, cells, I, J, K, sm);
  }
  __syncthreads();
  for (int k = tid; k < 2 * K.B; k += kBlock) out[k] = sm.unit_acc[k];
  __syncthreads();
}

// ------------------------------------------------------------ grid pieces

// A particle relative to the grid: v = x M / L split as v = g0 + delta with
// g0 the nearest node and |delta| <= 1/2, q = dx / h and the weight 1/h.
// The distance to node g in cells is then |k - delta| with k = g - g0
// taken into [-M/2, M/2], which keeps float's relative accuracy near the
// particle. A half-width outside (0, L/2] gives a NaN weight.
template <typename T>
struct TriGeo {
  int g0;
  T delta, q, w;
};

template <typename T>
__device__ __forceinline__ TriGeo<T> tri_geo(double xi, double h, double L, int M) {
  TriGeo<T> p;
  const double xw = xi - L * floor(xi / L);
  const double v = xw * (double(M) / L);
  double g0 = floor(v + 0.5);
  const double d = v - g0;
  if (g0 >= double(M)) g0 -= double(M);
  p.g0 = int(g0);
  p.delta = T(d);
  const bool ok = (h > 0.0) && (h <= 0.5 * L);
  p.q = T((L / double(M)) / h);
  p.w = ok ? T(1.0 / h) : T(NAN);
  if (!isfinite(xi)) p.w = T(NAN);
  return p;
}

// max(0, 1 - |d|/h) for node g (the raw triangle; the caller weights it).
template <typename T>
__device__ __forceinline__ T tri_node(const TriGeo<T>& p, int g, int M) {
  int k = g - p.g0;
  if (k > M / 2) k -= M;
  if (k < -(M / 2)) k += M;
  T d = fabs(T(k) - p.delta);
  d = fmin(d, T(M) - d);
  return fmax(T(0), T(1) - d * p.q);
}

template <typename T>
struct TriDepSmem {
  TriGeo<T> pg[kDepMaxChunk];
  double red[kBlock];
};

// One deposit chunk with triangles (same layout of work and of the fixed-
// order sums as the von Mises deposit): particles [lo, lo + cnt) onto all
// M nodes, written to out[M], unnormalised by N. Ends with a barrier.
template <typename T, bool PER, int G>
__device__ __forceinline__ void tri_deposit_block(const T* __restrict__ x, const T* __restrict__ hi, double h_g,
                                                  int M, double L, int64_t lo, int cnt, double* __restrict__ out,
                                                  TriDepSmem<T>& sm, uint32_t* status) {
  const int tid = threadIdx.x;
  for (int k = tid; k < cnt; k += kBlock) {
    const double xi = double(x[lo + k]);
    const double h = PER ? double(hi[lo + k]) : h_g;
    note_numeric(status, !isfinite(xi), PER && !(h > 0.0 && h <= 0.5 * L));
    sm.pg[k] = tri_geo<T>(xi, h, L, M);
  }
  __syncthreads();
  const double gscale = PER ? 1.0 : 1.0 / h_g;
  if (M <= kBlock) {
    const int S = kBlock / M;
    const int g = tid % M, sub = tid / M;
    double tot = 0.0;
    if (sub < S) {
      SumOf<T> acc;
      for (int p = sub; p < cnt; p += S) {
        const T t = tri_node(sm.pg[p], g, M);
        acc.add(PER ? sm.pg[p].w * t : t);
      }
      tot = acc.value();
    }
    sm.red[tid] = tot;
    __syncthreads();
    if (tid < M) {
      double v = 0.0;
      for (int q = 0; q < S; ++q) v += sm.red[q * M + tid];
      out[tid] = v * gscale;
    }
  } else {
    SumOf<T> acc[G];
    for (int p = 0; p < cnt; ++p) {
      const TriGeo<T> gp = sm.pg[p];
#pragma unroll
      for (int k = 0; k < G; ++k) {
        const int g = tid + k * kBlock;
        if (g < M) {
          const T t = tri_node(gp, g, M);
          acc[k].add(PER ? gp.w * t : t);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < G; ++k) {
      const int g = tid + k * kBlock;
      if (g < M) out[g] = acc[k].value() * gscale;
    }
  }
  __syncthreads();
}

}  // namespace kde
