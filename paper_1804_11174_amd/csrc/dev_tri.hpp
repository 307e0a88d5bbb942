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
// periodic separation). With a = max(0, 1 - u/2) and c = max(0, 1 - u),
// 6 B(u) = 8 (a^3 - c^3 / 2): each of a and c is one multiply-add of the
// distance clamped to [0, 1]. The image term needs only its a (its u is at
// least L / (2 h) >= 1), the same multiply-add of the image distance
// L - d; for h <= L/4 that a is 0. Partial sums are raw: sum of 6 B(u) / 8
// and sum of max(0, 1 - u); the finalize divides by 3 h / 4 and h.
#include "dev_cv.hpp"
#include "dev_density.hpp"

namespace kde {

// Per-width constants of the pair kernel, for a periodic distance r in
// the packed unit (1 or 2^-32 of the period) and s_b = L / h_b in that
// unit: a = 1 + r ka[b] (ka = -s/2) and c = 1 + r kc[b] (kc = -s), each
// clamped to [0, 1]; the image's a is 1 + (period - r) ka[b], `period` in
// the packed unit. hfrac2[b] = 2 h_b / L is the distance (in fractions of
// the period) from which width b contributes nothing; `reach` is the
// largest of them; image bit b is set when h_b > L/4 (with ascending
// widths, the top ones).
template <typename T>
struct TriConsts {
  int B;
  uint64_t image;
  double reach;
  T period;
  T ka[KDE_MAX_KAPPAS], kc[KDE_MAX_KAPPAS];
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
    const double sb = unit * L / widths[b];
    K.ka[b] = T(-0.5 * sb);
    K.kc[b] = T(-sb);
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

__device__ __forceinline__ float clamp01(float v) { return __builtin_amdgcn_fmed3f(v, 0.0f, 1.0f); }
__device__ __forceinline__ double clamp01(double v) { return fmin(fmax(v, 0.0), 1.0); }

template <typename T, int BC>
struct TriSmem {
  typename TriPacked<T>::type tj[kCvTile];
  double red[kBlock / 64][2 * BC];
  double unit_acc[2 * KDE_MAX_KAPPAS];
  int bstart;
};

// The terms of one (pair, width): a = max(0, 1 - u/2) given, c and the
// cubic, and with IMG the image's a (r and rp the distance and the
// image's distance).
template <typename T, bool LIVE_ALL, bool IMG>
__device__ __forceinline__ void tri_add(T r, T rp, T a, T kc, T ka, bool live, Acc<T>& s1, Acc<T>& s2) {
  const T c = clamp01(fma(r, kc, T(1)));
  T kb = fma(T(-0.5), c * c * c, a * a * a);
  if (IMG) {
    const T ai = clamp01(fma(rp, ka, T(1)));
    kb = fma(ai * ai, ai, kb);
  }
  if (LIVE_ALL) {
    s1.add(kb);
    s2.add(c);
  } else {
    s1.add(live ? kb : T(0));
    s2.add(live ? c : T(0));
  }
}

// Whether the pair kernel votes at every width (double) or once per j and
// pass (float). A vote lets the wave stop at the first width, widest
// first, whose support no lane reaches (the narrower ones are zero as
// well); it costs a compare and about seven scalar instructions and
// branches. Float terms issue at twice the rate of double ones, and there
// the scalar issue of a vote per width bounded the loop (7.2 ms against
// 4.4 ms with one vote per j at the paper-scale scan); in double the
// terms a vote per width saves are worth more (6.8 ms against 7.4 ms).
template <typename T>
constexpr bool kTriVoteEach = std::is_same<T, double>::value;

// One pass of a tile pair over widths [b_lo, b_hi). With a vote per width
// the wave stops at the first one, widest first, that no lane reaches.
// With one vote per j, on the pass's widest width, a j that no lane
// reaches is skipped and otherwise every width of the pass adds its terms,
// zero outside their supports; a pass narrower than BC evaluates its last
// width in the spare slots, whose sums are dropped. Either way a skipped
// term is an exact zero, so the sums do not depend on the voting.
// LIVE_ALL: every (i, j) of the pair is counted (an off-diagonal pair of
// full tiles), so no per-term mask. IMG: the pass holds a width that
// reaches its image; no vote stops such a width, and every width of the
// pass adds the image term, exactly 0 for those that do not reach their
// image (a branch per width on the image bit was 9 % slower in double).
// A pass without one has no image code (as a select per term it cost five
// instructions in float).
template <typename T, int BC, bool LIVE_ALL, bool IMG>
__device__ __forceinline__ void tri_pass(typename TriPacked<T>::type pi, bool valid_i, bool diag, int nj, int b_lo,
                                         int b_hi, const TriConsts<T>& K, Acc<T> (&s1)[BC], Acc<T> (&s2)[BC],
                                         const typename TriPacked<T>::type* tj) {
  const int tid = threadIdx.x;
  // the pass's constants, read into (scalar) registers once per pass
  // instead of once per term
  T ka[BC], kc[BC];
#pragma unroll
  for (int bb = 0; bb < BC; ++bb) {
    const int b = min(b_lo + bb, b_hi - 1);
    ka[bb] = K.ka[b];
    kc[bb] = K.kc[b];
  }
  const T ktop = K.ka[b_hi - 1];
  for (int jj = 0; jj < nj; ++jj) {
    const bool live = LIVE_ALL || (valid_i && (!diag || jj > tid));
    const T r = tri_dist(pi, tj[jj]);
    const T rp = K.period - r;  // the image's distance
    if (kTriVoteEach<T>) {
      bool go = true;  // uniform across the wave
#pragma unroll
      for (int bb = BC - 1; bb >= 0; --bb) {
        const int b = b_lo + bb;
        if (b < b_hi && go) {
          const T a = clamp01(fma(r, ka[bb], T(1)));
          const bool img = IMG && ((K.image >> b) & 1);
          go = img || !__all(!live || a == T(0));
          if (go) tri_add<T, LIVE_ALL, IMG>(r, rp, a, kc[bb], ka[bb], live, s1[bb], s2[bb]);
        }
      }
    } else if (IMG || !__all(!live || clamp01(fma(r, ktop, T(1))) == T(0))) {
#pragma unroll
      for (int bb = 0; bb < BC; ++bb)
        tri_add<T, LIVE_ALL, IMG>(r, rp, clamp01(fma(r, ka[bb], T(1))), kc[bb], ka[bb], live, s1[bb], s2[bb]);
    }
    if ((jj & (kRun - 1)) == kRun - 1) fold_all(s1, s2);
  }
  fold_all(s1, s2);
}

// The passes of one tile pair over widths [b_start, B), widest first.
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
    // ascending widths: the pass reaches an image if its widest width does
    if ((K.image >> (b_hi - 1)) & 1)
      tri_pass<T, BC, LIVE_ALL, true>(pi, valid_i, diag, nj, b_lo, b_hi, K, s1, s2, sm.tj);
    else
      tri_pass<T, BC, LIVE_ALL, false>(pi, valid_i, diag, nj, b_lo, b_hi, K, s1, s2, sm.tj);
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
// [Tbar sums x 3 h / 4 | T sums x h] into the slot's running sums sm.unit_acc.
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
struct __align__(16) TriGeo {
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
      // groups of eight particles without a bound test inside a group (their
      // LDS reads in flight together), runs of kRun terms folded into a
      // compensated sum, as in the von Mises deposit
      auto term = [&](int p) {
        const TriGeo<T> gp = sm.pg[p];
        const T t = tri_node(gp, g, M);
        return PER ? gp.w * t : t;
      };
      Acc<T> acc;
      acc.zero();
      int p = sub, q = 0;
      for (; p + 7 * S < cnt; p += 8 * S, q += 8) {
        T e[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) e[u] = term(p + u * S);
#pragma unroll
        for (int u = 0; u < 8; ++u) acc.add(e[u]);
        if (((q + 8) & (kRun - 1)) == 0) acc.fold();
      }
      for (; p < cnt; p += S, ++q) {
        acc.add(term(p));
        if ((q & (kRun - 1)) == kRun - 1) acc.fold();
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
    // runs folded into Kahan sums, or for 16 nodes per thread a Kahan step
    // per term (registers)
    using Sum = typename std::conditional<(G <= 8), Acc<T>, SumOf<T>>::type;
    Sum acc[G];
#pragma unroll
    for (int k = 0; k < G; ++k) acc[k].zero();
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
      if ((p & (kRun - 1)) == kRun - 1) {
#pragma unroll
        for (int k = 0; k < G; ++k) acc[k].fold();
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
