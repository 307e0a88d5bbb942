#pragma once
// Device pieces of the least-squares cross-validation over a batch of
// concentrations (Sec. II.B, Eq. cv_def): the O(N^2) pair sums and the final
// combination. Shared by the one-set kernels of cv.hip and the batched engine.
//
// For the von Mises kernel both pair terms depend on a pair only through
// its half-angle difference phi = pi (x_i - x_j) / L, via s = sin(phi) and
// c = |cos(phi)|:
//   K-term    exp(-2 kappa s^2)                           (kernel, unnormalised)
//   Kbar-term exp(-2 kappa (1 - c)) I0e(2 kappa c)        (two-fold convolution)
// Both exponents are formed without cancellation:
//   double: from half-angle vectors (a, b) = (cos(pi x/L), sin(pi x/L)),
//           c = |a_i a_j + b_i b_j|, s = b_i a_j - a_i b_j, 1 - c = s^2 / (1 + c).
//           The vectors carry an absolute rounding of about one unit, so for
//           near-coincident pairs (|s| < 2^-8) s is taken instead from the
//           exact difference of the wrapped positions, d = w_i - w_j (with
//           the periodic image when |d| > L/2), as sin(pi d / L) by its
//           Taylor series: the exponent -2 kappa s^2 then keeps full
//           relative accuracy at any kappa. A wave computes that only when
//           one of its pairs is that close, so it costs nothing away from
//           the diagonal tiles;
//   float : from 32-bit fixed-point phases, whose wrapped integer difference
//           gives phi in [-pi/2, pi/2) exactly up to one conversion; then
//           1 - c = phi^2 R(phi^2) with R the Taylor series of
//           (1 - cos phi) / phi^2 (6 terms, below float rounding on that
//           range) and s^2 = (1 - c)(1 + c) = q (2 - q). Normalisers 1/(L I0e(kappa)) and
// 1/(L I0e(kappa)^2) are applied once, in double, by the finalize kernel.
//
// Work decomposition: particles (sorted by angular cell) are cut into tiles
// of 256. A tile pair (I <= J) is taken one i-particle per thread against
// the J tile staged in LDS (every lane reads the same j: an LDS
// broadcast). Concentrations are processed in chunks of up to 16, each with
// per-thread accumulators; at the end of a chunk the 256 per-thread sums
// are reduced in double in a fixed order into the workgroup's running
// sums. A workgroup owns one slot: the tile pairs k = slot, slot + S, ...
// of the list ordered by circular tile distance (pair_decode), S =
// min(tile pairs, 32768), and writes the slot's 2B sums to its own row, so
// the partial sums take at most 32768 x 2B doubles at any N. No
// floating-point atomics are used.
//
// Terms whose exponent is below -70 need not be evaluated: each is below
// e^-70 (4e-31) times the largest term of its sum (the pair at distance 0
// has exponent 0 and I0e <= 1). Concentrations are ascending and the
// exponent scales with kappa, so once every lane of a wave is below the
// bound for one concentration, the wave skips the rest for that j (the
// power-sum route below skips none of its terms: its K-bar terms cost
// nothing per term, and its K terms are taken for every pair).
//
// Concentrations run in chunks of three kinds. The leading ones with
// 2 kappa below X0 (1.01 X0 in double; pure_branch), where the
// small-argument fit covers every pair: no
// term can reach the skip bound, so there is no vote, and the pair
// geometry is s^2 and c^2 alone; they have a loop of their own. In float,
// with only that branch's polynomial live, its coefficients stay in scalar
// registers instead of being rebuilt for every term. In double, whose
// polynomial has 21 coefficients, the K-bar terms are summed through the
// power sums of c^2 (power_sums_f64): the polynomials of these
// concentrations differ only by a power of a per-concentration scale, so a
// thread sums the powers of c^2 over its pairs once and forms each
// concentration's sum from them; on two tiles far enough apart, larger
// concentrations whose every pair there takes the small-argument branch
// join them. Those up to `nsmall`, where a
// term may take either Bessel branch. And the rest, where every term that
// is not skipped takes the large-argument fit: in float a loop of its own
// with two constants per concentration (in double the previous loop,
// which takes the fit for them). From npure on, the K-bar terms leave out
// a factor 1/sqrt(kappa) (the large-argument fit's 1/sqrt(2 kappa c) and
// the small-argument constant are scaled to match), which the finalize
// applies to their sums (KappaList::scale). Which loop a concentration
// takes depends on kappa alone, so the sums still do not depend on the
// chunk or group size.
#include "dev_sum.hpp"
#include "device_bessel.hpp"
#include "kde_internal.hpp"

namespace kde {


// The double small-argument fit keeps its accuracy a little past t = 1: up
// to x = 1.01 X0 (t = 1.0201) Horner's rule stays within 1.5e-15 relative,
// as on [0, X0] (against mpmath; pinned by a CPU test of the coefficient
// table). The float fit grows to 5.3e-7 there against 3.5e-7 on [0, X0],
// too close to the float form's bound, so it keeps X0.
template <typename T>
struct PureReach {
  static constexpr double value = 1.0;
};
template <>
struct PureReach<double> {
  static constexpr double value = 1.01;
};

template <typename T>
struct CvConsts {
  T A[KDE_MAX_KAPPAS];     // -2 kappa (double) or -2 kappa log2(e) (float)
  T vk[KDE_MAX_KAPPAS];    // X0 / kappa: v = X0 / (2 kappa c) = vk / (2 c)
  T em2k[KDE_MAX_KAPPAS];  // small-argument branch: exp(-2 kappa), times sqrt(kappa) from npure on
  T twok[KDE_MAX_KAPPAS];  // 2 kappa
  T tk[KDE_MAX_KAPPAS];    // (2 kappa / X0)^2: t = (R / X0)^2 = tk c^2
  int B;
  int npure;   // leading concentrations with pure_branch: every term takes the small-argument branch
  int nsmall;  // leading concentrations that may need the small-argument I0e branch
  T skip;      // exponent bound (in the unit of A)
};


// Pair-kernel exponents lie in [-2 kappa, 0] with kappa <= KDE_MAX_CV_KAPPA
// (checked on the host), inside the table exponential's domain; `tab` is
// the unit's LDS copy of KDE_EXP_TABLE (unused in float, where the exponent
// is in base 2 and the hardware exp2 serves).
__device__ __forceinline__ double exp_unit(double a, const double* __restrict__ tab) {
  return exp_nonpos_table(a, tab);
}
__device__ __forceinline__ float exp_unit(float a, const double* __restrict__) { return __builtin_amdgcn_exp2f(a); }

__device__ __forceinline__ double rcp_unit(double a) { return 1.0 / a; }
__device__ __forceinline__ float rcp_unit(float a) { return __builtin_amdgcn_rcpf(a); }
__device__ __forceinline__ double rsqrt_unit(double a) { return 1.0 / sqrt(a); }
__device__ __forceinline__ float rsqrt_unit(float a) { return __builtin_amdgcn_rsqf(a); }

__device__ __forceinline__ double i0_small(double t) { return i0_small_f64(t); }
__device__ __forceinline__ float i0_small(float t) { return i0_small_f32(t); }
__device__ __forceinline__ double i0e_sqrt_large(double t) { return i0e_sqrt_large_f64(t); }
__device__ __forceinline__ float i0e_sqrt_large(float t) { return i0e_sqrt_large_f32(t); }

template <typename T>
struct I0eBounds;
template <>
struct I0eBounds<double> {
  static constexpr double X0 = KDE_I0E_F64_X0;
};
template <>
struct I0eBounds<float> {
  static constexpr float X0 = KDE_I0E_F32_X0;
};

// Position of packed particle i as a fraction of the period, from its
// packed form: the wrapped position w (third component of the double
// form) times 1/L, the double position fraction, or the 32-bit phase.
__device__ __forceinline__ double packed_frac(const double* __restrict__ packed, int64_t i, double inv_L) {
  return packed[3 * i + 2] * inv_L;
}
__device__ __forceinline__ double packed_frac(const FracPos* __restrict__ packed, int64_t i, double) {
  return packed[i].f;
}
__device__ __forceinline__ double packed_frac(const uint32_t* __restrict__ packed, int64_t i, double) {
  return double(packed[i]) * (1.0 / 4294967296.0);
}

// Lower bound, in fractions of the period, on the periodic distance between
// any particle of tile [i0, i0 + ni) and any of tile [j0, j0 + nj), tiles of
// a sort by cell (`cells` cells) with the first tile before the second; a
// value <= 0 means no bound (overlapping or adjacent tiles). A tile spans the
// cells of its first and last particle; the cell read back from a packed
// value may differ from the sort's by one at a boundary (the packing
// rounds), so two cells of slack are added each way. A position within one
// phase step of L packs to 0 although it sorts into the last cell, so a
// tile whose last fraction is below its first reaches the end of the period.
// The two candidate gaps add up to at most 1, so the bound is at most 1/2.
template <typename P>
__device__ __forceinline__ double tile_gap(const P* __restrict__ packed, int64_t i0, int ni, int64_t j0, int nj,
                                           int cells, double inv_L) {
  const double c = double(cells);
  const double fI0 = packed_frac(packed, i0, inv_L), fI1 = packed_frac(packed, i0 + ni - 1, inv_L);
  const double fJ0 = packed_frac(packed, j0, inv_L), fJ1 = packed_frac(packed, j0 + nj - 1, inv_L);
  const double loI = (floor(fI0 * c) - 2.0) / c;
  const double hiI = (floor((fI1 < fI0 ? 1.0 : fI1) * c) + 3.0) / c;
  const double loJ = (floor(fJ0 * c) - 2.0) / c;
  const double hiJ = (floor((fJ1 < fJ0 ? 1.0 : fJ1) * c) + 3.0) / c;
  return fmin(loJ - hiI, 1.0 + loI - hiJ);
}

// A lower bound on 1 - cos(pi g) = 2 sin^2(pi g / 2) for a gap g in
// (0, 1/2]: sin y >= y - y^3 / 6 for y >= 0, and y = pi g / 2 <= pi / 4
// keeps that bound positive (it is below the sine by at most 0.4 %, which
// only makes the tile test that uses it a little less eager). Two constants
// instead of a sine's polynomial: the pair kernels keep this test's
// constants live across their loop over tile pairs.
__device__ __forceinline__ double one_minus_cos_pi_lower(double g) {
  const double y = 1.5707963267948966 * g;
  const double sl = y * fma(y * y, -1.0 / 6.0, 1.0);
  return 2.0 * sl * sl;
}

// Geometry of one pair: s^2, q = 1 - c, c, c^2, 1/(2c'), 1/sqrt(2c') with
// c' = max(c, X0 / (X0 + S)), S the skip exponent. c' = c wherever the
// large-argument Bessel fit is used for a term that is not negligible:
// for a concentration with 2 kappa <= X0 + S (which takes that fit only
// when 2 kappa c >= X0) c >= X0 / (2 kappa) >= X0 / (X0 + S); for one with
// 2 kappa > X0 + S, a pair with c below the floor has exponent -2 kappa
// (1 - c) < -S. Then v = X0 / (2 kappa c') <= 1 always, so the fit never
// leaves its interval and needs no per-term clamp.
template <typename T>
struct Geo {
  T s2, q, c, c2, inv2c, rs2c;
};

// The period, for the exact separation of near-coincident pairs.
struct Period {
  double L, half, pi_over_L;
};
__device__ __forceinline__ Period make_period(double L) { return Period{L, 0.5 * L, 3.141592653589793 / L}; }

constexpr double kNearS = 0.00390625;  // 2^-8: |s| below this takes the exact separation

template <typename T>
__device__ __forceinline__ T c_floor() {
  return T(double(I0eBounds<T>::X0) / (double(I0eBounds<T>::X0) + kSkipExponent));
}

// i-particle state held in registers.
template <typename T>
struct IPart;
template <>
struct IPart<double> {
  double a, b, w;
};
template <>
struct IPart<float> {
  uint32_t u;
};

__device__ __forceinline__ IPart<double> load_i(const double* __restrict__ packed, int64_t i, bool valid) {
  return IPart<double>{valid ? packed[3 * i] : 1.0, valid ? packed[3 * i + 1] : 0.0, valid ? packed[3 * i + 2] : 0.0};
}
__device__ __forceinline__ IPart<float> load_i(const uint32_t* __restrict__ packed, int64_t i, bool valid) {
  return IPart<float>{valid ? packed[i] : 0u};
}

// 1/d for d in [1, 2] and 1/sqrt(x) for x in [0.37, 2] (no zeros,
// infinities or subnormals can reach them): the hardware estimate and two
// Newton steps, which square its relative error twice to below 2^-53 --
// a few FMAs in place of the IEEE division and square-root sequences with
// their special-case scaling.
__device__ __forceinline__ double rcp_newton(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double rsqrt_newton(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);  // 1 - x y^2
  y = fma(0.5 * y, e, y);
  e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}

__device__ __forceinline__ Geo<double> pair_geo(const IPart<double>& p, const double* __restrict__ tj, int jj,
                                                const Period& per) {
  const double aj = tj[3 * jj], bj = tj[3 * jj + 1];
  const double c = fabs(p.a * aj + p.b * bj);
  double s = p.b * aj - p.a * bj;
  const bool near = fabs(s) < kNearS;
  if (__any(near)) {
    // d exact (Sterbenz) for close w; the image across the period by an
    // exact shift of the larger position. Only s^2 is used, so the sign
    // the image flips does not matter. |pi d / L| < 2^-7 here, where the
    // series' next term is below 1e-24 of the value.
    const double wj = tj[3 * jj + 2];
    double d = p.w - wj;
    d = (d > per.half) ? (p.w - per.L) - wj : ((d < -per.half) ? p.w - (wj - per.L) : d);
    const double ph = d * per.pi_over_L;
    const double p2 = ph * ph;
    const double sn = ph * fma(p2, fma(p2, fma(p2, -1.0 / 5040.0, 1.0 / 120.0), -1.0 / 6.0), 1.0);
    s = near ? sn : s;
  }
  Geo<double> g;
  g.s2 = s * s;
  g.q = g.s2 * rcp_newton(1.0 + c);  // 1 - c without cancellation
  g.c = c;
  g.c2 = c * c;
  const double cf = fmax(c, c_floor<double>());
  g.rs2c = rsqrt_newton(2.0 * cf);
  g.inv2c = g.rs2c * g.rs2c;
  return g;
}

// (1 - cos phi) / phi^2 for |phi| <= pi/2 as a polynomial in y = phi^2:
// its Taylor series to y^5. The first term left out, y^6 / 14!, is below
// 7e-9 of the value on that range (the value is at least 0.40 there), a
// tenth of a float unit.
__device__ __forceinline__ float one_minus_cos_ratio(float y) {
  float r = -1.0f / 479001600.0f;
  r = fmaf(r, y, 1.0f / 3628800.0f);
  r = fmaf(r, y, -1.0f / 40320.0f);
  r = fmaf(r, y, 1.0f / 720.0f);
  r = fmaf(r, y, -1.0f / 24.0f);
  return fmaf(r, y, 0.5f);
}

__device__ __forceinline__ Geo<float> pair_geo(const IPart<float>& p, const uint32_t* __restrict__ tj, int jj,
                                               const Period&) {
  // pi / 2^32 turns a wrapped phase difference into the half-angle difference
  const float phi = float(int32_t(p.u - tj[jj])) * 7.3145904152e-10f;
  const float y = phi * phi;
  const float r = one_minus_cos_ratio(y);
  Geo<float> g;
  g.q = y * r;
  g.c = 1.0f - g.q;
  g.s2 = g.q * (2.0f - g.q);
  g.c2 = g.c * g.c;
  const float cf = fmaxf(g.c, c_floor<float>());
  g.rs2c = __builtin_amdgcn_rsqf(2.0f * cf);
  g.inv2c = g.rs2c * g.rs2c;
  return g;
}

// s^2 and c^2 of one pair: all that the small-argument terms need.
template <typename T>
struct GeoS {
  T s2, c2;
};
__device__ __forceinline__ GeoS<double> pair_geo_small(const IPart<double>& p, const double* __restrict__ tj, int jj) {
  const double aj = tj[3 * jj], bj = tj[3 * jj + 1];
  const double c = p.a * aj + p.b * bj;
  const double s = p.b * aj - p.a * bj;
  return GeoS<double>{s * s, c * c};
}
__device__ __forceinline__ GeoS<float> pair_geo_small(const IPart<float>& p, const uint32_t* __restrict__ tj, int jj) {
  const float phi = float(int32_t(p.u - tj[jj])) * 7.3145904152e-10f;
  const float y = phi * phi;
  const float r = one_minus_cos_ratio(y);
  const float q = y * r;
  const float c = 1.0f - q;
  return GeoS<float>{q * (2.0f - q), c * c};
}

// Double concentrations whose every pair of a tile pair takes the
// small-argument branch: those with pure_branch (2 kappa < 1.01 X0), and on
// a tile pair whose two tiles are at least a gap g apart, also those with
// 2 kappa cos(pi g) < 1.01 X0 (c = |cos(pi d / L)| <= cos(pi g) there). Their
// K-bar terms are one polynomial, em2k Q(tk c^2), of every pair's c^2, with
// coefficients q_m common to all of these concentrations and only the
// scale tk (and em2k) differing; so the sum over j of a thread's terms is
// em2k sum_m q_m tk^m W_m with W_m = sum_j c^2m, the same sum reassociated.
// power_sums_f64 adds each pair's powers c^2m once per tile pair (m =
// 0..20: twenty multiplies and twenty-one adds per pair, however many such
// concentrations the tile pair has, against a 21-coefficient Horner per
// pair and concentration); kbar_from_sums_f64 forms each concentration's
// K-bar sum from the W_m; k_terms_f64 then takes their K terms over the
// tile, a pass at a time, in the order of the per-term loop. Every product
// q_m tk^m W_m is positive but the one of m = 19, which is below 2e-5 of
// the total, so the reassociation adds no cancellation. Which
// concentrations take this route on a tile pair depends on the tile pair
// and kappa alone, so the sums do not depend on the chunk or group size.
// (The float form keeps the per-term loop: its power sums, eleven
// compensated float sums, cost registers that the float kernel's eight
// waves do not have, and were not a consistent gain.)
template <bool MASKED>
__device__ __forceinline__ void power_sums_f64(const double* __restrict__ tj, int nj, const IPart<double>& ip,
                                               bool valid_i, bool diag, double (&W)[KDE_I0E_F64_NSMALL]) {
  constexpr int NS = KDE_I0E_F64_NSMALL;
#pragma unroll
  for (int m = 0; m < NS; ++m) W[m] = 0.0;
  for (int jj = 0; jj < nj; ++jj) {
    const double c = ip.a * tj[3 * jj] + ip.b * tj[3 * jj + 1];
    const double c2 = c * c;
    double p = 1.0;
    if (MASKED) p = (valid_i && (!diag || jj > int(threadIdx.x))) ? 1.0 : 0.0;
    W[0] += p;
#pragma unroll
    for (int m = 1; m < NS; ++m) {
      p *= c2;
      W[m] += p;
    }
  }
}

// The K-bar sum of concentration b from the power sums, per thread:
// em2k sum_m q_m tk^m W_m by Horner's rule in tk.
__device__ __forceinline__ double kbar_from_sums_f64(int b, const CvConsts<double>& K,
                                                     const double (&W)[KDE_I0E_F64_NSMALL]) {
  constexpr int NS = KDE_I0E_F64_NSMALL;
  constexpr double q[NS] = KDE_I0E_F64_SMALL;
  const double tk = K.tk[b];
  double r = q[NS - 1] * W[NS - 1];
#pragma unroll
  for (int m = NS - 2; m >= 0; --m) r = fma(r, tk, q[m] * W[m]);
  return K.em2k[b] * r;
}

// The K terms of concentrations [b0, b_end) (at most BC) over the tile,
// per thread, in the order of the per-term loop.
template <int BC, bool MASKED>
__device__ __forceinline__ void k_terms_f64(const double* __restrict__ tj, int nj, const IPart<double>& ip,
                                            bool valid_i, bool diag, int b0, int b_end, const CvConsts<double>& K,
                                            const double* __restrict__ etab, double (&v2)[BC]) {
  const int nb = min(BC, b_end - b0);
#pragma unroll
  for (int bb = 0; bb < BC; ++bb) v2[bb] = 0.0;
  for (int jj = 0; jj < nj; ++jj) {
    const double s = ip.b * tj[3 * jj] - ip.a * tj[3 * jj + 1];
    const double s2 = s * s;
    bool live = true;
    if (MASKED) live = valid_i && (!diag || jj > int(threadIdx.x));
#pragma unroll
    for (int bb = 0; bb < BC; ++bb) {
      if (bb < nb) {
        double t2 = exp_unit(K.A[b0 + bb] * s2, etab);
        if (MASKED) t2 = live ? t2 : 0.0;
        v2[bb] += t2;
      }
    }
  }
}

// Float concentrations [b0, b_end) with pure_branch (2 kappa < X0): every
// term takes the small-argument branch, and no exponent reaches -X0 > -S,
// so nothing is skipped. Same accumulation order as pair_chunk. The
// chunk's three constants per concentration sit in (scalar) registers. (The
// double form sums its K-bar terms through power sums: power_sums_f64.)
template <typename T, int BC, bool MASKED>
__device__ __forceinline__ void pair_chunk_pure(const typename Packed<T>::type* __restrict__ tj, int nj,
                                                const IPart<T>& ip, bool valid_i, bool diag, int b0, int b_end,
                                                const CvConsts<T>& K, const double* __restrict__ etab,
                                                Acc<T> (&acc1)[BC], Acc<T> (&acc2)[BC]) {
  constexpr bool hold = std::is_same<T, float>::value;
  const int nb = min(BC, b_end - b0);
  T Ab[BC], Eb[BC], Tb[BC];
#pragma unroll
  for (int bb = 0; bb < BC; ++bb) {
    Ab[bb] = (hold && bb < nb) ? K.A[b0 + bb] : T(0);
    Eb[bb] = (hold && bb < nb) ? K.em2k[b0 + bb] : T(0);
    Tb[bb] = (hold && bb < nb) ? K.tk[b0 + bb] : T(0);
  }
  for (int jj = 0; jj < nj; ++jj) {
    const GeoS<T> g = pair_geo_small(ip, tj, jj);
    bool live = true;
    if (MASKED) live = valid_i && (!diag || jj > int(threadIdx.x));
#pragma unroll
    for (int bb = 0; bb < BC; ++bb) {
      if (bb < nb) {
        const int b = b0 + bb;
        T t2 = exp_unit((hold ? Ab[bb] : K.A[b]) * g.s2, etab);
        T t1 = (hold ? Eb[bb] : K.em2k[b]) * i0_small((hold ? Tb[bb] : K.tk[b]) * g.c2);
        if (MASKED) {
          t1 = live ? t1 : T(0);
          t2 = live ? t2 : T(0);
        }
        acc1[bb].add(t1);
        acc2[bb].add(t2);
      }
    }
    if ((jj & (kRun - 1)) == kRun - 1) fold_all(acc1, acc2);
  }
  fold_all(acc1, acc2);
}

// Whether the concentrations from nsmall on run through a loop of their own
// (pair_chunk_large) in chunks that do not straddle nsmall. In float that
// loop holds its constants in scalar registers; in double it has nothing to
// gain, and the extra chunk boundary would cost a pass over the tile (its
// pair geometry) whenever the two ranges share a chunk's worth of
// concentrations: 3 % at 16 concentrations in [1, 1e4].
template <typename T>
constexpr bool kSplitLarge = std::is_same<T, float>::value;

// Concentrations [b0, b_end) from npure on (in float, below nsmall): a
// term of a concentration below nsmall takes the small-argument Bessel
// branch when 2 kappa c < X0, else the large-argument fit (both without the
// factor 1/sqrt(kappa)); from nsmall on, always the fit.
template <typename T, int BC, bool MASKED>
__device__ __forceinline__ void pair_chunk(const typename Packed<T>::type* __restrict__ tj, int nj,
                                           const IPart<T>& ip, bool valid_i, bool diag, int b0, int b_end,
                                           const CvConsts<T>& K, const Period& per, const double* __restrict__ etab,
                                           Acc<T> (&acc1)[BC], Acc<T> (&acc2)[BC]) {
  const int nb = min(BC, b_end - b0);
  const T X0 = I0eBounds<T>::X0;
  for (int jj = 0; jj < nj; ++jj) {
    const Geo<T> g = pair_geo(ip, tj, jj, per);
    bool live = true;
    if (MASKED) live = valid_i && (!diag || jj > int(threadIdx.x));
    // `go` is uniform across the wave: it turns false at the first
    // concentration for which every live pair of the wave is negligible
    bool go = true;
#pragma unroll
    for (int bb = 0; bb < BC; ++bb) {
      const int b = b0 + bb;
      go = go && (bb < nb);
      T A = T(0), Aq = T(0);
      if (go) {
        A = K.A[b];
        Aq = A * g.q;
        go = !__all(!live || Aq < K.skip);
      }
      if (go) {
        T t2 = exp_unit(A * g.s2, etab);
        T t1;
        const T R = K.twok[b] * g.c;
        if ((kSplitLarge<T> || b < K.nsmall) && R < X0) {
          t1 = K.em2k[b] * i0_small(K.tk[b] * g.c2);
        } else {
          t1 = exp_unit(Aq, etab) * (i0e_sqrt_large(g.inv2c * K.vk[b]) * g.rs2c);
        }
        if (MASKED) {
          t1 = live ? t1 : T(0);
          t2 = live ? t2 : T(0);
        }
        acc1[bb].add(t1);
        acc2[bb].add(t2);
      }
    }
    if ((jj & (kRun - 1)) == kRun - 1) fold_all(acc1, acc2);
  }
  fold_all(acc1, acc2);
}

// Concentrations [b0, b_end) at or above nsmall: a term that is not
// skipped takes the large-argument fit, exp(-2 kappa q) sqrt(x) I0e(x) /
// sqrt(x) with x = 2 kappa c; the 1/sqrt(kappa) of 1/sqrt(x) is left out
// here (the finalize applies it to the sum), so each concentration needs
// only its exponent factor and X0/kappa. In float those are read into
// (scalar) registers once per chunk instead of once per term; in double
// the registers they would take cost more than the loads.
template <typename T, int BC, bool MASKED>
__device__ __forceinline__ void pair_chunk_large(const typename Packed<T>::type* __restrict__ tj, int nj,
                                                 const IPart<T>& ip, bool valid_i, bool diag, int b0, int b_end,
                                                 const CvConsts<T>& K, const Period& per,
                                                 const double* __restrict__ etab, Acc<T> (&acc1)[BC],
                                                 Acc<T> (&acc2)[BC]) {
  constexpr bool hold = std::is_same<T, float>::value;
  const int nb = min(BC, b_end - b0);
  T Ab[BC], Vb[BC];
#pragma unroll
  for (int bb = 0; bb < BC; ++bb) {
    Ab[bb] = (hold && bb < nb) ? K.A[b0 + bb] : T(0);
    Vb[bb] = (hold && bb < nb) ? K.vk[b0 + bb] : T(0);
  }
  for (int jj = 0; jj < nj; ++jj) {
    const Geo<T> g = pair_geo(ip, tj, jj, per);
    bool live = true;
    if (MASKED) live = valid_i && (!diag || jj > int(threadIdx.x));
    bool go = true;
#pragma unroll
    for (int bb = 0; bb < BC; ++bb) {
      go = go && (bb < nb);
      T A = T(0), Aq = T(0);
      if (go) {
        A = hold ? Ab[bb] : K.A[b0 + bb];
        Aq = A * g.q;
        go = !__all(!live || Aq < K.skip);
      }
      if (go) {
        const T V = hold ? Vb[bb] : K.vk[b0 + bb];
        T t2 = exp_unit(A * g.s2, etab);
        T t1 = exp_unit(Aq, etab) * (i0e_sqrt_large(g.inv2c * V) * g.rs2c);
        if (MASKED) {
          t1 = live ? t1 : T(0);
          t2 = live ? t2 : T(0);
        }
        acc1[bb].add(t1);
        acc2[bb].add(t2);
      }
    }
    if ((jj & (kRun - 1)) == kRun - 1) fold_all(acc1, acc2);
  }
  fold_all(acc1, acc2);
}

// Waves per SIMD the pair kernels are compiled for, by (precision, pass
// size): the occupancy the register use of the tile-pair body allows on
// its own. Without the hint the loop over a slot's tile pairs lets the
// compiler keep more values live across it (hoisted constants, scalar
// values spilled to vector lanes), which costs one to four waves; with it,
// the few values that no longer fit are reloaded once per tile pair.
template <typename T, int BC>
struct PairWaves {
  static constexpr int value = 4;
};
template <> struct PairWaves<double, 4> { static constexpr int value = 6; };
template <> struct PairWaves<double, 8> { static constexpr int value = 5; };
template <> struct PairWaves<double, 16> { static constexpr int value = 4; };
template <> struct PairWaves<float, 4> { static constexpr int value = 8; };
template <> struct PairWaves<float, 8> { static constexpr int value = 6; };

// Shared memory of one tile-pair unit.
template <typename T, int BC>
struct CvSmem {
  typename Packed<T>::type tj[Packed<T>::per_particle * kCvTile];
  double red[kBlock / 64][2 * BC];
  double unit_acc[2 * KDE_MAX_KAPPAS];
  double etab[std::is_same<T, double>::value ? 256 : 1];  // exponential table (double form)
  // double: per-wave K-bar sums of the power-sum route, by concentration
  double kbar_red[kBlock / 64][std::is_same<T, double>::value ? KDE_MAX_KAPPAS : 1];
  int b_end;
  int p_end;  // double: concentrations [b_lo, p_end) take the power-sum route on this tile pair
};

// The workgroup's sums of one pass, concentrations [b0, bc_end): each
// thread's sums v1 (K-bar) and v2 (K) in double (WHICH: 1 the K-bar sums
// only, 2 the K sums only, 3 both), reduced over the wave by a fixed
// butterfly, over the waves in wave order, and added to the slot's running
// sums sm.unit_acc. Ends with a barrier.
template <typename T, int BC, int WHICH = 3>
__device__ __forceinline__ void reduce_chunk_values(const double (&v1)[BC], const double (&v2)[BC], int b0,
                                                    int bc_end, int B, CvSmem<T, BC>& sm) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int bb = 0; bb < BC; ++bb) {
    if (WHICH & 1) {
      const double w1 = wave_sum(v1[bb]);
      if (lane == 0) sm.red[wave][bb] = w1;
    }
    if (WHICH & 2) {
      const double w2 = wave_sum(v2[bb]);
      if (lane == 0) sm.red[wave][BC + bb] = w2;
    }
  }
  __syncthreads();
  if (tid < 2 * BC) {
    const int bb = tid % BC;
    const int which = tid / BC;  // 0: Kbar sums, 1: K sums
    if (b0 + bb < bc_end && (WHICH & (1 << which))) {
      double v = 0.0;
      for (int w = 0; w < kBlock / 64; ++w) v += sm.red[w][tid];
      sm.unit_acc[which * B + b0 + bb] += v;
    }
  }
  __syncthreads();
}

// One tile pair of the pair sums: tile I (one i per thread) against tile J
// (staged in LDS), concentrations [b_lo, b_hi); adds this pair's sums into
// the slot's running sums sm.unit_acc ([Kbar sums | K sums], 2B entries,
// each one added to in a fixed order: chunk reductions in wave order,
// tile pairs in the order of the slot's list). The exponential table
// (double form) must be staged and visible. A tile pair may be split over
// several units by concentration range: every concentration accumulates
// the same terms in the same order whatever the range. Ends with a
// barrier, so the caller may reuse `sm`.
//
// Concentrations are ascending, and a pair's K-bar exponent -2 kappa q
// (q = 1 - cos(pi d / L), growing with the periodic distance d) is the
// larger of its two exponents. With gap the lower bound on the distance
// between the two tiles (from `cells`, the sort's cell count), every term
// of a concentration with kappa q_min > S/2 (q_min a lower bound on
// 1 - cos(pi gap), S the skip exponent) is below the skip bound, so the unit stops before the
// first such concentration; the margin of 1e-6 keeps this a subset of what
// the per-term test would skip, so the sums are those of the full loop.
template <typename T, int BC>
__device__ __forceinline__ void cv_tile_pair(const typename Packed<T>::type* __restrict__ packed, int64_t n,
                                             int cells, double L, int I, int J, const CvConsts<T>& K, int b_lo,
                                             int b_hi, CvSmem<T, BC>& sm) {
  constexpr int pp = Packed<T>::per_particle;
  const Period per = make_period(L);
  const int tid = threadIdx.x;
  const int64_t i0 = int64_t(I) * kCvTile, j0 = int64_t(J) * kCvTile;
  const int nj = int(min(int64_t(kCvTile), n - j0));
  if (tid == 0) {
    int be = b_hi;
    int pe = max(b_lo, min(K.npure, b_hi));
    if (I != J) {
      const double gap = tile_gap(packed, i0, int(min(int64_t(kCvTile), n - i0)), j0, nj, cells, 1.0 / L);
      if (gap > 0.0) {
        const double qmin = one_minus_cos_pi_lower(gap);
        be = b_lo;
        while (be < b_hi && !(double(K.twok[be]) * qmin > kSkipExponent * (1.0 + 1e-6))) ++be;
        if constexpr (std::is_same<T, double>::value) {
          // every pair has c <= cos(pi gap) (gap <= 1/2) <= 1 - x^2/2 + x^4/24
          // with x = pi gap (the cosine's Taylor bound from above, a few
          // operations instead of a library call); the margin covers the
          // rounding of c itself
          const double x2 = (3.141592653589793 * gap) * (3.141592653589793 * gap);
          const double cmax = fma(x2, fma(x2, 1.0 / 24.0, -0.5), 1.0) + 1e-12;
          while (pe < be && double(K.twok[pe]) * cmax < PureReach<double>::value * double(I0eBounds<double>::X0)) ++pe;
        }
      }
    }
    sm.b_end = be;
    sm.p_end = min(pe, be);
  }
  for (int k = tid; k < pp * nj; k += kBlock) sm.tj[k] = packed[pp * j0 + k];
  const int64_t i = i0 + tid;
  const bool valid_i = i < n;
  const IPart<T> ip = load_i(packed, i, valid_i);
  const bool diag = (I == J);
  const bool masked = diag || (int64_t(I + 1) * kCvTile > n);
  __syncthreads();
  const int b_end = sm.b_end;

  int b0 = b_lo;
  if constexpr (std::is_same<T, double>::value) {
    const int p_end = sm.p_end;
    if (b0 < p_end) {
      double W[KDE_I0E_F64_NSMALL];
      if (masked)
        power_sums_f64<true>(sm.tj, nj, ip, valid_i, diag, W);
      else
        power_sums_f64<false>(sm.tj, nj, ip, valid_i, diag, W);
      // the K-bar sums of the whole range first, with no barrier between
      // them, so that the power sums are dead before the K terms' passes:
      // per concentration the thread's sum, its wave's sum into LDS; then
      // the waves' sums in wave order into the running sums
      const int lane = tid & 63, wave = tid >> 6;
      for (int b = b0; b < p_end; ++b) {
        const double w = wave_sum(kbar_from_sums_f64(b, K, W));
        if (lane == 0) sm.kbar_red[wave][b] = w;
      }
      __syncthreads();
      for (int b = b0 + tid; b < p_end; b += kBlock) {
        double v = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) v += sm.kbar_red[w][b];
        sm.unit_acc[b] += v;
      }
      __syncthreads();
    }
    while (b0 < p_end) {
      const int bc_end = min(b0 + BC, p_end);
      double v2[BC];
      if (masked)
        k_terms_f64<BC, true>(sm.tj, nj, ip, valid_i, diag, b0, bc_end, K, sm.etab, v2);
      else
        k_terms_f64<BC, false>(sm.tj, nj, ip, valid_i, diag, b0, bc_end, K, sm.etab, v2);
      reduce_chunk_values<T, BC, 2>(v2, v2, b0, bc_end, K.B, sm);
      b0 = bc_end;
    }
  }
  for (; b0 < b_end;) {
    // chunks do not straddle npure, nor in float nsmall
    const int bc_end = min(b0 + BC, b0 < K.npure ? min(b_end, K.npure)
                                                 : (kSplitLarge<T> && b0 < K.nsmall ? min(b_end, K.nsmall) : b_end));
    Acc<T> s1[BC], s2[BC];
#pragma unroll
    for (int bb = 0; bb < BC; ++bb) {
      s1[bb].zero();
      s2[bb].zero();
    }
    if (b0 < K.npure) {  // float only: in double these took the power-sum route above
      if constexpr (std::is_same<T, float>::value) {
        if (masked)
          pair_chunk_pure<T, BC, true>(sm.tj, nj, ip, valid_i, diag, b0, bc_end, K, sm.etab, s1, s2);
        else
          pair_chunk_pure<T, BC, false>(sm.tj, nj, ip, valid_i, diag, b0, bc_end, K, sm.etab, s1, s2);
      }
    } else if (!kSplitLarge<T> || b0 < K.nsmall) {
      if (masked)
        pair_chunk<T, BC, true>(sm.tj, nj, ip, valid_i, diag, b0, bc_end, K, per, sm.etab, s1, s2);
      else
        pair_chunk<T, BC, false>(sm.tj, nj, ip, valid_i, diag, b0, bc_end, K, per, sm.etab, s1, s2);
    } else {
      if (masked)
        pair_chunk_large<T, BC, true>(sm.tj, nj, ip, valid_i, diag, b0, bc_end, K, per, sm.etab, s1, s2);
      else
        pair_chunk_large<T, BC, false>(sm.tj, nj, ip, valid_i, diag, b0, bc_end, K, per, sm.etab, s1, s2);
    }
    double v1[BC], v2[BC];
#pragma unroll
    for (int bb = 0; bb < BC; ++bb) {
      v1[bb] = s1[bb].value();
      v2[bb] = s2[bb].value();
    }
    reduce_chunk_values<T, BC>(v1, v2, b0, bc_end, K.B, sm);
    b0 = bc_end;
  }
}

// Item k of the list of the T(T+1)/2 tile pairs of T sorted tiles in
// order of circular tile distance e = min(J - I, T - (J - I)): band e holds
// the pairs with J - I = e (I ascending) and then those with J - I = T - e
// (the pairs that are neighbours across the period), T items per band (the
// last band T/2 when T is even). Tiles hold equal particle counts of the
// cell-sorted positions, so the separation of a pair, and with it the work
// of its tile pair, falls with e: the list runs roughly from the most to
// the least expensive tile pair.
__device__ __forceinline__ void pair_decode(int64_t k, int T, int& I, int& J) {
  const int64_t t = T;
  const int64_t e = k / t;
  const int64_t r = k - e * t;
  if (r < t - e) {
    I = int(r);
    J = int(r + e);
  } else {
    I = int(r - (t - e));
    J = int(r);
  }
}

// One slot of the pair sums: the tile pairs k = slot, slot + nslots,
// slot + 2 nslots, ... of the list of pair_decode, in that order, for
// concentrations [b_lo, b_hi); writes those entries of the slot's row of
// 2B running sums [Kbar sums | K sums] at `out`. Up to kCvMaxSlots tile
// pairs every slot holds one, and the workgroups, dispatched in slot order,
// take the most expensive tile pairs first; beyond that the partial sums
// stay at kCvMaxSlots rows and each slot takes tile pairs from every band.
// Used by the one-set kernel and by the batched engine (the same slots and
// order, so their sums are bitwise equal). Ends with a barrier.
template <typename T, int BC>
__device__ __forceinline__ void cv_slot(const typename Packed<T>::type* __restrict__ packed, int64_t n, int cells,
                                        double L, int64_t slot, int64_t nslots, const CvConsts<T>& K, int b_lo,
                                        int b_hi, double* __restrict__ out, CvSmem<T, BC>& sm) {
  const int tid = threadIdx.x;
  for (int k = tid; k < 2 * KDE_MAX_KAPPAS; k += kBlock) sm.unit_acc[k] = 0.0;
  if constexpr (std::is_same<T, double>::value) {
    constexpr double etab_src[256] = KDE_EXP_TABLE;
    for (int k = tid; k < 256; k += kBlock) sm.etab[k] = etab_src[k];
  }
  const int ntiles = int((n + kCvTile - 1) / kCvTile);
  const int64_t items = int64_t(ntiles) * (ntiles + 1) / 2;
  for (int64_t k = slot; k < items; k += nslots) {
    int I, J;
    pair_decode(k, ntiles, I, J);
    cv_tile_pair<T, BC>(packed, n, cells, L, I, J, K, b_lo, b_hi, sm);
  }
  __syncthreads();
  const int nk = b_hi - b_lo;
  for (int k = tid; k < 2 * nk; k += kBlock) {
    const int e = (k / nk) * K.B + b_lo + k % nk;
    out[e] = sm.unit_acc[e];
  }
  __syncthreads();
}

// Whether a term of concentration k may take the small-argument Bessel
// branch (2 kappa |c| < X0) without being negligible: such a term carries
// weight exp(-2 kappa (1 - |c|)) <= exp(-(2 kappa - X0)), below the skip
// bound once 2 kappa - X0 exceeds it. With pure_branch, decides the chunk
// kind of k.
template <typename T>
inline bool small_branch_live(double k) {
  return 2.0 * k - double(I0eBounds<T>::X0) <= kSkipExponent;
}

// Whether every term of concentration k takes the small-argument branch:
// 2 kappa < reach X0, so 2 kappa |c| < reach X0 for every pair and t =
// (2 kappa c / X0)^2 stays where the fit holds. (In double, without the
// stretch a concentration just above X0/2, such as 10^(28/31) = 8.0003 of
// 32 values log-spaced in [1, 1e4], would take the general loop: per term
// a skip vote, the reciprocal geometry and either branch.)
template <typename T>
inline bool pure_branch(double k) {
  return 2.0 * k < PureReach<T>::value * double(I0eBounds<T>::X0);
}

// Per-concentration constants of the pair kernel, computed on the host.
template <typename T>
inline CvConsts<T> make_consts(const double* kappas, int B) {
  CvConsts<T> K{};
  const double log2e = 1.4426950408889634;
  const double unit = std::is_same<T, float>::value ? log2e : 1.0;
  const double X0 = double(I0eBounds<T>::X0);
  K.B = B;
  K.nsmall = 0;
  K.npure = 0;
  for (int b = 0; b < B; ++b) {
    const double k = kappas[b];
    K.A[b] = T(-2.0 * k * unit);
    K.vk[b] = T(X0 / k);
    K.em2k[b] = T(std::exp(-2.0 * k) * (pure_branch<T>(k) ? 1.0 : std::sqrt(k)));
    K.twok[b] = T(2.0 * k);
    K.tk[b] = T((2.0 * k / X0) * (2.0 * k / X0));
    if (small_branch_live<T>(k)) K.nsmall = b + 1;
    if (pure_branch<T>(k)) K.npure = b + 1;
  }
  K.skip = T(-kSkipExponent * unit);
  return K;
}

// Concentrations of a scan as the finalize takes them, with the factor
// scale[b] it applies to the raw K-bar sum of b: 1/sqrt(kappa) where the
// pair loops left it out of the terms (from npure on), else 1.
struct KappaList {
  double k[KDE_MAX_KAPPAS];
  double scale[KDE_MAX_KAPPAS];
};

template <typename T>
inline KappaList make_kappa_list(const double* kappas, int B) {
  KappaList kl{};
  for (int b = 0; b < B; ++b) {
    kl.k[b] = kappas[b];
    kl.scale[b] = pure_branch<T>(kappas[b]) ? 1.0 : 1.0 / std::sqrt(kappas[b]);
  }
  return kl;
}

// The objective from the unordered pair sums of one set, by one workgroup
// (thread b handles concentration b): raw[0..B) = sum_{i<j} exp(-2k(1-c))
// I0e(2kc), raw[B..2B) = sum_{i<j} exp(-2k s^2). Normalisers in double;
// writes cv[B], optional sums[2B] (normalised), and returns nothing; the
// first-minimum index is written by thread 0 into *argmin (if not NULL)
// and into `v` (LDS, B doubles) the objective values.
__device__ __forceinline__ void cv_finalize_block(const double* __restrict__ raw, int B, double n, double L,
                                                  const KappaList& kap, double* __restrict__ cv,
                                                  double* __restrict__ sums, int32_t* __restrict__ argmin,
                                                  double* v, int* best_out) {
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    const double k = kap.k[b];
    const double ik = i0e_f64(k);
    const double i2k = i0e_f64(2.0 * k);
    const double S1 = raw[b] * kap.scale[b] / (L * ik * ik);
    const double S2 = raw[B + b] / (L * ik);
    const double kbar0 = i2k / (L * ik * ik);
    const double val = (n * kbar0 + 2.0 * S1) / (n * n) - 4.0 * S2 / (n * (n - 1.0));
    if (cv) cv[b] = val;
    v[b] = val;
    if (sums) {
      sums[b] = S1;
      sums[B + b] = S2;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int best = 0;
    for (int t = 1; t < B; ++t)
      if (v[t] < v[best]) best = t;
    if (argmin) *argmin = best;
    if (best_out) *best_out = best;
  }
  __syncthreads();
}

}  // namespace kde
