// HIP kernels for gfx950 (MI355X): one pass of a batched complex FFT of
// power-of-two length L, applied along rows (contiguous vectors) or down
// columns (vectors strided by the row length).
//
// Algorithm. The paper's FFT (Section 2.2, Listing 1, Fig. 2) is radix-2
// Cooley-Tukey by decimation in time: bit-reversal reordering, then log2 L
// butterfly steps whose span doubles each step, each butterfly computing
// f = d1 * w, d1 = d0 - f, d0 = d0 + f with a precomputed twiddle w. Here the
// log2 L steps are grouped into a few passes of radix R = 2^s:
//   * inside a pass, each thread holds R points in registers and runs s
//     radix-2 DIT steps on them, on bit-reversed register order (the
//     bit-reversal is a renaming of registers, free at run time; the in-pass
//     twiddles W_2^q ... W_R^q are compile-time constants evaluated in double
//     precision and rounded once);
//   * between passes, the points are multiplied by the inter-pass twiddles
//     W_{Ns R}^{k r} (FP32 table, computed in FP64 on the host) and written
//     back through LDS directly into the order the next pass reads (a Stockham
//     auto-sort). The paper makes the same move on the Tensix (Section 4,
//     Fig. 5): each step reorders straight into the next step's order rather
//     than back to the natural order. Here that reordering happens on-chip,
//     so the digit reversal of the whole transform costs no HBM traffic.
// Each pass kernel therefore reads every point from HBM once, coalesced, and
// writes it once, coalesced (first pass loads point tt + T*j into register j,
// the last pass stores register j to point tt + T*j).
//
// Pass p (radix R, Ns = product of the earlier radices) in Stockham form:
// butterfly b in [0, L/R) takes points b + r L/R (r < R), multiplies point r
// by W_{Ns R}^{(b mod Ns) r}, transforms the R points, and sends output s to
// position (b div Ns) Ns R + (b mod Ns) + s Ns.
//
// Column mode: a workgroup owns C adjacent columns; lanes run over the
// columns first, so each load/store instruction touches rows of C*8 bytes.
// Where C*8 is less than a 128-byte line, column workgroups are remapped so
// that each of the 8 XCDs (each with its own L2) works through a contiguous
// range of column tiles: neighbouring tiles share cache lines and are then
// served by the same L2 (PassArgs::remap; the plan decides).
#pragma once

#include "fft_internal.h"

#include <hip/hip_ext.h>

#include <type_traits>

namespace fft2d {
namespace dev {

// ---------------------------------------------------------------- utilities
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n >> 1); }

template <int R>
constexpr int bitrev(int x) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) {
    r = (r << 1) | (x & 1);
    x >>= 1;
  }
  return r;
}

// Compile-time cos/sin of 2 pi q / n in double precision: the angle is
// reduced to an octant in integers, then a Taylor series on [0, pi/4].
constexpr double kQuarterPi = 0.78539816339744830961566084581988;

constexpr double series_sin(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double series_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

struct CosSin {
  double c, s;
};

constexpr CosSin unit_root(long q, long n) {
  q %= n;
  if (q < 0) q += n;
  const long o = (8 * q) / n;        // octant of 2 pi q / n
  const long rem = 8 * q - o * n;    // angle inside the octant: (pi/4) rem / n
  double cphi = 0.0, sphi = 0.0;     // angle inside the quadrant
  if ((o & 1) == 0) {
    const double a = kQuarterPi * (double)rem / (double)n;
    cphi = series_cos(a);
    sphi = series_sin(a);
  } else {
    const double b = kQuarterPi * (double)(n - rem) / (double)n;  // pi/2 - phi
    cphi = series_sin(b);
    sphi = series_cos(b);
  }
  switch (o >> 1) {
    case 0: return {cphi, sphi};
    case 1: return {-sphi, cphi};
    case 2: return {-cphi, -sphi};
    default: return {sphi, -cphi};
  }
}

typedef float f2v __attribute__((ext_vector_type(2)));

// Global loads/stores of one complex64; NT selects the nontemporal (streaming) form.
template <bool NT>
__device__ __forceinline__ float2 gload(const float2* p) {
  if constexpr (NT) {
    const f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(p));
    return make_float2(v.x, v.y);
  } else {
    return *p;
  }
}
template <bool NT>
__device__ __forceinline__ void gstore(float2* p, float2 v) {
  if constexpr (NT) {
    f2v w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, reinterpret_cast<f2v*>(p));
  } else {
    *p = v;
  }
}

// Raw buffer access: a wave-uniform resource (base address and size in bytes)
// plus a per-lane byte offset and a uniform byte offset. Accesses at or past
// `bytes` read zero and drop stores (hardware range check).
constexpr int kBufferDword3 = 0x00020000;
constexpr int kAuxNontemporal = 2;
constexpr int kAuxDevice = 16;  // sc1: device-scope load, not served from the CU's L1

struct Buf {
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ Buf(const void* base, uint32_t bytes)
      : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufferDword3)) {}
  template <int AUX = 0>
  __device__ __forceinline__ float2 load(uint32_t voff, uint32_t soff) const {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, AUX));
  }
  __device__ __forceinline__ void store(float2 v, uint32_t voff, uint32_t soff) const {
    using raw = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(raw, v), r, (int)voff, (int)soff, 0);
  }
};

// Byte size of the range [base_point, total_points) of a complex64 buffer, as
// a buffer resource size (every tile's accesses lie below 2^28 points).
__device__ __forceinline__ uint32_t span_bytes(int64_t total_points, int64_t base_point) {
  int64_t n = total_points - base_point;
  if (n < 0) n = 0;
  if (n > (int64_t(1) << 28)) n = int64_t(1) << 28;
  return (uint32_t)(n * 8);
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// v * exp(DIR * 2 pi i Q / N), with the trivial rotations done by swaps.
template <int DIR, int N, int Q>
__device__ __forceinline__ float2 rotate(float2 v) {
  constexpr int q = ((Q % N) + N) % N;
  if constexpr (q == 0) {
    return v;
  } else if constexpr (2 * q == N) {
    return make_float2(-v.x, -v.y);
  } else if constexpr (4 * q == N) {  // exp(DIR i pi / 2) = DIR i
    if constexpr (DIR < 0) return make_float2(v.y, -v.x);
    else return make_float2(-v.y, v.x);
  } else if constexpr (4 * q == 3 * N) {  // = -DIR i
    if constexpr (DIR < 0) return make_float2(-v.y, v.x);
    else return make_float2(v.y, -v.x);
  } else {
    constexpr CosSin w = unit_root(q, N);
    constexpr float c = (float)w.c;
    constexpr float s = (float)(DIR * w.s);
    return make_float2(v.x * c - v.y * s, v.x * s + v.y * c);
  }
}

// Radix-2 butterfly with the twiddle w = W_N^Q (exponent sign DIR):
// (lo, hi) <- (lo + w hi, lo - w hi). Trivial twiddles (1, -1, +-i) are
// swaps. For odd multiples of pi/4 (|cos| = |sin| = c) w hi = c (u, v) with
// u, v one addition each, and each output component is one FMA. A general
// twiddle gives lo - w hi in two FMAs per component and lo + w hi as
// 2 lo - (lo - w hi), one FMA per component: six instructions where a complex
// multiplication and two complex additions take eight.
template <int DIR, int N, int Q>
__device__ __forceinline__ void bfly(float2& lo, float2& hi) {
  constexpr int q = ((Q % N) + N) % N;
  if constexpr (q == 0 || 2 * q == N || 4 * q == N || 4 * q == 3 * N) {
    const float2 f = rotate<DIR, N, Q>(hi);
    hi = csub(lo, f);
    lo = cadd(lo, f);
  } else if constexpr ((8 * q) % N == 0) {
    constexpr CosSin w = unit_root(q, N);
    constexpr float c = (float)w.c;
    constexpr float s = (float)(DIR * w.s);
    static_assert(s == c || s == -c, "an odd multiple of pi/4 has |cos| = |sin|");
    constexpr float sg = (s == c) ? 1.0f : -1.0f;
    const float u = hi.x - sg * hi.y;
    const float v = sg * hi.x + hi.y;
    hi = make_float2(fmaf(-c, u, lo.x), fmaf(-c, v, lo.y));
    lo = make_float2(fmaf(c, u, lo.x), fmaf(c, v, lo.y));
  } else {
    constexpr CosSin w = unit_root(q, N);
    constexpr float c = (float)w.c;
    constexpr float s = (float)(DIR * w.s);
    const float2 h = make_float2(fmaf(-c, hi.x, fmaf(s, hi.y, lo.x)), fmaf(-c, hi.y, fmaf(-s, hi.x, lo.y)));
    lo = make_float2(fmaf(2.0f, lo.x, -h.x), fmaf(2.0f, lo.y, -h.y));
    hi = h;
  }
}

// First radix-2 step of an R-point DFT whose inputs a[k] are multiplied by
// run-time twiddles w[k] first (w[0] = 1): the pair (a[k] w[k], a[k + R/2]
// w[k + R/2]) gives lo - w' hi in two FMAs per component after the complex
// product a[k] w[k], and lo + w' hi = 2 lo - (lo - w' hi) in one.
__device__ __forceinline__ void bfly_tw(float2& lo, float2& hi, float2 wl, float2 wh, bool lo_one) {
  const float2 l = lo_one ? lo : cmul(lo, wl);
  const float2 h = make_float2(fmaf(-wh.x, hi.x, fmaf(wh.y, hi.y, l.x)), fmaf(-wh.x, hi.y, fmaf(-wh.y, hi.x, l.y)));
  lo = make_float2(fmaf(2.0f, l.x, -h.x), fmaf(2.0f, l.y, -h.y));
  hi = h;
}

// In-register R-point DFT (exponent sign DIR), natural order in and out,
// computed as log2 R radix-2 decimation-in-time steps on bit-reversed data:
// at the step of span h, points lo and lo + h (lo mod h = q) combine with the
// twiddle W_{2h}^q. With TW, input k is first multiplied by w[k] (k >= 1;
// w[0] is not read), fused into the first step.
template <int R, int DIR, bool TW = false>
__device__ __forceinline__ void dft_impl(float2 (&a)[R], const float2 (&w)[R]) {
  float2 b[R];
  static_for<0, R>([&](auto I) {
    constexpr int i = decltype(I)::value;
    b[bitrev<R>(i)] = a[i];
  });
  static_for<0, ilog2c(R)>([&](auto S) {
    constexpr int h = 1 << decltype(S)::value;
    static_for<0, R / (2 * h)>([&](auto G) {
      static_for<0, h>([&](auto Qv) {
        constexpr int q = decltype(Qv)::value;
        constexpr int lo = decltype(G)::value * 2 * h + q;
        constexpr int hi = lo + h;
        if constexpr (TW && h == 1) {
          // b[lo] = a[k], b[hi] = a[k + R/2] with k = bitrev(lo)
          constexpr int k = bitrev<R>(lo);
          bfly_tw(b[lo], b[hi], w[k], w[k + R / 2], k == 0);
        } else {
          bfly<DIR, 2 * h, q>(b[lo], b[hi]);
        }
      });
    });
  });
  static_for<0, R>([&](auto I) {
    constexpr int i = decltype(I)::value;
    a[i] = b[i];
  });
}

template <int R, int DIR>
__device__ __forceinline__ void dft(float2 (&a)[R]) {
  const float2 none[R] = {};
  dft_impl<R, DIR, false>(a, none);
}

// R-point DFT of a[k] * w[k] (w[0] = 1 is not read).
template <int R, int DIR>
__device__ __forceinline__ void dft_tw(float2 (&a)[R], const float2 (&w)[R]) {
  dft_impl<R, DIR, true>(a, w);
}

// ------------------------------------------------------------ configuration
template <int L_, int E_, int C_, int Q_, bool COL_, int... Rs>
struct Cfg {
  static constexpr int L = L_;   // FFT length
  static constexpr int E = E_;   // points per thread
  static constexpr int C = C_;   // vectors per workgroup
  static constexpr int Q = Q_;   // LDS exchange rounds
  static constexpr bool COL = COL_;
  static constexpr int P = sizeof...(Rs);
  static constexpr int T = L / E;  // threads per vector
  static constexpr int THREADS = T * C;
  static constexpr int LQ = L / Q;  // points of one vector exchanged per round

  static constexpr int radix(int p) {
    const int r[] = {Rs...};
    return r[p];
  }
  static constexpr int ns(int p) {
    int v = 1;
    for (int q = 0; q < p; ++q) v *= radix(q);
    return v;
  }
  static constexpr int tw_off(int p) {
    int o = 0;
    for (int q = 1; q < p; ++q) o += ns(q) * (radix(q) - 1);
    return o;
  }
  static constexpr int max_exchanged_radix() {  // largest radix of a pass followed by an LDS exchange
    int m = 1;
    for (int p = 0; p + 1 < P; ++p) m = radix(p) > m ? radix(p) : m;
    return m;
  }
  // LDS rows get one padding slot per 2^PADSHIFT points: every 16 for radix-16
  // write patterns; every 32 where a pass followed by an exchange has radix 32
  // or more (its lanes write slots 32 apart: one pad per 16 would put lanes k
  // and k + 16 on the same banks), except for row vectors shorter than 32
  // threads, whose rows are offset from each other already (ROWSTRIDE).
  static constexpr int PADSHIFT = (max_exchanged_radix() >= 32 && (COL || T >= 32)) ? 5 : 4;
  static constexpr int PADSPAN = 1 << PADSHIFT;
  static constexpr int pad(int e) { return e + (e >> PADSHIFT); }
  static constexpr int LQP = pad(LQ - 1) + 1;
  // Row mode: consecutive vectors of one wave start T banks-pairs apart.
  static constexpr int ROWSTRIDE = (T >= 32) ? LQP : (LQP + T);
  static constexpr int LDS_ELEMS = (P > 1) ? (COL ? LQP * C : ROWSTRIDE * C) : 1;

  __device__ static __forceinline__ int lds_index(int c, int e) {
    if constexpr (COL) return pad(e) * C + c;
    else return c * ROWSTRIDE + pad(e);
  }
  // Slot distance of point e0 + x from point e0 when the low PADSHIFT bits of
  // e0 and of x never carry into bit PADSHIFT (then pad(e0 + x) = pad(e0) +
  // pad(x)), so that an address is a per-thread base plus a compile-time
  // offset.
  static constexpr int lds_delta(int x) { return COL ? pad(x) * C : pad(x); }

  // Exchange rounds. Output s of butterfly b of pass p goes to position
  // (b div Ns) Ns R + (b mod Ns) + s Ns, inside a block of Ns R positions; with
  // Ns R <= L/Q every butterfly's outputs fall in one round, round b div
  // (L/(Q R)). Where a thread has at least Q butterflies per pass (E/R a
  // multiple of Q) that round depends on the butterfly's index i only
  // (by_index); otherwise (fewer butterflies than rounds) also on the thread.
  static constexpr bool by_index(int p) { return (E / radix(p)) % Q == 0; }

  static constexpr bool valid() {
    int prod = 1;
    for (int p = 0; p < P; ++p) {
      if (E % radix(p) != 0) return false;
      prod *= radix(p);
    }
    if (prod != L || L % E != 0 || THREADS > 1024 || THREADS % 64 != 0) return false;
    if (Q > 1) {
      for (int p = 0; p + 1 < P; ++p) {
        if (by_index(p)) {
          if (ns(p) > T) return false;  // destinations of one butterfly stay in one round
        } else if (ns(p) * radix(p) > LQ) {
          return false;
        }
      }
    }
    return E % Q == 0 && LDS_ELEMS * 8 <= 160 * 1024;
  }
};

constexpr int kKindPass = 0;
constexpr int kKindCombine = 1;
constexpr int kKindCrossRow = 2;
constexpr int kKindWaveRow = 3;

__device__ __forceinline__ int xcd_remap(int b, int nb) {
  // Consecutive workgroup ids are dispatched round-robin over the 8 XCDs; give
  // XCD x the contiguous id range [x q + min(x, r), ...) in dispatch order.
  const int x = b & 7, i = b >> 3;
  const int q = nb >> 3, r = nb & 7;
  return x * q + (x < r ? x : r) + i;
}

// One pass: butterflies of this thread, then (unless last) the LDS exchange.
// `tw` covers this pass kernel's twiddle table.
// ARITH = false keeps the data movement of the pass (the LDS exchange in the
// same order) and drops its arithmetic (twiddle loads, multiplications and the
// butterflies): the "compute off" variant used to measure the pass's
// data-movement ceiling.
// RD selects what each thread reads back after the exchange: 0, the points
// tt + T j of its own vector (the next pass's inputs); 1 (row mode, last
// exchange of a row pass with cross-row last stage, see rowx_tile), for every
// row c' of the workgroup the points t + r L/RL (r < RL, RL = the last radix)
// into d[c' RL + r], t the thread's index in the workgroup; 2, no exchange:
// output s of butterfly i stays in d[i R + s].
template <class K, int DIR, int p, int SB = 0, bool ARITH = true, int RD = 0>
__device__ __forceinline__ void run_pass(float2 (&d)[K::E], float2* lds, int tt, int c, const Buf& tw) {
  constexpr int R = K::radix(p);
  constexpr int Ns = K::ns(p);
  constexpr int NB = K::E / R;
  constexpr bool last = (p == K::P - 1);
  float2 o[K::E];
  static_for<0, NB>([&](auto I) {
    constexpr int i = decltype(I)::value;
    const int b = tt + K::T * i;
    float2 x[R];
    static_for<0, R>([&](auto Rr) {
      constexpr int r = decltype(Rr)::value;
      x[r] = d[i + NB * r];
    });
    if constexpr (p > 0 && ARITH) {
      const uint32_t voff = (uint32_t)(b & (Ns - 1)) * 8u;
      float2 w[R];
      w[0] = make_float2(1.0f, 0.0f);
      static_for<1, R>([&](auto Rr) {
        constexpr int r = decltype(Rr)::value;
        w[r] = tw.load(voff, (uint32_t)(K::tw_off(p) + (r - 1) * Ns) * 8u);
        if constexpr (DIR > 0) w[r].y = -w[r].y;
      });
      dft_tw<R, DIR>(x, w);
    } else if constexpr (ARITH) {
      dft<R, DIR>(x);
    }
    static_for<0, R>([&](auto S) {
      constexpr int s = decltype(S)::value;
      if constexpr (last) d[i + NB * s] = x[s];
      else o[i * R + s] = x[s];
    });
    // SB: keep the scheduler from hoisting the next butterfly's twiddle loads
    // above this one (bounds register pressure at some latency cost).
    if constexpr (SB != 0) __builtin_amdgcn_sched_barrier(0);
  });
  if constexpr (!last && RD == 2) {
    // no exchange: output s of butterfly i stays in d[i R + s] (the caller moves it)
    static_for<0, K::E>([&](auto J) { d[decltype(J)::value] = o[decltype(J)::value]; });
  } else if constexpr (!last) {
    constexpr int EQ = K::E / K::Q;
    // writes of butterfly i (positions relative to round h's first point)
    auto put = [&](auto I, int h) {
      constexpr int i = decltype(I)::value;
      const int b = tt + K::T * i;
      const int dst = (b / Ns) * Ns * R + (b & (Ns - 1)) - h * K::LQ;
      if constexpr (Ns * R >= K::PADSPAN) {
        // dst's low PADSHIFT bits are b mod Ns (< Ns), and s Ns adds multiples of Ns
        const int wbase = K::lds_index(c, dst);
        static_for<0, R>([&](auto S) {
          constexpr int s = decltype(S)::value;
          lds[wbase + K::lds_delta(s * Ns)] = o[i * R + s];
        });
      } else {
        static_for<0, R>([&](auto S) {
          constexpr int s = decltype(S)::value;
          lds[K::lds_index(c, dst + s * Ns)] = o[i * R + s];
        });
      }
    };
    static_for<0, K::Q>([&](auto H) {
      constexpr int h = decltype(H)::value;
      if constexpr (K::by_index(p)) {
        constexpr int NBQ = NB / K::Q;
        static_for<h * NBQ, (h + 1) * NBQ>([&](auto I) { put(I, h); });
      } else {
        // fewer butterflies than rounds: butterfly b's round is b div (L/(Q R))
        static_for<0, NB>([&](auto I) {
          if ((tt + K::T * decltype(I)::value) / (K::LQ / R) == h) put(I, h);
        });
      }
      __syncthreads();
      if constexpr (RD == 0) {
        // reads: point tt + T j' (j' < EQ) of the round, tt < T, so the slot is
        // lds_index(c, tt) + lds_delta(T j')
        const int rbase = K::lds_index(c, tt);
        static_for<0, EQ>([&](auto J) {
          constexpr int jj = decltype(J)::value;
          d[h * EQ + jj] = lds[rbase + K::lds_delta(K::T * jj)];
        });
      } else {
        constexpr int RL = K::radix(K::P - 1);
        constexpr int RLQ = RL / K::Q;  // last-stage inputs r of round h: h RLQ <= r < (h + 1) RLQ
        constexpr int SPAN = K::L / RL;  // = THREADS, a multiple of PADSPAN
        const int t = (int)threadIdx.x;
        static_for<0, K::C>([&](auto Cc) {
          constexpr int cr = decltype(Cc)::value;
          static_for<0, RLQ>([&](auto Rq) {
            constexpr int r = h * RLQ + decltype(Rq)::value;
            d[cr * RL + r] = lds[cr * K::ROWSTRIDE + K::pad(t) + K::pad(decltype(Rq)::value * SPAN)];
          });
        });
      }
      __syncthreads();
    });
  }
}

// Exchange of 4 x 4 blocks across a wave's four 16-lane rows in registers:
// for every B < 4 the registers v[4B + c] (c < 4) become w[A] with w[A] on
// row c equal to v[4B + c] on row A, stored to v[4A + B] (lanes within a row
// keep their data). Two v_permlane32_swap (rows 2, 3 of one register against
// rows 0, 1 of another) and two v_permlane16_swap (odd rows against even
// rows) per block and component.
__device__ __forceinline__ void swap32(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b),
                                                  false, false);
  a = __builtin_bit_cast(float, (unsigned)r[0]);
  b = __builtin_bit_cast(float, (unsigned)r[1]);
}
__device__ __forceinline__ void swap16(float& a, float& b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b),
                                                  false, false);
  a = __builtin_bit_cast(float, (unsigned)r[0]);
  b = __builtin_bit_cast(float, (unsigned)r[1]);
}
__device__ __forceinline__ void transpose_rows4x4(float2 (&v)[16]) {
  float2 w[16];
  static_for<0, 4>([&](auto Bb) {
    constexpr int B = decltype(Bb)::value;
    float2 x0 = v[4 * B], x1 = v[4 * B + 1], x2 = v[4 * B + 2], x3 = v[4 * B + 3];
    swap32(x0.x, x2.x);
    swap32(x0.y, x2.y);
    swap32(x1.x, x3.x);
    swap32(x1.y, x3.y);
    swap16(x0.x, x1.x);
    swap16(x0.y, x1.y);
    swap16(x2.x, x3.x);
    swap16(x2.y, x3.y);
    w[B] = x0;
    w[4 + B] = x1;
    w[8 + B] = x2;
    w[12 + B] = x3;
  });
  static_for<0, 16>([&](auto I) { v[decltype(I)::value] = w[decltype(I)::value]; });
}

// One 1024-point row per 64-lane wave (radix 16, 16, 4; 16 points per lane):
// the exchange after the first pass goes through the LDS, the one after the
// second runs in registers. Pass 1 sends output s = 4B + c of lane 16A + l to
// point 256 A + l + 64 B + 16 c, which the last pass reads as register 4A + B
// of lane 16c + l: a 4 x 4 transpose of (16-lane row, register) blocks.
template <class K, int DIR, int AUX, int MODE = 0>
__device__ __forceinline__ void row_wave_tile(const PassArgs& a, int w, float2* lds) {
  static_assert(K::L == 1024 && K::T == 64 && K::C == 1 && K::E == 16 && K::P == 3 && K::Q == 1 &&
                    K::radix(0) == 16 && K::radix(1) == 16 && K::radix(2) == 4 && !K::COL,
                "one 1024-point row per wave, radix 16 x 16 x 4");
  const int tt = threadIdx.x;
  const int64_t base = (int64_t)w * K::L;
  const Buf src(a.in + base, span_bytes(a.total, base));
  const Buf dst(a.out + base, span_bytes(a.total, base));
  const Buf tw(a.tw, (uint32_t)a.tw_count * 8u);
  float2 d[K::E];
  static_for<0, K::E>([&](auto J) {
    d[decltype(J)::value] = src.load<AUX>((uint32_t)tt * 8u, (uint32_t)(K::T * decltype(J)::value) * 8u);
  });
  if constexpr (MODE < 2) {
    run_pass<K, DIR, 0, 0, MODE == 0>(d, lds, tt, 0, tw);
    run_pass<K, DIR, 1, 0, MODE == 0, 2>(d, lds, tt, 0, tw);
    transpose_rows4x4(d);
    run_pass<K, DIR, 2, 0, MODE == 0>(d, lds, tt, 0, tw);
  }
  if (w < a.nvec) {
    const float sc = a.scale;
    static_for<0, K::E>([&](auto J) {
      constexpr int j = decltype(J)::value;
      dst.store(make_float2(d[j].x * sc, d[j].y * sc), (uint32_t)tt * 8u, (uint32_t)(K::T * j) * 8u);
    });
  }
}

// MODE as for fft_tile (1: loads, exchanges and stores only; 2: loads and
// stores only).
template <class K, int DIR, bool NT, int MODE = 0>
__global__ __launch_bounds__(64) void row_wave_kernel(PassArgs a) {
  __shared__ float2 lds[K::LDS_ELEMS];
  row_wave_tile<K, DIR, NT ? kAuxNontemporal : 0, MODE>(a, blockIdx.x, lds);
}

// Conjugation and scaling of one tile's input and output. A forward-sign
// kernel computes the inverse transform as conj(F(conj(x))) / (M N); the
// batched path uses this instead of a second set of kernels.
struct TileIO {
  bool conj_in = false;
  bool conj_out = false;
  float scale = 1.0f;
};

// One workgroup's tile of a pass: C vectors starting at vector w*C (w must be
// wave-uniform). Global memory is reached through buffer resources based at
// the tile's first point, so every lane needs one 32-bit offset register and
// the E points differ by uniform offsets.
// AUX: cache policy of the input loads (0, kAuxNontemporal, or kAuxDevice).
// MODE: 0 the FFT; 1 its data movement only (loads, LDS exchanges, stores;
// no arithmetic); 2 loads and stores only (a copy with the tile's access
// pattern). Modes 1 and 2 are measurement variants (the paper's Table 2
// times its FFT with components switched off in the same way).
template <class K, int DIR, int AUX = 0, int SB = 0, int MODE = 0>
__device__ __forceinline__ void fft_tile(const PassArgs& a, int w, float2* lds, TileIO io) {
  const int t = threadIdx.x;
  const int c = K::COL ? (t % K::C) : (t / K::T);
  const int tt = K::COL ? (t / K::C) : (t % K::T);
  const int64_t v0 = (int64_t)w * K::C;
  const bool active = v0 + c < a.nvec;
  int64_t base_in, base_out, es_in, es_out;
  uint32_t lane_in, lane_out;  // point offsets of this lane's vector from the tile bases
  if constexpr (K::COL) {
    // vector v = (grid g, residue k1, column col); element e is row
    // k1 + M1*e of grid g on input and on output (M1 = a.m1; plain column
    // pass: M1 = 1), so a tile reads and writes the same points.
    const int64_t per_g = a.m1 * a.ncols;
    auto start = [&](int64_t v) {
      const int64_t g = v / per_g;
      const int64_t rem = v - g * per_g;  // = k1 * ncols + col
      return g * (int64_t)K::L * per_g + rem;
    };
    base_in = base_out = start(v0);
    if (a.ncols >= K::C) {  // the tile's columns share one grid and residue
      lane_in = lane_out = (uint32_t)c;
    } else {
      lane_in = lane_out = (uint32_t)(start(v0 + c) - base_in);
    }
    es_in = es_out = per_g;
  } else {
    base_in = base_out = v0 * K::L;
    lane_in = lane_out = (uint32_t)(c * K::L);
    es_in = es_out = 1;
  }
  const Buf src(a.in + base_in, span_bytes(a.total, base_in));
  const Buf dst(a.out + base_out, span_bytes(a.total, base_out));
  const Buf tw(a.tw, (uint32_t)a.tw_count * 8u);
  const uint32_t voff_in = (lane_in + (uint32_t)(tt * es_in)) * 8u;
  const uint32_t voff_out = (lane_out + (uint32_t)(tt * es_out)) * 8u;
  const uint32_t sj_in = (uint32_t)(K::T * es_in) * 8u;
  const uint32_t sj_out = (uint32_t)(K::T * es_out) * 8u;
  float2 d[K::E];
  static_for<0, K::E>([&](auto J) {
    constexpr int j = decltype(J)::value;
    d[j] = src.load<AUX>(voff_in, sj_in * j);
  });
  if (io.conj_in) static_for<0, K::E>([&](auto J) { d[decltype(J)::value].y = -d[decltype(J)::value].y; });
  if constexpr (MODE < 2)
    static_for<0, K::P>([&](auto Pp) { run_pass<K, DIR, decltype(Pp)::value, SB, MODE == 0>(d, lds, tt, c, tw); });
  if (active) {
    const float sc = io.scale;
    const float sy = io.conj_out ? -sc : sc;
    static_for<0, K::E>([&](auto J) {
      constexpr int j = decltype(J)::value;
      dst.store(make_float2(d[j].x * sc, d[j].y * sy), voff_out, sj_out * j);
    });
  }
}

template <class K, int DIR, bool NT = false, int WPE = 1, int SB = 0, int MODE = 0>
__global__ __launch_bounds__(K::THREADS) __attribute__((amdgpu_waves_per_eu(WPE))) void pass_kernel(PassArgs a) {
  static_assert(K::valid(), "invalid pass configuration");
  __shared__ float2 lds[K::LDS_ELEMS];
  const int w = (K::COL && a.remap) ? xcd_remap(blockIdx.x, a.nblocks) : (int)blockIdx.x;
  TileIO io;
  io.scale = a.scale;
  fft_tile<K, DIR, NT ? kAuxNontemporal : 0, SB, MODE>(a, w, lds, io);
}

// Row pass with combine (first half of a split column transform, see
// PassArgs): tile w = (grid g, m2) transforms the M1 = C rows M2*m1 + m2,
// then for every column position an M1-point DFT across those rows and the
// twiddle W_M^(m2 k1), stored to row M1*m2 + k1 (the tile's output is the M1
// consecutive rows starting at row M1*m2). The rows' transformed points
// are exchanged through LDS in Q rounds of L/Q positions; in each round every
// thread owns L/(Q*THREADS) positions and all M1 rows of each. Only
// io.conj_in is honoured (the output is an intermediate, never final).
// MODE as for fft_tile: 1 keeps the loads, both LDS exchanges and the stores
// (no row FFTs, no combine DFT, no twiddles); 2 stores each loaded row to its
// output row (row M2*c + m2 to row M1*m2 + c) without LDS.
template <class K, int DIR, int AUX = 0, int SB = 0, int MODE = 0>
__device__ __forceinline__ void rowc_tile(const PassArgs& a, int64_t w, float2* lds, TileIO io) {
  static_assert(K::valid() && !K::COL && K::C >= 2 && K::P > 1, "invalid combine configuration");
  constexpr int M1 = K::C;
  constexpr int NQ = K::L / K::Q;
  constexpr int NPOS = NQ / K::THREADS;
  static_assert(NPOS >= 1 && NQ % K::THREADS == 0, "positions per thread must be whole");
  const int t = threadIdx.x;
  const int c = t / K::T;
  const int tt = t % K::T;
  const int64_t g = w / a.m2;
  const int64_t m2 = w - g * a.m2;
  const int64_t gbase = g * a.m2 * M1 * K::L;
  // input rows M2*c + m2 of grid g: the tile base is row m2, lane rows c*M2
  // further; output rows M1*m2 + k1
  const int64_t base = gbase + m2 * K::L;
  const int64_t obase = gbase + m2 * M1 * K::L;
  const Buf src(a.in + base, span_bytes(a.total, base));
  const Buf dst(a.out + obase, span_bytes(a.total, obase));
  const Buf tw(a.tw, (uint32_t)a.tw_count * 8u);
  const uint32_t row_bytes = (uint32_t)(a.m2 * K::L) * 8u;  // from row m2 + M2*k to row m2 + M2*(k+1)
  const uint32_t voff_in = (uint32_t)c * row_bytes + (uint32_t)tt * 8u;
  float2 d[K::E];
  static_for<0, K::E>([&](auto J) {
    constexpr int j = decltype(J)::value;
    d[j] = src.load<AUX>(voff_in, (uint32_t)(K::T * j) * 8u);
  });
  if (io.conj_in) static_for<0, K::E>([&](auto J) { d[decltype(J)::value].y = -d[decltype(J)::value].y; });
  if constexpr (MODE == 2) {
    const uint32_t voff_out = (uint32_t)c * (uint32_t)(K::L * 8) + (uint32_t)tt * 8u;
    static_for<0, K::E>([&](auto J) {
      constexpr int j = decltype(J)::value;
      dst.store(d[j], voff_out, (uint32_t)(K::T * j) * 8u);
    });
    return;
  }
  static_for<0, K::P>([&](auto Pp) { run_pass<K, DIR, decltype(Pp)::value, SB, MODE == 0>(d, lds, tt, c, tw); });
  float2 wk[M1];
  if constexpr (MODE == 0) {
    static_for<1, M1>([&](auto Kk) {
      constexpr int k1 = decltype(Kk)::value;
      float2 w1 = a.twc[m2 * k1];
      if constexpr (DIR > 0) w1.y = -w1.y;
      wk[k1] = w1;
    });
  }
  static_for<0, K::Q>([&](auto H) {
    constexpr int h = decltype(H)::value;
    constexpr int EQ = K::E / K::Q;
    const int wbase = K::lds_index(c, tt);
    static_for<0, EQ>([&](auto J) {
      constexpr int jj = decltype(J)::value;
      lds[wbase + K::lds_delta(K::T * jj)] = d[h * EQ + jj];
    });
    __syncthreads();
    const int rbase = K::lds_index(0, t);
    static_for<0, NPOS>([&](auto I) {
      constexpr int i = decltype(I)::value;
      float2 x[M1];
      static_for<0, M1>([&](auto R) {
        constexpr int r = decltype(R)::value;
        x[r] = lds[rbase + r * K::ROWSTRIDE + K::lds_delta(K::THREADS * i)];
      });
      if constexpr (MODE == 0) dft<M1, DIR>(x);
      const uint32_t voff = (uint32_t)(h * NQ + K::THREADS * i + t) * 8u;
      static_for<0, M1>([&](auto Kk) {
        constexpr int k1 = decltype(Kk)::value;
        dst.store((k1 == 0 || MODE != 0) ? x[k1] : cmul(x[k1], wk[k1]), voff, (uint32_t)(k1 * K::L) * 8u);
      });
    });
    __syncthreads();
  });
}

template <class K, int DIR, int WPE = 1, int SB = 0, bool NT = false, int MODE = 0>
__global__ __launch_bounds__(K::THREADS) __attribute__((amdgpu_waves_per_eu(WPE))) void rowc_kernel(PassArgs a) {
  __shared__ float2 lds[K::LDS_ELEMS];
  rowc_tile<K, DIR, NT ? kAuxNontemporal : 0, SB, MODE>(a, blockIdx.x, lds, TileIO{});
}

// Row pass with combine whose last FFT stage runs across the workgroup's rows
// (the same result as rowc_tile with one LDS exchange fewer). The length-L
// row FFT's last stage has radix RL = E / M1 and L / RL = THREADS butterflies
// per row; its inputs cross the LDS in the exchange after the stage before,
// and thread t takes butterfly t of every one of the M1 rows (RL points each).
// The stage's outputs t + s L/RL of the M1 rows are then exactly the points
// the M1-point combine needs, so the combine DFT and its twiddle W_M^(m2 k1)
// run in registers and store row k1's points t + s L/RL (coalesced over t).
// The twiddles of the last stage, W_L^(t r), are the same for every row and
// loaded once. MODE as for rowc_tile.
template <class K, int DIR, int AUX = 0, int SB = 0, int MODE = 0>
__device__ __forceinline__ void rowx_tile(const PassArgs& a, int64_t w, float2* lds, TileIO io) {
  constexpr int M1 = K::C;
  constexpr int RL = K::radix(K::P - 1);
  constexpr int SPAN = K::L / RL;
  static_assert(K::valid() && !K::COL && M1 >= 2 && K::P > 1, "invalid combine configuration");
  static_assert(RL * M1 == K::E && SPAN == K::THREADS && RL % K::Q == 0 && SPAN % K::PADSPAN == 0,
                "the last stage must take one butterfly of every row per thread");
  const int t = threadIdx.x;
  const int c = t / K::T;
  const int tt = t % K::T;
  const int64_t g = w / a.m2;
  const int64_t m2 = w - g * a.m2;
  const int64_t gbase = g * a.m2 * M1 * K::L;
  const int64_t base = gbase + m2 * K::L;
  const int64_t obase = gbase + m2 * M1 * K::L;
  const Buf src(a.in + base, span_bytes(a.total, base));
  const Buf dst(a.out + obase, span_bytes(a.total, obase));
  const Buf tw(a.tw, (uint32_t)a.tw_count * 8u);
  const uint32_t row_bytes = (uint32_t)(a.m2 * K::L) * 8u;  // from row m2 + M2*k to row m2 + M2*(k+1)
  const uint32_t voff_in = (uint32_t)c * row_bytes + (uint32_t)tt * 8u;
  float2 d[K::E];
  static_for<0, K::E>([&](auto J) {
    constexpr int j = decltype(J)::value;
    d[j] = src.load<AUX>(voff_in, (uint32_t)(K::T * j) * 8u);
  });
  if (io.conj_in) static_for<0, K::E>([&](auto J) { d[decltype(J)::value].y = -d[decltype(J)::value].y; });
  if constexpr (MODE == 2) {
    const uint32_t voff_out = (uint32_t)c * (uint32_t)(K::L * 8) + (uint32_t)tt * 8u;
    static_for<0, K::E>([&](auto J) {
      constexpr int j = decltype(J)::value;
      dst.store(d[j], voff_out, (uint32_t)(K::T * j) * 8u);
    });
    return;
  }
  static_for<0, K::P - 2>([&](auto Pp) { run_pass<K, DIR, decltype(Pp)::value, SB, MODE == 0>(d, lds, tt, c, tw); });
  run_pass<K, DIR, K::P - 2, SB, MODE == 0, 1>(d, lds, tt, c, tw);
  float2 wk[M1];
  if constexpr (MODE == 0) {
    float2 wl[RL];
    wl[0] = make_float2(1.0f, 0.0f);
    static_for<1, RL>([&](auto Rr) {
      constexpr int r = decltype(Rr)::value;
      float2 v = tw.load((uint32_t)t * 8u, (uint32_t)(K::tw_off(K::P - 1) + (r - 1) * SPAN) * 8u);
      if constexpr (DIR > 0) v.y = -v.y;
      wl[r] = v;
    });
    static_for<1, M1>([&](auto Kk) {
      constexpr int k1 = decltype(Kk)::value;
      float2 w1 = a.twc[m2 * k1];
      if constexpr (DIR > 0) w1.y = -w1.y;
      wk[k1] = w1;
    });
    static_for<0, M1>([&](auto Cc) {
      constexpr int cr = decltype(Cc)::value;
      float2 x[RL];
      static_for<0, RL>([&](auto Rr) { x[decltype(Rr)::value] = d[cr * RL + decltype(Rr)::value]; });
      dft_tw<RL, DIR>(x, wl);
      static_for<0, RL>([&](auto S) { d[cr * RL + decltype(S)::value] = x[decltype(S)::value]; });
    });
  }
  static_for<0, RL>([&](auto S) {
    constexpr int s = decltype(S)::value;
    float2 z[M1];
    static_for<0, M1>([&](auto Cc) { z[decltype(Cc)::value] = d[decltype(Cc)::value * RL + s]; });
    if constexpr (MODE == 0) dft<M1, DIR>(z);
    static_for<0, M1>([&](auto Kk) {
      constexpr int k1 = decltype(Kk)::value;
      dst.store((k1 == 0 || MODE != 0) ? z[k1] : cmul(z[k1], wk[k1]), (uint32_t)t * 8u,
                (uint32_t)(k1 * K::L + s * SPAN) * 8u);
    });
  });
}

template <class K, int DIR, int WPE = 1, int SB = 0, bool NT = false, int MODE = 0>
__global__ __launch_bounds__(K::THREADS) __attribute__((amdgpu_waves_per_eu(WPE))) void rowx_kernel(PassArgs a) {
  __shared__ float2 lds[K::LDS_ELEMS];
  rowx_tile<K, DIR, NT ? kAuxNontemporal : 0, SB, MODE>(a, blockIdx.x, lds, TileIO{});
}

// Whole-grid tile: one workgroup computes the complete 2D transform of one
// M x N grid (M = KC::L rows, N = KR::L columns), reading and writing every
// point once. Row tiles of KR::C rows are loaded and transformed in turn; each
// passes through the LDS, where every thread picks up the points of the
// columns it owns in KC's layout (column v*KC::C + cc, points ttc + KC::T*j)
// and keeps them in registers; then the columns are transformed and stored.
// src/dst cover the grid (row-major, N contiguous); tr/tc are the twiddle
// tables of KR's and KC's schedules.
template <class KR, class KC>
constexpr int grid_lds_elems() {
  int m = KR::LDS_ELEMS > KC::LDS_ELEMS ? KR::LDS_ELEMS : KC::LDS_ELEMS;
  return KR::C * KR::L > m ? KR::C * KR::L : m;
}

template <class KR, class KC, int DIR>
__device__ __forceinline__ void grid_tile(const Buf& src, const Buf& dst, const Buf& tr, const Buf& tc, TileIO io,
                                          float2* lds) {
  constexpr int M = KC::L;
  constexpr int N = KR::L;
  static_assert(KR::valid() && KC::valid() && !KR::COL && KC::COL, "row and column configurations");
  static_assert(KR::THREADS == KC::THREADS, "one workgroup runs both");
  static_assert(M % KR::C == 0 && N % KC::C == 0, "whole tiles");
  static_assert(KR::C % KC::T == 0, "a row tile holds whole point blocks of the column layout");
  constexpr int NRT = M / KR::C;
  constexpr int NCT = N / KC::C;
  constexpr int JR = KR::C / KC::T;  // column points j of row tile u: u * JR <= j < (u + 1) * JR
  const int t = threadIdx.x;
  const int cr = t / KR::T, ttr = t % KR::T;  // row tiles: row cr of the tile, points ttr + T j
  const int cc = t % KC::C, ttc = t / KC::C;  // column tiles: column cc of the tile, points ttc + T j
  float2 dcl[NCT][KC::E];
  static_for<0, NRT>([&](auto U) {
    constexpr int u = decltype(U)::value;
    float2 dr[KR::E];
    const uint32_t voff = (uint32_t)((u * KR::C + cr) * N + ttr) * 8u;
    static_for<0, KR::E>([&](auto J) {
      constexpr int j = decltype(J)::value;
      dr[j] = src.load(voff, (uint32_t)(KR::T * j) * 8u);
      if (io.conj_in) dr[j].y = -dr[j].y;
    });
    if constexpr (u > 0) __syncthreads();  // the previous row tile's points have been read from LDS
    static_for<0, KR::P>([&](auto Pp) { run_pass<KR, DIR, decltype(Pp)::value>(dr, lds, ttr, cr, tr); });
    __syncthreads();
    static_for<0, KR::E>([&](auto J) {
      constexpr int j = decltype(J)::value;
      lds[cr * N + ttr + KR::T * j] = dr[j];
    });
    __syncthreads();
    static_for<0, NCT>([&](auto V) {
      constexpr int v = decltype(V)::value;
      static_for<0, JR>([&](auto J) {
        constexpr int j = u * JR + decltype(J)::value;
        dcl[v][j] = lds[(ttc + KC::T * j - u * KR::C) * N + v * KC::C + cc];
      });
    });
  });
  __syncthreads();  // the column passes reuse the LDS
  const float sc = io.scale;
  const float sy = io.conj_out ? -sc : sc;
  static_for<0, NCT>([&](auto V) {
    constexpr int v = decltype(V)::value;
    static_for<0, KC::P>([&](auto Pp) { run_pass<KC, DIR, decltype(Pp)::value>(dcl[v], lds, ttc, cc, tc); });
    const uint32_t voff = (uint32_t)(ttc * N + v * KC::C + cc) * 8u;
    static_for<0, KC::E>([&](auto J) {
      constexpr int j = decltype(J)::value;
      dst.store(make_float2(dcl[v][j].x * sc, dcl[v][j].y * sy), voff, (uint32_t)(KC::T * j * N) * 8u);
    });
  });
}

// Whole-grid kernel: workgroup g transforms grid g of the batch (a.nvec grids
// of KC::L x KR::L; a.tw = KR's table, a.twc = KC's table).
template <class KR, class KC, int DIR>
__global__ __launch_bounds__(KR::THREADS) void grid_kernel(PassArgs a) {
  __shared__ float2 lds[grid_lds_elems<KR, KC>()];
  constexpr int64_t P = (int64_t)KR::L * KC::L;
  const int64_t base = (int64_t)blockIdx.x * P;
  const Buf src(a.in + base, span_bytes(a.total, base));
  const Buf dst(a.out + base, span_bytes(a.total, base));
  const Buf tr(a.tw, (uint32_t)KR::tw_off(KR::P) * 8u);
  const Buf tc(a.twc, (uint32_t)KC::tw_off(KC::P) * 8u);
  TileIO io;
  io.scale = a.scale;
  grid_tile<KR, KC, DIR>(src, dst, tr, tc, io, lds);
}

// Launch through hipExtLaunchKernel with start and stop events, which then
// take the kernel's own begin and end times.
inline hipError_t launch_timed(void (*kernel)(PassArgs), const PassArgs& a, int threads, hipStream_t s,
                               hipEvent_t t0, hipEvent_t t1) {
  PassArgs copy = a;
  void* args[] = {&copy};
  return hipExtLaunchKernel(reinterpret_cast<const void*>(kernel), dim3(a.nblocks), dim3(threads), args, 0, s,
                            t0, t1, 0);
}

template <class K, int WPE, bool NT>
hipError_t launch_pass(const PassArgs& a, int dir, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  if (t0 != nullptr || t1 != nullptr)
    return launch_timed(dir < 0 ? pass_kernel<K, -1, NT, WPE> : pass_kernel<K, +1, NT, WPE>, a, K::THREADS, s,
                        t0, t1);
  if (dir < 0) hipLaunchKernelGGL((pass_kernel<K, -1, NT, WPE>), dim3(a.nblocks), dim3(K::THREADS), 0, s, a);
  else hipLaunchKernelGGL((pass_kernel<K, +1, NT, WPE>), dim3(a.nblocks), dim3(K::THREADS), 0, s, a);
  return hipGetLastError();
}

template <class K, int WPE, bool NT>
hipError_t launch_rowc(const PassArgs& a, int dir, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  if (t0 != nullptr || t1 != nullptr)
    return launch_timed(dir < 0 ? rowc_kernel<K, -1, WPE, 0, NT> : rowc_kernel<K, +1, WPE, 0, NT>, a, K::THREADS,
                        s, t0, t1);
  if (dir < 0) hipLaunchKernelGGL((rowc_kernel<K, -1, WPE, 0, NT>), dim3(a.nblocks), dim3(K::THREADS), 0, s, a);
  else hipLaunchKernelGGL((rowc_kernel<K, +1, WPE, 0, NT>), dim3(a.nblocks), dim3(K::THREADS), 0, s, a);
  return hipGetLastError();
}

template <class K, int WPE, bool NT>
hipError_t launch_rowx(const PassArgs& a, int dir, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  if (t0 != nullptr || t1 != nullptr)
    return launch_timed(dir < 0 ? rowx_kernel<K, -1, WPE, 0, NT> : rowx_kernel<K, +1, WPE, 0, NT>, a, K::THREADS,
                        s, t0, t1);
  if (dir < 0) hipLaunchKernelGGL((rowx_kernel<K, -1, WPE, 0, NT>), dim3(a.nblocks), dim3(K::THREADS), 0, s, a);
  else hipLaunchKernelGGL((rowx_kernel<K, +1, WPE, 0, NT>), dim3(a.nblocks), dim3(K::THREADS), 0, s, a);
  return hipGetLastError();
}

template <class K, int WPE, bool NT>
hipError_t launch_wave(const PassArgs& a, int dir, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  if (t0 != nullptr || t1 != nullptr)
    return launch_timed(dir < 0 ? row_wave_kernel<K, -1, NT> : row_wave_kernel<K, +1, NT>, a, K::THREADS, s, t0, t1);
  if (dir < 0) hipLaunchKernelGGL((row_wave_kernel<K, -1, NT>), dim3(a.nblocks), dim3(K::THREADS), 0, s, a);
  else hipLaunchKernelGGL((row_wave_kernel<K, +1, NT>), dim3(a.nblocks), dim3(K::THREADS), 0, s, a);
  return hipGetLastError();
}

// Measurement variants (MODE 1: data movement without arithmetic, MODE 2:
// loads and stores only) of a pass, launched like launch_pass/launch_rowc
// with the forward sign (events optional).
template <class K, int WPE, bool NT, int KIND>
hipError_t launch_probe(const PassArgs& a, int mode, hipStream_t s, hipEvent_t t0, hipEvent_t t1) {
  void (*k)(PassArgs) = nullptr;
  if constexpr (KIND == kKindCombine)
    k = mode == 1 ? rowc_kernel<K, -1, WPE, 0, NT, 1> : rowc_kernel<K, -1, WPE, 0, NT, 2>;
  else if constexpr (KIND == kKindCrossRow)
    k = mode == 1 ? rowx_kernel<K, -1, WPE, 0, NT, 1> : rowx_kernel<K, -1, WPE, 0, NT, 2>;
  else if constexpr (KIND == kKindWaveRow)
    k = mode == 1 ? row_wave_kernel<K, -1, NT, 1> : row_wave_kernel<K, -1, NT, 2>;
  else k = mode == 1 ? pass_kernel<K, -1, NT, WPE, 0, 1> : pass_kernel<K, -1, NT, WPE, 0, 2>;
  if (t0 != nullptr || t1 != nullptr) return launch_timed(k, a, K::THREADS, s, t0, t1);
  hipLaunchKernelGGL(k, dim3(a.nblocks), dim3(K::THREADS), 0, s, a);
  return hipGetLastError();
}

// Shape metadata of a configuration (no kernel instantiated).
template <class K>
constexpr PassKernel meta() {
  PassKernel k{};
  k.L = K::L;
  k.E = K::E;
  k.T = K::T;
  k.C = K::C;
  k.Q = K::Q;
  k.threads = K::THREADS;
  k.colmode = K::COL ? 1 : 0;
  k.npass = K::P;
  for (int p = 0; p < kMaxPasses; ++p) k.radix[p] = p < K::P ? K::radix(p) : 0;
  k.lds_bytes = (size_t)K::LDS_ELEMS * 8;
  k.launch = nullptr;
  return k;
}

// KIND: kKindPass (a plain row or column pass), kKindCombine (row pass with
// an M1 = C point combine, rowc_kernel) or kKindCrossRow (the same with the
// last stage across rows, rowx_kernel) or kKindWaveRow (one 1024-point row
// per wave with its second exchange in registers, row_wave_kernel).
// WPE: minimum waves per SIMD the compiler must allow (bounds VGPR use).
// NT: nontemporal loads of the input (row passes read data not reused soon;
// measured faster from HBM, slower when the data already sits in the MALL).
// PROBE: also compile the measurement variants (launch_probe).
template <class K, int KIND = kKindPass, int WPE = 1, bool NT = !K::COL, bool PROBE = false>
constexpr PassKernel describe() {
  PassKernel k{};
  k.combine = (KIND == kKindCombine || KIND == kKindCrossRow) ? K::C : 0;
  k.xrow = KIND == kKindCrossRow ? 1 : 0;
  k.shuffle = KIND == kKindWaveRow ? 1 : 0;
  k.L = K::L;
  k.E = K::E;
  k.T = K::T;
  k.C = K::C;
  k.Q = K::Q;
  k.threads = K::THREADS;
  k.colmode = K::COL ? 1 : 0;
  k.npass = K::P;
  for (int p = 0; p < kMaxPasses; ++p) k.radix[p] = p < K::P ? K::radix(p) : 0;
  k.lds_bytes = (size_t)K::LDS_ELEMS * 8;
  k.wpe = WPE;
  k.nt = NT ? 1 : 0;
  if constexpr (KIND == kKindCombine) k.launch = &launch_rowc<K, WPE, NT>;
  else if constexpr (KIND == kKindCrossRow) k.launch = &launch_rowx<K, WPE, NT>;
  else if constexpr (KIND == kKindWaveRow) k.launch = &launch_wave<K, WPE, NT>;
  else k.launch = &launch_pass<K, WPE, NT>;
  if constexpr (PROBE) k.launch_probe = &launch_probe<K, WPE, NT, KIND>;
  return k;
}

}  // namespace dev
}  // namespace fft2d
