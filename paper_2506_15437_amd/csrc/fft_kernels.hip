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
//     auto-sort), which is the paper's "one data reordering per step" idea
//     (Section 4, Fig. 5) moved on-chip: the digit reversal of the whole
//     transform costs no HBM traffic at all.
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
// Column workgroups are remapped so that each of the 8 XCDs (each with its own
// L2) works through a contiguous range of column tiles; neighbouring tiles
// share cache lines and are then served by the same L2.
#include "fft_internal.h"

#include <type_traits>

namespace fft2d {
namespace {

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
  double cphi, sphi;                 // angle inside the quadrant
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

// In-register R-point DFT (exponent sign DIR), natural order in and out,
// computed as log2 R radix-2 decimation-in-time steps on bit-reversed data:
// at the step of span h, points lo and lo + h (lo mod h = q) combine with the
// twiddle W_{2h}^q.
template <int R, int DIR>
__device__ __forceinline__ void dft(float2 (&a)[R]) {
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
        const float2 f = rotate<DIR, 2 * h, q>(b[hi]);
        b[hi] = csub(b[lo], f);
        b[lo] = cadd(b[lo], f);
      });
    });
  });
  static_for<0, R>([&](auto I) {
    constexpr int i = decltype(I)::value;
    a[i] = b[i];
  });
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
  static constexpr int pad(int e) { return e + (e >> 4); }
  static constexpr int LQP = pad(LQ - 1) + 1;
  // Row mode: consecutive vectors of one wave start T banks-pairs apart.
  static constexpr int ROWSTRIDE = (T >= 32) ? LQP : (LQP + T);
  static constexpr int LDS_ELEMS = (P > 1) ? (COL ? LQP * C : ROWSTRIDE * C) : 1;

  __device__ static __forceinline__ int lds_index(int c, int e) {
    if constexpr (COL) return pad(e) * C + c;
    else return c * ROWSTRIDE + pad(e);
  }

  static constexpr bool valid() {
    int prod = 1;
    for (int p = 0; p < P; ++p) {
      if (E % radix(p) != 0) return false;
      prod *= radix(p);
    }
    if (prod != L || L % E != 0 || THREADS > 1024 || THREADS % 64 != 0) return false;
    if (Q > 1) {
      for (int p = 0; p + 1 < P; ++p) {
        if ((E / radix(p)) % Q != 0) return false;  // whole butterflies per round
        if (ns(p) > T) return false;                // destinations of one butterfly stay in one round
      }
    }
    return LDS_ELEMS * 8 <= 160 * 1024;
  }
};

__device__ __forceinline__ int xcd_remap(int b, int nb) {
  // Consecutive workgroup ids are dispatched round-robin over the 8 XCDs; give
  // XCD x the contiguous id range [x q + min(x, r), ...) in dispatch order.
  const int x = b & 7, i = b >> 3;
  const int q = nb >> 3, r = nb & 7;
  return x * q + (x < r ? x : r) + i;
}

// One pass: butterflies of this thread, then (unless last) the LDS exchange.
template <class K, int DIR, int p>
__device__ __forceinline__ void run_pass(float2 (&d)[K::E], float2* lds, int tt, int c, const float2* __restrict__ tw) {
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
    if constexpr (p > 0) {
      const float2* twp = tw + K::tw_off(p) + (b & (Ns - 1));
      static_for<1, R>([&](auto Rr) {
        constexpr int r = decltype(Rr)::value;
        float2 w = twp[(r - 1) * Ns];
        if constexpr (DIR > 0) w.y = -w.y;
        x[r] = cmul(x[r], w);
      });
    }
    dft<R, DIR>(x);
    static_for<0, R>([&](auto S) {
      constexpr int s = decltype(S)::value;
      if constexpr (last) d[i + NB * s] = x[s];
      else o[i * R + s] = x[s];
    });
  });
  if constexpr (!last) {
    constexpr int NBQ = NB / K::Q;
    constexpr int EQ = K::E / K::Q;
    static_for<0, K::Q>([&](auto H) {
      constexpr int h = decltype(H)::value;
      static_for<0, NBQ>([&](auto I) {
        constexpr int i = h * NBQ + decltype(I)::value;
        const int b = tt + K::T * i;
        const int dst = (b / Ns) * Ns * R + (b & (Ns - 1)) - h * K::LQ;
        static_for<0, R>([&](auto S) {
          constexpr int s = decltype(S)::value;
          lds[K::lds_index(c, dst + s * Ns)] = o[i * R + s];
        });
      });
      __syncthreads();
      static_for<0, EQ>([&](auto J) {
        constexpr int j = h * EQ + decltype(J)::value;
        d[j] = lds[K::lds_index(c, tt + K::T * j - h * K::LQ)];
      });
      __syncthreads();
    });
  }
}

template <class K, int DIR>
__global__ __launch_bounds__(K::THREADS) void pass_kernel(PassArgs a) {
  static_assert(K::valid(), "invalid pass configuration");
  __shared__ float2 lds[K::LDS_ELEMS];
  const int t = threadIdx.x;
  const int c = K::COL ? (t % K::C) : (t / K::T);
  const int tt = K::COL ? (t / K::C) : (t % K::T);
  const int w = K::COL ? xcd_remap(blockIdx.x, a.nblocks) : (int)blockIdx.x;
  const int64_t v = (int64_t)w * K::C + c;
  const bool active = v < a.nvec;
  int64_t base, es;
  if constexpr (K::COL) {
    const int64_t g = v / a.ncols;
    const int64_t col = v - g * a.ncols;
    base = g * (int64_t)K::L * a.ncols + col;
    es = a.ncols;
  } else {
    base = v * K::L;
    es = 1;
  }
  float2 d[K::E];
  if (active) {
    static_for<0, K::E>([&](auto J) {
      constexpr int j = decltype(J)::value;
      d[j] = a.in[base + (int64_t)(tt + K::T * j) * es];
    });
  } else {
    static_for<0, K::E>([&](auto J) { d[decltype(J)::value] = make_float2(0.f, 0.f); });
  }
  static_for<0, K::P>([&](auto Pp) { run_pass<K, DIR, decltype(Pp)::value>(d, lds, tt, c, a.tw); });
  if (active) {
    const float sc = a.scale;
    static_for<0, K::E>([&](auto J) {
      constexpr int j = decltype(J)::value;
      a.out[base + (int64_t)(tt + K::T * j) * es] = make_float2(d[j].x * sc, d[j].y * sc);
    });
  }
}

template <class K>
hipError_t launch_pass(const PassArgs& a, int dir, hipStream_t s) {
  if (dir < 0) hipLaunchKernelGGL((pass_kernel<K, -1>), dim3(a.nblocks), dim3(K::THREADS), 0, s, a);
  else hipLaunchKernelGGL((pass_kernel<K, +1>), dim3(a.nblocks), dim3(K::THREADS), 0, s, a);
  return hipGetLastError();
}

template <class K>
constexpr PassKernel describe() {
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
  k.launch = &launch_pass<K>;
  return k;
}

__global__ void scale_copy_kernel(const float2* __restrict__ in, float2* __restrict__ out, int64_t n, float sc) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    const float2 v = in[i];
    out[i] = make_float2(v.x * sc, v.y * sc);
  }
}

// ------------------------------------------------------------ kernel table
// Row mode: vectors are contiguous; a few rows per workgroup for short rows.
using R2 = Cfg<2, 2, 128, 1, false, 2>;
using R4 = Cfg<4, 4, 128, 1, false, 4>;
using R8 = Cfg<8, 8, 64, 1, false, 8>;
using R16 = Cfg<16, 16, 64, 1, false, 16>;
using R32 = Cfg<32, 8, 32, 1, false, 8, 4>;
using R64 = Cfg<64, 8, 16, 1, false, 8, 8>;
using R128 = Cfg<128, 16, 16, 1, false, 16, 8>;
using R256 = Cfg<256, 16, 8, 1, false, 16, 16>;
using R512 = Cfg<512, 32, 8, 1, false, 32, 16>;
using R1024 = Cfg<1024, 32, 4, 1, false, 32, 32>;
using R2048 = Cfg<2048, 16, 2, 1, false, 16, 16, 8>;
using R4096 = Cfg<4096, 16, 1, 1, false, 16, 16, 16>;
using R8192 = Cfg<8192, 32, 1, 1, false, 32, 16, 16>;
using R16384 = Cfg<16384, 32, 1, 1, false, 32, 32, 16>;

// Column mode: C columns per workgroup (C*8-byte row segments), the LDS
// exchange split into Q rounds where C*L points would not fit 160 KiB.
using C2 = Cfg<2, 2, 256, 1, true, 2>;
using C4 = Cfg<4, 4, 256, 1, true, 4>;
using C8 = Cfg<8, 8, 128, 1, true, 8>;
using C16 = Cfg<16, 16, 128, 1, true, 16>;
using C32 = Cfg<32, 8, 64, 1, true, 8, 4>;
using C64 = Cfg<64, 8, 32, 1, true, 8, 8>;
using C128 = Cfg<128, 16, 32, 1, true, 16, 8>;
using C256 = Cfg<256, 16, 16, 1, true, 16, 16>;
using C512 = Cfg<512, 32, 16, 1, true, 32, 16>;
using C1024 = Cfg<1024, 32, 16, 1, true, 32, 32>;
using C2048 = Cfg<2048, 16, 8, 1, true, 16, 16, 8>;
using C4096 = Cfg<4096, 32, 8, 2, true, 16, 16, 16>;
using C8192 = Cfg<8192, 32, 4, 2, true, 16, 16, 32>;
using C16384 = Cfg<16384, 32, 2, 2, true, 16, 16, 16, 4>;

const PassKernel kRowKernels[] = {
    describe<R2>(),   describe<R4>(),   describe<R8>(),    describe<R16>(),   describe<R32>(),
    describe<R64>(),  describe<R128>(), describe<R256>(),  describe<R512>(),  describe<R1024>(),
    describe<R2048>(), describe<R4096>(), describe<R8192>(), describe<R16384>(),
};
const PassKernel kColKernels[] = {
    describe<C2>(),   describe<C4>(),   describe<C8>(),    describe<C16>(),   describe<C32>(),
    describe<C64>(),  describe<C128>(), describe<C256>(),  describe<C512>(),  describe<C1024>(),
    describe<C2048>(), describe<C4096>(), describe<C8192>(), describe<C16384>(),
};

}  // namespace

const PassKernel* find_pass_kernel(int L, bool colmode) {
  const PassKernel* tab = colmode ? kColKernels : kRowKernels;
  const int n = colmode ? (int)(sizeof(kColKernels) / sizeof(kColKernels[0]))
                        : (int)(sizeof(kRowKernels) / sizeof(kRowKernels[0]));
  for (int i = 0; i < n; ++i)
    if (tab[i].L == L) return &tab[i];
  return nullptr;
}

int list_pass_kernels(int L, bool colmode, const PassKernel** out, int cap) {
  const PassKernel* k = find_pass_kernel(L, colmode);
  if (!k) return 0;
  if (cap > 0) out[0] = k;
  return 1;
}

size_t twiddle_count(const PassKernel& k) {
  size_t n = 0, ns = 1;
  for (int p = 0; p < k.npass; ++p) {
    if (p > 0) n += ns * (size_t)(k.radix[p] - 1);
    ns *= (size_t)k.radix[p];
  }
  return n;
}

hipError_t launch_scale_copy(const float2* in, float2* out, int64_t n, float scale, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(scale_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s, in, out, n, scale);
  return hipGetLastError();
}

}  // namespace fft2d
