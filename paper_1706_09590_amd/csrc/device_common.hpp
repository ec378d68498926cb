// Device building blocks: complex arithmetic, register-resident small DFTs
// with compile-time twiddles, and Hermitian-packed state helpers.
#pragma once

#include <hip/hip_runtime.h>

namespace qhfpe {

template <typename T>
struct cx {
  T re, im;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {  // a * conj(b)
  return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im};
}

// cos and sin of 2 pi e / 48, e = 0..47 (every radix used below divides 48).
__device__ constexpr double kCos48[48] = {
    1.0, 0.9914448613738104, 0.9659258262890683, 0.9238795325112867, 0.8660254037844387,
    0.7933533402912352, 0.7071067811865476, 0.6087614290087207, 0.5000000000000001,
    0.38268343236508984, 0.25881904510252074, 0.1305261922200517, 0.0, -0.1305261922200516,
    -0.25881904510252063, -0.3826834323650895, -0.4999999999999998, -0.6087614290087207,
    -0.7071067811865475, -0.793353340291235, -0.8660254037844387, -0.9238795325112867,
    -0.9659258262890682, -0.9914448613738104, -1.0, -0.9914448613738104, -0.9659258262890683,
    -0.9238795325112868, -0.8660254037844388, -0.7933533402912352, -0.7071067811865479,
    -0.6087614290087209, -0.5000000000000004, -0.3826834323650895, -0.25881904510252063,
    -0.13052619222005163, 0.0, 0.13052619222005127, 0.2588190451025203, 0.38268343236508917,
    0.5000000000000001, 0.6087614290087199, 0.7071067811865474, 0.7933533402912349,
    0.8660254037844384, 0.9238795325112868, 0.9659258262890681, 0.9914448613738104};
__device__ constexpr double kSin48[48] = {
    0.0, 0.13052619222005157, 0.25881904510252074, 0.3826834323650898, 0.49999999999999994,
    0.6087614290087207, 0.7071067811865475, 0.7933533402912352, 0.8660254037844386,
    0.9238795325112867, 0.9659258262890683, 0.9914448613738104, 1.0, 0.9914448613738104,
    0.9659258262890683, 0.9238795325112868, 0.8660254037844387, 0.7933533402912352,
    0.7071067811865476, 0.6087614290087209, 0.49999999999999994, 0.3826834323650899,
    0.258819045102521, 0.130526192220052, 0.0, -0.13052619222005177, -0.2588190451025208,
    -0.38268343236508967, -0.4999999999999997, -0.6087614290087207, -0.7071067811865471,
    -0.7933533402912349, -0.8660254037844384, -0.9238795325112868, -0.9659258262890683,
    -0.9914448613738104, -1.0, -0.9914448613738105, -0.9659258262890684, -0.923879532511287,
    -0.8660254037844386, -0.7933533402912357, -0.7071067811865477, -0.6087614290087209,
    -0.5000000000000004, -0.38268343236508956, -0.25881904510252157, -0.13052619222005168};

// x * exp(2 pi i E / 48) with the angle known at compile time; multiples of
// a quarter turn are exact swaps and sign flips.
template <int E, typename T>
__device__ __forceinline__ cx<T> rot48(cx<T> x) {
  constexpr int e = ((E % 48) + 48) % 48;
  if constexpr (e == 0) {
    return x;
  } else if constexpr (e == 12) {
    return {-x.im, x.re};
  } else if constexpr (e == 24) {
    return {-x.re, -x.im};
  } else if constexpr (e == 36) {
    return {x.im, -x.re};
  } else if constexpr (e % 6 == 0) {
    // odd multiples of an eighth turn: (+-1 +- i)/sqrt(2)
    const T h = T(0.70710678118654752440);
    constexpr int cs = (e == 6 || e == 42) ? 1 : -1;
    constexpr int sn = (e == 6 || e == 18) ? 1 : -1;
    return {h * (T(cs) * x.re - T(sn) * x.im), h * (T(sn) * x.re + T(cs) * x.im)};
  } else {
    const T c = T(kCos48[e]);
    const T s = T(kSin48[e]);
    return {x.re * c - x.im * s, x.re * s + x.im * c};
  }
}

// In-place R-point DFT, y_k = sum_n x_n exp(S 2 pi i n k / R), natural order
// in and out.  Composite R = A * B runs A-point DFTs over n = B n1 + n2,
// twiddles, then B-point DFTs (output index k = k1 + A k2).
template <int R, int S, typename T>
struct SmallDft;

template <int S, typename T>
struct SmallDft<1, S, T> {
  __device__ __forceinline__ static void run(cx<T>*) {}
};

template <int S, typename T>
struct SmallDft<2, S, T> {
  __device__ __forceinline__ static void run(cx<T>* x) {
    cx<T> a = x[0], b = x[1];
    x[0] = a + b;
    x[1] = a - b;
  }
};

template <int S, typename T>
struct SmallDft<3, S, T> {
  __device__ __forceinline__ static void run(cx<T>* x) {
    const T h = T(0.8660254037844386);  // sin(2 pi / 3)
    cx<T> t1 = x[1] + x[2];
    cx<T> t2 = {x[0].re - T(0.5) * t1.re, x[0].im - T(0.5) * t1.im};
    cx<T> d = x[1] - x[2];
    // S i h d
    cx<T> t3 = {-T(S) * h * d.im, T(S) * h * d.re};
    x[0] = x[0] + t1;
    x[1] = t2 + t3;
    x[2] = t2 - t3;
  }
};

template <int S, typename T>
struct SmallDft<4, S, T> {
  __device__ __forceinline__ static void run(cx<T>* x) {
    cx<T> a = x[0] + x[2], b = x[0] - x[2];
    cx<T> c = x[1] + x[3], d = x[1] - x[3];
    cx<T> sd = (S > 0) ? cx<T>{-d.im, d.re} : cx<T>{d.im, -d.re};  // S i d
    x[0] = a + c;
    x[2] = a - c;
    x[1] = b + sd;
    x[3] = b - sd;
  }
};

template <int R, int S, typename T>
struct SmallDft {
  static constexpr int A = (R % 4 == 0) ? 4 : ((R % 2 == 0) ? 2 : 3);
  static constexpr int B = R / A;
  static_assert(48 % R == 0, "radix must divide 48");

  template <int N2, int K1>
  __device__ __forceinline__ static void twiddle_col(cx<T>* y) {
    if constexpr (N2 < B) {
      // y[N2*A + K1] *= exp(S 2 pi i N2 K1 / R)
      y[N2 * A + K1] = rot48<S * N2 * K1 * (48 / R), T>(y[N2 * A + K1]);
      twiddle_col<N2 + 1, K1>(y);
    }
  }
  template <int K1>
  __device__ __forceinline__ static void twiddle_all(cx<T>* y) {
    if constexpr (K1 < A) {
      twiddle_col<0, K1>(y);
      twiddle_all<K1 + 1>(y);
    }
  }

  __device__ __forceinline__ static void run(cx<T>* x) {
    cx<T> y[R];  // y[n2*A + k1]
#pragma unroll
    for (int n2 = 0; n2 < B; ++n2) {
      cx<T> t[A];
#pragma unroll
      for (int n1 = 0; n1 < A; ++n1) t[n1] = x[B * n1 + n2];
      SmallDft<A, S, T>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) y[n2 * A + k1] = t[k1];
    }
    twiddle_all<0>(y);
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      cx<T> t[B];
#pragma unroll
      for (int n2 = 0; n2 < B; ++n2) t[n2] = y[n2 * A + k1];
      SmallDft<B, S, T>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) x[k1 + A * k2] = t[k2];
    }
  }
};

// ---------------------------------------------------------------------------
// Buffer-resource memory access: a 32-bit per-lane byte offset (voffset)
// plus a wave-uniform byte offset (soffset) from a uniform base, with the
// hardware range check of raw buffers (reads past num_records return 0,
// writes past it are dropped).
// ---------------------------------------------------------------------------
using rsrc_t = __amdgpu_buffer_rsrc_t;
constexpr int kBufferDword3 = 0x00020000;  // raw buffer, gfx9-family data format bits

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, kBufferDword3);
}
template <typename T>
__device__ __forceinline__ T buf_load(rsrc_t r, unsigned voff, unsigned soff);
template <>
__device__ __forceinline__ float buf_load<float>(rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <>
__device__ __forceinline__ double buf_load<double>(rsrc_t r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void buf_store(float v, rsrc_t r, unsigned voff, unsigned soff) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void buf_store(double v, rsrc_t r, unsigned voff, unsigned soff) {
  using u2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, (int)voff, (int)soff, 0);
}

// Four consecutive elements per lane (one 16-byte access for float, two for
// double); voff must be 16-byte aligned.  The loaded vector is bit-cast as a
// whole: taking single 32-bit elements out of it and bit-casting those makes
// this compiler shrink the load to one dword at offset 0 (every element
// then reads element 0).
typedef float qhfpe_f2 __attribute__((ext_vector_type(2)));
typedef float qhfpe_f4 __attribute__((ext_vector_type(4)));
typedef double qhfpe_d2 __attribute__((ext_vector_type(2)));
template <typename T>
struct Quad {
  T v[4];
};
__device__ __forceinline__ Quad<float> buf_load4(rsrc_t r, unsigned voff, unsigned soff, float) {
  const qhfpe_f4 x = __builtin_bit_cast(qhfpe_f4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
  return {{x[0], x[1], x[2], x[3]}};
}
__device__ __forceinline__ Quad<double> buf_load4(rsrc_t r, unsigned voff, unsigned soff, double) {
  const qhfpe_d2 x = __builtin_bit_cast(qhfpe_d2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
  const qhfpe_d2 y =
      __builtin_bit_cast(qhfpe_d2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff + 16, (int)soff, 0));
  return {{x[0], x[1], y[0], y[1]}};
}
// CPOL: cache policy of the store (0, or kStoreNT for non-temporal stores)
constexpr int kStoreNT = 2;  // the nt bit of the buffer instructions' cache policy
template <int CPOL = 0>
__device__ __forceinline__ void buf_store4(const Quad<float>& q, rsrc_t r, unsigned voff, unsigned soff) {
  using u4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
  const qhfpe_f4 x = {q.v[0], q.v[1], q.v[2], q.v[3]};
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, x), r, (int)voff, (int)soff, CPOL);
}
template <int CPOL = 0>
__device__ __forceinline__ void buf_store4(const Quad<double>& q, rsrc_t r, unsigned voff, unsigned soff) {
  using u4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(r, 0, 0, 0));
  const qhfpe_d2 x = {q.v[0], q.v[1]}, y = {q.v[2], q.v[3]};
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, x), r, (int)voff, (int)soff, CPOL);
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u4, y), r, (int)voff + 16, (int)soff, CPOL);
}

// M consecutive elements per lane (M * sizeof(T) = 8, 16 or 32 bytes; voff
// aligned to that size, at most 16).
template <int M>
__device__ __forceinline__ void buf_load_n(rsrc_t r, unsigned voff, unsigned soff, float* out) {
  static_assert(M == 2 || M == 4, "2 or 4 floats");
  if constexpr (M == 2) {
    const qhfpe_f2 x = __builtin_bit_cast(qhfpe_f2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
    out[0] = x[0];
    out[1] = x[1];
  } else {
    const Quad<float> q = buf_load4(r, voff, soff, 0.0f);
    for (int j = 0; j < 4; ++j) out[j] = q.v[j];
  }
}
template <int M>
__device__ __forceinline__ void buf_load_n(rsrc_t r, unsigned voff, unsigned soff, double* out) {
  static_assert(M == 2 || M == 4, "2 or 4 doubles");
  if constexpr (M == 2) {
    const qhfpe_d2 x = __builtin_bit_cast(qhfpe_d2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0));
    out[0] = x[0];
    out[1] = x[1];
  } else {
    const Quad<double> q = buf_load4(r, voff, soff, 0.0);
    for (int j = 0; j < 4; ++j) out[j] = q.v[j];
  }
}

// Cross-lane rotations over the whole 64-lane wave (DPP wave_ror:1 /
// wave_rol:1): lane_prev returns lane l-1's value (lane 0 gets lane 63's),
// lane_next lane l+1's (lane 63 gets lane 0's).
__device__ __forceinline__ int dpp_prev(int x) { return __builtin_amdgcn_mov_dpp(x, 0x13C, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_next(int x) { return __builtin_amdgcn_mov_dpp(x, 0x134, 0xf, 0xf, false); }
__device__ __forceinline__ float lane_prev(float x) { return __builtin_bit_cast(float, dpp_prev(__builtin_bit_cast(int, x))); }
__device__ __forceinline__ float lane_next(float x) { return __builtin_bit_cast(float, dpp_next(__builtin_bit_cast(int, x))); }
__device__ __forceinline__ double lane_prev(double x) {
  const auto v = __builtin_bit_cast(int __attribute__((ext_vector_type(2))), x);
  return __builtin_bit_cast(double, (int __attribute__((ext_vector_type(2)))){dpp_prev(v[0]), dpp_prev(v[1])});
}
__device__ __forceinline__ double lane_next(double x) {
  const auto v = __builtin_bit_cast(int __attribute__((ext_vector_type(2))), x);
  return __builtin_bit_cast(double, (int __attribute__((ext_vector_type(2)))){dpp_next(v[0]), dpp_next(v[1])});
}

// Orders LDS accesses of one wave: accesses before it (of any lane) are
// performed before accesses after it.  LDS executes a wave's instructions
// in order, so only the compiler has to be kept from moving them across.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// Hermitian-packed electronic matrices.  Component order: diagonal j at j;
// off-diagonal pair (j, k), j < k, at NS + 2 * pair(j, k) (re) and +1 (im),
// pairs enumerated (0,1), (0,2), (1,2).
// ---------------------------------------------------------------------------
template <int NS>
struct Packing {
  static constexpr int NC = NS * NS;
  __host__ __device__ static constexpr int pair(int j, int k) {
    // j < k
    return (NS == 2) ? 0 : (j == 0 ? (k == 1 ? 0 : 1) : 2);
  }
  __host__ __device__ static constexpr int re(int j, int k) { return NS + 2 * pair(j, k); }
};

// Entry (j, k) of the Hermitian matrix held in packed form h[NC].
template <int NS, typename T>
__device__ __forceinline__ cx<T> herm_get(const T* h, int j, int k) {
  if (j == k) return {h[j], T(0)};
  if (j < k) return {h[Packing<NS>::re(j, k)], h[Packing<NS>::re(j, k) + 1]};
  return {h[Packing<NS>::re(k, j)], -h[Packing<NS>::re(k, j) + 1]};
}

// out = -i (A H - H A) for real symmetric A (diagonal of A ignored is fine:
// it cancels) and Hermitian H; the result is Hermitian.  Packed in/out.
template <int NS, typename T>
__device__ __forceinline__ void commutator_mi(const T A[NS][NS], const T* h, T* out) {
#pragma unroll
  for (int j = 0; j < NS; ++j) {
#pragma unroll
    for (int k = j; k < NS; ++k) {
      cx<T> c = {T(0), T(0)};
#pragma unroll
      for (int l = 0; l < NS; ++l) {
        cx<T> hl = herm_get<NS>(h, l, k);
        cx<T> hr = herm_get<NS>(h, j, l);
        c.re += A[j][l] * hl.re - hr.re * A[l][k];
        c.im += A[j][l] * hl.im - hr.im * A[l][k];
      }
      // -i c
      if (j == k) {
        out[j] = c.im;
      } else {
        out[Packing<NS>::re(j, k)] = c.im;
        out[Packing<NS>::re(j, k) + 1] = -c.re;
      }
    }
  }
}

}  // namespace qhfpe
