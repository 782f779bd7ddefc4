// fl_common.h -- device-side types shared by the HIP kernels of the loop
// library: complex arithmetic, spinor and link storage formats, the
// checkerboard geometry, the multi-lattice tile map and wave reductions.
//
// Data layout in HBM (per lattice, per parity, structure of arrays):
//   spinor field of one right-hand side: NC vectors x Vh sites, vector c of
//     site i at base[c*Vh + i]; consecutive right-hand sides follow each
//     other (stride NC*Vh vectors).  FP64: 12 x double2, FP32: 6 x float4.
//   links: [mu][parity][NCg][Vh] vectors.  FP64 18 reals: 9 x double2;
//     FP32 12 reals: 3 x float4 (rows 0 and 1); FP32 18 reals: 9 x float2;
//     BF16 12 reals: 3 x (4 bf16).  Row 2 of a 12-real link is rebuilt as
//     conj(row0 x row1), exact for SU(3).
// Each wavefront (64 lanes) works on 64 consecutive checkerboard sites of
// ONE right-hand side, so per-RHS masks and reductions are wave-uniform and
// every reduction partial covers a fixed block of 64 sites, whatever the
// batch composition.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#define FL_MAXLAT 4
#define FL_WAVE 64

// ---------------------------------------------------------------------------
// complex numbers
// ---------------------------------------------------------------------------
template <typename R>
struct cx {
    R re, im;
};

template <typename R>
__device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return cx<R>{a.re + b.re, a.im + b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return cx<R>{a.re - b.re, a.im - b.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a) { return cx<R>{-a.re, -a.im}; }
template <typename R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b)
{
    return cx<R>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return cx<R>{s * a.re, s * a.im}; }
// i * a
template <typename R>
__device__ __forceinline__ cx<R> ti(cx<R> a) { return cx<R>{-a.im, a.re}; }
template <typename R>
__device__ __forceinline__ cx<R> cj(cx<R> a) { return cx<R>{a.re, -a.im}; }
// conj(a) * b
template <typename R>
__device__ __forceinline__ cx<R> cjmul(cx<R> a, cx<R> b)
{
    return cx<R>{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}

// acc + a * b as four fused multiply-adds (the compiler cannot reassociate
// acc + (a*b) into this form by itself)
template <typename R>
__device__ __forceinline__ cx<R> cmad(cx<R> acc, cx<R> a, cx<R> b)
{
    R re = fma(a.re, b.re, acc.re);
    R im = fma(a.re, b.im, acc.im);
    re = fma(-a.im, b.im, re);
    im = fma(a.im, b.re, im);
    return cx<R>{re, im};
}

// acc + conj(a) * b
template <typename R>
__device__ __forceinline__ cx<R> cjmad(cx<R> acc, cx<R> a, cx<R> b)
{
    R re = fma(a.re, b.re, acc.re);
    R im = fma(a.re, b.im, acc.im);
    re = fma(a.im, b.im, re);
    im = fma(-a.im, b.re, im);
    return cx<R>{re, im};
}

// acc - a * b
template <typename R>
__device__ __forceinline__ cx<R> cmsub(cx<R> acc, cx<R> a, cx<R> b)
{
    R re = fma(-a.re, b.re, acc.re);
    R im = fma(-a.re, b.im, acc.im);
    re = fma(a.im, b.im, re);
    im = fma(-a.im, b.re, im);
    return cx<R>{re, im};
}

// ---------------------------------------------------------------------------
// buffer views: a raw buffer resource per field and wavefront (scalar
// registers), so that each load is one buffer instruction with a 32-bit
// per-lane offset and a scalar component offset, and no 64-bit address
// arithmetic per lane
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));
typedef unsigned v2u __attribute__((ext_vector_type(2)));

struct Buf {
    __amdgpu_buffer_rsrc_t r;
};

__device__ __forceinline__ Buf make_buf(const void *base, unsigned bytes)
{
    Buf b;
    b.r = __builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)bytes, 0x00020000);
    return b;
}

__device__ __forceinline__ v4f buf_ld16(const Buf &b, int voff, int soff)
{
    return __builtin_amdgcn_raw_buffer_load_b128(b.r, voff, soff, 0);
}

__device__ __forceinline__ v2f buf_ld8(const Buf &b, int voff, int soff)
{
    return __builtin_amdgcn_raw_buffer_load_b64(b.r, voff, soff, 0);
}

// CP: cache policy of the store (0: default; ST_STREAM: non-temporal, for
// results no later access of the same kernel reads); LD_STREAM: the same
// policy for a load of data no other access of the kernel reads
enum { ST_STREAM = 2, LD_STREAM = 2 };

template <int CP = 0>
__device__ __forceinline__ void buf_st16(const Buf &b, v4f v, int voff, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b128(v, b.r, voff, soff, CP);
}

// Store groups.  Measured on gfx950: a vector instruction issued shortly
// after a vector-memory store can overwrite the store's data registers
// before the store has read them when the memory pipeline is congested (the
// compiler's hazard model does not cover stores with a scalar offset
// register), which corrupts the stored data.  Every group of stores in this
// library is therefore issued back to back from registers prepared before
// it, with no vector instruction in between (scalar component offsets and
// one lane offset, or precomputed addresses), and followed by store_drain()
// before any further vector work; a store that ends a kernel needs no drain.
__device__ __forceinline__ void store_drain()
{
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), gfx9 encoding
    __builtin_amdgcn_sched_barrier(0);
}

__device__ __forceinline__ void store_fence_begin() { __builtin_amdgcn_sched_barrier(0); }

__device__ __forceinline__ void buf_st8(const Buf &b, v2f v, int voff, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b64(v, b.r, voff, soff, 0);
}

// N 16-byte vectors of one lane at byte offsets voff + c * cstride (cstride
// wave-uniform), as one store group
template <int N, int CP = 0>
__device__ __forceinline__ void st16_group(const Buf &b, const v4f (&v)[N], int voff, int cstride)
{
    store_fence_begin();
#pragma unroll
    for (int c = 0; c < N; ++c) buf_st16<CP>(b, v[c], voff, c * cstride);
    store_drain();
}

// N values through precomputed addresses, as one store group
template <int N, typename T>
__device__ __forceinline__ void ptr_store_group(T *const (&p)[N], const T (&v)[N])
{
    store_fence_begin();
#pragma unroll
    for (int c = 0; c < N; ++c) *p[c] = v[c];
    store_drain();
}

__device__ __forceinline__ float buf_ld4(const Buf &b, int voff, int soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(b.r, voff, soff, 0));
}

template <int CP = 0>
__device__ __forceinline__ void buf_st4(const Buf &b, float v, int voff, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), b.r, voff, soff, CP);
}

__device__ __forceinline__ double2 v4f_to_d2(v4f v)
{
    union {
        v4f f;
        double2 d;
    } u;
    u.f = v;
    return u.d;
}

__device__ __forceinline__ v4f d2_to_v4f(double2 d)
{
    union {
        v4f f;
        double2 d;
    } u;
    u.d = d;
    return u.f;
}

// ---------------------------------------------------------------------------
// spinor storage: 24 reals (spin-major, colour, re/im) per site
// ---------------------------------------------------------------------------
template <typename R>
struct SpinorFmt;

//
// Every format provides, for the component-major layout of one right-hand
// side's field on Vh sites (SITE_BYTES per site):
//   load/store    through a per-wave buffer view (and plain pointers for
//                 FP64/FP32),
//   load_raw      the values up to one common per-site factor, returned
//                 (1 for FP64/FP32) so that a stencil can fold it into the
//                 scalar it multiplies the hop by,
//   to_lds/lds_load_raw  the raw site copied into, and read back from, a
//                 wave's LDS window of wsmax sites.
template <>
struct SpinorFmt<double> {
    typedef double R;
    typedef double2 V;
    static constexpr int NC = 12;
    static constexpr int SITE_BYTES = 192;
    __device__ static __forceinline__ void load(const V *__restrict__ f, int Vh, int i, cx<double> s[12])
    {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            V v = f[(size_t)c * Vh + i];
            s[c] = cx<double>{v.x, v.y};
        }
    }
    __device__ static __forceinline__ void store(V *__restrict__ f, int Vh, int i, const cx<double> s[12])
    {
        V *p[12];
        V v[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            p[c] = f + (size_t)c * Vh + i;
            v[c] = make_double2(s[c].re, s[c].im);
        }
        ptr_store_group(p, v);
    }
    // buffer views of one right-hand side's field (component stride Vh*16 bytes)
    __device__ static __forceinline__ void load(const Buf &b, int Vh, int i, cx<double> s[12])
    {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            double2 v = v4f_to_d2(buf_ld16(b, i * 16, c * Vh * 16));
            s[c] = cx<double>{v.x, v.y};
        }
    }
    template <int CP = 0>
    __device__ static __forceinline__ void store(const Buf &b, int Vh, int i, const cx<double> s[12])
    {
        v4f v[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = d2_to_v4f(make_double2(s[c].re, s[c].im));
        st16_group<12, CP>(b, v, i * 16, Vh * 16);
    }
    __device__ static __forceinline__ double load_raw(const Buf &b, int Vh, int i, cx<double> s[12])
    {
        load(b, Vh, i, s);
        return 1.0;
    }
    __device__ static __forceinline__ void to_lds(const Buf &b, int Vh, int i, unsigned char *w, int wsmax, int j)
    {
#pragma unroll
        for (int c = 0; c < 12; ++c) ((v4f *)w)[c * wsmax + j] = buf_ld16(b, i * 16, c * Vh * 16);
    }
    __device__ static __forceinline__ double lds_load_raw(const unsigned char *w, int wsmax, int j, cx<double> s[12])
    {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
            double2 v = v4f_to_d2(((const v4f *)w)[c * wsmax + j]);
            s[c] = cx<double>{v.x, v.y};
        }
        return 1.0;
    }
};

template <>
struct SpinorFmt<float> {
    typedef float R;
    typedef float4 V;
    static constexpr int NC = 6;
    static constexpr int SITE_BYTES = 96;
    __device__ static __forceinline__ void load(const V *__restrict__ f, int Vh, int i, cx<float> s[12])
    {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            V v = f[(size_t)c * Vh + i];
            s[2 * c] = cx<float>{v.x, v.y};
            s[2 * c + 1] = cx<float>{v.z, v.w};
        }
    }
    __device__ static __forceinline__ void store(V *__restrict__ f, int Vh, int i, const cx<float> s[12])
    {
        V *p[6];
        V v[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            p[c] = f + (size_t)c * Vh + i;
            v[c] = make_float4(s[2 * c].re, s[2 * c].im, s[2 * c + 1].re, s[2 * c + 1].im);
        }
        ptr_store_group(p, v);
    }
    __device__ static __forceinline__ void load(const Buf &b, int Vh, int i, cx<float> s[12])
    {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            v4f v = buf_ld16(b, i * 16, c * Vh * 16);
            s[2 * c] = cx<float>{v.x, v.y};
            s[2 * c + 1] = cx<float>{v.z, v.w};
        }
    }
    template <int CP = 0>
    __device__ static __forceinline__ void store(const Buf &b, int Vh, int i, const cx<float> s[12])
    {
        v4f v[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] = v4f{s[2 * c].re, s[2 * c].im, s[2 * c + 1].re, s[2 * c + 1].im};
        st16_group<6, CP>(b, v, i * 16, Vh * 16);
    }
    __device__ static __forceinline__ float load_raw(const Buf &b, int Vh, int i, cx<float> s[12])
    {
        load(b, Vh, i, s);
        return 1.0f;
    }
    __device__ static __forceinline__ void to_lds(const Buf &b, int Vh, int i, unsigned char *w, int wsmax, int j)
    {
#pragma unroll
        for (int c = 0; c < 6; ++c) ((v4f *)w)[c * wsmax + j] = buf_ld16(b, i * 16, c * Vh * 16);
    }
    __device__ static __forceinline__ float lds_load_raw(const unsigned char *w, int wsmax, int j, cx<float> s[12])
    {
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            v4f v = ((const v4f *)w)[c * wsmax + j];
            s[2 * c] = cx<float>{v.x, v.y};
            s[2 * c + 1] = cx<float>{v.z, v.w};
        }
        return 1.0f;
    }
};

// 16-bit fixed-point spinor storage with one FP32 scale per site: the 24
// reals of a site are divided by their largest magnitude m and stored as
// round(16383 v / m) in int16 (three 16-byte vectors, complex entry 4c + w in
// word w of vector c, real part in the low half); the scale m / 16383 follows
// the three vector arrays as an FP32 array.  Relative rounding error per
// component <= 1 / 32766 of the site's largest component.  The 15-bit range
// leaves room for the sum or difference of two stored values in int16, which
// the packed hop uses for its spin projection.
struct H16 {};

__device__ __forceinline__ cx<float> h16_pair(unsigned w)
{
    return cx<float>{(float)(int)(short)(w & 0xffffu), (float)((int)w >> 16)};
}


__device__ __forceinline__ unsigned h16_pack(float a, float b)
{
    // a, b in [-1, 1] (clamped) -> round(32767 a) | round(32767 b) << 16
    return __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_pknorm_i16(a, b));
}

// a complex number as two int16 in one 32-bit word (real part low)
typedef short s2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ s2 as_s2(unsigned w) { return __builtin_bit_cast(s2, w); }
__device__ __forceinline__ s2 swp(s2 z) { return __builtin_shufflevector(z, z, 1, 0); }

// u . h (the products summed exactly in int32) as the three-operand form with
// an inline zero accumulator: the builtin with a zero accumulator becomes
// the two-operand v_dot2c form, which needs a v_mov to clear its register
__device__ __forceinline__ int sdot2_first(s2 u, s2 h)
{
    int r;
    asm("v_dot2_i32_i16 %0, %1, %2, 0" : "=v"(r) : "v"(u), "v"(h));
    return r;
}

// swp(l) * k + u as one packed multiply-add: op_sel feeds the high half of l
// to the low lane and its low half to the high lane
__device__ __forceinline__ s2 mad_swp(s2 l, s2 k, s2 u)
{
    unsigned r;
    asm("v_pk_mad_i16 %0, %1, %2, %3 op_sel:[1,0,0] op_sel_hi:[0,1,1]"
        : "=v"(r)
        : "v"(__builtin_bit_cast(unsigned, l)), "s"(__builtin_bit_cast(unsigned, k)),
          "v"(__builtin_bit_cast(unsigned, u)));
    return as_s2(r);
}

// |v|^2 of a stored 16-bit site (words w, scale sc) from its integers: exact
// int32 sums of squares over three groups of four words (each <= 8 * 16383^2
// < 2^31), scaled once
__device__ __forceinline__ float h16_norm2(const unsigned w[12], float sc)
{
    float t = 0.0f;
#pragma unroll
    for (int g = 0; g < 3; ++g) {
        int n = sdot2_first(as_s2(w[4 * g]), as_s2(w[4 * g]));
#pragma unroll
        for (int k = 1; k < 4; ++k) n = __builtin_amdgcn_sdot2(as_s2(w[4 * g + k]), as_s2(w[4 * g + k]), n, false);
        t += (float)n;
    }
    return t * sc * sc;
}

template <>
struct SpinorFmt<H16> {
    typedef float R;
    static constexpr int NC = 3;
    static constexpr int SITE_BYTES = 52;
    __device__ static __forceinline__ void unpack(const v4f v[3], cx<float> s[12])
    {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            // reinterpret the whole vector: a bit cast of one element
            // accessor (v[c].y) reads the bytes of element 0
            const v4u u = __builtin_bit_cast(v4u, v[c]);
            s[4 * c] = h16_pair(u.x);
            s[4 * c + 1] = h16_pair(u.y);
            s[4 * c + 2] = h16_pair(u.z);
            s[4 * c + 3] = h16_pair(u.w);
        }
    }
    __device__ static __forceinline__ float load_raw(const Buf &b, int Vh, int i, cx<float> s[12])
    {
        v4f v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = buf_ld16(b, i * 16, c * Vh * 16);
        const float sc = buf_ld4(b, i * 4, 3 * Vh * 16);
        unpack(v, s);
        return sc;
    }
    __device__ static __forceinline__ void load(const Buf &b, int Vh, int i, cx<float> s[12])
    {
        const float sc = load_raw(b, Vh, i, s);
#pragma unroll
        for (int k = 0; k < 12; ++k) s[k] = cx<float>{s[k].re * sc, s[k].im * sc};
    }
    // stores f s; returns the site scale and the stored words (the factor
    // f only enters the scale and the sign of the words: f s rounds to the
    // same integers as s)
    template <int CP = 0>
    __device__ static __forceinline__ float store_words(const Buf &b, int Vh, int i, const cx<float> s[12],
                                                        unsigned w[12], float f = 1.0f)
    {
        float m = 0.0f;
#pragma unroll
        for (int k = 0; k < 12; ++k) m = fmaxf(m, fmaxf(fabsf(s[k].re), fabsf(s[k].im)));
        // h16_pack(x) = round(32767 x): x = v / m * (16383 / 32767)
        const float inv = m > 0.0f ? copysignf((16383.0f / 32767.0f) / m, f) : 0.0f;
        const float sc = m * fabsf(f) * (1.0f / 16383.0f);
#pragma unroll
        for (int k = 0; k < 12; ++k) w[k] = h16_pack(s[k].re * inv, s[k].im * inv);
        v4f v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const v4u u = {w[4 * c], w[4 * c + 1], w[4 * c + 2], w[4 * c + 3]};
            v[c] = __builtin_bit_cast(v4f, u);
        }
        // both lane offsets exist before the group, so no vector instruction
        // runs between its stores
        int vo16 = i * 16, vo4 = i * 4;
        float scv = sc;
        asm volatile("" : "+v"(vo16), "+v"(vo4), "+v"(scv));
        store_fence_begin();
#pragma unroll
        for (int c = 0; c < 3; ++c) buf_st16<CP>(b, v[c], vo16, c * Vh * 16);
        buf_st4<CP>(b, scv, vo4, 3 * Vh * 16);
        store_drain();
        return sc;
    }
    // stores s and replaces it by the stored (rounded) values
    template <int CP = 0>
    __device__ static __forceinline__ void store(const Buf &b, int Vh, int i, cx<float> s[12])
    {
        unsigned w[12];
        const float sc = store_words<CP>(b, Vh, i, s, w);
#pragma unroll
        for (int k = 0; k < 12; ++k) {
            const cx<float> q = h16_pair(w[k]);
            s[k] = cx<float>{q.re * sc, q.im * sc};
        }
    }
    __device__ static __forceinline__ void to_lds(const Buf &b, int Vh, int i, unsigned char *w, int wsmax, int j)
    {
#pragma unroll
        for (int c = 0; c < 3; ++c) ((v4f *)w)[c * wsmax + j] = buf_ld16(b, i * 16, c * Vh * 16);
        ((float *)(w + (size_t)3 * 16 * wsmax))[j] = buf_ld4(b, i * 4, 3 * Vh * 16);
    }
    __device__ static __forceinline__ float lds_load_raw(const unsigned char *w, int wsmax, int j, cx<float> s[12])
    {
        v4f v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) v[c] = ((const v4f *)w)[c * wsmax + j];
        unpack(v, s);
        return ((const float *)(w + (size_t)3 * 16 * wsmax))[j];
    }
    // integer form for the packed hop: the stored words of site i (one
    // complex entry each) and the site's scale
    __device__ static __forceinline__ float load_i16(const Buf &b, int Vh, int i, s2 p[12])
    {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const v4u u = __builtin_bit_cast(v4u, buf_ld16(b, i * 16, c * Vh * 16));
            p[4 * c] = as_s2(u.x);
            p[4 * c + 1] = as_s2(u.y);
            p[4 * c + 2] = as_s2(u.z);
            p[4 * c + 3] = as_s2(u.w);
        }
        return buf_ld4(b, i * 4, 3 * Vh * 16);
    }
    __device__ static __forceinline__ float lds_load_i16(const unsigned char *w, int wsmax, int j, s2 p[12])
    {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const v4u u = ((const v4u *)w)[c * wsmax + j];
            p[4 * c] = as_s2(u.x);
            p[4 * c + 1] = as_s2(u.y);
            p[4 * c + 2] = as_s2(u.z);
            p[4 * c + 3] = as_s2(u.w);
        }
        return ((const float *)(w + (size_t)3 * 16 * wsmax))[j];
    }
};

// store of a kernel's result that no later access of the same kernel reads:
// non-temporal, so that it does not evict the inputs that neighbouring
// workgroups still read from L2
template <typename S>
__device__ __forceinline__ void store_result(const Buf &b, int Vh, int i, cx<typename SpinorFmt<S>::R> s[12])
{
    SpinorFmt<S>::template store<ST_STREAM>(b, Vh, i, s);
}

// per-wave buffer view of right-hand side `rhs` of a field in format S
template <typename S>
__device__ __forceinline__ Buf spinor_buf(const void *base, int Vh, int rhs)
{
    const size_t per = (size_t)SpinorFmt<S>::SITE_BYTES * (size_t)Vh;
    return make_buf((const unsigned char *)base + (size_t)rhs * per, (unsigned)per);
}

// ---------------------------------------------------------------------------
// bfloat16: round-to-nearest-even from fp32 (the top 16 bits of the fp32
// pattern after adding half an ulp of the kept part, ties to even)
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    union {
        float f;
        uint32_t u;
    } v;
    v.f = f;
    if ((v.u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((v.u >> 16) | ((v.u & 0xffffu) ? 0x40u : 0u));
    uint32_t lsb = (v.u >> 16) & 1u;
    v.u += 0x7fffu + lsb;
    return (uint16_t)(v.u >> 16);
}

__host__ __device__ __forceinline__ float bf16_to_f32(uint32_t h)
{
    union {
        float f;
        uint32_t u;
    } v;
    v.u = h << 16;
    return v.f;
}

// ---------------------------------------------------------------------------
// link storage formats
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void rebuild_row2(cx<R> U[3][3])
{
    // row2 = conj(row0 x row1)
    U[2][0] = cj(cmsub(U[0][1] * U[1][2], U[0][2], U[1][1]));
    U[2][1] = cj(cmsub(U[0][2] * U[1][0], U[0][0], U[1][2]));
    U[2][2] = cj(cmsub(U[0][0] * U[1][1], U[0][1], U[1][0]));
}

// Each format stores one link as NC vectors of type V; unpack() turns the
// NC vectors into the 3x3 matrix (rebuilding row 2 for 12-real storage), so
// global, buffer and LDS reads share the decoding.
struct LinkF64R18 {
    typedef double R;
    typedef double2 V;
    static constexpr int NC = 9;
    static constexpr int REALS = 18;
    static constexpr int BYTES = 144;
    static constexpr int ESZ = 16;
    static constexpr R UNIT = 1.0;  // unpack() returns the link itself
    // staged (LDS) form: the stored vectors themselves
    typedef V SV;
    static constexpr int SNC = NC;
    __device__ static __forceinline__ void stage(const V v[NC], SV w[SNC])
    {
#pragma unroll
        for (int c = 0; c < NC; ++c) w[c] = v[c];
    }
    __device__ static __forceinline__ void unpack(const V v[NC], cx<double> U[3][3])
    {
#pragma unroll
        for (int c = 0; c < 9; ++c) U[c / 3][c % 3] = cx<double>{v[c].x, v[c].y};
    }
    __device__ static __forceinline__ void unpack_staged(const SV w[SNC], cx<R> U[3][3]) { unpack(w, U); }
    __device__ static __forceinline__ V buf_get(const Buf &g, int voff, int soff)
    {
        return v4f_to_d2(buf_ld16(g, voff, soff));
    }
};

struct LinkF32R18 {
    typedef float R;
    typedef float2 V;
    static constexpr int NC = 9;
    static constexpr int REALS = 18;
    static constexpr int BYTES = 72;
    static constexpr int ESZ = 8;
    static constexpr R UNIT = 1.0f;  // unpack() returns the link itself
    // staged (LDS) form: the stored vectors themselves
    typedef V SV;
    static constexpr int SNC = NC;
    __device__ static __forceinline__ void stage(const V v[NC], SV w[SNC])
    {
#pragma unroll
        for (int c = 0; c < NC; ++c) w[c] = v[c];
    }
    __device__ static __forceinline__ void unpack(const V v[NC], cx<float> U[3][3])
    {
#pragma unroll
        for (int c = 0; c < 9; ++c) U[c / 3][c % 3] = cx<float>{v[c].x, v[c].y};
    }
    __device__ static __forceinline__ void unpack_staged(const SV w[SNC], cx<R> U[3][3]) { unpack(w, U); }
    __device__ static __forceinline__ V buf_get(const Buf &g, int voff, int soff)
    {
        v2f f = buf_ld8(g, voff, soff);
        return make_float2(f.x, f.y);
    }
};

struct LinkF32R12 {
    typedef float R;
    typedef float4 V;
    static constexpr int NC = 3;
    static constexpr int REALS = 12;
    static constexpr int BYTES = 48;
    static constexpr int ESZ = 16;
    static constexpr R UNIT = 1.0f;  // unpack() returns the link itself
    // staged (LDS) form: the stored vectors themselves
    typedef V SV;
    static constexpr int SNC = NC;
    __device__ static __forceinline__ void stage(const V v[NC], SV w[SNC])
    {
#pragma unroll
        for (int c = 0; c < NC; ++c) w[c] = v[c];
    }
    __device__ static __forceinline__ void unpack(const V v[NC], cx<float> U[3][3])
    {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            int e = 2 * c;  // complex entries 2c, 2c+1 of rows 0..1
            U[e / 3][e % 3] = cx<float>{v[c].x, v[c].y};
            U[(e + 1) / 3][(e + 1) % 3] = cx<float>{v[c].z, v[c].w};
        }
        rebuild_row2(U);
    }
    __device__ static __forceinline__ void unpack_staged(const SV w[SNC], cx<R> U[3][3]) { unpack(w, U); }
    __device__ static __forceinline__ V buf_get(const Buf &g, int voff, int soff)
    {
        v4f f = buf_ld16(g, voff, soff);
        return make_float4(f.x, f.y, f.z, f.w);
    }
};

struct LinkBF16R12 {
    typedef float R;
    typedef uint2 V;  // four bf16 values
    static constexpr int NC = 3;
    static constexpr int REALS = 12;
    static constexpr int BYTES = 24;
    static constexpr int ESZ = 8;
    static constexpr R UNIT = 1.0f;  // unpack() returns the link itself
    // staged (LDS) form: the stored vectors themselves
    typedef V SV;
    static constexpr int SNC = NC;
    __device__ static __forceinline__ void stage(const V v[NC], SV w[SNC])
    {
#pragma unroll
        for (int c = 0; c < NC; ++c) w[c] = v[c];
    }
    __device__ static __forceinline__ void unpack(const V v[NC], cx<float> U[3][3])
    {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            int e = 2 * c;
            U[e / 3][e % 3] = cx<float>{bf16_to_f32(v[c].x & 0xffffu), bf16_to_f32(v[c].x >> 16)};
            U[(e + 1) / 3][(e + 1) % 3] = cx<float>{bf16_to_f32(v[c].y & 0xffffu), bf16_to_f32(v[c].y >> 16)};
        }
        rebuild_row2(U);
    }
    __device__ static __forceinline__ void unpack_staged(const SV w[SNC], cx<R> U[3][3]) { unpack(w, U); }
    __device__ static __forceinline__ V buf_get(const Buf &g, int voff, int soff)
    {
        v2f f = buf_ld8(g, voff, soff);
        union {
            v2f f;
            uint2 u;
        } cv;
        cv.f = f;
        return cv.u;
    }
};

// 16-bit fixed point, rows 0 and 1: every entry of an SU(3) matrix has
// |re|, |im| <= 1, so each real is stored as round(32767 u) (absolute error
// <= 1/65534), four per 8-byte vector
struct LinkQ16R12 {
    typedef float R;
    typedef uint2 V;
    static constexpr int NC = 3;
    static constexpr int REALS = 12;
    static constexpr int BYTES = 24;
    static constexpr int ESZ = 8;
    static constexpr R UNIT = 1.0f / 32767.0f;  // unpack() returns 32767 U
    __device__ static __forceinline__ void unpack(const V v[NC], cx<float> U[3][3])
    {
        // rows 0 and 1 as stored (32767 u); row 2 rebuilt from them carries
        // 32767^2 and is brought to the same 32767 scale
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            int e = 2 * c;
            U[e / 3][e % 3] = h16_pair(v[c].x);
            U[(e + 1) / 3][(e + 1) % 3] = h16_pair(v[c].y);
        }
        rebuild_row2(U);
#pragma unroll
        for (int b = 0; b < 3; ++b) U[2][b] = cx<float>{U[2][b].re * UNIT, U[2][b].im * UNIT};
    }
    __device__ static __forceinline__ V buf_get(const Buf &g, int voff, int soff)
    {
        const v2u u = __builtin_bit_cast(v2u, buf_ld8(g, voff, soff));
        return make_uint2(u.x, u.y);
    }
    // staged (LDS) form: all nine entries as int16 pairs at the 32767
    // scale, row 2 rebuilt once per workgroup (its rounding to int16 adds
    // at most 1/65534 per real, as for the stored rows)
    typedef unsigned SV;
    static constexpr int SNC = 9;
    __device__ static __forceinline__ void stage(const V v[NC], SV w[SNC])
    {
        cx<float> U[3][3];
        unpack(v, U);
        w[0] = v[0].x;
        w[1] = v[0].y;
        w[2] = v[1].x;
        w[3] = v[1].y;
        w[4] = v[2].x;
        w[5] = v[2].y;
#pragma unroll
        for (int b = 0; b < 3; ++b)
            w[6 + b] = h16_pack(U[2][b].re * UNIT, U[2][b].im * UNIT);
    }
    __device__ static __forceinline__ void unpack_staged(const SV w[SNC], cx<float> U[3][3])
    {
#pragma unroll
        for (int e = 0; e < 9; ++e) U[e / 3][e % 3] = h16_pair(w[e]);
    }
    // staged form of the packed integer hop: at half scale, round(16383.5 u)
    // (|entry| <= 16384), each entry as the two int16 pairs whose dot
    // products with a colour component h = (hr, hi) give the real and the
    // imaginary part of the product: for the link itself (forward hop)
    //   u h:        (ur, -ui) . h,   (ui, ur) . h
    // and for its adjoint (backward hop), entry (a, b) of U^+ = conj(u_ba):
    //   conj(u) h:  (ur, ui) . h,    (-ui, ur) . h
    // in words 2e, 2e + 1 of entry e = 3a + b of the matrix applied
    static constexpr float HALF_UNIT = 2.0f / 32767.0f;
    static constexpr int PK_SNC = 18;
    template <bool ADJ>
    __device__ static __forceinline__ void stage_pk(const V v[NC], SV w[PK_SNC])
    {
        cx<float> U[3][3];
        unpack(v, U);
        const float k = 0.5f * UNIT;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const cx<float> u = ADJ ? U[b][a] : U[a][b];
                const float ur = u.re * k, ui = u.im * k;
                const int e = 3 * a + b;
                w[2 * e] = ADJ ? h16_pack(ur, ui) : h16_pack(ur, -ui);
                w[2 * e + 1] = ADJ ? h16_pack(-ui, ur) : h16_pack(ui, ur);
            }
    }
};

// links of (direction mu, parity par) at checkerboard site i
template <class LK>
__device__ __forceinline__ void link_load(const typename LK::V *__restrict__ g, int Vh, int i,
                                          cx<typename LK::R> U[3][3])
{
    typename LK::V v[LK::NC];
#pragma unroll
    for (int c = 0; c < LK::NC; ++c) v[c] = g[(size_t)c * Vh + i];
    LK::unpack(v, U);
}

template <class LK>
__device__ __forceinline__ void link_load(const Buf &g, int Vh, int soff0, int i, cx<typename LK::R> U[3][3])
{
    typename LK::V v[LK::NC];
#pragma unroll
    for (int c = 0; c < LK::NC; ++c) v[c] = LK::buf_get(g, i * LK::ESZ, soff0 + c * Vh * LK::ESZ);
    LK::unpack(v, U);
}

// ---------------------------------------------------------------------------
// geometry of a batch of lattices and the tile map
// ---------------------------------------------------------------------------
// Division by a run-time constant d >= 1 for numerators n < 2^31
// (Granlund and Montgomery 1994): q = (mulhi(m, n) + n) >> l with
// l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1; the sum stays
// below 2^32 because mulhi(m, n) < n.
struct FastDiv {
    unsigned m;
    int l;
};

inline FastDiv make_fastdiv(unsigned d)
{
    FastDiv f;
    int s = 0;
    while ((1ull << s) < d) ++s;
    f.l = s;
    f.m = (unsigned)((((1ull << 32) * ((1ull << s) - d)) / d) + 1);
    return f;
}

__device__ __forceinline__ int fdiv(int n, FastDiv f)
{
    return (int)((__umulhi(f.m, (unsigned)n) + (unsigned)n) >> f.l);
}

struct LatGeom {
    int L[4];     // extents x, y, z, t
    int Lh0;      // Lx / 2
    int Vh;       // sites per parity
    int bc_t;     // +1 or -1
    int nsb;      // 64-site blocks per parity: ceil(Vh / 64)
    int nrhs;     // right-hand sides of this lattice in the batch
    int sys0;     // index of its first right-hand side in per-system arrays
    int tile0;    // first tile of this lattice in the flat grid
    int nrb;      // right-hand-side blocks: ceil(nrhs / RT)
    FastDiv fLh0, fLy, fLz, fnsb;  // division by Lh0, L[1], L[2], nsb
};

struct BatchGeom {
    int nlat;
    int ntiles;
    int RT;       // right-hand sides (wavefronts) per workgroup
    int G;        // right-hand-side blocks that sweep the site blocks together
    int nsb_max;  // stride of per-system partial arrays
    LatGeom lat[FL_MAXLAT];
    // 1: each XCD sweeps its tiles in reverse order.  The solver alternates
    // it launch by launch, so that a kernel starts on the tiles whose fields
    // its predecessor wrote last (still in the caches): +0.5 % solves/s at
    // 16^3x32 with 384 right-hand sides
    int rev = 0;
};

// Workgroups are dispatched round-robin over the 8 XCDs of the chip (block b
// runs on XCD b % 8).  Renumber them so that each XCD receives a contiguous
// range of tiles: neighbouring sites and the right-hand sides of one site
// block then share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int n, int rev)
{
    const int nx = 8;
    int x = b % nx, k = b / nx;
    int q = n / nx, r = n % nx;
    if (rev) k = q + (x < r ? 1 : 0) - 1 - k;  // the XCD's range from its end
    return x * q + (x < r ? x : r) + k;
}

struct TileInfo {
    int lat;   // lattice index in the batch
    int sb;    // site block
    int rhs;   // right-hand side within the lattice (this wave's)
    int sys;   // global system index
    int site;  // checkerboard site of this lane
    bool valid_rhs;
    bool valid_site;
};

__device__ __forceinline__ TileInfo tile_info(const BatchGeom &B)
{
    int tile = xcd_tile(blockIdx.x, gridDim.x, B.rev);
    int l = 0;
#pragma unroll
    for (int k = 1; k < FL_MAXLAT; ++k)
        if (k < B.nlat && tile >= B.lat[k].tile0) l = k;
    const LatGeom &g = B.lat[l];
    // tiles of a lattice: groups of G right-hand-side blocks; within a group
    // the site blocks are swept in order with the group's blocks innermost
    int local = tile - g.tile0;
    int G = B.G < g.nrb ? B.G : g.nrb;
    int sb, rb;
    if (G == 1) {  // one right-hand-side block sweeps the site blocks
        rb = fdiv(local, g.fnsb);
        sb = local - rb * g.nsb;
    } else {
        int span = g.nsb * G;
        int grp = local / span;
        int rem = local - grp * span;
        int Gg = g.nrb - grp * G;
        if (Gg > G) Gg = G;
        sb = rem / Gg;
        rb = grp * G + (rem - sb * Gg);
    }
    int wave = threadIdx.x / FL_WAVE;
    int lane = threadIdx.x % FL_WAVE;
    TileInfo t;
    t.lat = l;
    t.sb = sb;
    t.rhs = rb * B.RT + wave;
    t.sys = g.sys0 + t.rhs;
    t.site = sb * FL_WAVE + lane;
    t.valid_rhs = t.rhs < g.nrhs;
    t.valid_site = t.site < g.Vh;
    return t;
}

// coordinates of checkerboard site i of parity p
struct Coord {
    int x, y, z, t;
    int rest;  // y + Ly*(z + Lz*t)
};

__device__ __forceinline__ Coord cb_coords(const LatGeom &g, int p, int i)
{
    Coord c;
    c.rest = fdiv(i, g.fLh0);
    const int xh = i - c.rest * g.Lh0;
    const int r = fdiv(c.rest, g.fLy);
    c.y = c.rest - r * g.L[1];
    c.t = fdiv(r, g.fLz);
    c.z = r - c.t * g.L[2];
    c.x = 2 * xh + ((p + c.y + c.z + c.t) & 1);
    return c;
}

__device__ __forceinline__ int cb_index(const LatGeom &g, int x, int y, int z, int t)
{
    return (x >> 1) + g.Lh0 * (y + g.L[1] * (z + g.L[2] * t));
}

// wave-wide sums in a fixed butterfly order (deterministic)
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, FL_WAVE);
    return v;
}

// per-system partial sums: partial[(slot * nsys + sys) * nsb_max + sb]
__device__ __forceinline__ size_t pidx(int slot, int nsys, int sys, int nsb_max, int sb)
{
    return ((size_t)slot * nsys + sys) * nsb_max + sb;
}

// A wave's sums s0, s1, s2 (equal in every lane) as a single store
// instruction at the end of a kernel: lane k < 3 writes slot slot0 + k when
// bit k of `which` is set.
__device__ __forceinline__ void write_partials(double *partial, int slot0, int nsys, int sys, int nsb_max, int sb,
                                               double s0, double s1, double s2, int which)
{
    const int lane = threadIdx.x % FL_WAVE;
    const double v = lane == 0 ? s0 : (lane == 1 ? s1 : s2);
    if (lane < 3 && ((which >> lane) & 1)) partial[pidx(slot0 + lane, nsys, sys, nsb_max, sb)] = v;
}
