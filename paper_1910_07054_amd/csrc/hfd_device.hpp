// Device-side building blocks for gfx950: complex arithmetic and a
// wavefront-local Stockham FFT engine.
//
// One FFT of length L is owned by a group of GT = L / V lanes of a single
// 64-wide wavefront; every lane holds V complex values in registers.  Passes
// use radix 8 (4 or 2 for the remainder).  Between passes the group exchanges
// data through its own LDS region of fft_region(L) slots (L values with one
// padding slot per eight, see lds_pad); because the group never spans two
// wavefronts, no workgroup barrier is needed inside a transform.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hfd {

template <typename R>
struct alignas(2 * sizeof(R)) cpx {
    R x, y;
};

template <typename R>
__device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b)
{
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cpx<R> cconj(cpx<R> a) { return {a.x, -a.y}; }
template <typename R>
__device__ __forceinline__ cpx<R> cscale(cpx<R> a, R s) { return {a.x * s, a.y * s}; }
// multiply by -i (forward transforms) or +i (inverse transforms)
template <typename R, bool INV>
__device__ __forceinline__ cpx<R> mul_mi(cpx<R> a)
{
    return INV ? cpx<R>{-a.y, a.x} : cpx<R>{a.y, -a.x};
}

// Row order of the tensor tables (the Fourier tensor's pair slots and the
// derivative offsets): kx = 0, kx = M = Lx/2, then kx = 1 .. M - 1, so that
// the two rows the packed column 0 reads are adjacent.
__host__ __device__ inline int tab_row(int kx, int M) { return kx == 0 ? 0 : (kx == M ? 1 : kx + 1); }

// Ordering point for LDS traffic inside one wavefront.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Read-only view of `bytes` bytes at a wave-uniform base, loaded with raw buffer
// instructions: a per-lane 32-bit byte offset plus a wave-uniform (scalar) byte
// offset, so no per-lane 64-bit address arithmetic.  Loads beyond `bytes`
// return zero instead of touching memory.
template <typename R>
struct UniformBuf {
    __amdgpu_buffer_rsrc_t rsrc;
    __device__ __forceinline__ UniformBuf(const R* base, unsigned bytes)
        : rsrc(__builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)bytes, 0x00020000))
    {
    }
    // element at (scalar element offset s) + (lane element offset v)
    __device__ __forceinline__ R ld(unsigned v, unsigned s) const
    {
        if constexpr (sizeof(R) == 4)
            return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b32(rsrc, (int)(v * 4u),
                                                                              (int)(s * 4u), 0));
        else
            return __builtin_bit_cast(R, __builtin_amdgcn_raw_buffer_load_b64(rsrc, (int)(v * 8u),
                                                                              (int)(s * 8u), 0));
    }
};

// values per lane for a transform of length L
__host__ __device__ constexpr int fft_vals(int L) { return L <= 8 ? L : (L <= 512 ? 8 : L / 64); }

// --- small DFTs in registers (natural order in and out) -------------------
template <typename R, bool INV>
__device__ __forceinline__ void dft2(cpx<R>* v)
{
    cpx<R> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
}

template <typename R, bool INV>
__device__ __forceinline__ void dft4(cpx<R>& a0, cpx<R>& a1, cpx<R>& a2, cpx<R>& a3)
{
    cpx<R> t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3);
    cpx<R> t3 = mul_mi<R, INV>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

template <typename R, bool INV>
__device__ __forceinline__ void dft8(cpx<R>* v)
{
    const R c = R(0.70710678118654752440084436210484903928);
    cpx<R> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cpx<R> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<R, INV>(e0, e1, e2, e3);
    dft4<R, INV>(o0, o1, o2, o3);
    // o_k *= w8^k (w8 = exp(-+ 2 pi i / 8))
    if (!INV) {
        o1 = {c * (o1.x + o1.y), c * (o1.y - o1.x)};
        o3 = {c * (o3.y - o3.x), -c * (o3.x + o3.y)};
    } else {
        o1 = {c * (o1.x - o1.y), c * (o1.x + o1.y)};
        o3 = {-c * (o3.x + o3.y), c * (o3.x - o3.y)};
    }
    o2 = mul_mi<R, INV>(o2);
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1);
    v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2);
    v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3);
    v[7] = csub(e3, o3);
}

template <typename R, int RAD, bool INV>
__device__ __forceinline__ void dft(cpx<R>* v)
{
    if constexpr (RAD == 8) dft8<R, INV>(v);
    else if constexpr (RAD == 4) dft4<R, INV>(v[0], v[1], v[2], v[3]);
    else dft2<R, INV>(v);
}

// Radix-RAD DFT of inputs whose upper half v[RAD/2 ..] is zero (the first
// pass of a transform of a zero-padded sequence): the butterflies that only
// add zeros are dropped.
template <typename R, int RAD, bool INV>
__device__ __forceinline__ void dft_half_in(cpx<R>* v)
{
    // DFT4 of (a0, a1, 0, 0): (a0 + a1, a0 + rot(a1), a0 - a1, a0 - rot(a1)),
    // rot = multiplication by -i (forward) or +i (inverse)
    auto dft4h = [](cpx<R> a0, cpx<R> a1, cpx<R>& b0, cpx<R>& b1, cpx<R>& b2, cpx<R>& b3) {
        const cpx<R> t = mul_mi<R, INV>(a1);
        b0 = cadd(a0, a1);
        b2 = csub(a0, a1);
        b1 = cadd(a0, t);
        b3 = csub(a0, t);
    };
    if constexpr (RAD == 8) {
        const R c = R(0.70710678118654752440084436210484903928);
        cpx<R> e0, e1, e2, e3, o0, o1, o2, o3;
        dft4h(v[0], v[2], e0, e1, e2, e3);
        dft4h(v[1], v[3], o0, o1, o2, o3);
        if (!INV) {
            o1 = {c * (o1.x + o1.y), c * (o1.y - o1.x)};
            o3 = {c * (o3.y - o3.x), -c * (o3.x + o3.y)};
        } else {
            o1 = {c * (o1.x - o1.y), c * (o1.x + o1.y)};
            o3 = {-c * (o3.x + o3.y), c * (o3.x - o3.y)};
        }
        o2 = mul_mi<R, INV>(o2);
        v[0] = cadd(e0, o0);
        v[4] = csub(e0, o0);
        v[1] = cadd(e1, o1);
        v[5] = csub(e1, o1);
        v[2] = cadd(e2, o2);
        v[6] = csub(e2, o2);
        v[3] = cadd(e3, o3);
        v[7] = csub(e3, o3);
    } else if constexpr (RAD == 4) {
        dft4h(v[0], v[1], v[0], v[1], v[2], v[3]);
    } else {
        v[1] = v[0];
    }
}

// LDS slot of element `pos` in the intermediate passes of a transform: one
// padding slot after every eight elements, so a transform of length L uses
// fft_region(L) slots.  The writes of a radix-8 pass go to positions 8j + r
// (first pass, lane j) and 64q + 8r + k (later passes, lane j = 8q + k); in
// natural order a half-wave's writes fall on 4 or 8 of the 32 eight-byte bank
// slots, padded on 32 distinct ones.  A lane's positions differ by multiples
// of 8 (or by r < 8 from a multiple of 8 in the first pass), so their padded
// slots differ by compile-time constants and cost no address arithmetic.
__host__ __device__ constexpr int fft_region(int L) { return L + (L >> 3); }
__device__ __forceinline__ int lds_pad(int pos) { return pos + (pos >> 3); }

// --- Stockham engine -------------------------------------------------------
// X[k] = sum_n x[n] exp(-+2 pi i n k / L) (unnormalized in both directions).
// Twiddles: table of exp(-2 pi i m / (L * tws)) read at index m * tws,
// m in [0, L).  A lane's twiddles depend only on its position g in the group,
// so they are loaded once (Twiddles::load) and reused for every transform the
// lane runs; inverse transforms use their conjugates.
// load(pos) supplies x[pos] for the first pass; store(pos, v) receives X[pos]
// from the last pass; sh is the group's LDS region of fft_region(L) slots
// (the last pass stores through `store`, which may write the region's first
// L slots in natural order).
template <int L, int V, int NS>
struct PassShape {
    static constexpr int REM = L / NS;
    static constexpr int RAD = (REM >= 8 && V % 8 == 0) ? 8 : ((REM >= 4 && V % 4 == 0) ? 4 : 2);
    static constexpr int NB = V / RAD;
    static constexpr bool LAST = (NS * RAD == L);
    static constexpr int NEXT = LAST ? L : NS * RAD;
};

// twiddle registers of all passes after the first, in pass order
template <int L, int V, int NS = 1>
struct TwCount {
    using P = PassShape<L, V, NS>;
    static constexpr int here = NS > 1 ? P::NB * (P::RAD - 1) : 0;
    static constexpr int value = here + (P::LAST ? 0 : TwCount<L, V, P::NEXT>::value);
};
template <int L, int V>
struct TwCount<L, V, L> {
    static constexpr int value = 0;
};

template <typename R, int L>
struct Twiddles {
    static constexpr int V = fft_vals(L);
    static constexpr int GT = L / V;
    static constexpr int N = TwCount<L, V>::value > 0 ? TwCount<L, V>::value : 1;
    cpx<R> w[N];

    template <int NS, int OFF>
    __device__ __forceinline__ void fill(int g, const cpx<R>* __restrict__ tw, int tws)
    {
        using P = PassShape<L, V, NS>;
        constexpr int here = NS > 1 ? P::NB * (P::RAD - 1) : 0;
        if constexpr (NS > 1) {
#pragma unroll
            for (int u = 0; u < P::NB; ++u) {
                const int j = g + GT * u;
                const int k = j & (NS - 1);
#pragma unroll
                for (int r = 1; r < P::RAD; ++r)
                    w[OFF + u * (P::RAD - 1) + r - 1] = tw[r * k * (L / (NS * P::RAD)) * tws];
            }
        }
        if constexpr (!P::LAST) fill<P::NEXT, OFF + here>(g, tw, tws);
    }
    __device__ __forceinline__ void load(int g, const cpx<R>* __restrict__ tw, int tws)
    {
        fill<1, 0>(g, tw, tws);
    }
};

// HIN: the input positions L/2 .. L-1 are zero (zero-padded sequence): the
// first pass neither loads nor transforms them.  HOUT: only the output
// positions 0 .. L/2-1 are wanted (cropped result): the last pass stores only
// those, and what feeds nothing else is not computed.
template <typename R, int L, int V, bool INV, int NS, int OFF, bool PRE = false, bool HIN = false,
          bool HOUT = false, class Load, class Store>
__device__ __forceinline__ void fft_pass(cpx<R> (&v)[V], cpx<R>* sh, int g, const cpx<R>* w,
                                         Load& load, Store& store)
{
    using P = PassShape<L, V, NS>;
    constexpr int GT = L / V;
    constexpr int RAD = P::RAD, NB = P::NB;
    constexpr int STRIDE = L / RAD;
    constexpr bool FIRST = (NS == 1);
    constexpr bool LAST = P::LAST;
    constexpr bool HALF_IN = FIRST && HIN;
    static_assert(L % (NS * RAD) == 0, "radix schedule");
    static_assert(FIRST || STRIDE % 8 == 0, "later passes read at multiples of 8");
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int j = g + GT * u;
        const int pj = lds_pad(j);
#pragma unroll
        for (int r = 0; r < RAD; ++r) {
            if constexpr (FIRST) {
                // positions j + r STRIDE >= L/2 exactly when r >= RAD/2
                if constexpr (HALF_IN) {
                    if (r >= RAD / 2) {
                        v[u * RAD + r] = {R(0), R(0)};
                        continue;
                    }
                }
                if constexpr (!PRE) v[u * RAD + r] = load(j + r * STRIDE);
            } else {
                v[u * RAD + r] = sh[pj + r * (STRIDE + STRIDE / 8)];
            }
        }
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        if constexpr (NS > 1) {
#pragma unroll
            for (int r = 1; r < RAD; ++r) {
                cpx<R> t = w[OFF + u * (RAD - 1) + r - 1];
                if (INV) t.y = -t.y;
                v[u * RAD + r] = cmul(v[u * RAD + r], t);
            }
        }
        if constexpr (HALF_IN) dft_half_in<R, RAD, INV>(&v[u * RAD]);
        else dft<R, RAD, INV>(&v[u * RAD]);
    }
    if constexpr (!FIRST) wave_sync();
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int j = g + GT * u;
        const int k = j & (NS - 1);
        const int base = (j - k) * RAD + k;
        const int pb = lds_pad(base);
#pragma unroll
        for (int r = 0; r < RAD; ++r) {
            if constexpr (LAST) {
                // positions base + r NS >= L/2 exactly when r >= RAD/2
                if (!HOUT || r < RAD / 2) store(base + r * NS, v[u * RAD + r]);
            } else {
                // first pass: (base & 7) + r < 8, so the padded slot is pb + r
                sh[pb + r * (NS + NS / 8)] = v[u * RAD + r];
            }
        }
    }
    if constexpr (!LAST) {
        wave_sync();
        constexpr int here = NS > 1 ? NB * (RAD - 1) : 0;
        fft_pass<R, L, V, INV, P::NEXT, OFF + here, false, false, HOUT>(v, sh, g, w, load, store);
    }
}

// The values a lane reads in the first pass, in register order, so that the
// input of several transforms can be requested before any of them starts
// (HIN: the zero upper half is not requested).
template <typename R, int L, bool HIN = false, class Load>
__device__ __forceinline__ void fft_first_loads(cpx<R> (&v)[fft_vals(L)], int g, Load load)
{
    constexpr int V = fft_vals(L), GT = L / V;
    using P = PassShape<L, V, 1>;
    constexpr int STRIDE = L / P::RAD;
#pragma unroll
    for (int u = 0; u < P::NB; ++u)
#pragma unroll
        for (int r = 0; r < P::RAD; ++r)
            v[u * P::RAD + r] = (HIN && r >= P::RAD / 2) ? cpx<R>{R(0), R(0)}
                                                           : load(g + GT * u + r * STRIDE);
}

// One transform whose first-pass values are already in v (fft_first_loads).
// sh: the group's LDS region of fft_region(L) values.
template <typename R, int L, bool INV, bool HIN = false, bool HOUT = false, class Store>
__device__ __forceinline__ void wave_fft_pre(cpx<R>* sh, int g, const Twiddles<R, L>& tw,
                                             cpx<R> (&v)[fft_vals(L)], Store store)
{
    constexpr int V = fft_vals(L);
    static_assert(L / V <= 64, "one transform must fit in a wavefront");
    auto none = [](int) { return cpx<R>{R(0), R(0)}; };
    fft_pass<R, L, V, INV, 1, 0, true, HIN, HOUT>(v, sh, g, tw.w, none, store);
}

// One transform with preloaded twiddles.
template <typename R, int L, bool INV, bool HIN = false, bool HOUT = false, class Load, class Store>
__device__ __forceinline__ void wave_fft(cpx<R>* sh, int g, const Twiddles<R, L>& tw, Load load,
                                         Store store)
{
    constexpr int V = fft_vals(L);
    static_assert(L / V <= 64, "one transform must fit in a wavefront");
    cpx<R> v[V];
    fft_pass<R, L, V, INV, 1, 0, false, HIN, HOUT>(v, sh, g, tw.w, load, store);
}

// One transform loading its own twiddles (single-use callers).
template <typename R, int L, bool INV, bool HIN = false, bool HOUT = false, class Load, class Store>
__device__ __forceinline__ void wave_fft(cpx<R>* sh, int g, const cpx<R>* __restrict__ tw, int tws,
                                         Load load, Store store)
{
    Twiddles<R, L> t;
    t.load(g, tw, tws);
    wave_fft<R, L, INV, HIN, HOUT>(sh, g, t, load, store);
}

}  // namespace hfd
