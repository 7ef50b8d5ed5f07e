// Device-side building blocks for gfx950: complex arithmetic and a
// wavefront-local Stockham FFT engine.
//
// One FFT of length L is owned by a group of GT = L / V lanes of a single
// 64-wide wavefront; every lane holds V complex values in registers.  Passes
// use radix 8 (4 or 2 for the remainder).  Between passes the group exchanges
// data through its own LDS region of L values; because the group never spans
// two wavefronts, no workgroup barrier is needed inside a transform.
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

// Ordering point for LDS traffic inside one wavefront.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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

// --- Stockham engine -------------------------------------------------------
// X[k] = sum_n x[n] exp(-+2 pi i n k / L) (unnormalized in both directions).
// tw: table of exp(-2 pi i m / (L * tws)) read at index m * tws, m in [0, L).
// load(pos) supplies x[pos] for the first pass; store(pos, v) receives X[pos]
// from the last pass; sh is the group's LDS region of L values.
template <typename R, int L, int V, bool INV, int NS, class Load, class Store>
__device__ __forceinline__ void fft_pass(cpx<R> (&v)[V], cpx<R>* sh, int g,
                                         const cpx<R>* __restrict__ tw, int tws, Load& load,
                                         Store& store)
{
    constexpr int GT = L / V;
    constexpr int REM = L / NS;
    constexpr int RAD = (REM >= 8 && V % 8 == 0) ? 8 : ((REM >= 4 && V % 4 == 0) ? 4 : 2);
    constexpr int NB = V / RAD;
    constexpr int STRIDE = L / RAD;
    constexpr bool FIRST = (NS == 1);
    constexpr bool LAST = (NS * RAD == L);
    static_assert(L % (NS * RAD) == 0, "radix schedule");
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int j = g + GT * u;
#pragma unroll
        for (int r = 0; r < RAD; ++r) {
            const int pos = j + r * STRIDE;
            if constexpr (FIRST) v[u * RAD + r] = load(pos);
            else v[u * RAD + r] = sh[pos];
        }
    }
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int j = g + GT * u;
        if constexpr (NS > 1) {
            const int k = j & (NS - 1);
#pragma unroll
            for (int r = 1; r < RAD; ++r) {
                cpx<R> w = tw[r * k * (L / (NS * RAD)) * tws];
                if (INV) w.y = -w.y;
                v[u * RAD + r] = cmul(v[u * RAD + r], w);
            }
        }
        dft<R, RAD, INV>(&v[u * RAD]);
    }
    if constexpr (!FIRST) wave_sync();
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int j = g + GT * u;
        const int k = j & (NS - 1);
        const int base = (j - k) * RAD + k;
#pragma unroll
        for (int r = 0; r < RAD; ++r) {
            const int pos = base + r * NS;
            if constexpr (LAST) store(pos, v[u * RAD + r]);
            else sh[pos] = v[u * RAD + r];
        }
    }
    if constexpr (!LAST) {
        wave_sync();
        fft_pass<R, L, V, INV, NS * RAD>(v, sh, g, tw, tws, load, store);
    }
}

template <typename R, int L, bool INV, class Load, class Store>
__device__ __forceinline__ void wave_fft(cpx<R>* sh, int g, const cpx<R>* __restrict__ tw, int tws,
                                         Load load, Store store)
{
    constexpr int V = fft_vals(L);
    static_assert(L / V <= 64, "one transform must fit in a wavefront");
    cpx<R> v[V];
    fft_pass<R, L, V, INV, 1>(v, sh, g, tw, tws, load, store);
}

}  // namespace hfd
