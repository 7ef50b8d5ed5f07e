// Batched z-mixing on matrix cores (five-pass path, many states).
//
// For a lateral frequency k the mixing is H(k) = S(k) M(k) with S the 3nz x 3nz
// block matrix of the layer-pair tensors (real xx, yy, zz, xy; imaginary xz, yz)
// and M the 3nz spectra of every state: with several states this is a dense
// product.  Written as a real product
//      [Hr]   [Sr  -Si] [Mr]
//      [Hi] = [Si   Sr] [Mi]      (6nz x 6nz) x (6nz x states)
// it runs on v_mfma_f32_16x16x16_bf16 with both operands split into three
// BF16 terms (a = a0 + a1 + a2, each the BF16 rounding of the remainder) and
// the six products of combined order <= 2 accumulated in FP32, which keeps
// about 24 bits per product.  A block owns one kx column, 16 consecutive ky
// and 16 states; spectra and tensor are staged in LDS with coalesced loads.
// The FP32 variant performs the same product with VALU FMAs on the same
// staging, so the two differ only in the arithmetic.
// The packed column kx = 0 (kx = 0 and Lx/2 together) is mixed by the generic
// kernel.
#include "field_kernels.hpp"
#include "launch.hpp"

namespace hfd {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int TK = 16;       // frequencies per block
constexpr int NBS = 16;      // states per block
constexpr int NZ_MFMA = 8;   // largest nz (6 nz <= 48 -> three 16-row tiles)
constexpr int MT_MAX = 3;

// round-to-nearest-even FP32 -> BF16 (bits) and back
__device__ __forceinline__ unsigned short bf16_bits(float x)
{
    const unsigned u = __float_as_uint(x);
    const unsigned r = u + 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(r >> 16);
}
__device__ __forceinline__ float bf16_float(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

__device__ __forceinline__ void split3(float x, short& h, short& m, short& l)
{
    const unsigned short bh = bf16_bits(x);
    const float r1 = x - bf16_float(bh);
    const unsigned short bm = bf16_bits(r1);
    const float r2 = r1 - bf16_float(bm);
    h = (short)bh;
    m = (short)bm;
    l = (short)bf16_bits(r2);
}

}  // namespace

template <bool MFMA>
__global__ __launch_bounds__(256) void k_mix_batched(const cpx<float>* __restrict__ Mh,
                                                     cpx<float>* __restrict__ Hh, int nz, int M,
                                                     int LY, int B, const float* __restrict__ Q,
                                                     long long q_geom_stride, int QY,
                                                     const float* __restrict__ lp, int bpg,
                                                     int adjoint)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int S = 3 * nz, S6 = 6 * nz, P = nz * (nz + 1) / 2;
    const int KT = (S6 + 15) / 16;
    cpx<float>* sm = reinterpret_cast<cpx<float>*>(smem_raw);                  // [TK][S][NBS]
    float* st = reinterpret_cast<float*>(sm + TK * S * NBS);                   // [TK][P][5]
    float* sa = st + TK * P * 5;                                               // [4 waves][S6][S6]
    const int kx = 1 + blockIdx.y;
    const int ky0 = blockIdx.x * TK;
    const int b0 = blockIdx.z * NBS;
    const int geom = b0 / bpg;  // a block never spans two stacks (bpg % 16 == 0 or B == bpg)
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const long long sst = (long long)M * LY;

    // stage spectra: 16 consecutive ky per (state, signal)
    for (int idx = tid; idx < TK * S * NBS; idx += 256) {
        const int kyl = idx % TK, s = (idx / TK) % S, bl = idx / (TK * S);
        const int b = b0 + bl, ky = ky0 + kyl;
        cpx<float> v = {0.f, 0.f};
        if (b < B && ky < LY) v = Mh[((long long)b * S + s) * sst + (long long)kx * LY + ky];
        sm[(kyl * S + s) * NBS + bl] = v;
    }
    // stage the tensor quadrant values; the ky-odd components (xy, yz) change
    // sign for ky > LY/2.  The sign is applied as a bit flip: a nested
    // conditional negation here was compiled with the xy case dropped.
    const float* Qcol = Q + (long long)geom * q_geom_stride + (long long)kx * P * 5 * QY;
    for (int idx = tid; idx < TK * P * 5; idx += 256) {
        const int kyl = idx % TK, c = (idx / TK) % 5, u = idx / (TK * 5);
        const int ky = ky0 + kyl;
        const int kq = ky <= LY / 2 ? ky : LY - ky;
        float v = 0.f;
        if (ky < LY) v = Qcol[(long long)(u * 5 + c) * QY + kq];
        // c in {2, 4}: even and non-zero
        const unsigned flip = (unsigned)(ky > LY / 2) & (unsigned)((c & 1) == 0) & (unsigned)(c != 0);
        st[(kyl * P + u) * 5 + c] = __uint_as_float(__float_as_uint(v) ^ (flip << 31));
    }
    __syncthreads();

    const float* lpg = lp + (long long)geom * 2 * nz;
    float* A = sa + w * S6 * S6;
    for (int kyl = w; kyl < TK; kyl += 4) {
        if (ky0 + kyl >= LY) break;
        // real 6nz x 6nz matrix of this frequency: rows (part, c, i), columns (part, c', j)
        const float* tq = st + kyl * P * 5;
        for (int e = l; e < S6 * S6; e += 64) {
            const int r = e / S6, k = e - r * S6;
            const int pr = r / S, rr = r - pr * S, c = rr / nz, i = rr - c * nz;
            const int pk = k / S, kk = k - pk * S, cc = kk / nz, j = kk - cc * nz;
            const int a = i < j ? i : j, bq = i < j ? j : i;
            const float* q = tq + (a * nz - a * (a - 1) / 2 + (bq - a)) * 5;
            float re = 0.f, im = 0.f;
            if (c == cc) {
                re = c == 0 ? q[0] : (c == 1 ? q[1] : -(q[0] + q[1]) + (i == j ? lpg[nz + i] : 0.f));
            } else if (c + cc == 1) {
                re = q[2];  // xy
            } else {
                im = (c + cc == 2) ? q[3] : q[4];  // xz or yz
                if (i > j) im = -im;               // conj for the transposed pair
            }
            float v = (pr == pk) ? re : (pr == 0 ? -im : im);
            v *= adjoint ? lpg[j] : lpg[i];
            A[e] = v;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        cpx<float>* mk = sm + kyl * S * NBS;   // spectra of this frequency, [S][NBS]
        const int n = l & 15, q4 = l >> 4;
        auto bval = [&](int k) -> float {
            if (k >= S6) return 0.f;
            const int pk = k / S, s = k - pk * S;
            const cpx<float> z = mk[s * NBS + n];
            return pk == 0 ? z.x : z.y;
        };
        auto aval = [&](int r, int k) -> float { return (r < S6 && k < S6) ? A[r * S6 + k] : 0.f; };
        const int MT = KT;
        f32x4 D[MT_MAX];
        for (int mt = 0; mt < MT_MAX; ++mt) D[mt] = (f32x4){0.f, 0.f, 0.f, 0.f};
        if constexpr (MFMA) {
            for (int kt = 0; kt < KT; ++kt) {
                bf16x4 bh, bm, bl;
                for (int e = 0; e < 4; ++e) {
                    short h, m, lo;
                    split3(bval(kt * 16 + 4 * q4 + e), h, m, lo);
                    bh[e] = h; bm[e] = m; bl[e] = lo;
                }
                for (int mt = 0; mt < MT; ++mt) {
                    bf16x4 ah, am, al;
                    for (int e = 0; e < 4; ++e) {
                        short h, m, lo;
                        split3(aval(mt * 16 + (l & 15), kt * 16 + 4 * q4 + e), h, m, lo);
                        ah[e] = h; am[e] = m; al[e] = lo;
                    }
                    f32x4 d = D[mt];
                    d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, d, 0, 0, 0);
                    d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(am, bm, d, 0, 0, 0);
                    d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, d, 0, 0, 0);
                    d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(am, bh, d, 0, 0, 0);
                    d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bm, d, 0, 0, 0);
                    d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, d, 0, 0, 0);
                    D[mt] = d;
                }
            }
        } else {
            // same product on the VALU: lane owns rows 4 q4 + e of each tile, column n
            for (int mt = 0; mt < MT; ++mt)
                for (int e = 0; e < 4; ++e) {
                    const int r = mt * 16 + 4 * q4 + e;
                    float acc = 0.f;
                    if (r < S6)
                        for (int k = 0; k < S6; ++k) acc = fmaf(A[r * S6 + k], bval(k), acc);
                    D[mt][e] = acc;
                }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // D[mt][e] = output row r = mt 16 + 4 q4 + e (part, c, i), state n
        for (int mt = 0; mt < MT; ++mt)
            for (int e = 0; e < 4; ++e) {
                const int r = mt * 16 + 4 * q4 + e;
                if (r < S6) {
                    const int pr = r / S, s = r - pr * S;
                    float* dst = reinterpret_cast<float*>(&mk[s * NBS + n]);
                    dst[pr] = D[mt][e];
                }
            }
    }
    __syncthreads();
    for (int idx = tid; idx < TK * S * NBS; idx += 256) {
        const int kyl = idx % TK, s = (idx / TK) % S, bl = idx / (TK * S);
        const int b = b0 + bl, ky = ky0 + kyl;
        if (b < B && ky < LY) Hh[((long long)b * S + s) * sst + (long long)kx * LY + ky] = sm[(kyl * S + s) * NBS + bl];
    }
}

bool mix_batched_supported(int nz, int B, int G)
{
    if (nz < 1 || nz > NZ_MFMA) return false;
    const int bpg = B / G;
    return G == 1 || bpg % NBS == 0;
}

size_t mix_batched_lds(int nz)
{
    const int S = 3 * nz, S6 = 6 * nz, P = nz * (nz + 1) / 2;
    return sizeof(cpx<float>) * TK * S * NBS + sizeof(float) * (TK * P * 5 + 4 * S6 * S6);
}

hipError_t launch_mix_batched(bool mfma, const void* Mh, void* Hh, int nz, int M, int LY, int B,
                              const void* Q, long long qgs, int QY, const void* lp, int bpg,
                              int adjoint, hipStream_t s)
{
    if (M < 2) return hipSuccess;
    const size_t lds = mix_batched_lds(nz);
    dim3 grid((LY + TK - 1) / TK, M - 1, (B + NBS - 1) / NBS);
    if (mfma) {
        static bool done = false;
        if (!done && lds > 65536) {
            hipError_t e = hipFuncSetAttribute((const void*)k_mix_batched<true>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, 163840);
            if (e != hipSuccess) return e;
            done = true;
        }
        hipLaunchKernelGGL(k_mix_batched<true>, grid, dim3(256), lds, s, (const cpx<float>*)Mh,
                           (cpx<float>*)Hh, nz, M, LY, B, (const float*)Q, qgs, QY,
                           (const float*)lp, bpg, adjoint);
    } else {
        static bool done = false;
        if (!done && lds > 65536) {
            hipError_t e = hipFuncSetAttribute((const void*)k_mix_batched<false>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, 163840);
            if (e != hipSuccess) return e;
            done = true;
        }
        hipLaunchKernelGGL(k_mix_batched<false>, grid, dim3(256), lds, s, (const cpx<float>*)Mh,
                           (cpx<float>*)Hh, nz, M, LY, B, (const float*)Q, qgs, QY,
                           (const float*)lp, bpg, adjoint);
    }
    return hipGetLastError();
}

}  // namespace hfd
