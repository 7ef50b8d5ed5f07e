// Batched z-mixing on matrix cores (five-pass path, many states).
//
// For a lateral frequency k the mixing is H(k) = S(k) M(k) with S the 3nz x 3nz
// block matrix of the layer-pair tensors (real xx, yy, zz, xy; imaginary xz, yz)
// and M the 3nz spectra of every state: with several states this is a dense
// product.  Written as a real product
//      [Hr]   [Sr  -Si] [Mr]
//      [Hi] = [Si   Sr] [Mi]      (6nz x 6nz) x (6nz x states)
// it runs on v_mfma_f32_16x16x32_bf16 with both operands split into three
// BF16 terms (a = a0 + a1 + a2, each the BF16 rounding of the remainder) and
// the six products of combined order <= 2 accumulated in FP32, which keeps
// about 24 bits per product.  A block owns 16 (8 above five layers)
// consecutive ky of one kx column and all states of one stack: the frequency
// matrices are built and split once, then applied to the states 16 at a time
// (the 16 columns of one product); spectra and tensor are staged in LDS with
// coalesced loads.  The FP32 variant performs the same product with VALU FMAs
// on the same staging, so the two differ only in the arithmetic.
// The packed column kx = 0 (kx = 0 and Lx/2 together) is mixed by the generic
// kernel.
#include "field_kernels.hpp"
#include "launch.hpp"

namespace hfd {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int NBS = 16;      // states per chunk (the 16 columns of one product)
constexpr int NZ_MFMA = 8;   // largest nz (6 nz <= 48 -> three 16-row tiles)

// round-to-nearest-even FP32 -> BF16 (bits) and back
__device__ __forceinline__ unsigned short bf16_bits(float x)
{
    const unsigned u = __float_as_uint(x);
    const unsigned r = u + 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(r >> 16);
}
__device__ __forceinline__ float bf16_float(unsigned short b) { return __uint_as_float((unsigned)b << 16); }

__device__ __forceinline__ void split3(float x, __bf16& h, __bf16& m, __bf16& l)
{
    const unsigned short bh = bf16_bits(x);
    const float r1 = x - bf16_float(bh);
    const unsigned short bm = bf16_bits(r1);
    const float r2 = r1 - bf16_float(bm);
    h = __builtin_bit_cast(__bf16, bh);
    m = __builtin_bit_cast(__bf16, bm);
    l = __builtin_bit_cast(__bf16, bf16_bits(r2));
}

}  // namespace

template <int NZ>
struct BatchedShape {
    static constexpr int S = 3 * NZ, S6 = 6 * NZ, P = NZ * (NZ + 1) / 2;
    static constexpr int KT = (S6 + 15) / 16;       // 16-row tiles (rows of A and of the output)
    static constexpr int KT2 = (S6 + 31) / 32;      // 32-wide tiles of the sum (one product)
    static constexpr int TK = 8;                      // frequencies per block
    static constexpr int FW = TK / 4;                 // frequencies per wave
    static constexpr int AS = (S6 + 3) & ~3;          // row stride of the FP32 matrix
    static constexpr size_t sm_bytes = sizeof(cpx<float>) * TK * S * NBS;
    static constexpr size_t st_bytes = sizeof(float) * TK * P * 5;
    static constexpr size_t sa_bytes(bool mfma) { return sizeof(float) * (mfma ? 4 : TK) * S6 * AS; }
    static constexpr size_t lds(bool mfma) { return sm_bytes + st_bytes + sa_bytes(mfma); }
};

// Real 6nz x 6nz matrix of one frequency (rows (part, c, i), columns
// (part, c', j)), from the staged tensor values tq[pair][5], into A (row
// stride AS).  Entries are spread over the 64 lanes of the wave.
template <int NZ>
__device__ __forceinline__ void build_real_matrix(float* A, const float* tq, const float* lpg, int l,
                                                  int adjoint)
{
    using SH = BatchedShape<NZ>;
    constexpr int S = SH::S, S6 = SH::S6;
    for (int e = l; e < S6 * S6; e += 64) {
        const int r = e / S6, k = e - r * S6;
        const int pr = r / S, rr = r - pr * S, c = rr / NZ, i = rr - c * NZ;
        const int pk = k / S, kk = k - pk * S, cc = kk / NZ, j = kk - cc * NZ;
        const int a = i < j ? i : j, bq = i < j ? j : i;
        const float* q = tq + (a * NZ - a * (a - 1) / 2 + (bq - a)) * 5;
        float re = 0.f, im = 0.f;
        if (c == cc) {
            re = c == 0 ? q[0] : (c == 1 ? q[1] : -(q[0] + q[1]) + (i == j ? lpg[NZ + i] : 0.f));
        } else if (c + cc == 1) {
            re = q[2];  // xy
        } else {
            im = (c + cc == 2) ? q[3] : q[4];  // xz or yz
            if (i > j) im = -im;               // conj for the transposed pair
        }
        float v = (pr == pk) ? re : (pr == 0 ? -im : im);
        v *= adjoint ? lpg[j] : lpg[i];
        A[r * SH::AS + k] = v;
    }
}

// Grid: (ceil(LY / TK), M - 1, G).  A block owns TK consecutive ky of one kx
// column and all bpg states of one stack; each wave owns FW of the
// frequencies.  The frequency matrices are built once per block (for the
// matrix cores: split into BF16 triples held in registers) and applied to the
// states in chunks of NBS, staged through LDS with coalesced loads and stores.
template <bool MFMA, int NZ>
__global__ __launch_bounds__(256) void k_mix_batched(const cpx<float>* __restrict__ Mh,
                                                     cpx<float>* __restrict__ Hh, int M, int LY,
                                                     const float* __restrict__ Q,
                                                     long long qcs, const int* __restrict__ qslot,
                                                     int QY,
                                                     const float* __restrict__ lp, int bpg,
                                                     int adjoint)
{
    using SH = BatchedShape<NZ>;
    constexpr int S = SH::S, S6 = SH::S6, P = SH::P, KT = SH::KT, KT2 = SH::KT2, TK = SH::TK,
                  FW = SH::FW, AS = SH::AS;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<float>* sm = reinterpret_cast<cpx<float>*>(smem_raw);                      // [TK][S][NBS]
    float* st = reinterpret_cast<float*>(smem_raw + SH::sm_bytes);                 // [TK][P][5]
    float* sa = reinterpret_cast<float*>(smem_raw + SH::sm_bytes + SH::st_bytes);  // matrices
    const int kx = 1 + blockIdx.y;
    const int ky0 = blockIdx.x * TK;
    const int geom = blockIdx.z;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int n = l & 15, q4 = l >> 4;
    const long long sst = (long long)M * LY;

    // tensor quadrant values; the ky-odd components (xy, yz) change sign for
    // ky > LY/2.  The sign is applied as a bit flip: a nested conditional
    // negation here was compiled with the xy case dropped.
    const float* Qcol = Q + (long long)tab_row(kx, M) * qcs;
    const int* sl = qslot + geom * P;  // the stack's pair slots
    for (int idx = tid; idx < TK * P * 5; idx += 256) {
        const int kyl = idx % TK, c = (idx / TK) % 5, u = idx / (TK * 5);
        const int ky = ky0 + kyl;
        const int kq = ky <= LY / 2 ? ky : LY - ky;
        float v = 0.f;
        if (ky < LY) v = Qcol[(long long)(sl[u] * 5 + c) * QY + kq];
        // c in {2, 4}: even and non-zero
        const unsigned flip = (unsigned)(ky > LY / 2) & (unsigned)((c & 1) == 0) & (unsigned)(c != 0);
        st[(kyl * P + u) * 5 + c] = __uint_as_float(__float_as_uint(v) ^ (flip << 31));
    }
    __syncthreads();

    const float* lpg = lp + (long long)geom * 2 * NZ;
    bf16x8 ah[MFMA ? FW : 1][KT][KT2], am[MFMA ? FW : 1][KT][KT2], al[MFMA ? FW : 1][KT][KT2];
#pragma unroll
    for (int f = 0; f < FW; ++f) {
        const int kyl = w + 4 * f;
        float* A = MFMA ? sa + w * S6 * AS : sa + kyl * S6 * AS;
        build_real_matrix<NZ>(A, st + kyl * P * 5, lpg, l, adjoint);
        if constexpr (MFMA) {
            wave_sync();
            // A operand layout of the 16x16x32 product: lane l holds row l % 16,
            // sum indices 8 (l / 16) + e
#pragma unroll
            for (int mt = 0; mt < KT; ++mt)
#pragma unroll
                for (int kt = 0; kt < KT2; ++kt)
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int r = mt * 16 + (l & 15), k = kt * 32 + 8 * q4 + e;
                        const float v = (r < S6 && k < S6) ? A[r * AS + k] : 0.f;
                        __bf16 h, m, lo;
                        split3(v, h, m, lo);
                        ah[f][mt][kt][e] = h;
                        am[f][mt][kt][e] = m;
                        al[f][mt][kt][e] = lo;
                    }
            wave_sync();
        }
    }
    if constexpr (!MFMA) wave_sync();

    const int b_begin = geom * bpg, b_end = b_begin + bpg;
    for (int c0 = b_begin; c0 < b_end; c0 += NBS) {
        // stage the spectra of this chunk: TK consecutive ky per (state, signal)
        __syncthreads();
        for (int idx = tid; idx < TK * S * NBS; idx += 256) {
            const int kyl = idx % TK, s = (idx / TK) % S, bl = idx / (TK * S);
            const int b = c0 + bl, ky = ky0 + kyl;
            cpx<float> v = {0.f, 0.f};
            if (b < b_end && ky < LY) v = Mh[((long long)b * S + s) * sst + (long long)kx * LY + ky];
            sm[(kyl * S + s) * NBS + bl] = v;
        }
        __syncthreads();
#pragma unroll
        for (int f = 0; f < FW; ++f) {
            const int kyl = w + 4 * f;
            cpx<float>* mk = sm + kyl * S * NBS;   // spectra of this frequency, [S][NBS]
            f32x4 D[KT];
            if constexpr (MFMA) {
#pragma unroll
                for (int mt = 0; mt < KT; ++mt) D[mt] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kt = 0; kt < KT2; ++kt) {
                    // B operand: lane l holds sum indices 8 (l / 16) + e of state l % 16
                    bf16x8 bh, bm, bl;
#pragma unroll
                    for (int e = 0; e < 8; ++e) {
                        const int k = kt * 32 + 8 * q4 + e;
                        float v = 0.f;
                        if (k < S6) {
                            const int pk = k / S, s = k - pk * S;
                            const cpx<float> z = mk[s * NBS + n];
                            v = pk == 0 ? z.x : z.y;
                        }
                        __bf16 h, m, lo;
                        split3(v, h, m, lo);
                        bh[e] = h; bm[e] = m; bl[e] = lo;
                    }
#pragma unroll
                    for (int mt = 0; mt < KT; ++mt) {
                        f32x4 d = D[mt];
                        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[f][mt][kt], bh, d, 0, 0, 0);
                        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[f][mt][kt], bm, d, 0, 0, 0);
                        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[f][mt][kt], bl, d, 0, 0, 0);
                        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(am[f][mt][kt], bh, d, 0, 0, 0);
                        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[f][mt][kt], bm, d, 0, 0, 0);
                        d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[f][mt][kt], bh, d, 0, 0, 0);
                        D[mt] = d;
                    }
                }
            } else {
                // same product on the VALU: lane owns rows 4 q4 + e of each tile, state n
                const float* A = sa + kyl * S6 * AS;
                float acc[KT][4];
#pragma unroll
                for (int mt = 0; mt < KT; ++mt)
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc[mt][e] = 0.f;
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    const cpx<float> z = mk[s * NBS + n];
#pragma unroll
                    for (int mt = 0; mt < KT; ++mt)
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            const int r = mt * 16 + 4 * q4 + e;
                            if (r < S6) {
                                acc[mt][e] = fmaf(A[r * AS + s], z.x, acc[mt][e]);
                                acc[mt][e] = fmaf(A[r * AS + S + s], z.y, acc[mt][e]);
                            }
                        }
                }
#pragma unroll
                for (int mt = 0; mt < KT; ++mt) D[mt] = (f32x4){acc[mt][0], acc[mt][1], acc[mt][2], acc[mt][3]};
            }
            wave_sync();
            // D[mt][e] = output row r = 16 mt + 4 q4 + e (part, c, i), state n
#pragma unroll
            for (int mt = 0; mt < KT; ++mt)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int r = mt * 16 + 4 * q4 + e;
                    if (r < S6) {
                        const int pr = r / S, s = r - pr * S;
                        reinterpret_cast<float*>(&mk[s * NBS + n])[pr] = D[mt][e];
                    }
                }
        }
        __syncthreads();
        for (int idx = tid; idx < TK * S * NBS; idx += 256) {
            const int kyl = idx % TK, s = (idx / TK) % S, bl = idx / (TK * S);
            const int b = c0 + bl, ky = ky0 + kyl;
            if (b < b_end && ky < LY)
                Hh[((long long)b * S + s) * sst + (long long)kx * LY + ky] = sm[(kyl * S + s) * NBS + bl];
        }
    }
}

bool mix_batched_supported(int nz, int B, int G)
{
    (void)B;
    (void)G;
    return nz >= 1 && nz <= NZ_MFMA;
}

namespace {

template <bool MFMA, int NZ>
hipError_t launch_batched_nz(const void* Mh, void* Hh, int M, int LY, int G, const void* Q,
                             long long qcs, const int* qslot, int QY, const void* lp, int bpg,
                             int adjoint, hipStream_t s)
{
    using SH = BatchedShape<NZ>;
    const size_t lds = SH::lds(MFMA);
    hipError_t e = ensure_lds_limit((const void*)k_mix_batched<MFMA, NZ>, (int)lds);
    if (e != hipSuccess) return e;
    dim3 grid((LY + SH::TK - 1) / SH::TK, M - 1, G);
    hipLaunchKernelGGL((k_mix_batched<MFMA, NZ>), grid, dim3(256), lds, s, (const cpx<float>*)Mh,
                       (cpx<float>*)Hh, M, LY, (const float*)Q, qcs, qslot, QY, (const float*)lp,
                       bpg, adjoint);
    return hipGetLastError();
}

template <bool MFMA>
hipError_t launch_batched(int nz, const void* Mh, void* Hh, int M, int LY, int G, const void* Q,
                          long long qcs, const int* qslot, int QY, const void* lp, int bpg,
                          int adjoint, hipStream_t s)
{
#define HFD_BATCHED_CASE(N) \
    case N: return launch_batched_nz<MFMA, N>(Mh, Hh, M, LY, G, Q, qcs, qslot, QY, lp, bpg, adjoint, s)
    switch (nz) {
    HFD_BATCHED_CASE(1);
    HFD_BATCHED_CASE(2);
    HFD_BATCHED_CASE(3);
    HFD_BATCHED_CASE(4);
    HFD_BATCHED_CASE(5);
    HFD_BATCHED_CASE(6);
    HFD_BATCHED_CASE(7);
    HFD_BATCHED_CASE(8);
    default: return hipErrorInvalidValue;
    }
#undef HFD_BATCHED_CASE
}

}  // namespace

hipError_t launch_mix_batched(bool mfma, const void* Mh, void* Hh, int nz, int M, int LY, int B,
                              const void* Q, long long qcs, const int* qslot, int QY, const void* lp,
                              int bpg, int adjoint, hipStream_t s)
{
    if (M < 2) return hipSuccess;
    if (bpg < 1 || B % bpg) return hipErrorInvalidValue;
    const int G = B / bpg;
    return mfma ? launch_batched<true>(nz, Mh, Hh, M, LY, G, Q, qcs, qslot, QY, lp, bpg, adjoint, s)
                : launch_batched<false>(nz, Mh, Hh, M, LY, G, Q, qcs, qslot, QY, lp, bpg, adjoint, s);
}

}  // namespace hfd
