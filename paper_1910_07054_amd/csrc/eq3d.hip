// Equidistant layers: the convolution theorem along z as well (eq. FFT_3D of
// Sec. 3.1, the equidistant case the paper compares against in Sec. 3.2).
//
// With equal thickness t and a uniform pitch p (z_i = z_0 + i p) the tensor of
// layers i, j depends on the offset d = i - j only, so the layer sum
// h_i = -sum_j N(d = i - j) * m_j is a convolution along z.  After the x and y
// transforms it is done per lateral frequency by a length-Lz transform along
// the layer axis (zero padded, Lz >= 2 nz), a 3x3 product with the 3-D Fourier
// tensor, and the inverse transform: O(nz log nz) per frequency instead of the
// O(nz^2) explicit sum.
//
// 3-D Fourier tensor: the 2D spectra of N(d) for d in [-(nz-1), nz-1] are real
// (xx, yy, zz, xy) or imaginary (xz, yz) by lateral parity; xz and yz are odd
// in d, the others even, so their transforms along z are real as well:
//   T(kz) = sum_d Q(d) cos(2 pi kz d / Lz)   (xx, yy, zz, xy)
//   T(kz) = sum_d Q(d) sin(2 pi kz d / Lz)   (xz, yz; Q = imaginary part)
// stored on kx in [0, Lx/2], kz in [0, Lz/2], ky in [0, Ly/2]; xy is odd in ky,
// xz odd in kz, yz odd in ky and kz.
#include "field_kernels.hpp"
#include "launch.hpp"

namespace hfd {

// T3[kx][kz][c][ky] = (1/Lz) sum_d Q2[d][c][kx][ky] (cos | sin)(2 pi kz d / Lz)
// Q2: FP64 [2nz-1][6][QX][QY] (offset d at index d + nz - 1).
template <typename R>
__global__ __launch_bounds__(256) void k_zdft3(const double* __restrict__ Q2, R* __restrict__ T3,
                                               int nz, int LZ, int QX, int QY)
{
    const int LZH = LZ / 2 + 1;
    const long long n = (long long)QX * LZH * 6 * QY;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n) return;
    const int ky = (int)(idx % QY);
    const int c = (int)((idx / QY) % 6);
    const int kz = (int)((idx / ((long long)QY * 6)) % LZH);
    const int kx = (int)(idx / ((long long)QY * 6 * LZH));
    const bool odd = c == 4 || c == 5;
    const long long dstride = 6LL * QX * QY;
    const double* q = Q2 + ((long long)c * QX + kx) * QY + ky;
    double acc = 0.0;
    for (int d = -(nz - 1); d <= nz - 1; ++d) {
        double sn, cs;
        sincospi(2.0 * (double)kz * (double)d / (double)LZ, &sn, &cs);
        acc += q[(long long)(d + nz - 1) * dstride] * (odd ? sn : cs);
    }
    T3[idx] = (R)(acc / (double)LZ);
}

// The packed column 0 of every signal holds Z = A + iB with A, B the y-spectra
// of the real columns kx = 0 and kx = Lx/2.  Unpack: A into column 0, B into
// Bc[sig][ky]; one thread per ky pair (t, LY - t).
template <typename R>
__global__ __launch_bounds__(256) void k_unpack0(cpx<R>* __restrict__ Mh, cpx<R>* __restrict__ Bc,
                                                 int M, int LY, long long nsig)
{
    const int HP = LY / 2 + 1;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nsig * HP) return;
    const long long sig = idx / HP;
    const int t = (int)(idx % HP), tm = (LY - t) & (LY - 1);
    cpx<R>* col = Mh + sig * M * LY;
    cpx<R>* bc = Bc + sig * LY;
    const cpx<R> z1 = col[t], z2 = col[tm];
    const cpx<R> a = {R(0.5) * (z1.x + z2.x), R(0.5) * (z1.y - z2.y)};
    const cpx<R> b = {R(0.5) * (z1.y + z2.y), R(0.5) * (z2.x - z1.x)};
    col[t] = a;
    bc[t] = b;
    if (tm != t) {
        col[tm] = cconj(a);
        bc[tm] = cconj(b);
    }
}

// Repack after the z pass: column 0 = HA + i HB.
template <typename R>
__global__ __launch_bounds__(256) void k_repack0(cpx<R>* __restrict__ Hh, const cpx<R>* __restrict__ HBc,
                                                 int M, int LY, long long nsig)
{
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nsig * LY) return;
    const long long sig = idx / LY;
    const int ky = (int)(idx % LY);
    cpx<R>* col = Hh + sig * M * LY;
    const cpx<R> a = col[ky], b = HBc[sig * LY + ky];
    col[ky] = {a.x - b.y, a.y + b.x};
}

template <typename R, int LZ>
struct ZPassShape {
    static constexpr int V = fft_vals(LZ), GT = LZ / V;
    static constexpr int NT = 256, NG = NT / GT;
    // ky points per block: the tile holds 3 transforms of LZ values per point
    static constexpr int TP = (sizeof(cpx<R>) * 3 * 16 * fft_region(LZ) <= 49152) ? 16 : 8;
};

// z pass: block = TP consecutive ky of one kx column (kx = M is the split-off
// column Lx/2) of one state.  The 3 nz spectra of the tile are staged in LDS
// zero padded to LZ along the layer axis, transformed along z, multiplied by
// the real symmetric 3x3 tensor, transformed back, and the first nz layers
// written out.
template <typename R, int LZ>
__global__ __launch_bounds__(256) void k_zpass3(const cpx<R>* __restrict__ Mh, const cpx<R>* __restrict__ Bc,
                                                cpx<R>* __restrict__ Hh, cpx<R>* __restrict__ HBc, int nz,
                                                int M, int LY, const R* __restrict__ T3, int QY,
                                                const cpx<R>* __restrict__ twz)
{
    using SH = ZPassShape<R, LZ>;
    constexpr int TP = SH::TP, GT = SH::GT, NG = SH::NG, NT = SH::NT, LZH = LZ / 2 + 1;
    constexpr int LZP = fft_region(LZ);  // LDS slots per transform
    __shared__ cpx<R> sh[3 * TP * LZP];
    const int kx = blockIdx.y, b = blockIdx.z;
    const int ky0 = blockIdx.x * TP;
    const int S = 3 * nz;
    const int tid = threadIdx.x, grp = tid / GT, g = tid % GT;
    const bool split = kx == M;
    const long long sstride = split ? (long long)LY : (long long)M * LY;
    const cpx<R>* src = split ? Bc : Mh + (long long)kx * LY;
    cpx<R>* dst = split ? HBc : Hh + (long long)kx * LY;
    Twiddles<R, LZ> tw;
    tw.load(g, twz, 1);

    // stage: sh[(p * 3 + c) * LZP + l], zero for l >= nz
    for (int idx = tid; idx < TP * 3 * LZ; idx += NT) {
        const int p = idx % TP, r = idx / TP, c = r / LZ, l = r - c * LZ;
        const int ky = ky0 + p;
        cpx<R> v = {R(0), R(0)};
        if (l < nz && ky < LY) v = src[((long long)b * S + c * nz + l) * sstride + ky];
        sh[(p * 3 + c) * LZP + l] = v;
    }
    __syncthreads();
    for (int tr = grp; tr < 3 * TP; tr += NG) {
        cpx<R>* reg = sh + tr * LZP;
        wave_fft<R, LZ, false>(reg, g, tw, [&](int pos) -> cpx<R> { return reg[pos]; },
                               [&](int pos, cpx<R> v) { reg[pos] = v; });
    }
    __syncthreads();
    // 3x3 product per (point, kz)
    const R* Tk = T3 + (long long)kx * LZH * 6 * QY;
    for (int idx = tid; idx < TP * LZ; idx += NT) {
        const int p = idx % TP, kz = idx / TP;
        const int ky = ky0 + p;
        if (ky >= LY) continue;
        const int kyq = ky <= LY / 2 ? ky : LY - ky;
        const int kzq = kz <= LZ / 2 ? kz : LZ - kz;
        const R sy = ky <= LY / 2 ? R(1) : R(-1);
        const R sz = kz <= LZ / 2 ? R(1) : R(-1);
        const R* t = Tk + (long long)kzq * 6 * QY + kyq;
        const R xx = t[0], yy = t[QY], zz = t[2 * QY], xy = sy * t[3 * QY], xz = sz * t[4 * QY],
                yz = sy * sz * t[5 * QY];
        cpx<R>* v = sh + p * 3 * LZP + kz;
        const cpx<R> X = v[0], Y = v[LZP], Z = v[2 * LZP];
        v[0] = {xx * X.x + xy * Y.x + xz * Z.x, xx * X.y + xy * Y.y + xz * Z.y};
        v[LZP] = {xy * X.x + yy * Y.x + yz * Z.x, xy * X.y + yy * Y.y + yz * Z.y};
        v[2 * LZP] = {xz * X.x + yz * Y.x + zz * Z.x, xz * X.y + yz * Y.y + zz * Z.y};
    }
    __syncthreads();
    for (int tr = grp; tr < 3 * TP; tr += NG) {
        cpx<R>* reg = sh + tr * LZP;
        wave_fft<R, LZ, true>(reg, g, tw, [&](int pos) -> cpx<R> { return reg[pos]; },
                              [&](int pos, cpx<R> v) { reg[pos] = v; });
    }
    __syncthreads();
    for (int idx = tid; idx < TP * 3 * nz; idx += NT) {
        const int p = idx % TP, cl = idx / TP, c = cl / nz, l = cl - c * nz;
        const int ky = ky0 + p;
        if (ky < LY) dst[((long long)b * S + cl) * sstride + ky] = sh[(p * 3 + c) * LZP + l];
    }
}

namespace {

template <typename R>
hipError_t zpass_r(int LZ, const void* Mh, const void* Bc, void* Hh, void* HBc, int nz, int M,
                   int LY, int B, const void* T3, int QY, const void* twz, hipStream_t s)
{
#define HFD_ZPASS_CASE(L)                                                                          \
    case L: {                                                                                      \
        dim3 grid((LY + ZPassShape<R, L>::TP - 1) / ZPassShape<R, L>::TP, M + 1, B);               \
        hipLaunchKernelGGL((k_zpass3<R, L>), grid, dim3(256), 0, s, (const cpx<R>*)Mh,             \
                           (const cpx<R>*)Bc, (cpx<R>*)Hh, (cpx<R>*)HBc, nz, M, LY, (const R*)T3,  \
                           QY, (const cpx<R>*)twz);                                                \
        return hipGetLastError();                                                                  \
    }
    switch (LZ) {
        HFD_ZPASS_CASE(2)
        HFD_ZPASS_CASE(4)
        HFD_ZPASS_CASE(8)
        HFD_ZPASS_CASE(16)
        HFD_ZPASS_CASE(32)
        HFD_ZPASS_CASE(64)
        HFD_ZPASS_CASE(128)
    default: return hipErrorInvalidValue;
    }
#undef HFD_ZPASS_CASE
}

}  // namespace

hipError_t launch_zdft3(bool out_fp64, const double* Q2, void* T3, int nz, int LZ, int QX, int QY,
                        hipStream_t s)
{
    const long long n = (long long)QX * (LZ / 2 + 1) * 6 * QY;
    const long long nb = (n + 255) / 256;
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
    if (out_fp64)
        hipLaunchKernelGGL(k_zdft3<double>, dim3((unsigned)nb), dim3(256), 0, s, Q2, (double*)T3, nz,
                           LZ, QX, QY);
    else
        hipLaunchKernelGGL(k_zdft3<float>, dim3((unsigned)nb), dim3(256), 0, s, Q2, (float*)T3, nz,
                           LZ, QX, QY);
    return hipGetLastError();
}

hipError_t launch_eq3d_mix(bool fp64, int LZ, void* Mh, void* Bc, void* Hh, void* HBc, int nz, int M,
                           int LY, int B, const void* T3, int QY, const void* twz, hipStream_t s)
{
    if (!Mh || !Bc || !Hh || !HBc || !T3 || !twz) return hipErrorInvalidValue;
    const long long nsig = (long long)B * 3 * nz;
    const long long n1 = nsig * (LY / 2 + 1), n2 = nsig * LY;
    if ((n2 + 255) / 256 > 0x7fffffffLL) return hipErrorInvalidValue;
    hipError_t e;
    if (fp64) {
        hipLaunchKernelGGL(k_unpack0<double>, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s,
                           (cpx<double>*)Mh, (cpx<double>*)Bc, M, LY, nsig);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = zpass_r<double>(LZ, Mh, Bc, Hh, HBc, nz, M, LY, B, T3, QY, twz, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_repack0<double>, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s,
                           (cpx<double>*)Hh, (const cpx<double>*)HBc, M, LY, nsig);
    } else {
        hipLaunchKernelGGL(k_unpack0<float>, dim3((unsigned)((n1 + 255) / 256)), dim3(256), 0, s,
                           (cpx<float>*)Mh, (cpx<float>*)Bc, M, LY, nsig);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = zpass_r<float>(LZ, Mh, Bc, Hh, HBc, nz, M, LY, B, T3, QY, twz, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_repack0<float>, dim3((unsigned)((n2 + 255) / 256)), dim3(256), 0, s,
                           (cpx<float>*)Hh, (const cpx<float>*)HBc, M, LY, nsig);
    }
    return hipGetLastError();
}

}  // namespace hfd
