// Field-path kernels: h = -N * m by the hybrid scheme of Sec. 3.1 --
// 2D DFT along x and y (zero padded to Lx x Ly), an explicit sum over layers
// per lateral frequency, inverse 2D DFT, crop.
//
// Data layout (per state b, signal s = c * nz + l for component c, layer l):
//   m, h   [B][S][ny][nx]           real, x fastest
//   X1     [B][S][M][ny]            complex, M = Lx/2 columns of the x
//                                   half-spectrum, y fastest; column 0 packs
//                                   the two real columns kx = 0 and kx = Lx/2
//                                   as X(0) + i X(Lx/2)
//   Mh, Hh [B][S][M][Ly]            full y spectra (five-pass path only)
//   Q      [G][Lx/2+1][P][5][Ly/2+1] Fourier tensor on the quadrant kx in
//                                   [0, Lx/2], ky in [0, Ly/2] (contiguous per
//                                   kx column), unique pairs i <= j, components
//                                   xx, yy, xy, xz, yz of
//                                   t_i * (-DFT2(N^{ij}) / (Lx Ly)); real part
//                                   for xx, yy, xy, imaginary part for xz, yz
//   lp     [G][2][nz]               1 / t_l and -t_l / (Lx Ly) (trace of the
//                                   self-pair block, which fixes zz)
#pragma once
#include "hfd_device.hpp"

namespace hfd {

// Rows are numbered flat over all signals (row r = signal r / ny, y = r % ny)
// and a block takes TY consecutive rows, one wave or part of a wave per row.
// TYO = 0 picks the default: 16 rows (or one per group of a 256-thread block),
// halved until the tile fits in 80 KB of LDS.
template <typename R, int LX, int TYO = 0>
struct XPassShape {
    static constexpr int M = LX / 2;
    static constexpr int V = fft_vals(M);
    static constexpr int GT = M / V;
    static constexpr int RS = fft_region(M) | 1;   // LDS row stride: a transform's region, odd
    static constexpr int pick_ty()
    {
        if (TYO > 0) return TYO;
        const int ng = (GT * 16 < 256 ? 256 : (GT * 16 > 1024 ? 1024 : GT * 16)) / GT;
        int ty = ng > 16 ? ng : 16;
        while (ty > 1 && sizeof(cpx<R>) * (size_t)ty * RS > 81920) ty /= 2;
        return ty;
    }
    static constexpr int TY = pick_ty();
    // threads: one group per row, at least one wave, at most 1024
    static constexpr int NT0 = GT * TY;
    static constexpr int NT = NT0 < 64 ? 64 : (NT0 > 1024 ? 1024 : NT0);
    static constexpr int NG = NT / GT;
    static constexpr size_t LDS = sizeof(cpx<R>) * TY * RS;
    // waves per SIMD for two resident blocks (the register budget that allows it)
    static constexpr int WPE = NT / 128 > 8 ? 8 : (NT / 128 < 1 ? 1 : NT / 128);
};

// ---------------------------------------------------------------------------
// x pass, forward: each row of nx reals (zero padded to LX) -> packed half
// spectrum of LX/2 complex values, written transposed (y fastest).
// A length-LX real transform is one complex transform of length LX/2 on
// z[n] = x[2n] + i x[2n+1] followed by the even/odd split.
// ---------------------------------------------------------------------------
// Split of the packed real transform, per row: lane g of the row's group owns
// the frequency pairs (k, M - k) for k = g + GT i, i < KI; their twiddles
// exp(-2 pi i k / LX) are loaded once per lane (for the longest rows, whose
// transform needs the registers, they are read where used).
template <typename R, int LX>
struct RealSplit {
    static constexpr int M = LX / 2, GT = XPassShape<R, LX>::GT, HM = M / 2 + 1;
    static constexpr int KI = (HM + GT - 1) / GT;
    static constexpr bool CACHE = KI * sizeof(R) <= 32;
    cpx<R> w[CACHE ? KI : 1];
    const cpx<R>* tw;
    __device__ __forceinline__ void load(int g, const cpx<R>* __restrict__ twx)
    {
        tw = twx;
        if constexpr (CACHE) {
#pragma unroll
            for (int i = 0; i < KI; ++i) {
                const int k = g + GT * i;
                w[i] = k < HM ? twx[k] : cpx<R>{R(0), R(0)};
            }
        }
    }
    __device__ __forceinline__ cpx<R> wk(int i, int k) const
    {
        if constexpr (CACHE) return w[i];
        else return tw[k];
    }
    // forward: complex spectrum Z of z[n] = x[2n] + i x[2n+1] -> X[k], k < M,
    // with X[0] and X[M] packed as X[0] + i X[M]
    __device__ __forceinline__ void forward(cpx<R>* row, int g) const
    {
#pragma unroll
        for (int i = 0; i < KI; ++i) {
            const int k = g + GT * i;
            if (k >= HM) continue;
            if (k == 0) {
                const cpx<R> z = row[0];
                row[0] = {z.x + z.y, z.x - z.y};
            } else if (2 * k == M) {
                row[k] = cconj(row[k]);
            } else {
                const cpx<R> a = row[k], b = row[M - k];
                const cpx<R> E = {R(0.5) * (a.x + b.x), R(0.5) * (a.y - b.y)};
                const cpx<R> O = {R(0.5) * (a.y + b.y), R(0.5) * (b.x - a.x)};
                const cpx<R> wO = cmul(wk(i, k), O);
                row[k] = cadd(E, wO);
                row[M - k] = cconj(csub(E, wO));
            }
        }
    }
    // inverse: packed half spectrum -> spectrum of z (unnormalized, twice the
    // forward's input)
    __device__ __forceinline__ void inverse(cpx<R>* row, int g) const
    {
#pragma unroll
        for (int i = 0; i < KI; ++i) {
            const int k = g + GT * i;
            if (k >= HM) continue;
            if (k == 0) {
                const cpx<R> z = row[0];
                row[0] = {z.x + z.y, z.x - z.y};
            } else if (2 * k == M) {
                const cpx<R> z = row[k];
                row[k] = {R(2) * z.x, R(-2) * z.y};
            } else {
                const cpx<R> a = row[k], b = row[M - k];
                const cpx<R> P = {a.x + b.x, a.y - b.y};   // a + conj(b)
                const cpx<R> Qd = {a.x - b.x, a.y + b.y};  // a - conj(b)
                const cpx<R> T = cmul(cconj(wk(i, k)), Qd);
                row[k] = {P.x - T.y, P.y + T.x};
                row[M - k] = {P.x + T.y, T.x - P.y};
            }
        }
    }
};

// ---------------------------------------------------------------------------
// x pass, forward: each row of nx reals (zero padded to LX) -> packed half
// spectrum of LX/2 complex values, written transposed (y fastest).
// A length-LX real transform is one complex transform of length LX/2 on
// z[n] = x[2n] + i x[2n+1] followed by the even/odd split, which the row's
// group applies to its own row.  HALF: nx <= LX/2, so z[n] is zero for
// n >= LX/4 and the first radix pass skips that half (the field path; the
// tensor transforms run on full rows).
// ---------------------------------------------------------------------------
template <typename R, int LX, int TYO = 0, bool HALF = true>
__global__ __launch_bounds__((XPassShape<R, LX, TYO>::NT), (XPassShape<R, LX, TYO>::WPE)) void k_xfwd(
    const R* __restrict__ in, cpx<R>* __restrict__ out, int nx, int ny, int nrows,
    long long in_sig_stride, int in_row_stride, const cpx<R>* __restrict__ twx)
{
    using S = XPassShape<R, LX, TYO>;
    constexpr int M = S::M, GT = S::GT, NG = S::NG, TY = S::TY, RS = S::RS, NT = S::NT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<R>* sh = reinterpret_cast<cpx<R>*>(smem_raw);
    const int r0 = blockIdx.x * TY;
    const int tid = threadIdx.x, grp = tid / GT, g = tid % GT;
    Twiddles<R, M> tw;
    tw.load(g, twx, 2);
    RealSplit<R, LX> split;
    split.load(g, twx);

    for (int r = grp; r < TY; r += NG) {
        const int fr = r0 + r;
        if (fr >= nrows) break;
        const int sig = fr / ny, y = fr - sig * ny;
        cpx<R>* row = sh + r * RS;
        const R* src = in + (long long)sig * in_sig_stride + (long long)y * in_row_stride;
        if ((nx & 1) == 0 && (in_row_stride & 1) == 0 && (in_sig_stride & 1) == 0) {
            // even rows: (x[2n], x[2n+1]) is one aligned 2-element load
            const cpx<R>* src2 = reinterpret_cast<const cpx<R>*>(src);
            const int nh = nx >> 1;
            wave_fft<R, M, false, HALF>(
                row, g, tw,
                [&](int pos) -> cpx<R> { return pos < nh ? src2[pos] : cpx<R>{R(0), R(0)}; },
                [&](int pos, cpx<R> v) { row[pos] = v; });
        } else {
            wave_fft<R, M, false, HALF>(
                row, g, tw,
                [&](int pos) -> cpx<R> {
                    const int n0 = 2 * pos;
                    return {n0 < nx ? src[n0] : R(0), n0 + 1 < nx ? src[n0 + 1] : R(0)};
                },
                [&](int pos, cpx<R> v) { row[pos] = v; });
        }
        wave_sync();
        split.forward(row, g);
    }
    __syncthreads();
    // transposed store: consecutive threads take consecutive rows of one kx
    for (int idx = tid; idx < M * TY; idx += NT) {
        const int r = idx % TY, kx = idx / TY;
        const int fr = r0 + r;
        if (fr < nrows) {
            const int sig = fr / ny, y = fr - sig * ny;
            out[((long long)sig * M + kx) * ny + y] = sh[r * RS + kx];
        }
    }
}

// ---------------------------------------------------------------------------
// x pass of the tensor tables from their quadrants: row y < ny of array sig
// holds W(p, y), p < nx, of component sig % 6 (order xx yy zz xy xz yz); the
// full periodic row of length LX is W(p) at p and sx W(p) at LX - p (sx = -1
// for the x-odd components xy and xz), zero between.  Its transform is real
// for an x-even row and imaginary for an x-odd one; that part is stored
// transposed, out[sig][kx][y] for kx in [0, LX/2] (columns of ny reals; the
// rows kx = 0 and LX/2 of x-odd components are exactly zero).
// ---------------------------------------------------------------------------
template <int LX, int TYO = 0>
__global__ __launch_bounds__((XPassShape<double, LX, TYO>::NT), (XPassShape<double, LX, TYO>::WPE)) void k_xtab(
    const double* __restrict__ in, double* __restrict__ out, int nx, int ny, int nrows,
    const cpx<double>* __restrict__ twx)
{
    using R = double;
    using S = XPassShape<R, LX, TYO>;
    constexpr int M = S::M, GT = S::GT, NG = S::NG, TY = S::TY, RS = S::RS, NT = S::NT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<R>* sh = reinterpret_cast<cpx<R>*>(smem_raw);
    const int r0 = blockIdx.x * TY;
    const int tid = threadIdx.x, grp = tid / GT, g = tid % GT;
    Twiddles<R, M> tw;
    tw.load(g, twx, 2);
    RealSplit<R, LX> split;
    split.load(g, twx);
    for (int r = grp; r < TY; r += NG) {
        const int fr = r0 + r;
        if (fr >= nrows) break;
        const int sig = fr / ny, y = fr - sig * ny;
        const int c6 = sig % 6;
        const R sx = (c6 == 3 || c6 == 4) ? R(-1) : R(1);
        const R* src = in + ((long long)sig * ny + y) * nx;
        auto xv = [&](int x) -> R {
            if (x < nx) return src[x];
            const int m = LX - x;
            return m < nx ? sx * src[m] : R(0);
        };
        cpx<R>* row = sh + r * RS;
        wave_fft<R, M, false>(
            row, g, tw, [&](int pos) -> cpx<R> { return {xv(2 * pos), xv(2 * pos + 1)}; },
            [&](int pos, cpx<R> v) { row[pos] = v; });
        wave_sync();
        split.forward(row, g);
    }
    __syncthreads();
    for (int idx = tid; idx < (M + 1) * TY; idx += NT) {
        const int r = idx % TY, kx = idx / TY;
        const int fr = r0 + r;
        if (fr < nrows) {
            const int sig = fr / ny, y = fr - sig * ny;
            const int c6 = sig % 6;
            const bool xodd = (c6 == 3 || c6 == 4);
            // column 0 holds X[0] + i X[M] (both real for an x-even row)
            const cpx<R> z = sh[r * RS + (kx == M ? 0 : kx)];
            const R v = xodd ? (kx == 0 || kx == M ? R(0) : z.y) : (kx == M ? z.y : z.x);
            out[((long long)sig * (M + 1) + kx) * ny + y] = v;
        }
    }
}

// ---------------------------------------------------------------------------
// x pass, inverse: packed half spectrum (transposed) -> nx reals per row.
// Unnormalized; the 1/(Lx Ly) is folded into the tensor.  HALF: nx <= LX/2,
// only the first half of the transform is kept.
// ---------------------------------------------------------------------------
template <typename R, int LX, int TYO = 0, bool HALF = true>
__global__ __launch_bounds__((XPassShape<R, LX, TYO>::NT), (XPassShape<R, LX, TYO>::WPE)) void k_xinv(
    const cpx<R>* __restrict__ in, R* __restrict__ out, int nx, int ny, int nrows,
    long long out_sig_stride, int out_row_stride, const cpx<R>* __restrict__ twx)
{
    using S = XPassShape<R, LX, TYO>;
    constexpr int M = S::M, GT = S::GT, NG = S::NG, TY = S::TY, RS = S::RS, NT = S::NT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<R>* sh = reinterpret_cast<cpx<R>*>(smem_raw);
    const int r0 = blockIdx.x * TY;
    const int tid = threadIdx.x, grp = tid / GT, g = tid % GT;
    Twiddles<R, M> tw;
    tw.load(g, twx, 2);
    RealSplit<R, LX> split;
    split.load(g, twx);
    for (int idx = tid; idx < M * TY; idx += NT) {
        const int r = idx % TY, kx = idx / TY;
        const int fr = r0 + r;
        cpx<R> v = {R(0), R(0)};
        if (fr < nrows) {
            const int sig = fr / ny, y = fr - sig * ny;
            v = in[((long long)sig * M + kx) * ny + y];
        }
        sh[r * RS + kx] = v;
    }
    __syncthreads();
    for (int r = grp; r < TY; r += NG) {
        const int fr = r0 + r;
        if (fr >= nrows) break;
        const int sig = fr / ny, y = fr - sig * ny;
        cpx<R>* row = sh + r * RS;
        split.inverse(row, g);
        wave_sync();
        R* dst = out + (long long)sig * out_sig_stride + (long long)y * out_row_stride;
        if ((nx & 1) == 0 && (out_row_stride & 1) == 0 && (out_sig_stride & 1) == 0) {
            cpx<R>* dst2 = reinterpret_cast<cpx<R>*>(dst);
            const int nh = nx >> 1;
            wave_fft<R, M, true, false, HALF>(
                row, g, tw, [&](int pos) -> cpx<R> { return row[pos]; },
                [&](int pos, cpx<R> v) {
                    if (pos < nh) dst2[pos] = v;
                });
        } else {
            wave_fft<R, M, true, false, HALF>(
                row, g, tw, [&](int pos) -> cpx<R> { return row[pos]; },
                [&](int pos, cpx<R> v) {
                    const int n0 = 2 * pos;
                    if (n0 < nx) dst[n0] = v.x;
                    if (n0 + 1 < nx) dst[n0 + 1] = v.y;
                });
        }
    }
}

// ---------------------------------------------------------------------------
// z-mixing of one frequency pair.  For the unique layer pairs i <= j the
// stored block S^{ij} = t_i T^{ij} (T = -DFT2(N)/(Lx Ly)) is applied both
// ways: H_i += S^{ij} M_j and H_j += conj(S^{ij}) M_i (reciprocity
// t_j T^{ji} = conj(t_i T^{ij})).  Real components: xx, yy, zz, xy; imaginary
// components: xz, yz.  zz follows from the trace: sum of the diagonal of
// S^{ij} is dg_i on the self pair and 0 otherwise (the trace of N is the
// overlap volume over the target volume).  Point b carries the sign sb of the
// components that are odd in ky (xy, yz).
// Arrays are indexed [c * NZMAX + layer].
// ---------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void block_apply(cpx<R>& hx, cpx<R>& hy, cpx<R>& hz, cpx<R> X, cpx<R> Y,
                                            cpx<R> Z, R xx, R yy, R zz, R xy, R xz, R yz)
{
    // real parts (xx, yy, zz, xy) multiply, imaginary parts (i xz, i yz) rotate
    hx.x = fma(xx, X.x, hx.x); hx.x = fma(xy, Y.x, hx.x); hx.x = fma(-xz, Z.y, hx.x);
    hx.y = fma(xx, X.y, hx.y); hx.y = fma(xy, Y.y, hx.y); hx.y = fma(xz, Z.x, hx.y);
    hy.x = fma(xy, X.x, hy.x); hy.x = fma(yy, Y.x, hy.x); hy.x = fma(-yz, Z.y, hy.x);
    hy.y = fma(xy, X.y, hy.y); hy.y = fma(yy, Y.y, hy.y); hy.y = fma(yz, Z.x, hy.y);
    hz.x = fma(-xz, X.y, hz.x); hz.x = fma(-yz, Y.y, hz.x); hz.x = fma(zz, Z.x, hz.x);
    hz.y = fma(xz, X.x, hz.y); hz.y = fma(yz, Y.x, hz.y); hz.y = fma(zz, Z.y, hz.y);
}

// On the kx = 0 and kx = Lx/2 rows of the tensor xy and xz vanish (both are
// odd in x, lateral parity); EDGE = 1 drops them.
template <int EDGE, typename R>
__device__ __forceinline__ void block_apply_e(cpx<R>& hx, cpx<R>& hy, cpx<R>& hz, cpx<R> X, cpx<R> Y,
                                              cpx<R> Z, R xx, R yy, R zz, R xy, R xz, R yz)
{
    if constexpr (EDGE == 0) {
        block_apply(hx, hy, hz, X, Y, Z, xx, yy, zz, xy, xz, yz);
    } else {
        hx.x = fma(xx, X.x, hx.x); hx.y = fma(xx, X.y, hx.y);
        hy.x = fma(yy, Y.x, hy.x); hy.x = fma(-yz, Z.y, hy.x);
        hy.y = fma(yy, Y.y, hy.y); hy.y = fma(yz, Z.x, hy.y);
        hz.x = fma(-yz, Y.y, hz.x); hz.x = fma(zz, Z.x, hz.x);
        hz.y = fma(yz, Y.x, hz.y); hz.y = fma(zz, Z.y, hz.y);
    }
}

// Tensor values of one target row i (pairs (i, j), j >= i), 5 components each;
// sl maps the stack's pair u to its slot of the tensor table.
template <typename R, int NZMAX>
struct TensorRow {
    R v[NZMAX][5];
    // row i starts at pair index u = i nz - i (i - 1) / 2
    template <int EDGE = 0>
    __device__ __forceinline__ void load(const UniformBuf<R>& qcol, unsigned kq, int QY, int nz, int i,
                                         const int* __restrict__ sl)
    {
        const int u = i * nz - i * (i - 1) / 2;
#pragma unroll
        for (int j = 0; j < NZMAX; ++j)
            if (j >= i && j < nz) {
                const int slot = sl[u + j - i];
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    const bool need = EDGE == 0 || c < 2 || c == 4;
                    v[j][c] = need ? qcol.ld(kq, (unsigned)((slot * 5 + c) * QY)) : R(0);
                }
            }
    }
};

// One frequency point: H_i += S^{ij} M_j and, for i < j, H_j += conj(S^{ij}) M_i.
// qcol views the tensor table from a wave-uniform base (one kx row); kq is the
// lane's element offset (the quadrant ky, plus the row for the packed column);
// pair u, component c sits at (sl[u] * 5 + c) * QY + kq.
// sg is the sign of the ky-odd components (xy, yz).
// Row i + 1 of the tensor is loaded while row i is applied; `first` holds
// row 0, loaded by the caller ahead of time.
template <typename R, int NZMAX, int EDGE = 0, class In>
__device__ __forceinline__ void mix1(int nz, In in, cpx<R>* H, const UniformBuf<R>& qcol,
                                     unsigned kq, int QY, const int* __restrict__ sl, R sg,
                                     const R* dg, const TensorRow<R, NZMAX>& first)
{
#pragma unroll
    for (int k = 0; k < 3 * NZMAX; ++k) H[k] = {R(0), R(0)};
    // double buffering needs two rows of registers; above 8 layers the rows
    // are loaded one at a time
    constexpr bool DB = NZMAX <= 8;
    TensorRow<R, NZMAX> cur = first, nxt;
#pragma unroll
    for (int i = 0; i < NZMAX; ++i) {
        if (i < nz) {
            if constexpr (DB) {
                if (i + 1 < NZMAX && i + 1 < nz) nxt.template load<EDGE>(qcol, kq, QY, nz, i + 1, sl);
            } else if (i > 0) {
                cur.template load<EDGE>(qcol, kq, QY, nz, i, sl);
            }
            const cpx<R> ix = in(0, i), iy = in(1, i), iz = in(2, i);
#pragma unroll
            for (int j = i; j < NZMAX; ++j) {
                if (j < nz) {
                    const R xx = cur.v[j][0], yy = cur.v[j][1], xy = sg * cur.v[j][2],
                            xz = cur.v[j][3], yz = sg * cur.v[j][4];
                    R zz = -(xx + yy);
                    if (i == j) zz += dg[i];
                    if (i == j) {
                        block_apply_e<EDGE>(H[i], H[NZMAX + i], H[2 * NZMAX + i], ix, iy, iz, xx, yy,
                                            zz, xy, xz, yz);
                    } else {
                        const cpx<R> jx = in(0, j), jy = in(1, j), jz = in(2, j);
                        block_apply_e<EDGE>(H[i], H[NZMAX + i], H[2 * NZMAX + i], jx, jy, jz, xx, yy,
                                            zz, xy, xz, yz);
                        block_apply_e<EDGE>(H[j], H[NZMAX + j], H[2 * NZMAX + j], ix, iy, iz, xx, yy,
                                            zz, xy, -xz, -yz);
                    }
                }
            }
            if constexpr (DB) {
                if (i + 1 < NZMAX) cur = nxt;
            }
        }
    }
}

template <typename R, int NZMAX, int EDGE = 0, class In>
__device__ __forceinline__ void mix1(int nz, In in, cpx<R>* H, const UniformBuf<R>& qcol,
                                     unsigned kq, int QY, const int* __restrict__ sl, R sg,
                                     const R* dg)
{
    TensorRow<R, NZMAX> first;
    first.template load<EDGE>(qcol, kq, QY, nz, 0, sl);
    mix1<R, NZMAX, EDGE>(nz, in, H, qcol, kq, QY, sl, sg, dg, first);
}

// The two points of the packed column that are their own mirror (ky = 0 and
// LY/2) need four real mixings: A = Re Z with the kx = 0 row and B = Im Z with
// the kx = M row, at both points.  With LY lanes for LY + 2 mixings they are
// spread over the lanes of one wave: lane e takes one (point, part, target
// layer i) and sums over the source layers.  All blocks there are diagonal
// and real (xy, xz and yz vanish on those rows and columns).  Q is the tensor
// table, whose rows kx = 0 and kx = M come first (Q and Q + qcs), sl the
// stack's slot map; lpg holds 1/t and the trace terms.  The
// points are read by prep() and written by finish(), and no other lane touches
// them.  prep() requests the operands (called before the lane's own mixing, so that
// their latency overlaps it); finish() sums and writes the results.
template <typename R, int LY, int NZMAX, bool ADJ>
struct MirrorPoints {
    R xx[NZMAX], yy[NZMAX], v[3][NZMAX];
    int i, part, kp;
    bool act;

    __device__ __forceinline__ void prep(const cpx<R>* sh, int nz, int e, const R* __restrict__ Q,
                                         long long qcs, const int* __restrict__ sl, int QY,
                                         const R* lpg)
    {
        i = e % NZMAX;
        part = (e / NZMAX) & 1;
        const int pt = e / (2 * NZMAX);
        act = pt < 2 && i < nz;
        const int ii = i < nz ? i : nz - 1;
        kp = pt == 1 ? LY / 2 : 0;
        const UniformBuf<R> qb0(Q, (unsigned)(2 * qcs * sizeof(R)));
        const unsigned off = (unsigned)(kp + (part ? qcs : 0LL));
#pragma unroll
        for (int j = 0; j < NZMAX; ++j) {
            const int jj = j < nz ? j : ii;
            const int a = ii < jj ? ii : jj, b = ii < jj ? jj : ii;
            // the row and the slot differ between lanes, so they go into the
            // lane offset (the second offset of a buffer load must be wave-uniform)
            const unsigned o = off + (unsigned)(sl[a * nz - a * (a - 1) / 2 + (b - a)] * 5 * QY);
            xx[j] = qb0.ld(o, 0u);
            yy[j] = qb0.ld(o + QY, 0u);
        }
#pragma unroll
        for (int j = 0; j < NZMAX; ++j) {
            const int jj = j < nz ? j : 0;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const cpx<R> z = sh[(c * nz + jj) * fft_region(LY) + kp];
                R x = part ? z.y : z.x;
                if constexpr (ADJ) x *= lpg[jj];
                v[c][j] = (act && j < nz) ? x : R(0);
            }
        }
    }

    __device__ __forceinline__ void finish(cpx<R>* sh, int nz, const R* lpg)
    {
        wave_sync();  // the whole wave has read its operands
        const int ii = i < nz ? i : nz - 1;
        const R dgi = lpg[nz + ii];
        R acc[3] = {R(0), R(0), R(0)};
#pragma unroll
        for (int j = 0; j < NZMAX; ++j) {
            const R zz = (j == ii ? dgi : R(0)) - (xx[j] + yy[j]);
            acc[0] = fma(xx[j], v[0][j], acc[0]);
            acc[1] = fma(yy[j], v[1][j], acc[1]);
            acc[2] = fma(zz, v[2][j], acc[2]);
        }
        if (act) {
            const R sc = ADJ ? R(1) : lpg[i];
#pragma unroll
            for (int c = 0; c < 3; ++c)
                reinterpret_cast<R*>(&sh[(c * nz + i) * fft_region(LY) + kp])[part] = acc[c] * sc;
        }
    }
};

template <int LY>
struct FusedShape {
    // one thread per frequency from 512-point columns on; shorter columns
    // get 512 threads too, so that more of their transforms run at once
    static constexpr int NT = LY < 512 ? 512 : LY;
};

// ---------------------------------------------------------------------------
// Fused y pass for one kx column of one state: forward y-DFT of the 3 nz
// signals (input zero padded from ny to LY), z-mixing per ky, inverse y-DFT
// cropped to ny.  All 3 nz spectra stay in LDS.  Lanes 2t and 2t+1 mix the ky
// pair (t, LY - t) (t = 0: ky = 0 and LY/2), which share one quadrant tensor
// entry, so the two lanes read the same addresses.
// Column 0 carries kx = 0 and kx = Lx/2 packed as A + iB; they are separated
// with the Hermitian symmetry in ky, mixed with their own tensor rows and
// packed again.  adjoint != 0 applies the transpose (inputs scaled by 1/t
// instead of the outputs).
// ---------------------------------------------------------------------------
// Body of the fused y pass for column kx of state b (stack geom); the
// kernels below launch it on a grid (M, states per stack, stacks).
template <typename R, int LY, int NZMAX, bool ADJ>
__device__ __forceinline__ void ymix_column(int kx, int b, int geom, cpx<R>* __restrict__ X,
                                            int ny, int nz, int M, const R* __restrict__ Q,
                                            long long qcs, const int* __restrict__ qslot, int QY,
                                            const R* __restrict__ lp,
                                            const cpx<R>* __restrict__ twy)
{
    constexpr int NT = FusedShape<LY>::NT;
    constexpr int V = fft_vals(LY), GT = LY / V, NG = NT / GT;
    constexpr int LYP = fft_region(LY);  // LDS slots per signal
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<R>* sh = reinterpret_cast<cpx<R>*>(smem_raw);
    const int S = 3 * nz;
    const long long sstride = (long long)M * ny;
    cpx<R>* col = X + ((long long)b * S * M + kx) * ny;
    const int tid = threadIdx.x, grp = tid / GT, g = tid % GT;
    Twiddles<R, LY> tw;
    tw.load(g, twy, 1);

    // lane -> frequency point of the mixing phase (see below); the first tensor
    // row of an ordinary column is requested now so that its latency overlaps
    // the forward transforms
    const int t = tid >> 1, p = tid & 1;
    const int ky = p == 0 ? t : (t == 0 ? LY / 2 : LY - t);   // this lane's point
    const int kq = p == 0 ? t : (t == 0 ? LY / 2 : t);        // its quadrant column
    const int P = nz * (nz + 1) / 2;
    const int* sl = qslot + (long long)geom * P;              // the stack's pair slots
    const UniformBuf<R> qb(Q + tab_row(kx, M) * qcs, (unsigned)(qcs * sizeof(R)));
    // packed column: rows kx = 0 and kx = M (adjacent in the table) from one
    // uniform base, the row in the lane offset
    const UniformBuf<R> qb0(Q, (unsigned)(2 * qcs * sizeof(R)));
    const unsigned off0 = (unsigned)(t + (p == 0 ? 0LL : qcs));
    // (above 8 layers, or with 1024 threads per block, the registers do not
    // hold a prefetched row)
    constexpr bool EARLY_ROW = NZMAX <= 8 && NT <= 512;
    TensorRow<R, NZMAX> row0;
    if constexpr (EARLY_ROW) {
        if (kx != 0) {
            if (t < LY / 2) row0.load(qb, (unsigned)kq, QY, nz, 0, sl);
        } else if (t != 0 && t < LY / 2) {
            row0.template load<1>(qb0, off0, QY, nz, 0, sl);
        }
    }

    // forward transforms: the inputs of all of this group's signals are
    // requested first, then transformed one after the other
    constexpr int NR = (3 * NZMAX + NG - 1) / NG;   // signals per group, at most
    cpx<R> xin[NR][V];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int s = grp + r * NG;
        if (s < S) {
            const cpx<R>* src = col + s * sstride;
            fft_first_loads<R, LY, true>(xin[r], g, [&](int pos) -> cpx<R> {
                return pos < ny ? src[pos] : cpx<R>{R(0), R(0)};
            });
        }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        const int s = grp + r * NG;
        if (s < S) {
            cpx<R>* reg = sh + s * LYP;
            wave_fft_pre<R, LY, false, true>(reg, g, tw, xin[r], [&](int pos, cpx<R> v) { reg[pos] = v; });
        }
    }
    __syncthreads();

    // ky = 0 and LY/2 of the packed column are mixed by the first wave; its
    // operands are requested before the wave's own mixing where the register
    // budget allows (up to 512 threads per block)
    constexpr bool mirror_early = NT <= 512;
    MirrorPoints<R, LY, NZMAX, ADJ> mirror;
    const bool mirror_wave = kx == 0 && tid < 64;
    if (mirror_early && mirror_wave)
        mirror.prep(sh, nz, tid, Q, qcs, sl, QY, lp + (long long)geom * 2 * nz);

    if (t < LY / 2) {
        const R* lpg = lp + (long long)geom * 2 * nz;
        R invt[NZMAX], dg[NZMAX];
#pragma unroll
        for (int i = 0; i < NZMAX; ++i) {
            invt[i] = i < nz ? lpg[i] : R(0);
            dg[i] = i < nz ? lpg[nz + i] : R(0);
        }
        // sources scaled by 1/t for the transpose (T A T^-1), targets otherwise
        auto isc = [&](int l) -> R { return invt[l]; };
        cpx<R> H[3 * NZMAX];
        auto store = [&](int ky) {
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int l = 0; l < NZMAX; ++l)
                    if (l < nz) {
                        cpx<R> v = H[c * NZMAX + l];
                        if constexpr (!ADJ) v = cscale(v, invt[l]);
                        sh[(c * nz + l) * LYP + ky] = v;
                    }
        };
        auto ld = [&](int c, int l, int k) -> cpx<R> {
            cpx<R> v = sh[(c * nz + l) * LYP + k];
            if constexpr (ADJ) v = cscale(v, isc(l));
            return v;
        };
        const R sg = (p == 1 && t != 0) ? R(-1) : R(1);
        if (kx != 0) {
            auto in = [&](int c, int l) -> cpx<R> { return ld(c, l, ky); };
            if constexpr (EARLY_ROW) mix1<R, NZMAX>(nz, in, H, qb, (unsigned)kq, QY, sl, sg, dg, row0);
            else mix1<R, NZMAX>(nz, in, H, qb, (unsigned)kq, QY, sl, sg, dg);
            store(ky);
        } else if (t != 0) {
            // column 0 holds Z = A + iB with A the kx = 0 and B the kx = Lx/2
            // column: A(ky) = (Z(ky) + conj Z(-ky))/2, B(ky) = (Z(ky) - conj Z(-ky))/(2i).
            // Lane p = 0 mixes A(t) with row 0, lane p = 1 mixes B(t) with row M;
            // W(t) = HA + i HB, W(-t) = conj(HA) + i conj(HB).
            const int k1 = t, k2 = LY - t;
            auto in = [&](int c, int l) -> cpx<R> {
                const cpx<R> z1 = ld(c, l, k1), z2 = ld(c, l, k2);
                return p == 0 ? cpx<R>{R(0.5) * (z1.x + z2.x), R(0.5) * (z1.y - z2.y)}
                              : cpx<R>{R(0.5) * (z1.y + z2.y), R(0.5) * (z2.x - z1.x)};
            };
            // on the rows kx = 0 and kx = M only xx, yy, zz and yz are non-zero
            if constexpr (EARLY_ROW) mix1<R, NZMAX, 1>(nz, in, H, qb0, off0, QY, sl, R(1), dg, row0);
            else mix1<R, NZMAX, 1>(nz, in, H, qb0, off0, QY, sl, R(1), dg);
#pragma unroll
            for (int k = 0; k < 3 * NZMAX; ++k) {
                const cpx<R> o = {__shfl_xor(H[k].x, 1), __shfl_xor(H[k].y, 1)};
                const cpx<R> A = p == 0 ? H[k] : o, Bv = p == 0 ? o : H[k];
                H[k] = p == 0 ? cpx<R>{A.x - Bv.y, A.y + Bv.x} : cpx<R>{A.x + Bv.y, Bv.x - A.y};
            }
            store(p == 0 ? k1 : k2);
        }
    }
    if (mirror_wave) {
        if constexpr (!mirror_early)
            mirror.prep(sh, nz, tid, Q, qcs, sl, QY, lp + (long long)geom * 2 * nz);
        mirror.finish(sh, nz, lp + (long long)geom * 2 * nz);
    }
    __syncthreads();

    for (int s = grp; s < S; s += NG) {
        cpx<R>* dst = col + s * sstride;
        cpx<R>* reg = sh + s * LYP;
        wave_fft<R, LY, true, false, true>(
            reg, g, tw, [&](int pos) -> cpx<R> { return reg[pos]; },
            [&](int pos, cpx<R> v) {
                if (pos < ny) dst[pos] = v;
            });
    }
}

// Grid (M, states per stack, stacks): the stack index is blockIdx.z, so no
// integer division is needed (on gfx950 it runs on the vector unit, and a
// buffer descriptor built from its result is treated as a per-lane value).
template <typename R, int LY, int NZMAX, bool ADJ>
__global__ __launch_bounds__(FusedShape<LY>::NT) void k_ymix_fused(
    cpx<R>* __restrict__ X, int ny, int nz, int M, const R* __restrict__ Q, long long qcs,
    const int* __restrict__ qslot, int QY, const R* __restrict__ lp, int bpg,
    const cpx<R>* __restrict__ twy)
{
    const int geom = blockIdx.z;
    ymix_column<R, LY, NZMAX, ADJ>(blockIdx.x, geom * bpg + blockIdx.y, geom, X, ny, nz, M, Q, qcs,
                                   qslot, QY, lp, twy);
}

// ---------------------------------------------------------------------------
// Fused y pass for a stack of exactly NZ layers (single precision, 256-, 512-
// or 1024-point columns, 512 threads): the same three phases as ymix_column, with every loop over
// layers and layer pairs unrolled.  A lane's 3 NZ input values sit in
// registers for the whole mixing, which walks the NZ (NZ + 1) / 2 stored pairs
// in order (i, j >= i) and applies each block both ways; the tensor entries
// are plain loads that the compiler schedules ahead of their use.  The column
// spectra are read and written through buffer descriptors whose size is the
// column's ny values: the zero padding of the forward transform and the crop
// of the inverse come from the descriptor's range check.  Column 0 (the packed
// kx = 0 and Lx/2 columns) runs ymix_column (512-point columns) or a
// separate k_ymix_fused launch (1024-point columns).
// ---------------------------------------------------------------------------
template <int LY>
struct ExactShape {
    static constexpr int NT = 512;  // 8 waves at any column length: 256 VGPRs per lane
};

template <typename R, int LY, int NZ, bool ADJ, int PRE = 0>
__global__ __launch_bounds__(ExactShape<LY>::NT) void k_ymix_fused_nz(
    cpx<R>* __restrict__ X, int ny, int M, const R* __restrict__ Q, long long qcs,
    const int* __restrict__ qslot, int QY, const R* __restrict__ lp, int bpg,
    const cpx<R>* __restrict__ twy)
{
    constexpr int NT = ExactShape<LY>::NT;
    constexpr int V = fft_vals(LY), GT = LY / V, NG = NT / GT;
    constexpr int S = 3 * NZ, P = NZ * (NZ + 1) / 2;
    constexpr int TPL = LY / NT;           // frequency pairs per lane pair
    constexpr int LYP = fft_region(LY);    // LDS slots per signal
    constexpr int NR = (S + NG - 1) / NG;  // signals per wave, at most
    // one transform per wavefront (512- and 1024-point columns), or two
    // (256-point columns: each half-wave transforms its own signal, so the
    // column reads and writes use per-lane addresses instead of descriptors)
    static_assert(sizeof(R) == 4 && (GT == 64 || GT == 32), "single precision, 256 to 1024 points");
    constexpr bool WHOLE_WAVE = GT == 64;
    // 512-point columns: block 0 runs the packed column 0 with the generic
    // body (one thread per frequency, as here); longer columns leave column 0
    // to a separate launch of k_ymix_fused and start at kx = 1
    constexpr bool OWN_COL0 = LY <= NT;
    const int kx = blockIdx.x + (OWN_COL0 ? 0 : 1), geom = blockIdx.z, b = geom * bpg + blockIdx.y;
    if constexpr (OWN_COL0) {
        if (kx == 0) {
            ymix_column<R, LY, NZ, ADJ>(0, b, geom, X, ny, NZ, M, Q, qcs, qslot, QY, lp, twy);
            return;
        }
    }
    extern __shared__ __align__(16) unsigned char smem_raw[];
    cpx<R>* sh = reinterpret_cast<cpx<R>*>(smem_raw);
    const long long sstride = (long long)M * ny;
    cpx<R>* col = X + ((long long)b * S * M + kx) * ny;
    const int tid = threadIdx.x, grp = tid / GT, g = tid % GT;
    const int cbytes = ny * (int)sizeof(cpx<R>);
    const int p = tid & 1;
    const int* sl = qslot + geom * P;  // the stack's pair slots (scalar loads)
    const UniformBuf<R> qb(Q + (long long)tab_row(kx, M) * qcs, (unsigned)(qcs * sizeof(R)));
    static_assert(PRE == 0 || TPL == 1, "tensor prefetch for one frequency pair per lane");
    R qpre[PRE > 0 ? PRE : 1][5];

    // forward transforms: the inputs of all of this wave's signals are
    // requested first, then transformed one after the other
    {
        Twiddles<R, LY> tw;
        tw.load(g, twy, 1);
        cpx<R> xin[NR][V];
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if constexpr (WHOLE_WAVE) {
                const int s = __builtin_amdgcn_readfirstlane(grp + r * NG);
                if (s < S) {
                    const __amdgpu_buffer_rsrc_t src = __builtin_amdgcn_make_buffer_rsrc(
                        (void*)(col + s * sstride), (short)0, cbytes, 0x00020000);
                    fft_first_loads<R, LY, true>(xin[r], g, [&](int pos) -> cpx<R> {
                        return __builtin_bit_cast(cpx<R>, __builtin_amdgcn_raw_buffer_load_b64(
                                                              src, pos * (int)sizeof(cpx<R>), 0, 0));
                    });
                }
            } else {
                const int s = grp + r * NG;
                if (s < S) {
                    const cpx<R>* src = col + s * sstride;
                    fft_first_loads<R, LY, true>(xin[r], g, [&](int pos) -> cpx<R> {
                        return pos < ny ? src[pos] : cpx<R>{R(0), R(0)};
                    });
                }
            }
        }
        // the first PRE tensor pairs are requested behind the column values
        // (the wait counter is in order), to arrive while the transforms run
        {
            const int t = tid >> 1, kq = p == 0 ? t : (t == 0 ? LY / 2 : t);
#pragma unroll
            for (int u = 0; u < PRE; ++u)
#pragma unroll
                for (int c = 0; c < 5; ++c)
                    qpre[u][c] = qb.ld((unsigned)kq, (unsigned)((sl[u] * 5 + c) * QY));
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const int s = grp + r * NG;
            if (s < S) {
                cpx<R>* reg = sh + s * LYP;
                wave_fft_pre<R, LY, false, true>(reg, g, tw, xin[r],
                                           [&](int pos, cpx<R> v) { reg[pos] = v; });
            }
        }
    }
    __syncthreads();

    // mixing: lanes 2t and 2t+1 take ky = t and LY - t (t = 0: 0 and LY/2),
    // which share the quadrant tensor entry t; t steps by NT / 2
    const R* lpg = lp + (long long)geom * 2 * NZ;
    for (int t = tid >> 1; t < LY / 2; t += NT / 2) {
        const int ky = p == 0 ? t : (t == 0 ? LY / 2 : LY - t);
        const int kq = p == 0 ? t : (t == 0 ? LY / 2 : t);
        const R sg = (p == 1 && t != 0) ? R(-1) : R(1);
        {
            cpx<R> in[3][NZ], H[3][NZ];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int l = 0; l < NZ; ++l) {
                    cpx<R> v = sh[(c * NZ + l) * LYP + ky];
                    if constexpr (ADJ) v = cscale(v, lpg[l]);  // T A T^-1: sources scaled by 1/t
                    in[c][l] = v;
                    H[c][l] = {R(0), R(0)};
                }
#pragma unroll
            for (int i = 0; i < NZ; ++i)
#pragma unroll
                for (int j = i; j < NZ; ++j) {
                    const int u = i * NZ - i * (i - 1) / 2 + (j - i);
                    auto q = [&](int c) -> R {
                        if constexpr (PRE > 0)
                            if (u < PRE) return qpre[u < PRE ? u : 0][c];
                        return qb.ld((unsigned)kq, (unsigned)((sl[u] * 5 + c) * QY));
                    };
                    const R xx = q(0), yy = q(1), xy = sg * q(2), xz = q(3), yz = sg * q(4);
                    R zz = -(xx + yy);
                    if (i == j) {
                        zz += lpg[NZ + i];
                        block_apply(H[0][i], H[1][i], H[2][i], in[0][i], in[1][i], in[2][i], xx, yy,
                                    zz, xy, xz, yz);
                    } else {
                        block_apply(H[0][i], H[1][i], H[2][i], in[0][j], in[1][j], in[2][j], xx, yy,
                                    zz, xy, xz, yz);
                        block_apply(H[0][j], H[1][j], H[2][j], in[0][i], in[1][i], in[2][i], xx, yy,
                                    zz, xy, -xz, -yz);
                    }
                }
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int l = 0; l < NZ; ++l) {
                    cpx<R> v = H[c][l];
                    if constexpr (!ADJ) v = cscale(v, lpg[l]);  // targets scaled by 1/t
                    sh[(c * NZ + l) * LYP + ky] = v;
                }
        }
    }
    __syncthreads();

    // inverse transforms; stores beyond the column's ny values are dropped
    {
        Twiddles<R, LY> tw;
        tw.load(g, twy, 1);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if constexpr (WHOLE_WAVE) {
                const int s = __builtin_amdgcn_readfirstlane(grp + r * NG);
                if (s < S) {
                    const __amdgpu_buffer_rsrc_t dst = __builtin_amdgcn_make_buffer_rsrc(
                        (void*)(col + s * sstride), (short)0, cbytes, 0x00020000);
                    cpx<R>* reg = sh + s * LYP;
                    wave_fft<R, LY, true, false, true>(
                        reg, g, tw, [&](int pos) -> cpx<R> { return reg[pos]; },
                        [&](int pos, cpx<R> v) {
                            __builtin_amdgcn_raw_buffer_store_b64(
                                __builtin_bit_cast(__attribute__((__vector_size__(8))) unsigned, v),
                                dst, pos * (int)sizeof(cpx<R>), 0, 0);
                        });
                }
            } else {
                const int s = grp + r * NG;
                if (s < S) {
                    cpx<R>* dst = col + s * sstride;
                    cpx<R>* reg = sh + s * LYP;
                    wave_fft<R, LY, true, false, true>(
                        reg, g, tw, [&](int pos) -> cpx<R> { return reg[pos]; },
                        [&](int pos, cpx<R> v) {
                            if (pos < ny) dst[pos] = v;
                        });
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Five-pass path: y transforms and mixing as separate kernels (any nz).
// ---------------------------------------------------------------------------
template <typename R, int LY>
struct YPassShape {
    static constexpr int V = fft_vals(LY);
    static constexpr int GT = LY / V;
    static constexpr int NG0 = 256 / GT;
    static constexpr int NGL = (int)(65536 / (sizeof(cpx<R>) * fft_region(LY)));
    static constexpr int NG = NG0 < NGL ? NG0 : (NGL < 1 ? 1 : NGL);
    static constexpr int NT = NG * GT;
};

// columns of n_in complex values (zero padded to LY) -> LY spectrum values
// (HALF: n_in <= LY/2, the first radix pass skips the zero half)
template <typename R, int LY, bool HALF>
__global__ __launch_bounds__((YPassShape<R, LY>::NT)) void k_yfwd(const cpx<R>* __restrict__ in,
                                                                cpx<R>* __restrict__ out, int n_in,
                                                                long long ncols,
                                                                const cpx<R>* __restrict__ twy)
{
    using S = YPassShape<R, LY>;
    __shared__ cpx<R> sh[S::NG * fft_region(LY)];
    const int tid = threadIdx.x, grp = tid / S::GT, g = tid % S::GT;
    const long long c = (long long)blockIdx.x * S::NG + grp;
    if (c >= ncols) return;
    const cpx<R>* src = in + c * n_in;
    cpx<R>* dst = out + c * LY;
    wave_fft<R, LY, false, HALF>(
        sh + grp * fft_region(LY), g, twy, 1,
        [&](int pos) -> cpx<R> { return pos < n_in ? src[pos] : cpx<R>{R(0), R(0)}; },
        [&](int pos, cpx<R> v) { dst[pos] = v; });
}

// LY spectrum values -> first n_out values of the inverse transform
// (HALF: n_out <= LY/2, the last radix pass computes only that half)
template <typename R, int LY, bool HALF>
__global__ __launch_bounds__((YPassShape<R, LY>::NT)) void k_yinv(const cpx<R>* __restrict__ in,
                                                                cpx<R>* __restrict__ out, int n_out,
                                                                long long ncols,
                                                                const cpx<R>* __restrict__ twy)
{
    using S = YPassShape<R, LY>;
    __shared__ cpx<R> sh[S::NG * fft_region(LY)];
    const int tid = threadIdx.x, grp = tid / S::GT, g = tid % S::GT;
    const long long c = (long long)blockIdx.x * S::NG + grp;
    if (c >= ncols) return;
    const cpx<R>* src = in + c * LY;
    cpx<R>* dst = out + c * n_out;
    wave_fft<R, LY, true, false, HALF>(
        sh + grp * fft_region(LY), g, twy, 1, [&](int pos) -> cpx<R> { return src[pos]; },
        [&](int pos, cpx<R> v) {
            if (pos < n_out) dst[pos] = v;
        });
}

// Five-pass z-mixing on full spectra (any nz).  Lanes 2t' and 2t'+1 of a wave
// take the ky points t and LY - t (t = 0: ky = 0 and LY/2), which share one
// quadrant tensor entry; a block (one wave) takes one group of IB target
// layers of 32 ky pairs, each lane summing over all source layers with its IB
// targets' accumulators in registers.  One-dimensional grid, block 64.  Tiles
// (32 ky pairs of one kx column of one state) are numbered ky tile fastest;
// block L runs target group (L / 8) % ngrp of tile 8 ((L / 8) / ngrp) + L % 8,
// so the ngrp blocks of one tile are 8 apart and land on the same XCD (blocks
// are dispatched to the 8 XCDs in turn): they share the tile's spectra and
// tensor entries in that XCD's L2.
// Column 0 carries kx = 0 and Lx/2 packed as A + iB: lane p = 0 mixes A(t)
// with the kx = 0 row and lane p = 1 B(t) with the kx = Lx/2 row, and the pair
// repacks through a lane shuffle; the self-mirrored points t = 0 (ky = 0 and
// LY/2) mix both parts on one lane.
template <typename R, int IB>
__global__ __launch_bounds__(64, 4) void k_mix_pairs(const cpx<R>* __restrict__ Mh,
                                                    cpx<R>* __restrict__ Hh, int nz, int M, int LY,
                                                    const R* __restrict__ Q, long long qcs,
                                                    const int* __restrict__ qslot, int QY,
                                                    const R* __restrict__ lp, int bpg, int adjoint,
                                                    int kx0, int nkx, int B)
{
    const int ngrp = (nz + IB - 1) / IB;
    const int nkyb = (LY / 2 + 31) / 32;
    const long long L = blockIdx.x;
    const long long r = L >> 3;
    const long long tile = (r / ngrp) * 8 + (L & 7);
    if (tile >= (long long)nkyb * nkx * B) return;  // padding of the last tiles
    const int kyb = (int)(tile % nkyb);
    const int kx = kx0 + (int)((tile / nkyb) % nkx), b = (int)(tile / ((long long)nkyb * nkx));
    const int lane = threadIdx.x & 63, i0 = (int)(r % ngrp) * IB;
    const int t = kyb * 32 + (lane >> 1), p = lane & 1;
    if (t >= LY / 2) return;  // no block-level synchronization below
    const int S = 3 * nz, geom = b / bpg;
    const long long sst = (long long)M * LY;
    const cpx<R>* mb = Mh + ((long long)b * S * M + kx) * LY;
    cpx<R>* hb = Hh + ((long long)b * S * M + kx) * LY;
    const R* lpg = lp + (long long)geom * 2 * nz;
    const int* sl = qslot + (long long)geom * (nz * (nz + 1) / 2);  // the stack's pair slots
    const R* dg = lpg + nz;

    // H[IB][3] += S^{ij} v_j over all sources j; row: tensor row (kx) base,
    // kq: quadrant column, sg: sign of the ky-odd components
    auto mix = [&](cpx<R> (&H)[IB][3], const R* row, int kq, R sg, auto in) {
        for (int k = 0; k < IB; ++k)
            for (int c = 0; c < 3; ++c) H[k][c] = {R(0), R(0)};
        for (int j = 0; j < nz; ++j) {
            const R sc = adjoint ? lpg[j] : R(1);
            const cpx<R> X = cscale(in(0, j), sc), Y = cscale(in(1, j), sc), Z = cscale(in(2, j), sc);
#pragma unroll
            for (int k = 0; k < IB; ++k) {
                const int i = i0 + k;
                if (i < nz) {
                    const int a = i < j ? i : j, bq = i < j ? j : i;
                    const R* q = row + (long long)sl[a * nz - a * (a - 1) / 2 + (bq - a)] * 5 * QY + kq;
                    const R simag = i <= j ? R(1) : R(-1);  // conj for the transposed pair
                    const R xx = q[0], yy = q[QY], xy = sg * q[2 * QY], xz = simag * q[3 * QY],
                            yz = sg * simag * q[4 * QY];
                    const R zz = -(xx + yy) + (i == j ? dg[i] : R(0));
                    block_apply(H[k][0], H[k][1], H[k][2], X, Y, Z, xx, yy, zz, xy, xz, yz);
                }
            }
        }
    };
    auto store = [&](const cpx<R> (&H)[IB][3], int ky) {
#pragma unroll
        for (int k = 0; k < IB; ++k) {
            const int i = i0 + k;
            if (i < nz) {
                const R post = adjoint ? R(1) : lpg[i];
                for (int c = 0; c < 3; ++c) hb[(c * nz + i) * sst + ky] = cscale(H[k][c], post);
            }
        }
    };
    cpx<R> H[IB][3];
    if (kx != 0) {
        const int ky = p == 0 ? t : (t == 0 ? LY / 2 : LY - t);
        const int kq = p == 0 ? t : (t == 0 ? LY / 2 : t);
        const R sg = (p == 1 && t != 0) ? R(-1) : R(1);
        mix(H, Q + tab_row(kx, M) * qcs, kq, sg,
            [&](int c, int j) { return mb[(c * nz + j) * sst + ky]; });
        store(H, ky);
    } else if (t != 0) {
        // A(t) = (Z(t) + conj Z(-t)) / 2 on lane 0, B(t) = (Z(t) - conj Z(-t)) / (2i) on lane 1
        const int k1 = t, k2 = LY - t;
        mix(H, Q + (p == 0 ? 0 : tab_row(M, M)) * qcs, t, R(1), [&](int c, int j) {
            const cpx<R> z1 = mb[(c * nz + j) * sst + k1], z2 = mb[(c * nz + j) * sst + k2];
            return p == 0 ? cpx<R>{R(0.5) * (z1.x + z2.x), R(0.5) * (z1.y - z2.y)}
                          : cpx<R>{R(0.5) * (z1.y + z2.y), R(0.5) * (z2.x - z1.x)};
        });
        // W(t) = HA + i HB on lane 0, W(-t) = conj(HA) + i conj(HB) on lane 1
#pragma unroll
        for (int k = 0; k < IB; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const cpx<R> o = {__shfl_xor(H[k][c].x, 1), __shfl_xor(H[k][c].y, 1)};
                const cpx<R> A = p == 0 ? H[k][c] : o, Bv = p == 0 ? o : H[k][c];
                H[k][c] = p == 0 ? cpx<R>{A.x - Bv.y, A.y + Bv.x} : cpx<R>{A.x + Bv.y, Bv.x - A.y};
            }
        store(H, p == 0 ? k1 : k2);
    } else {
        // ky = 0 (lane 0) or LY/2 (lane 1), each its own mirror: A = Re Z, B = Im Z;
        // the point receives A' first and then A' + i B'
        const int kp = p == 0 ? 0 : LY / 2;
        mix(H, Q, kp, R(1), [&](int c, int j) { return cpx<R>{mb[(c * nz + j) * sst + kp].x, R(0)}; });
        cpx<R> keep[IB][3];
#pragma unroll
        for (int k = 0; k < IB; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) keep[k][c] = H[k][c];
        mix(H, Q + tab_row(M, M) * qcs, kp, R(1),
            [&](int c, int j) { return cpx<R>{mb[(c * nz + j) * sst + kp].y, R(0)}; });
#pragma unroll
        for (int k = 0; k < IB; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                H[k][c] = {keep[k][c].x - H[k][c].y, keep[k][c].y + H[k][c].x};
        store(H, kp);
    }
}

}  // namespace hfd
