// Thickness gradient of L = <g, h(m)> (h = -N * m) for every state.
//
// With T^{ij} = -DFT2(N^{ij}) / (Lx Ly) the field is H_i = sum_j T^{ij} M_j and
//   L = sum_k sum_{ij} conj(G_i(k)) . T^{ij}(k) M_j(k)   (full Lx x Ly grid),
// G, M the 2D DFTs of the zero-padded g and m.  N^{ij} depends on the four
// interfaces bot_i, top_i (target) and bot_j, top_j (source) through
// N = -1/(4 pi dx dy t_i) sum_c s_c Psi(zeta_c), zeta = {top_i - bot_j,
// bot_i - bot_j, top_i - top_j, bot_i - top_j}, s = {+1, -1, -1, +1}, Psi the
// lateral-stencilled Phi.  The sign s_c factors into a target sign (+1 top,
// -1 bottom) times a source sign (+1 bottom, -1 top), so with K(zeta) the
// normalized DFT of -Psi/(4 pi dx dy) and, per interface e of layer l,
//   Ghat_e = +-G_l / t_l (+ top, - bottom),  Mhat_e = -+M_l (- top, + bottom),
// the functional is a sum over interface pairs:
//   L = sum_{e,f} Re conj(Ghat_e) . K(z_e - z_f) Mhat_f.
// Interfaces that coincide (top_l touching bot_{l+1}) move together under
// every thickness change (gaps are fixed), so they are merged into one
// position p with summed Ghat_p, Mhat_p.  Moving position p alone changes L by
//   dL/dz_p = sum_q [P(p, q) - P(q, p)] + (1/t terms),
//   P(p, q) = Re conj(Ghat_p) . D(z_p - z_q) Mhat_q,
// D = dK/dzeta the normalized DFT of -1/(4 pi dx dy) dPsi/dz.  The 1/t_l
// factor of Ghat adds -L_l / t_l to the top of layer l and +L_l / t_l to its
// bottom, L_l = sum_j Re conj(G_l) . T^{lj} M_j the layer's share of L.  Each
// D(z_p - z_q) is read once per frequency, where a sum over ordered layer pairs
// and their four offsets reads it up to eight times.  The half spectrum holds
// kx in [1, M) once (weight 2, the mirror -kx is the complex conjugate) and
// the packed column 0 carries kx = 0 and kx = Lx/2 (weight 1 each).
// Position p has rank r_p (r = l for bot_l, l + 1 for top_l) and
// dz_p/dt_k = [k < r_p].  D is stored for |zeta| only: dPsi/dz is odd in zeta
// for xx, yy, zz, xy and even for xz, yz, so D(-zeta) is D(zeta) with the
// first four negated (the table entry of a pair carries the sign).
#include "field_kernels.hpp"
#include "launch.hpp"

namespace hfd {

namespace {

// sum over the 64 lanes, the same bits in every lane (xor butterfly)
__device__ inline double wave_sum(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T>
__device__ inline T block_sum(T v, T* red)
{
    // wave reduction then across waves (blockDim.x multiple of 64, <= 1024)
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    T s = T(0);
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
    return s;  // valid in thread 0
}

// Re conj(g) . A m for the symmetric block A with real xx, yy, zz, xy and
// imaginary i xz, i yz entries; g, m = (re, im) x 3, arithmetic in double.
template <typename T>
__device__ inline double gAm(const double g[6], double xx, double yy, double zz, double xy,
                             double xz, double yz, const T mm[6])
{
    const double m[6] = {mm[0], mm[1], mm[2], mm[3], mm[4], mm[5]};
    const double vxr = xx * m[0] + xy * m[2] - xz * m[5];
    const double vxi = xx * m[1] + xy * m[3] + xz * m[4];
    const double vyr = xy * m[0] + yy * m[2] - yz * m[5];
    const double vyi = xy * m[1] + yy * m[3] + yz * m[4];
    const double vzr = zz * m[4] - xz * m[1] - yz * m[3];
    const double vzi = zz * m[5] + xz * m[0] + yz * m[2];
    return g[0] * vxr + g[1] * vxi + g[2] * vyr + g[3] * vyi + g[4] * vzr + g[5] * vzi;
}

}  // namespace

// QC (4 or 8) consecutive table entries from a 4 QC-byte aligned address
template <int QC>
__device__ inline void load_chunk(const int* __restrict__ src, int (&dst)[QC])
{
    static_assert(QC == 4 || QC == 8, "interface chunks hold 4 or 8 positions");
#pragma unroll
    for (int h = 0; h < QC / 4; ++h) {
        const int4 a = reinterpret_cast<const int4*>(src)[h];
        dst[4 * h] = a.x; dst[4 * h + 1] = a.y; dst[4 * h + 2] = a.z; dst[4 * h + 3] = a.w;
    }
}

// Per-position gradient sums of one wave over its 64 frequencies of row kx
// (PACKED: the packed column, rows 0 and M from the unpacked pair A, B).
// Sources (interface positions, then layers) are taken in chunks of QC held
// in registers; for each target the loads of the next target are issued
// before the arithmetic of the current one (software pipelining), and no
// load sits behind a branch: the two layers of a position are always read
// (clamped index, weight 0 when absent), source slots past the end read a
// valid slot against a zero source.
template <typename R, int QC, bool PACKED>
__device__ inline void tgrad_row(const cpx<R>* __restrict__ mb, const cpx<R>* __restrict__ gb,
                                 long long sst, int nz, int M, int kx, int ky, int kyn, int kq,
                                 double sgy, double wgt0, const R* __restrict__ Q, long long qcs,
                                 const int* __restrict__ sl, const R* __restrict__ Dg, int nzt,
                                 const int* __restrict__ it,
                                 const R* __restrict__ lpg, int QY, double* __restrict__ acc)
{
    constexpr int NV = PACKED ? 2 : 1;  // raw spectrum values per entry (ky, and LY - ky)
    const int lane = threadIdx.x;
    const ITabLayout lay = itab_layout(nz);
    const int NI = it[0];
    const int* pinfo = it + lay.info;
    const int* pbot = it + lay.pbot;
    const int* ptop = it + lay.ptop;
    const int* zpq = it + lay.zpq;
    // acc[v][64]: lane-owned partial sums of position v (LDS, fire-and-forget adds)
    auto add_out = [&](int v, double val) { atomicAdd(&acc[v * 64 + lane], val); };
    for (int ps = 0; ps < NV; ++ps) {
        const int row = PACKED ? (ps ? M : 0) : kx;
        // rows of D ([QX][nzt][6][QY]) and of the tensor table ([QX][slots][5][QY])
        // as buffers: the lane offset is kq, the slot and component offsets are scalar
        const int trow = tab_row(row, M);
        const UniformBuf<R> dbuf(Dg + (long long)trow * nzt * 6 * QY, (unsigned)(nzt * 6 * QY * sizeof(R)));
        const UniformBuf<R> qbuf(Q + (long long)trow * qcs, (unsigned)(qcs * sizeof(R)));
        // component c of layer l: raw loads, then (re, im) at this point
        auto raw = [&](const cpx<R>* base, int c, int l, cpx<R> (&z)[NV]) {
            z[0] = base[(c * nz + l) * sst + ky];
            if (PACKED) z[NV - 1] = base[(c * nz + l) * sst + kyn];
        };
        auto comb = [&](const cpx<R> (&z)[NV], double& re, double& im) {
            if (!PACKED) {
                re = z[0].x;
                im = z[0].y;
            } else {
                const cpx<R> z1 = z[0], z2 = z[NV - 1];
                const double ar = 0.5 * ((double)z1.x + z2.x), ai = 0.5 * ((double)z1.y - z2.y);
                const double br = 0.5 * ((double)z1.y + z2.y), bi = 0.5 * ((double)z2.x - z1.x);
                re = ps ? br : ar;
                im = ps ? bi : ai;
            }
        };
        // ---- interface pairs ------------------------------------------------
        struct PosLoads {
            R d[QC][6];
            cpx<R> g[2][3][NV];
            int zi[QC];
        };
        for (int qc = 0; qc < NI; qc += QC) {
            R mh[QC][6];  // Mhat in plan precision
            {
                int pi[QC];
                load_chunk(pinfo + qc, pi);
                cpx<R> zm[QC][2][3][NV];
#pragma unroll
                for (int q = 0; q < QC; ++q) {
                    const int rk = pi[q] >> 2;
                    const int la = rk > 0 ? rk - 1 : 0, lb = rk < nz ? rk : nz - 1;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        raw(mb, c, la, zm[q][0][c]);
                        raw(mb, c, lb, zm[q][1][c]);
                    }
                }
#pragma unroll
                for (int q = 0; q < QC; ++q) {
                    const bool live = qc + q < NI;
                    const int info = pi[q];
                    const double wa = live && (info & 1) ? -1.0 : 0.0;  // top of rk - 1: -M
                    const double wb = live && (info & 2) ? 1.0 : 0.0;   // bottom of rk: +M
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        double ra, ia, rb, ib;
                        comb(zm[q][0][c], ra, ia);
                        comb(zm[q][1][c], rb, ib);
                        mh[q][2 * c] = (R)(wa * ra + wb * rb);
                        mh[q][2 * c + 1] = (R)(wa * ia + wb * ib);
                    }
                }
            }
            auto fetch = [&](int p, PosLoads& f) {
                const int rk = pinfo[p] >> 2;
                const int la = rk > 0 ? rk - 1 : 0, lb = rk < nz ? rk : nz - 1;
                load_chunk(zpq + p * lay.nsp + qc, f.zi);
#pragma unroll
                for (int q = 0; q < QC; ++q)
#pragma unroll
                    for (int c = 0; c < 6; ++c)
                        f.d[q][c] = dbuf.ld(kq, (unsigned)(((f.zi[q] >> 1) * 6 + c) * QY));
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    raw(gb, c, la, f.g[0][c]);
                    raw(gb, c, lb, f.g[1][c]);
                }
            };
            double gq[QC];
#pragma unroll
            for (int q = 0; q < QC; ++q) gq[q] = 0.0;
            PosLoads nxt;
            fetch(0, nxt);
            for (int p = 0; p < NI; ++p) {
                const PosLoads cur = nxt;
                if (p + 1 < NI) fetch(p + 1, nxt);
                const int info = pinfo[p], rk = info >> 2;
                const int la = rk > 0 ? rk - 1 : 0, lb = rk < nz ? rk : nz - 1;
                // top of rk - 1: +G / t; bottom of rk: -G / t (lp holds 1/t)
                const double wa = (info & 1) ? wgt0 * (double)lpg[la] : 0.0;
                const double wb = (info & 2) ? -wgt0 * (double)lpg[lb] : 0.0;
                double gh[6];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    double ra, ia, rb, ib;
                    comb(cur.g[0][c], ra, ia);
                    comb(cur.g[1][c], rb, ib);
                    gh[2 * c] = wa * ra + wb * rb;
                    gh[2 * c + 1] = wa * ia + wb * ib;
                }
                double ga = 0.0;
#pragma unroll
                for (int q = 0; q < QC; ++q) {
                    const R* d = cur.d[q];
                    // z_p < z_q: D(-zeta) = D(zeta) with xx, yy, zz, xy negated
                    const double sz = (cur.zi[q] & 1) ? -1.0 : 1.0;
                    const double pd = gAm(gh, sz * d[0], sz * d[1], sz * d[2], sz * sgy * (double)d[3],
                                          d[4], sgy * (double)d[5], mh[q]);
                    ga += pd;
                    gq[q] -= pd;
                }
                add_out(p, ga);
            }
#pragma unroll
            for (int q = 0; q < QC; ++q)
                if (qc + q < NI) add_out(qc + q, gq[q]);
        }
        // ---- the 1/t_l factor ----------------------------------------------
        // top_l gets -L_l / t_l, bot_l gets +L_l / t_l, L_l = sum_j
        // Re conj(G_l) . T^{lj} M_j; the stored blocks are t_l T^{lj}
        struct LayerLoads {
            R a[QC][5];
            cpx<R> g[3][NV];
        };
        for (int jc = 0; jc < nz; jc += QC) {
            R mj[QC][6];
            {
                cpx<R> zm[QC][3][NV];
#pragma unroll
                for (int q = 0; q < QC; ++q) {
                    const int j = jc + q < nz ? jc + q : nz - 1;
#pragma unroll
                    for (int c = 0; c < 3; ++c) raw(mb, c, j, zm[q][c]);
                }
#pragma unroll
                for (int q = 0; q < QC; ++q) {
                    const double w = jc + q < nz ? 1.0 : 0.0;
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        double re, im;
                        comb(zm[q][c], re, im);
                        mj[q][2 * c] = (R)(w * re);
                        mj[q][2 * c + 1] = (R)(w * im);
                    }
                }
            }
            auto fetch = [&](int l, LayerLoads& f) {
#pragma unroll
                for (int q = 0; q < QC; ++q) {
                    const int j = jc + q < nz ? jc + q : nz - 1;
                    const int a = l < j ? l : j, bq = l < j ? j : l;
                    const int slot = sl[a * nz - a * (a - 1) / 2 + (bq - a)];
#pragma unroll
                    for (int c = 0; c < 5; ++c) f.a[q][c] = qbuf.ld(kq, (unsigned)((slot * 5 + c) * QY));
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) raw(gb, c, l, f.g[c]);
            };
            LayerLoads nxt;
            fetch(0, nxt);
            for (int l = 0; l < nz; ++l) {
                const LayerLoads cur = nxt;
                if (l + 1 < nz) fetch(l + 1, nxt);
                const double it_l = lpg[l];  // lp holds 1/t
                const double w = wgt0 * it_l * it_l;
                const double trace = lpg[nz + l];
                double g6[6];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    double re, im;
                    comb(cur.g[c], re, im);
                    g6[2 * c] = w * re;
                    g6[2 * c + 1] = w * im;
                }
                double sl = 0.0;
#pragma unroll
                for (int q = 0; q < QC; ++q) {
                    const int j = jc + q;
                    const double simag = l <= j ? 1.0 : -1.0;
                    const double xx = cur.a[q][0], yy = cur.a[q][1];
                    const double zz = -(xx + yy) + (l == j ? trace : 0.0);
                    sl += gAm(g6, xx, yy, zz, sgy * (double)cur.a[q][2], simag * (double)cur.a[q][3],
                              simag * sgy * (double)cur.a[q][4], mj[q]);
                }
                add_out(ptop[l], -sl);
                add_out(pbot[l], sl);
            }
        }
    }
}

// One wave per (state, kx, 32 lateral frequency pairs): lanes 2s and 2s+1 take
// ky = t and LY - t (t = ty*32 + s; lane 2s+1 of t = 0 takes ky = LY/2), which
// share every quadrant value of D and Q.  Each lane accumulates its own
// per-position sums in LDS; the block sums them over the lanes at the end.
// Block order: groups of 8 tiles, within a group every state of the launch,
// with the 8 tiles on consecutive block indices: the states of one tile are 8
// indices apart, so they run one after the other on one XCD and read that
// tile's slice of the offset table D (shared by every stack when stored) and
// of their geometry's Q through its L2, instead of streaming the whole table
// once per state.
// itab per geometry: see itab_layout.  D per geometry: [QX][nzt][6][QY], nzt D slots per row.
// lp per geometry: 1/t_l, then the trace term of the diagonal blocks.
// partial[b][tile][2nz]: the block's position gradients.
template <typename R, int QC>
__global__ __launch_bounds__(64) void k_tgrad(const cpx<R>* __restrict__ Mh,
                                              const cpx<R>* __restrict__ Gh, int nz, int M, int LY,
                                              const R* __restrict__ Q, long long qcs,
                                              const int* __restrict__ qslot,
                                              const R* __restrict__ D, int nzt,
                                              const int* __restrict__ itab, int itab_stride,
                                              const R* __restrict__ lp, int bpg,
                                              int QY, int b0, int nst, int ntiles,
                                              double* __restrict__ partial)
{
    const int L = blockIdx.x, r8 = L >> 3;
    const int tile = (r8 / nst) * 8 + (L & 7);
    if (tile >= ntiles) return;
    const int b = b0 + r8 % nst;
    const int geom = b / bpg;
    const int half = LY >> 1;
    const int tpk = (half + 31) >> 5;
    const int kx = tile / tpk, ty = tile - kx * tpk;
    const int lane = threadIdx.x;
    const int t0 = ty * 32 + (lane >> 1);
    const bool active = t0 < half;
    const int t = active ? t0 : 0;
    const int ky = (lane & 1) == 0 ? t : (t == 0 ? half : LY - t);
    const int kq = ky <= half ? ky : LY - ky;
    const double sgy = ky <= half ? 1.0 : -1.0;
    const int kyn = (LY - ky) & (LY - 1);
    const int S = 3 * nz;
    const long long sst = (long long)M * LY;
    const cpx<R>* mb = Mh + ((long long)b * S * M + kx) * LY;
    const cpx<R>* gb = Gh + ((long long)b * S * M + kx) * LY;
    const int* sl = qslot + (long long)geom * (nz * (nz + 1) / 2);  // the stack's pair slots
    const R* lpg = lp + (long long)geom * 2 * nz;
    const int* it = itab + (long long)geom * itab_stride;
    const int NI = it[0], NS = 2 * nz;
    extern __shared__ double acc[];  // [NI][64]
    for (int v = 0; v < NI; ++v) acc[v * 64 + lane] = 0.0;
    if (kx == 0)
        tgrad_row<R, QC, true>(mb, gb, sst, nz, M, kx, ky, kyn, kq, sgy, active ? 1.0 : 0.0, Q, qcs,
                               sl, D, nzt, it, lpg, QY, acc);
    else
        tgrad_row<R, QC, false>(mb, gb, sst, nz, M, kx, ky, kyn, kq, sgy, active ? 2.0 : 0.0, Q,
                                qcs, sl, D, nzt, it, lpg, QY, acc);
    __syncthreads();
    double* out = partial + ((long long)b * ntiles + tile) * NS;
    for (int v = 0; v < NI; ++v) {
        const double sv = wave_sum(acc[v * 64 + lane]);
        if (lane == 0) out[v] = sv;
    }
}

// Sum the tile partials of each position (fixed order) and apply the stacking
// chain rule dL/dt_k = sum_p [k < r_p] dL/dz_p.
__global__ __launch_bounds__(256) void k_tgrad_finish(const double* __restrict__ partial, int nparts,
                                                      int nz, const int* __restrict__ itab,
                                                      int itab_stride, int bpg,
                                                      double* __restrict__ grad_t)
{
    __shared__ double red[4];
    __shared__ double gp[128];
    const int b = blockIdx.x;
    const int* it = itab + (long long)(b / bpg) * itab_stride;
    const int NI = it[0], NS = 2 * nz;
    for (int v = 0; v < NI; ++v) {
        double s = 0.0;
        for (int k = threadIdx.x; k < nparts; k += blockDim.x)
            s += partial[((long long)b * nparts + k) * NS + v];
        s = block_sum(s, red);
        if (threadIdx.x == 0) gp[v] = s;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nz; k += blockDim.x) {
        double s = 0.0;
        for (int p = 0; p < NI; ++p)
            if (k < (it[itab_layout(nz).info + p] >> 2)) s += gp[p];
        grad_t[(long long)b * nz + k] = s;
    }
}

int tgrad_tiles(int M, int LY)
{
    return M * ((LY / 2 + 31) / 32);
}

hipError_t launch_tgrad(bool fp64, const void* Mh, const void* Gh, int nz, int M, int LY, int b0,
                        int nb, const void* Q, long long qcs, const int* qslot, const void* D, int nzt,
                        const int* itab, int itab_stride, const void* lp, int bpg,
                        int QX, int QY, double* partial, hipStream_t s)
{
    if (nz < 1 || nz > 64 || nb < 1 || bpg < 1 || nb % bpg || LY < 2 || (LY & (LY - 1)))
        return hipErrorInvalidValue;
    (void)QX;  // D and Q rows are addressed through nzt, qcs and QY
    // one row of D or Q is a buffer with 32-bit byte offsets
    const long long rsz = fp64 ? 8 : 4;
    if ((long long)nzt * 6 * QY * rsz >= (1LL << 31) || qcs * rsz >= (1LL << 31))
        return hipErrorInvalidValue;
    const int ntiles = tgrad_tiles(M, LY);
    const long long nblk = (long long)((ntiles + 7) / 8) * 8 * nb;
    if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
    const size_t lds = sizeof(double) * 64 * 2 * nz;  // >= NI x 64
    if (fp64)
        hipLaunchKernelGGL((k_tgrad<double, 4>), dim3((unsigned)nblk), dim3(64), lds, s,
                           (const cpx<double>*)Mh, (const cpx<double>*)Gh, nz, M, LY,
                           (const double*)Q, qcs, qslot, (const double*)D, nzt, itab, itab_stride,
                           (const double*)lp, bpg, QY, b0, nb, ntiles, partial);
    else
        hipLaunchKernelGGL((k_tgrad<float, 4>), dim3((unsigned)nblk), dim3(64), lds, s,
                           (const cpx<float>*)Mh, (const cpx<float>*)Gh, nz, M, LY,
                           (const float*)Q, qcs, qslot, (const float*)D, nzt, itab, itab_stride,
                           (const float*)lp, bpg, QY, b0, nb, ntiles, partial);
    return hipGetLastError();
}

hipError_t launch_tgrad_finish(const double* partial, int nparts, int B, int nz, const int* itab,
                               int itab_stride, int bpg, double* grad_t, hipStream_t s)
{
    if (nz < 1 || nz > 64 || B < 1 || bpg < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_tgrad_finish, dim3(B), dim3(256), 0, s, partial, nparts, nz, itab,
                       itab_stride, bpg, grad_t);
    return hipGetLastError();
}

}  // namespace hfd
