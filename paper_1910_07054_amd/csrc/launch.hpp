// Host-side launch wrappers: map run-time sizes onto the compiled template
// instances.  Each returns hipErrorInvalidValue for a size outside the
// compiled range (the API layer checks ranges first).
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/hfd.h"

namespace hfd {

// set the message returned by hfd_last_error (api.hip) and return s
hfd_status report_error(hfd_status s, const std::string& msg);

constexpr int kMinL = 8;
constexpr int kMaxL = 4096;

// Raise the dynamic-LDS limit of `kernel` on the current device to `bytes`
// (no-op up to 64 KB).  Remembered per (kernel, device) once the runtime has
// accepted it; thread safe.
hipError_t ensure_lds_limit(const void* kernel, int bytes);

// x pass, forward / inverse (R = float if !fp64 else double) over nsig * ny
// rows; ty = rows per block (0: the default tile; else one of 4, 8, 12, 16, 24,
// 32 where x_tile_supported, for rows of nx <= LX/2 values only)
bool x_tile_supported(bool fp64, int LX, int ty);
// x transforms of nsig tensor quadrants in[nsig][ny][nx] (FP64; component
// sig % 6, extended to length LX by its x parity) -> out[nsig][LX/2 + 1][ny],
// the real part of each transform (x-even components) or the imaginary part
// (x-odd ones), which is the non-zero one
hipError_t launch_xtab(int LX, const double* in, void* out, int nx, int ny, int nsig, const void* twx64,
                       hipStream_t s);
hipError_t launch_xfwd(bool fp64, int LX, const void* in, void* out, int nx, int ny,
                       long long in_sig_stride, int in_row_stride, int nsig, const void* twx,
                       hipStream_t s, int ty = 0);
hipError_t launch_xinv(bool fp64, int LX, const void* in, void* out, int nx, int ny,
                       long long out_sig_stride, int out_row_stride, int nsig, const void* twx,
                       hipStream_t s, int ty = 0);

// y pass on columns: forward (n_in values padded to LY) / inverse (first n_out kept)
hipError_t launch_yfwd(bool fp64, int LY, const void* in, void* out, int n_in, long long ncols,
                       const void* twy, hipStream_t s);
hipError_t launch_yinv(bool fp64, int LY, const void* in, void* out, int n_out, long long ncols,
                       const void* twy, hipStream_t s);

// The Fourier tensor of a plan is one table of pair slots, Q[QX][nslot][5][QY]
// (kx row outer, qcs = nslot * 5 * QY elements per row); pair u (i <= j,
// u = i nz - i (i - 1) / 2 + j - i) of stack g reads slot qslot[g * P + u].
// Stacks that share a pair geometry (thicknesses and offset) share its slot.
// Consumers take (Q, qcs, qslot) with qslot already offset to their first
// stack.

// fused y pass: does a compiled instance exist for (fp64, LY, nz) with lds bytes?
bool fused_supported(bool fp64, int LY, int nz, size_t* lds_bytes);
// generic = true: the run-time layer-count kernel even where an exact-layer
// kernel exists (the autotuner times both)
hipError_t launch_fused(bool fp64, int LY, int nz, void* X, int ny, int M, int B, const void* Q,
                        long long qcs, const int* qslot, int QX, int QY, const void* lp, int bpg,
                        int adjoint, const void* twy, hipStream_t s, bool generic = false);

// exact-layer-count fused y pass (single precision; LY = 256 or 512 with
// 1 <= nz <= 10, LY = 1024 with 1 <= nz <= 4): grid (M, bpg, G); units 1-3
// cover 1-4, 5-7 and 8-10 layers of 512-point columns, unit 4 the 1024-point
// columns, unit 5 the 256-point columns
hipError_t launch_fused_exact_1(int nz, int adjoint, void* X, int ny, int M, int bpg, int G,
                                const void* Q, long long qcs, const int* qslot, int QY,
                                const void* lp, const void* tw, hipStream_t s);
hipError_t launch_fused_exact_2(int nz, int adjoint, void* X, int ny, int M, int bpg, int G,
                                const void* Q, long long qcs, const int* qslot, int QY,
                                const void* lp, const void* tw, hipStream_t s);
hipError_t launch_fused_exact_3(int nz, int adjoint, void* X, int ny, int M, int bpg, int G,
                                const void* Q, long long qcs, const int* qslot, int QY,
                                const void* lp, const void* tw, hipStream_t s);
hipError_t launch_fused_exact_4(int nz, int adjoint, void* X, int ny, int M, int bpg, int G,
                                const void* Q, long long qcs, const int* qslot, int QY,
                                const void* lp, const void* tw, hipStream_t s);
hipError_t launch_fused_exact_5(int nz, int adjoint, void* X, int ny, int M, int bpg, int G,
                                const void* Q, long long qcs, const int* qslot, int QY,
                                const void* lp, const void* tw, hipStream_t s);
inline bool fused_exact_supported(bool fp64, int LY, int nz)
{
    return !fp64 && nz >= 1 && ((LY == 256 && nz <= 10) || (LY == 512 && nz <= 10) || (LY == 1024 && nz <= 4));
}
inline hipError_t launch_fused_exact(int LY, int nz, int adjoint, void* X, int ny, int M, int bpg,
                                     int G, const void* Q, long long qcs, const int* qslot, int QY,
                                     const void* lp, const void* tw, hipStream_t s)
{
    if (LY == 1024) return launch_fused_exact_4(nz, adjoint, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, tw, s);
    if (LY == 256) return launch_fused_exact_5(nz, adjoint, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, tw, s);
    if (nz <= 4) return launch_fused_exact_1(nz, adjoint, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, tw, s);
    if (nz <= 7) return launch_fused_exact_2(nz, adjoint, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, tw, s);
    return launch_fused_exact_3(nz, adjoint, X, ny, M, bpg, G, Q, qcs, qslot, QY, lp, tw, s);
}

// generic mixing of the kx columns [kx0, kx0 + nkx)
hipError_t launch_mix_generic(bool fp64, const void* Mh, void* Hh, int nz, int M, int LY, int B,
                              const void* Q, long long qcs, const int* qslot, int QX, int QY,
                              const void* lp, int bpg, int adjoint, int kx0, int nkx, hipStream_t s);

// batched mixing of the kx columns 1 .. M-1 (all states of one stack per block,
// 16 at a time): matrix cores with the three-way BF16 split (mfma = true) or
// FP32 VALU on the same staging
bool mix_batched_supported(int nz, int B, int G);
hipError_t launch_mix_batched(bool mfma, const void* Mh, void* Hh, int nz, int M, int LY, int B,
                              const void* Q, long long qcs, const int* qslot, int QY, const void* lp,
                              int bpg, int adjoint, hipStream_t s);

// equidistant stacks: 3-D Fourier tensor from the per-offset 2D spectra, and
// the z pass on the five-pass spectra (packed column unpacked into Bc and
// repacked; Bc, HBc: [B][3nz][LY])
hipError_t launch_zdft3(bool out_fp64, const double* Q2, void* T3, int nz, int LZ, int QX, int QY,
                        hipStream_t s);
hipError_t launch_eq3d_mix(bool fp64, int LZ, void* Mh, void* Bc, void* Hh, void* HBc, int nz, int M,
                           int LY, int B, const void* T3, int QY, const void* twz, hipStream_t s);

// thickness-gradient reduction over the spectra (states b0 .. b0+nb-1, nb a
// multiple of bpg); partial: [states][tgrad_tiles(M, LY)][2 nz]
int tgrad_tiles(int M, int LY);
// Per-geometry interface table of the thickness gradient (ints): [0] NI, the
// number of interface positions; pinfo[nsp] at `info` (rank r*4 + 1 if the top
// of layer r-1 is there + 2 if the bottom of layer r is there); pos_bot[nz],
// pos_top[nz]; zpq[nsp][nsp] at `zpq`: 2 x (D slot of |z_p - z_q|) + 1 when
// z_p < z_q.  nsp = 2nz rounded up to 8 and every row 32-byte aligned, so a
// chunk of 8 entries is two aligned 16-byte loads; padding entries are slot 0.
struct ITabLayout {
    int nsp, info, pbot, ptop, zpq, stride;
};
__host__ __device__ inline ITabLayout itab_layout(int nz)
{
    ITabLayout t;
    t.nsp = (2 * nz + 7) & ~7;
    t.info = 8;
    t.pbot = t.info + t.nsp;
    t.ptop = t.pbot + nz;
    t.zpq = (t.ptop + nz + 7) & ~7;
    t.stride = t.zpq + t.nsp * t.nsp;
    return t;
}
hipError_t launch_tgrad(bool fp64, const void* Mh, const void* Gh, int nz, int M, int LY, int b0,
                        int nb, const void* Q, long long qcs, const int* qslot, const void* D, int nzt,
                        const int* itab, int itab_stride, const void* lp, int bpg,
                        int QX, int QY, double* partial, hipStream_t s);
hipError_t launch_tgrad_finish(const double* partial, int nparts, int B, int nz, const int* itab,
                               int itab_stride, int bpg, double* grad_t, hipStream_t s);

// tensor setup (FP64)
struct PairGeoH {
    double ti, tj, Z, pad;
};
// tmax: the largest thickness among the npairs pair records (bounds the near box);
// mode 1: offset table [pair][6][2ny-1][2nx-1], 2: the quadrant [pair][6][ny][nx]
hipError_t launch_tensor_real(double* W, const PairGeoH* pg, int npairs, int nx, int ny, int Lx,
                              int Ly, double dx, double dy, double tmax, int mode, hipStream_t s);
// zero n doubles (a kernel, so that graph captures hold no memset node)
hipError_t launch_zero64(double* p, long long n, hipStream_t s);
// quadrants W[nzeta][6][ny][nx] of the lateral-stencilled z-derivative tables
hipError_t launch_dtensor_real(double* W, const double* zeta, int nzeta, int nx, int ny, double dx,
                               double dy, hipStream_t s);
// y transforms of x-pass tensor spectra F[pair][6][M + 1][ny] (FP64 reals as
// launch_xtab writes them, columns extended to Ly by each component's y
// parity) and their
// packing into the quadrant: comps 5 (field tensor) or 6 (all components);
// row_outer: [QX][pair_total][comps][QY] at pairs pair0.., else
// [npairs][comps][QX][QY]; times scale[u].  src (device, optional): for output
// pair u the index of its spectra in F, or -1 to leave the pair alone
// (default: u itself).  twy64: the FP64 twiddles of length Ly.
hipError_t launch_ytab(bool out_fp64, const void* F, void* Q, const double* scale, int npairs,
                       int comps, int M, int ny, int Ly, int QX, int QY, int pair0, int pair_total,
                       int row_outer, const void* twy64, hipStream_t s, const int* src = nullptr);

}  // namespace hfd
