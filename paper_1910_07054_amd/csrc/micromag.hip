// Micromagnetic energy of one layer on the lateral grid (include/hfd_mm.h):
// exchange, uniaxial anisotropy, applied and bias fields in the kernels here,
// the demagnetizing field through hfd_demag_field.  These are the energy
// terms of the hysteresis simulation of Sec. 4 (free layer of the MRAM cell);
// the finite-difference form is the usual one (the paper gives only the terms
// and the CoFe constants).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "../../include/hfd_mm.h"
#include "launch.hpp"

using namespace hfd;

namespace {

constexpr int kBlock = 256;

// m = u / |u| on the mask, 0 elsewhere; rinv = 1 / |u| (0 off the mask).
// A zero vector inside the mask raises *bad.
__global__ __launch_bounds__(kBlock) void k_mm_normalize(const double* __restrict__ u,
                                                         const unsigned char* __restrict__ mask,
                                                         double* __restrict__ m,
                                                         double* __restrict__ rinv, int n,
                                                         int* __restrict__ bad)
{
    const int c = blockIdx.x * kBlock + threadIdx.x;
    if (c >= n) return;
    double x = 0, y = 0, z = 0, ri = 0;
    if (mask[c]) {
        const double ux = u[c], uy = u[n + c], uz = u[2 * n + c];
        const double r2 = ux * ux + uy * uy + uz * uz;
        if (r2 > 0) {
            ri = 1.0 / sqrt(r2);
            x = ux * ri;
            y = uy * ri;
            z = uz * ri;
        } else {
            *bad = 1;
        }
    }
    m[c] = x;
    m[n + c] = y;
    m[2 * n + c] = z;
    rinv[c] = ri;
}

// Effective field, reduced energy per cell (summed per block into part[]) and
// the gradient with respect to u (see hfd_mm.h).
__global__ __launch_bounds__(kBlock) void k_mm_heff(
    const double* __restrict__ m, const double* __restrict__ rinv,
    const unsigned char* __restrict__ mask, const double* __restrict__ hd,
    const double* __restrict__ hb, int nx, int ny, double cex_x, double cex_y, double hk,
    double hx_ext, double hy_ext, double hz_ext, double* __restrict__ grad,
    double* __restrict__ heff, double* __restrict__ part)
{
    __shared__ double red[kBlock];
    const int n = nx * ny;
    const int c = blockIdx.x * kBlock + threadIdx.x;
    double e = 0;
    if (c < n) {
        double g[3] = {0, 0, 0}, h[3] = {0, 0, 0};
        if (mask[c]) {
            const int x = c % nx, y = c / nx;
            const double mc[3] = {m[c], m[n + c], m[2 * n + c]};
            double hex[3] = {0, 0, 0};
            // free surfaces: only neighbours inside the grid and the mask couple
            auto couple = [&](int nb, double w) {
                if (mask[nb])
                    for (int k = 0; k < 3; ++k) hex[k] += w * (m[k * n + nb] - mc[k]);
            };
            if (x > 0) couple(c - 1, cex_x);
            if (x + 1 < nx) couple(c + 1, cex_x);
            if (y > 0) couple(c - nx, cex_y);
            if (y + 1 < ny) couple(c + nx, cex_y);
            const double han[3] = {0, 0, hk * mc[2]};
            const double hext[3] = {hx_ext, hy_ext, hz_ext};
            double mh = 0;
            for (int k = 0; k < 3; ++k) {
                const double quad = hex[k] + han[k] + hd[k * n + c];
                const double lin = hext[k] + hb[k * n + c];
                h[k] = quad + lin;
                e += -0.5 * mc[k] * quad - mc[k] * lin;
                mh += mc[k] * h[k];
            }
            const double ri = rinv[c];
            for (int k = 0; k < 3; ++k) g[k] = -(h[k] - mh * mc[k]) * ri;
        }
        for (int k = 0; k < 3; ++k) {
            grad[k * n + c] = g[k];
            if (heff) heff[k * n + c] = h[k];
        }
    }
    red[threadIdx.x] = e;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_mm_clear(int* __restrict__ flag) { *flag = 0; }

// sum of the block partials (one block, fixed order)
__global__ __launch_bounds__(kBlock) void k_mm_sum(const double* __restrict__ part, int np,
                                                   double* __restrict__ out)
{
    __shared__ double red[kBlock];
    double s = 0;
    for (int i = threadIdx.x; i < np; i += kBlock) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

std::mutex g_mm_mu;
std::unordered_set<const void*> g_mm_live;

}  // namespace

struct hfd_mm_s {
    hfd_plan plan = nullptr;
    int nx = 0, ny = 0, dev = 0, nblk = 0;
    double cex_x = 0, cex_y = 0, hk = 0;
    unsigned char* mask = nullptr;
    double *m = nullptr, *rinv = nullptr, *hd = nullptr, *hb = nullptr, *part = nullptr,
           *sum = nullptr;
    int* bad = nullptr;
};

namespace {

hfd_status mm_free(hfd_mm p)
{
    void* bufs[] = {p->mask, p->m, p->rinv, p->hd, p->hb, p->part, p->sum, p->bad};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    delete p;
    return HFD_OK;
}

hfd_status mm_check(hfd_mm p)
{
    if (!p) return report_error(HFD_EHANDLE, "micromagnetic object is NULL");
    std::lock_guard<std::mutex> lk(g_mm_mu);
    if (!g_mm_live.count(p)) return report_error(HFD_EHANDLE, "unknown or destroyed micromagnetic object");
    return HFD_OK;
}

#define MM_HIP(call)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return report_error(HFD_EHIP, std::string(#call) + " failed: " + hipGetErrorString(e_)); \
    } while (0)

// restores the caller's device on scope exit
struct DevScope {
    int prev = -1;
    hipError_t enter(int dev)
    {
        hipError_t e = hipGetDevice(&prev);
        return e != hipSuccess ? e : hipSetDevice(dev);
    }
    ~DevScope()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace

extern "C" {

hfd_status hfd_mm_create(hfd_mm* out, hfd_plan plan, const unsigned char* mask, double cex_x,
                         double cex_y, double hk, void* stream)
{
    if (!out) return report_error(HFD_EINVAL, "out is NULL");
    *out = nullptr;
    if (!mask) return report_error(HFD_EINVAL, "mask is NULL");
    if (!std::isfinite(cex_x) || !std::isfinite(cex_y) || cex_x < 0 || cex_y < 0 || !std::isfinite(hk))
        return report_error(HFD_EINVAL, "cex_x, cex_y must be finite and >= 0, hk finite");
    hfd_info inf;
    hfd_status st = hfd_get_info(plan, &inf);
    if (st) return st;
    if (inf.nz != 1 || inf.n_geom != 1 || !inf.fp64 || inf.equidistant)
        return report_error(HFD_EINVAL, "the demagnetization plan must be FP64 with one layer and one stack");
    hfd_mm p = new (std::nothrow) hfd_mm_s();
    if (!p) return report_error(HFD_ENOMEM, "host allocation failed");
    p->plan = plan;
    p->nx = inf.nx;
    p->ny = inf.ny;
    p->cex_x = cex_x;
    p->cex_y = cex_y;
    p->hk = hk;
    const size_t n = (size_t)p->nx * p->ny;
    p->nblk = (int)((n + kBlock - 1) / kBlock);
    if (hipGetDevice(&p->dev) != hipSuccess) {
        mm_free(p);
        return report_error(HFD_EHIP, "hipGetDevice failed");
    }
    hipStream_t s = (hipStream_t)stream;
    bool ok = hipMalloc(&p->mask, n) == hipSuccess && hipMalloc(&p->m, 3 * n * 8) == hipSuccess &&
              hipMalloc(&p->rinv, n * 8) == hipSuccess && hipMalloc(&p->hd, 3 * n * 8) == hipSuccess &&
              hipMalloc(&p->hb, 3 * n * 8) == hipSuccess &&
              hipMalloc(&p->part, (size_t)p->nblk * 8) == hipSuccess &&
              hipMalloc(&p->sum, 8) == hipSuccess && hipMalloc(&p->bad, sizeof(int)) == hipSuccess;
    if (!ok) {
        mm_free(p);
        return report_error(HFD_ENOMEM, "device allocation of the micromagnetic workspace failed");
    }
    std::vector<unsigned char> mk(mask, mask + n);
    for (auto& v : mk) v = v ? 1 : 0;
    std::vector<double> zero(3 * n, 0.0);
    ok = hipMemcpyAsync(p->mask, mk.data(), n, hipMemcpyHostToDevice, s) == hipSuccess &&
         hipMemcpyAsync(p->hb, zero.data(), 3 * n * 8, hipMemcpyHostToDevice, s) == hipSuccess &&
         hipStreamSynchronize(s) == hipSuccess;
    if (!ok) {
        mm_free(p);
        return report_error(HFD_EHIP, "upload of the mask failed");
    }
    {
        std::lock_guard<std::mutex> lk(g_mm_mu);
        g_mm_live.insert(p);
    }
    *out = p;
    return HFD_OK;
}

hfd_status hfd_mm_set_bias(hfd_mm p, const double* h_bias, void* stream)
{
    hfd_status st = mm_check(p);
    if (st) return st;
    if (!h_bias) return report_error(HFD_EINVAL, "h_bias is NULL");
    DevScope ds;
    MM_HIP(ds.enter(p->dev));
    MM_HIP(hipMemcpyAsync(p->hb, h_bias, 3 * (size_t)p->nx * p->ny * 8, hipMemcpyDeviceToDevice,
                          (hipStream_t)stream));
    return HFD_OK;
}

hfd_status hfd_mm_energy_grad(hfd_mm p, const double* u, const double* h_ext, double* grad,
                              double* h_eff, double* m_out, double* energy, void* stream)
{
    hfd_status st = mm_check(p);
    if (st) return st;
    if (!u || !h_ext || !grad || !energy) return report_error(HFD_EINVAL, "u, h_ext, grad and energy are required");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(h_ext[k])) return report_error(HFD_EINVAL, "h_ext must be finite");
    const int n = p->nx * p->ny;
    if ((const void*)u == (const void*)grad) return report_error(HFD_EINVAL, "u and grad must not alias");
    DevScope ds;
    MM_HIP(ds.enter(p->dev));
    hipStream_t s = (hipStream_t)stream;
    // the flag is cleared by a kernel (no memset node in captured work)
    hipLaunchKernelGGL(k_mm_clear, dim3(1), dim3(1), 0, s, p->bad);
    hipLaunchKernelGGL(k_mm_normalize, dim3(p->nblk), dim3(kBlock), 0, s, u, p->mask, p->m, p->rinv, n,
                       p->bad);
    MM_HIP(hipGetLastError());
    st = hfd_demag_field(p->plan, p->m, p->hd, 1, stream);
    if (st) return st;
    hipLaunchKernelGGL(k_mm_heff, dim3(p->nblk), dim3(kBlock), 0, s, p->m, p->rinv, p->mask, p->hd,
                       p->hb, p->nx, p->ny, p->cex_x, p->cex_y, p->hk, h_ext[0], h_ext[1], h_ext[2],
                       grad, h_eff, p->part);
    hipLaunchKernelGGL(k_mm_sum, dim3(1), dim3(kBlock), 0, s, p->part, p->nblk, p->sum);
    MM_HIP(hipGetLastError());
    if (m_out) MM_HIP(hipMemcpyAsync(m_out, p->m, 3 * (size_t)n * 8, hipMemcpyDeviceToDevice, s));
    int bad = 0;
    MM_HIP(hipMemcpyAsync(energy, p->sum, 8, hipMemcpyDeviceToHost, s));
    MM_HIP(hipMemcpyAsync(&bad, p->bad, sizeof(int), hipMemcpyDeviceToHost, s));
    MM_HIP(hipStreamSynchronize(s));
    if (bad) return report_error(HFD_EINVAL, "u is the zero vector on a magnetic cell");
    return HFD_OK;
}

hfd_status hfd_mm_destroy(hfd_mm p)
{
    hfd_status st = mm_check(p);
    if (st) return st;
    {
        std::lock_guard<std::mutex> lk(g_mm_mu);
        g_mm_live.erase(p);
    }
    DevScope ds;
    (void)ds.enter(p->dev);
    return mm_free(p);
}

}  // extern "C"
