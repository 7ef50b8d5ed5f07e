// C ABI of the hybrid-FFT demagnetization-field library (include/hfd.h).
// Host logic only: argument validation, plan ownership, tensor setup
// orchestration and kernel dispatch.  All arithmetic runs in the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <iterator>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <unordered_set>
#include <vector>

#include "../../include/hfd.h"
#include "launch.hpp"

using namespace hfd;

namespace hfd {
hipError_t ensure_lds_limit(const void* kernel, int bytes)
{
    if (bytes <= 65536) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, int> done;  // (kernel, device) -> limit set
    std::lock_guard<std::mutex> lk(mu);
    const auto key = std::make_pair(kernel, dev);
    const auto it = done.find(key);
    if (it != done.end() && it->second >= bytes) return hipSuccess;
    e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    done[key] = bytes;
    return hipSuccess;
}
}  // namespace hfd

// Device scratch of hfd_demag_field_noalloc: the x-pass spectra of one call
// (batch * 3 nz * (Lx/2) * ny complex values).  One copy per GPU, held until
// the process ends; its device address is looked up once per device when the
// first plan is created there (plan setup), never taken from the host-side name.
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

thread_local std::string g_err;

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device -> address of `scratch` on that device

hfd_status fail(hfd_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

#define HFD_HIP(call)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (call);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(HFD_EHIP, std::string(#call) + " failed: " + hipGetErrorString(e_)); \
    } while (0)

#define HFD_TRY(expr)                    \
    do {                                 \
        hfd_status st_ = (expr);         \
        if (st_ != HFD_OK) return st_;   \
    } while (0)

constexpr uint64_t kMagic = 0x31414c5044464848ull;
constexpr uint64_t kDead = 0xdeaddeaddeaddeadull;
constexpr unsigned kKnownFlags =
    HFD_FP64 | HFD_MIX_SPLIT_BF16 | HFD_SPLIT_PASSES | HFD_STORE_DTENSOR | HFD_MIX_BATCHED_FP32 |
    HFD_EQUIDISTANT;

int next_pow2(long long v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// safe products for size computations (overflow -> -1)
long long mul_ll(long long a, long long b)
{
    if (a < 0 || b < 0) return -1;
    if (a != 0 && b > (long long)(INT64_MAX / 4) / a) return -1;
    return a * b;
}

struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    hipError_t set(int dev)
    {
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        if (prev != dev) {
            changed = true;
            return hipSetDevice(dev);
        }
        return hipSuccess;
    }
    ~DeviceGuard()
    {
        if (changed) (void)hipSetDevice(prev);
    }
};

}  // namespace

namespace hfd {
// error reporting for the other translation units (hfd_last_error)
hfd_status report_error(hfd_status s, const std::string& msg) { return fail(s, msg); }
}  // namespace hfd

namespace {

// with the device current: record the address of `scratch` on it (once)
hfd_status scratch_init(int dev)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr.count(dev)) return HFD_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(HFD_EHIP, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
    return HFD_OK;
}

void* scratch_ptr(int dev)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    const auto it = g_scratch_ptr.find(dev);
    return it == g_scratch_ptr.end() ? nullptr : it->second;
}

}  // namespace

struct hfd_plan_s {
    uint64_t magic = kMagic;
    int dev = 0;
    int nx = 0, ny = 0, nz = 0, G = 0, batch_max = 0;
    double dx = 0, dy = 0;
    unsigned flags = 0;
    bool fp64 = false, bf16 = false, batched32 = false, fused = false;
    int Lx = 0, Ly = 0, M = 0, QX = 0, QY = 0, P = 0;
    size_t rsz = 4, csz = 8;
    std::vector<double> thick, zbot;  // [G][nz]
    // device
    // Fourier tensor.  Non-equidistant plans: one table of pair slots
    // [QX][nslot][5][QY] (qcs = nslot * 5 * QY elements per kx row, rows in
    // the order kx = 0, M, 1, .., M - 1, see tab_row); pair u of
    // stack g reads slot qslot[g * P + u], and stacks whose pairs have the same
    // geometry (thicknesses and offset) share the slot.  nslot = G * P, so any
    // geometry fits without reallocation.  Equidistant plans: the 3-D tensor.
    void* Q = nullptr;
    long long q_geom_stride = 0;  // elements of one stack's tensor ([QX][P][5][QY], export)
    long long qcs = 0;
    int nslot = 0;
    int nslot_used = 0;           // distinct pair geometries of the current thicknesses
    int* qslot = nullptr;         // device [G][P]
    std::vector<int> qslot_host;
    void* lp = nullptr;         // [G][2][nz]
    void* twx = nullptr;        // plan precision, length Lx
    void* twy = nullptr;        // plan precision, length Ly
    double* twx64 = nullptr;    // FP64 (tensor setup)
    double* twy64 = nullptr;
    void* X1 = nullptr;         // [batch_max][S][M][ny]
    void* Mh = nullptr;         // [batch_max][S][M][Ly]
    void* Hh = nullptr;
    size_t x1_bytes = 0, mh_bytes = 0;
    // thickness-derivative data
    void* D = nullptr;          // [QX][nzeta_max][6][QY] plan precision, one offset table
    int* itab = nullptr;        // [G][itab_stride] interface positions and D slots (k_tgrad)
    int itab_stride = 0;
    double* zeta_dev = nullptr; // [tables][nzeta_max]
    int nzeta_max = 0;
    std::vector<int> nzeta;     // per table (one shared table when stored, else per group)
    std::vector<int> dgroup;    // first stack of each table's group, then G
    std::vector<double> zeta_host;
    std::vector<int> itab_host;
    bool d_valid = false;       // D holds the current geometry (stored mode)
    double* dW = nullptr;       // FP64 quadrants of the derivative lattice [chunk][6][ny][nx]
    void* dF = nullptr;         // their x-pass spectra [chunk][6][Lx/2 + 1][ny]
    double* dscale = nullptr;   // -1/(Lx Ly) per zeta of a chunk
    int dchunk = 0;
    double* partial = nullptr;  // reduction partials [batch_max][ntiles][2 nz]
    int ntiles = 0;
    // equidistant stack: layer sum by FFT along z (path 4)
    bool eq3d = false;
    int Lz = 0;                 // padded length along z
    void* Bc = nullptr;         // [2][batch_max][S][Ly]: split-off column Lx/2 in / out
    void* twz = nullptr;        // plan precision, length Lz
    // field path: 0 fused y-pass, 1 five-pass generic mixing, 2 five-pass batched
    // FP32 mixing, 3 five-pass split-BF16 MFMA mixing, 4 equidistant (z FFT);
    // default from the flags, per-batch choice from hfd_autotune
    int path = 0;
    struct Tune {
        int path, xty;
        int chunk;    // states per launch of the fused path (0: the whole batch)
        int generic;  // fused path: 1 = run-time layer-count kernel instead of the exact one
    };
    std::map<int, Tune> tuned;
    // false while hfd_set_thickness rebuilds the plan and after it failed:
    // field and vjp calls are refused until a later set succeeds
    bool ready = true;
    // tensor-setup scratch, allocated once with the plan (set_thickness reuses it)
    double* sW = nullptr;       // real-space FP64 quadrants [chunk][6][ny][nx]
    void* sF = nullptr;         // their x-pass spectra [chunk][6][Lx/2 + 1][ny]
    void* spg = nullptr;        // pair geometries
    double* sscale = nullptr;   // per pair scale
    double* sQ2 = nullptr;      // equidistant plans: per-offset spectra
    int schunk = 0, spg_cap = 0;
};

namespace {

// live plans; a handle not in this set (never created, or destroyed) is rejected
std::mutex g_plans_mu;
std::unordered_set<const void*> g_plans;

hfd_status check_plan(hfd_plan p)
{
    if (!p) return fail(HFD_EHANDLE, "plan is NULL");
    {
        std::lock_guard<std::mutex> lk(g_plans_mu);
        if (!g_plans.count(p)) return fail(HFD_EHANDLE, "plan handle was destroyed or never created");
    }
    if (p->magic != kMagic) return fail(HFD_EHANDLE, "plan handle is corrupted");
    return HFD_OK;
}

hfd_status check_ready(hfd_plan p)
{
    HFD_TRY(check_plan(p));
    if (!p->ready)
        return fail(HFD_EINVAL, "the plan's tensor is not valid (the last hfd_set_thickness failed): "
                                "call hfd_set_thickness again or destroy the plan");
    return HFD_OK;
}

hfd_status validate_geometry(int nz, int G, const double* thick, const double* zbot,
                             std::vector<double>& t_out, std::vector<double>& z_out)
{
    if (!thick) return fail(HFD_EINVAL, "thickness is NULL");
    t_out.assign(thick, thick + (size_t)G * nz);
    z_out.resize((size_t)G * nz);
    for (int g = 0; g < G; ++g) {
        for (int l = 0; l < nz; ++l) {
            const double t = t_out[(size_t)g * nz + l];
            if (!std::isfinite(t) || !(t > 0.0))
                return fail(HFD_EINVAL, "thickness[" + std::to_string(g) + "][" + std::to_string(l) +
                                            "] must be finite and > 0");
        }
        if (zbot) {
            for (int l = 0; l < nz; ++l) {
                const double z = zbot[(size_t)g * nz + l];
                if (!std::isfinite(z)) return fail(HFD_EINVAL, "z_bottom must be finite");
                z_out[(size_t)g * nz + l] = z;
            }
            for (int l = 0; l + 1 < nz; ++l) {
                const double top = z_out[(size_t)g * nz + l] + t_out[(size_t)g * nz + l];
                const double nb = z_out[(size_t)g * nz + l + 1];
                const double tol = 1e-9 * std::max({std::fabs(top), std::fabs(nb), 1e-300}) +
                                   1e-12 * t_out[(size_t)g * nz + l];
                if (nb < top - tol)
                    return fail(HFD_EINVAL, "layers overlap: z_bottom[" + std::to_string(g) + "][" +
                                                std::to_string(l + 1) + "] is below the top of layer " +
                                                std::to_string(l) +
                                                " (layers must be ordered bottom to top and may touch)");
            }
        } else {
            double acc = 0.0;
            for (int l = 0; l < nz; ++l) {
                z_out[(size_t)g * nz + l] = acc;
                acc += t_out[(size_t)g * nz + l];
            }
        }
    }
    return HFD_OK;
}

template <typename T>
hfd_status dev_alloc(T** p, size_t bytes, const char* what)
{
    *p = nullptr;
    if (bytes == 0) return HFD_OK;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(HFD_ENOMEM, std::string("hipMalloc of ") + std::to_string(bytes) + " bytes for " +
                                    what + " failed: " + hipGetErrorString(e));
    }
    *p = (T*)q;
    return HFD_OK;
}

void free_plan_memory(hfd_plan p)
{
    if (p->twx == p->twx64) p->twx = nullptr;  // FP64 plans share the FP64 tables
    if (p->twy == p->twy64) p->twy = nullptr;
    void* bufs[] = {p->Q, p->lp, p->twx, p->twy, p->twx64, p->twy64, p->X1, p->Mh, p->Hh,
                    p->D, p->itab, p->zeta_dev, p->partial, p->dW, p->dF, p->dscale, p->Bc, p->twz,
                    p->sW, p->sF, p->spg, p->sscale, p->sQ2, p->qslot};
    for (void* b : bufs)
        if (b) (void)hipFree(b);
    p->dW = nullptr;
    p->dF = nullptr;
    p->dscale = nullptr;
    p->Q = p->lp = p->twx = p->twy = p->X1 = p->Mh = p->Hh = nullptr;
    p->twx64 = p->twy64 = nullptr;
    p->D = nullptr;
    p->itab = nullptr;
    p->zeta_dev = nullptr;
    p->partial = nullptr;
    p->Bc = p->twz = nullptr;
    p->sW = nullptr;
    p->sF = nullptr;
    p->spg = nullptr;
    p->sscale = nullptr;
    p->sQ2 = nullptr;
    p->qslot = nullptr;
}

// twiddle table exp(-2 pi i m / L), m in [0, L), in FP64 (exact octant reduction)
std::vector<double> twiddles(int L)
{
    std::vector<double> t(2 * (size_t)L);
    for (int m = 0; m < L; ++m) {
        // angle = 2 pi m / L; use sin/cos of reduced arguments for accuracy
        const long double a = 2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)L;
        t[2 * (size_t)m] = (double)cosl(a);
        t[2 * (size_t)m + 1] = (double)-sinl(a);
    }
    return t;
}

hfd_status upload_twiddles(hfd_plan p, hipStream_t s)
{
    auto tx = twiddles(p->Lx), ty = twiddles(p->Ly);
    HFD_TRY(dev_alloc(&p->twx64, tx.size() * 8, "twiddles"));
    HFD_TRY(dev_alloc(&p->twy64, ty.size() * 8, "twiddles"));
    HFD_HIP(hipMemcpyAsync(p->twx64, tx.data(), tx.size() * 8, hipMemcpyHostToDevice, s));
    HFD_HIP(hipMemcpyAsync(p->twy64, ty.data(), ty.size() * 8, hipMemcpyHostToDevice, s));
    if (p->eq3d) {  // z-transform table in the plan precision (both precisions)
        auto tz = twiddles(p->Lz);
        if (p->fp64) {
            HFD_TRY(dev_alloc(&p->twz, tz.size() * 8, "twiddles"));
            HFD_HIP(hipMemcpyAsync(p->twz, tz.data(), tz.size() * 8, hipMemcpyHostToDevice, s));
        } else {
            std::vector<float> fz(tz.begin(), tz.end());
            HFD_TRY(dev_alloc(&p->twz, fz.size() * 4, "twiddles"));
            HFD_HIP(hipMemcpyAsync(p->twz, fz.data(), fz.size() * 4, hipMemcpyHostToDevice, s));
        }
        HFD_HIP(hipStreamSynchronize(s));
    }
    if (p->fp64) {
        p->twx = p->twx64;
        p->twy = p->twy64;
        HFD_HIP(hipStreamSynchronize(s));
        return HFD_OK;
    }
    std::vector<float> fx(tx.begin(), tx.end()), fy(ty.begin(), ty.end());
    HFD_TRY(dev_alloc(&p->twx, fx.size() * 4, "twiddles"));
    HFD_TRY(dev_alloc(&p->twy, fy.size() * 4, "twiddles"));
    HFD_HIP(hipMemcpyAsync(p->twx, fx.data(), fx.size() * 4, hipMemcpyHostToDevice, s));
    HFD_HIP(hipMemcpyAsync(p->twy, fy.data(), fy.size() * 4, hipMemcpyHostToDevice, s));
    HFD_HIP(hipStreamSynchronize(s));
    return HFD_OK;
}

// Bytes per pair (or offset) of the FP64 quadrant tables [6][ny][nx] and of
// their x-pass spectra [6][Lx/2 + 1][ny] (reals).
static long long quadrant_bytes(hfd_plan p) { return 6LL * p->nx * p->ny * 8; }
static long long xspectra_bytes(hfd_plan p) { return 6LL * (p->M + 1) * p->ny * 8; }

// Tensor-setup scratch, allocated once per plan: quadrant tables and their
// x-pass spectra for a chunk of pair geometries (256 MB each at most), the
// pair list and scales, and for equidistant plans the per-offset spectra.
hfd_status alloc_setup_scratch(hfd_plan p)
{
    const long long per_pair = std::max(quadrant_bytes(p), xspectra_bytes(p));
    // distinct geometries of all stacks, at most
    const int ngeo = (int)std::max((long long)p->G * p->P, 2LL * p->nz - 1);
    const long long budget = 256LL << 20;
    p->schunk = (int)std::max(1LL, std::min<long long>(ngeo, budget / per_pair));
    p->spg_cap = ngeo;
    HFD_TRY(dev_alloc(&p->sW, (size_t)p->schunk * quadrant_bytes(p), "tensor setup (real space)"));
    HFD_TRY(dev_alloc(&p->sF, (size_t)p->schunk * xspectra_bytes(p), "tensor setup (spectra)"));
    HFD_TRY(dev_alloc(&p->spg, sizeof(PairGeoH) * (size_t)ngeo, "pair table"));
    HFD_TRY(dev_alloc(&p->sscale, sizeof(double) * (size_t)ngeo, "pair scales"));
    if (p->eq3d)
        HFD_TRY(dev_alloc(&p->sQ2, sizeof(double) * 6 * (size_t)p->QX * p->QY * (2 * p->nz - 1),
                          "per-offset spectra"));
    return HFD_OK;
}

static double max_thickness(const std::vector<PairGeoH>& geos, int first, int count)
{
    double t = 0.0;
    for (int u = first; u < first + count; ++u) t = std::max(t, std::max(geos[u].ti, geos[u].tj));
    return t;
}

// FP64 x-pass spectra of the real-space tensor quadrants (6 components each)
// of the cuboid-pair geometries `geos`, in chunks of the plan's setup scratch;
// after each chunk pack(first, count, F) enqueues the y transforms and packing
// (launch_ytab) of spectra F[count][6][M + 1][ny] (reals, launch_xtab).
// Synchronizes the stream at the end.

template <class Pack>
hfd_status tensor_spectra(hfd_plan p, const std::vector<PairGeoH>& geos, hipStream_t s, Pack pack)
{
    const int n = (int)geos.size();
    if (n > p->spg_cap) return fail(HFD_EINVAL, "internal: more pair geometries than the setup scratch holds");
    const int CP = p->schunk;
    double* W = p->sW;
    void* F = p->sF;
    PairGeoH* pg = (PairGeoH*)p->spg;
    hipError_t e = hipMemcpyAsync(pg, geos.data(), sizeof(PairGeoH) * n, hipMemcpyHostToDevice, s);
    for (int u0 = 0; u0 < n && e == hipSuccess; u0 += CP) {
        const int np = std::min(CP, n - u0);
        // quadrants; the transforms extend them by parity
        e = launch_tensor_real(W, pg + u0, np, p->nx, p->ny, p->Lx, p->Ly, p->dx, p->dy,
                               max_thickness(geos, u0, np), 2, s);
        if (e == hipSuccess) e = launch_xtab(p->Lx, W, F, p->nx, p->ny, np * 6, p->twx64, s);
        if (e == hipSuccess) e = pack(u0, np, (const double*)F);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(HFD_EHIP, std::string("tensor setup: ") + hipGetErrorString(e));
    return HFD_OK;
}

// Build the Fourier tensor of every stack (FP64 setup, stored in plan precision).
// Every distinct pair geometry (thicknesses and offset) of all stacks is
// computed once and stored in one slot: pairs at the same layer distance of an
// equal-thickness stack, and the pairs that thickness candidates of one stack
// have in common, share it.
hfd_status build_tensor(hfd_plan p, hipStream_t s)
{
    const long long plane = (long long)p->Lx * p->Ly;
    double* scale = p->sscale;
    hfd_status st = HFD_OK;
    std::vector<PairGeoH> ug;
    std::vector<double> hs;
    std::map<std::tuple<double, double, double>, int> seen;
    p->qslot_host.assign((size_t)p->G * p->P, 0);
    for (int g = 0; g < p->G; ++g) {
        const double* t = &p->thick[(size_t)g * p->nz];
        const double* z = &p->zbot[(size_t)g * p->nz];
        int u = 0;
        for (int i = 0; i < p->nz; ++i)
            for (int j = i; j < p->nz; ++j, ++u) {
                const auto key = std::make_tuple(t[i], t[j], z[i] - z[j]);
                auto it = seen.find(key);
                if (it == seen.end()) {
                    it = seen.emplace(key, (int)ug.size()).first;
                    ug.push_back({t[i], t[j], z[i] - z[j], 0.0});
                    hs.push_back(-t[i] / (double)plane);
                }
                p->qslot_host[(size_t)g * p->P + u] = it->second;
            }
    }
    if (hipMemcpyAsync(scale, hs.data(), sizeof(double) * hs.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(p->qslot, p->qslot_host.data(), sizeof(int) * p->qslot_host.size(),
                       hipMemcpyHostToDevice, s) != hipSuccess)
        st = fail(HFD_EHIP, "tensor setup: scale or slot upload failed");
    if (st == HFD_OK)
        st = tensor_spectra(p, ug, s, [&](int u0, int np, const double* F) -> hipError_t {
            return launch_ytab(p->fp64, F, p->Q, scale + u0, np, 5, p->M, p->ny, p->Ly, p->QX, p->QY, u0,
                               p->nslot, 1, p->twy64, s);
        });
    if (st == HFD_OK) p->nslot_used = (int)ug.size();
    (void)hipStreamSynchronize(s);
    if (st) return st;
    // layer parameters: 1/t and the self-pair trace -t/(Lx Ly)
    std::vector<double> lp((size_t)p->G * 2 * p->nz);
    for (int g = 0; g < p->G; ++g)
        for (int l = 0; l < p->nz; ++l) {
            const double t = p->thick[(size_t)g * p->nz + l];
            lp[((size_t)g * 2) * p->nz + l] = 1.0 / t;
            lp[((size_t)g * 2 + 1) * p->nz + l] = -t / (double)plane;
        }
    hipError_t e;
    if (p->fp64) {
        e = hipMemcpyAsync(p->lp, lp.data(), lp.size() * 8, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    } else {
        std::vector<float> lf(lp.begin(), lp.end());
        e = hipMemcpyAsync(p->lp, lf.data(), lf.size() * 4, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e != hipSuccess) return fail(HFD_EHIP, std::string("tensor setup: ") + hipGetErrorString(e));
    p->d_valid = false;
    return HFD_OK;
}

// Equidistant stack: the 2D spectra of N(d) for the 2nz - 1 layer offsets d
// (FP64, all 6 components on the quadrant), then the transform along z to the
// real 3-D Fourier tensor [kx][kz][6][ky] (eq. FFT_3D), scaled by -1/(Lx Ly Lz).
hfd_status build_tensor3d(hfd_plan p, hipStream_t s)
{
    const long long plane = (long long)p->Lx * p->Ly;
    const int nd = 2 * p->nz - 1;
    const double t = p->thick[0];
    const double pitch = p->nz > 1 ? p->zbot[1] - p->zbot[0] : t;
    std::vector<PairGeoH> geos((size_t)nd);
    for (int k = 0; k < nd; ++k) geos[k] = {t, t, (double)(k - (p->nz - 1)) * pitch, 0.0};
    std::vector<double> hs((size_t)nd, -1.0 / (double)plane);
    double* scale = p->sscale;
    double* Q2 = p->sQ2;
    const size_t per = (size_t)6 * p->QX * p->QY;
    hfd_status st = HFD_OK;
    if (hipMemcpyAsync(scale, hs.data(), sizeof(double) * nd, hipMemcpyHostToDevice, s) != hipSuccess)
        st = fail(HFD_EHIP, "tensor setup: scale upload failed");
    if (st == HFD_OK)
        st = tensor_spectra(p, geos, s, [&](int u0, int np, const double* F) -> hipError_t {
            return launch_ytab(true, F, Q2 + (size_t)u0 * per, scale + u0, np, 6, p->M, p->ny, p->Ly,
                               p->QX, p->QY, 0, np, 0, p->twy64, s);
        });
    if (st == HFD_OK) {
        hipError_t e = launch_zdft3(p->fp64, Q2, p->Q, p->nz, p->Lz, p->QX, p->QY, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = fail(HFD_EHIP, std::string("tensor setup: ") + hipGetErrorString(e));
    }
    (void)hipStreamSynchronize(s);
    return st;
}

// Equal thicknesses and a uniform pitch (relative tolerance 1e-12), one stack.
hfd_status check_equidistant(int nz, int G, const std::vector<double>& t, const std::vector<double>& z)
{
    if (G != 1) return fail(HFD_EINVAL, "HFD_EQUIDISTANT needs n_geom = 1");
    for (int l = 1; l < nz; ++l)
        if (std::fabs(t[l] - t[0]) > 1e-12 * t[0])
            return fail(HFD_EINVAL, "HFD_EQUIDISTANT needs equal thicknesses");
    if (nz > 2) {
        const double p0 = z[1] - z[0];
        for (int l = 2; l < nz; ++l) {
            const double pl = z[l] - z[l - 1];
            if (std::fabs(pl - p0) > 1e-12 * std::max(std::fabs(z[l]), p0))
                return fail(HFD_EINVAL, "HFD_EQUIDISTANT needs a uniform pitch z_bottom[l+1] - z_bottom[l]");
        }
    }
    return HFD_OK;
}


// Distinct offsets |zeta| = |(interface of the target) - (interface of the
// source)| over all ordered layer pairs, merged when equal to 1e-12 relative
// (D(-zeta) is D(zeta) with xx, yy, zz, xy negated: those derivatives are odd
// in zeta, xz and yz even), and per geometry the table of k_tgrad: interface
// positions (top_l and bot_{l+1} merged when they touch), their ranks, the
// position of every layer's bottom and top, and for every position pair the
// D slot of |z_p - z_q| times 2, plus 1 when z_p < z_q.
// sorted distinct |offsets| of stacks g0 .. g1-1 (the four interface
// differences of every ordered layer pair), values within rounding of zero
// snapped to exactly zero (touching interfaces)
static std::vector<double> distinct_offsets(hfd_plan p, int g0, int g1)
{
    const int nz = p->nz;
    std::vector<double> u;
    double sc = 0.0;
    for (int g = g0; g < g1; ++g) {
        const double* t = &p->thick[(size_t)g * nz];
        const double* z = &p->zbot[(size_t)g * nz];
        for (int l = 0; l < nz; ++l) sc = std::max(sc, std::fabs(z[l]) + t[l]);
        for (int i = 0; i < nz; ++i)
            for (int j = 0; j < nz; ++j) {
                const double ti = z[i] + t[i], bi = z[i], tj = z[j] + t[j], bj = z[j];
                u.insert(u.end(), {std::fabs(ti - bj), std::fabs(bi - bj), std::fabs(ti - tj),
                                   std::fabs(bi - tj)});
            }
    }
    std::sort(u.begin(), u.end());
    std::vector<double> m;
    for (double v : u) {
        if (!m.empty() && std::fabs(v - m.back()) <= 1e-12 * std::max(1.0, std::fabs(v))) continue;
        m.push_back(v);
    }
    for (double& v : m)
        if (std::fabs(v) <= 1e-12 * std::max(1.0, sc)) v = 0.0;
    return m;
}

// Groups of consecutive stacks that share one offset table: all stacks in one
// group when stored; otherwise stacks are added to a group while the union of
// their offsets stays within cap slots (a stack alone may exceed it).
// Returns the first stack of every group, then G.
static std::vector<int> derivative_groups(hfd_plan p, bool shared, int cap)
{
    std::vector<int> first{0};
    if (!shared) {
        std::vector<double> cur;
        for (int g = 0; g < p->G; ++g) {
            const std::vector<double> own = distinct_offsets(p, g, g + 1);
            std::vector<double> merged;
            std::merge(cur.begin(), cur.end(), own.begin(), own.end(), std::back_inserter(merged));
            std::vector<double> m;
            for (double v : merged)
                if (m.empty() || std::fabs(v - m.back()) > 1e-12 * std::max(1.0, std::fabs(v)))
                    m.push_back(v);
            if (g > first.back() && (int)m.size() > cap) {
                first.push_back(g);
                cur = own;
            } else {
                cur.swap(m);
            }
        }
    }
    first.push_back(p->G);
    return first;
}

// Offset tables of the groups `first` and the interface table itab of every
// stack, whose pair entries index its group's table.
void derivative_offsets(hfd_plan p, const std::vector<int>& first, std::vector<double>& zeta,
                        std::vector<int>& itab, std::vector<int>& count, int& nmax)
{
    const int nz = p->nz, G = p->G;
    const ITabLayout lay = itab_layout(nz);
    const int stride = lay.stride;
    itab.assign((size_t)G * stride, 0);
    auto geo = [&](int g, const double*& t, const double*& z) {
        t = &p->thick[(size_t)g * nz];
        z = &p->zbot[(size_t)g * nz];
    };
    auto scale_of = [&](int g) {
        const double *t, *z;
        geo(g, t, z);
        double sc = 0.0;
        for (int l = 0; l < nz; ++l) sc = std::max(sc, std::fabs(z[l]) + t[l]);
        return sc;
    };
    std::vector<std::vector<double>> tables;
    std::vector<int> table_of((size_t)G);
    for (size_t k = 0; k + 1 < first.size(); ++k) {
        tables.push_back(distinct_offsets(p, first[k], first[k + 1]));
        for (int g = first[k]; g < first[k + 1]; ++g) table_of[(size_t)g] = (int)k;
    }
    for (int g = 0; g < G; ++g) {
        const double *t, *z;
        geo(g, t, z);
        const std::vector<double>& m = tables[(size_t)table_of[(size_t)g]];
        const double ztol = 1e-12 * std::max(1.0, scale_of(g));
        auto nearest = [&](double v) {
            const auto it = std::lower_bound(m.begin(), m.end(), v);
            int k = (int)(it - m.begin());
            if (k == (int)m.size() || (k > 0 && std::fabs(m[k - 1] - v) <= std::fabs(m[k] - v))) --k;
            return k;
        };
        // interface positions bottom to top
        int* tab = &itab[(size_t)g * stride];
        int* pinfo = tab + lay.info;
        int* pbot = tab + lay.pbot;
        int* ptop = tab + lay.ptop;
        int* zpq = tab + lay.zpq;
        std::vector<double> pz;
        for (int l = 0; l < nz; ++l) {
            if (l > 0 && std::fabs(z[l] - pz.back()) <= ztol) {
                pinfo[pz.size() - 1] |= 2;  // bottom of l on the top of l - 1 (rank l)
            } else {
                pinfo[pz.size()] = l * 4 + 2;
                pz.push_back(z[l]);
            }
            pbot[l] = (int)pz.size() - 1;
            pinfo[pz.size()] = (l + 1) * 4 + 1;
            ptop[l] = (int)pz.size();
            pz.push_back(z[l] + t[l]);
        }
        const int NI = (int)pz.size();
        tab[0] = NI;
        for (int a = 0; a < NI; ++a)
            for (int c = 0; c < NI; ++c) {
                const double v = pz[a] - pz[c];
                const int k = nearest(std::fabs(v));
                zpq[a * lay.nsp + c] = 2 * k + (v < 0.0 && m[k] != 0.0 ? 1 : 0);
            }
    }
    const int T = (int)tables.size();
    count.assign(T, 0);
    nmax = 0;
    for (int k = 0; k < T; ++k) {
        count[k] = (int)tables[k].size();
        nmax = std::max(nmax, count[k]);
    }
    zeta.assign((size_t)T * nmax, 0.0);
    for (int k = 0; k < T; ++k)
        for (int i = 0; i < count[k]; ++i) zeta[(size_t)k * nmax + i] = tables[k][i];
}

// derivative spectra one recomputed table may hold (see setup_derivatives)
constexpr long long kRecomputeBytes = 256LL << 20;

// Allocate (or grow) the derivative buffers and upload the offsets.  New
// buffers are allocated before the old ones are released, so a failure leaves
// the previous buffers in place (the plan is then marked not ready by the
// caller).  Buffers only grow: a geometry with fewer distinct offsets keeps
// the allocated stride nzeta_max.
hfd_status setup_derivatives(hfd_plan p, hipStream_t s)
{
    std::vector<double> zeta;
    std::vector<int> itab, count;
    int nmax = 0;
    // stored: one table shared by all stacks; recomputed: one table per group
    // of stacks, built into the same buffer before that group's reduction.  A
    // group's table holds up to kRecomputeBytes of spectra (or one stack's
    // table where that is larger): neighbouring stacks (thickness candidates)
    // share most offsets, and each shared offset is built once per group.
    const bool stored = (p->flags & HFD_STORE_DTENSOR) != 0;
    const long long slot_bytes = 6LL * p->QX * p->QY * p->rsz;
    const int cap = (int)std::max(1LL, kRecomputeBytes / slot_bytes);
    const std::vector<int> first = derivative_groups(p, stored, cap);
    derivative_offsets(p, first, zeta, itab, count, nmax);
    auto swap_in = [](auto*& slot, auto* fresh) {
        if (slot) (void)hipFree(slot);
        slot = fresh;
    };
    if (nmax > p->nzeta_max || !p->D) {
        const long long per_table = (long long)nmax * 6 * p->QX * p->QY;
        void* nD = nullptr;
        double* nz_dev = nullptr;
        HFD_TRY(dev_alloc(&nD, (size_t)per_table * p->rsz, "derivative tensor"));
        hfd_status st = dev_alloc(&nz_dev, sizeof(double) * count.size() * (size_t)nmax,
                                  "derivative offsets");
        if (st) { (void)hipFree(nD); return st; }
        swap_in(p->D, nD);
        swap_in(p->zeta_dev, nz_dev);
        p->nzeta_max = nmax;
    }
    if (!p->itab) HFD_TRY(dev_alloc(&p->itab, sizeof(int) * itab.size(), "interface table"));
    p->itab_stride = itab_layout(p->nz).stride;
    const long long plane = (long long)p->Lx * p->Ly;
    const long long per_z = std::max(quadrant_bytes(p), xspectra_bytes(p));
    const int chunk = (int)std::max(1LL, std::min<long long>(nmax, (256LL << 20) / per_z));
    if (chunk > p->dchunk) {
        double *nW = nullptr, *nsc = nullptr;
        void* nF = nullptr;
        hfd_status st = dev_alloc(&nW, (size_t)chunk * per_z, "derivative scratch");
        if (st == HFD_OK) st = dev_alloc(&nF, (size_t)chunk * per_z, "derivative scratch");
        if (st == HFD_OK) st = dev_alloc(&nsc, sizeof(double) * chunk, "derivative scale");
        if (st) {
            if (nW) (void)hipFree(nW);
            if (nF) (void)hipFree(nF);
            return st;
        }
        swap_in(p->dW, nW);
        swap_in(p->dF, nF);
        swap_in(p->dscale, nsc);
        std::vector<double> sc((size_t)chunk, -1.0 / (double)plane);
        HFD_HIP(hipMemcpyAsync(p->dscale, sc.data(), sizeof(double) * chunk, hipMemcpyHostToDevice, s));
        p->dchunk = chunk;
    }
    // offsets of table k at k * nzeta_max (the allocated stride, which stays
    // larger than nmax when a new geometry has fewer distinct offsets)
    p->zeta_host.assign(count.size() * (size_t)p->nzeta_max, 0.0);
    for (size_t k = 0; k < count.size(); ++k)
        for (int i = 0; i < count[k]; ++i) p->zeta_host[k * p->nzeta_max + i] = zeta[k * nmax + i];
    p->itab_host = itab;
    p->nzeta = count;
    p->dgroup = first;
    HFD_HIP(hipMemcpyAsync(p->zeta_dev, p->zeta_host.data(), sizeof(double) * p->zeta_host.size(),
                           hipMemcpyHostToDevice, s));
    HFD_HIP(hipMemcpyAsync(p->itab, p->itab_host.data(), sizeof(int) * itab.size(),
                           hipMemcpyHostToDevice, s));
    // partial sums of the reduction
    const int ntiles = tgrad_tiles(p->M, p->Ly);
    if (ntiles != p->ntiles || !p->partial) {
        double* np_ = nullptr;
        HFD_TRY(dev_alloc(&np_, sizeof(double) * (size_t)p->batch_max * ntiles * 2 * p->nz,
                          "reduction partials"));
        swap_in(p->partial, np_);
        p->ntiles = ntiles;
    }
    HFD_HIP(hipStreamSynchronize(s));
    p->d_valid = false;
    return HFD_OK;
}

// D(|zeta|) of offset table k (the shared table when stored, else group k)
// into p->D: FP64 quadrant of the lateral-stencilled z-derivative, FP64 2D
// transforms by parity, packed to plan precision.
hfd_status compute_derivatives(hfd_plan p, int g, hipStream_t s)
{
    const int nzt = p->nzeta[g];
    char* dst = (char*)p->D;
    for (int z0 = 0; z0 < nzt; z0 += p->dchunk) {
        const int nc = std::min(p->dchunk, nzt - z0);
        HFD_HIP(launch_dtensor_real(p->dW, p->zeta_dev + (size_t)g * p->nzeta_max + z0, nc, p->nx,
                                    p->ny, p->dx, p->dy, s));
        HFD_HIP(launch_xtab(p->Lx, p->dW, p->dF, p->nx, p->ny, nc * 6, p->twx64, s));
        HFD_HIP(launch_ytab(p->fp64, p->dF, dst, p->dscale, nc, 6, p->M, p->ny, p->Ly, p->QX, p->QY, z0,
                            p->nzeta_max, 1, p->twy64, s));
    }
    return HFD_OK;
}

hfd_status check_field_args(hfd_plan p, const void* a, const void* b, int batch, const char* na,
                            const char* nb)
{
    if (!a) return fail(HFD_EINVAL, std::string(na) + " is NULL");
    if (!b) return fail(HFD_EINVAL, std::string(nb) + " is NULL");
    if (((uintptr_t)a & 15) || ((uintptr_t)b & 15))
        return fail(HFD_EINVAL, std::string(na) + " and " + nb + " must be 16-byte aligned");
    if (batch < 1) return fail(HFD_EINVAL, "batch must be >= 1");
    if (batch > p->batch_max)
        return fail(HFD_EBATCH, "batch " + std::to_string(batch) + " exceeds batch_max " +
                                    std::to_string(p->batch_max));
    if (batch % p->G)
        return fail(HFD_EINVAL, "batch must be a multiple of n_geom (" + std::to_string(p->G) + ")");
    const size_t bytes = (size_t)batch * 3 * p->nz * p->ny * p->nx * p->rsz;
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    if (a0 < b0 + bytes && b0 < a0 + bytes)
        return fail(HFD_EINVAL, std::string(na) + " and " + nb + " overlap");
    return HFD_OK;
}

int path_for(hfd_plan p, int batch)
{
    auto it = p->tuned.find(batch);
    return it != p->tuned.end() ? it->second.path : p->path;
}

// rows per block of the x passes: the tuned choice, else the largest compiled
// tile that still gives every CU at least one block
int xty_for(hfd_plan p, int batch)
{
    auto it = p->tuned.find(batch);
    if (it != p->tuned.end()) return it->second.xty;
    const long long rows = (long long)batch * 3 * p->nz * p->ny;
    int best = 0;
    for (int ty : {8, 16, 24, 32})
        if (x_tile_supported(p->fp64, p->Lx, ty) && (rows + ty - 1) / ty >= 256) best = ty;
    return best;
}

// Fused path, batch split into runs of `chunk` states launched one after the
// other (x pass, y pass, inverse x pass per run), so that the x-pass spectra
// of a run stay in the Infinity Cache between the three kernels.  A run lies
// inside one stack or covers whole stacks.
bool chunk_ok(hfd_plan p, int batch, int chunk)
{
    const int bpg = batch / p->G;
    return chunk >= 1 && chunk <= batch && batch % chunk == 0 &&
           (bpg % chunk == 0 || chunk % bpg == 0);
}

bool generic_for(hfd_plan p, int batch)
{
    auto it = p->tuned.find(batch);
    return it != p->tuned.end() && it->second.generic;
}

int chunk_for(hfd_plan p, int batch)
{
    auto it = p->tuned.find(batch);
    if (it != p->tuned.end() && it->second.chunk > 0 && chunk_ok(p, batch, it->second.chunk))
        return it->second.chunk;
    return batch;
}

const char* path_name(int path)
{
    switch (path) {
    case 0: return "fused";
    case 1: return "five_pass";
    case 2: return "five_pass_batched_fp32";
    case 3: return "five_pass_bf16_mfma";
    default: return "equidistant_z_fft";
    }
}

// Enqueue the field passes.  stage_ev: optional events recorded after each stage.
// `only` >= 0 launches the kernels of that stage alone (stage timing).
hfd_status run_field(hfd_plan p, const void* in, void* out, int batch, int adjoint, hipStream_t s,
                     hipEvent_t* stage_ev = nullptr, int* nstage = nullptr, int path = -1,
                     int only = -1, int xty = -1, void* x1 = nullptr, int chunk = -1,
                     int generic = -1)
{
    const bool gen = generic < 0 ? generic_for(p, batch) : generic != 0;
    if (!x1) x1 = p->X1;
    const int S = 3 * p->nz;
    const int nsig = batch * S;
    const int bpg = batch / p->G;
    if (path < 0) path = path_for(p, batch);
    if (xty < 0) xty = xty_for(p, batch);
    if (chunk < 0) chunk = chunk_for(p, batch);
    if (path == 0 && chunk < batch && chunk_ok(p, batch, chunk) && !stage_ev && only < 0) {
        // state-ordered runs of the fused path (see chunk_ok); one x-pass
        // buffer of `chunk` states is reused by every run
        const size_t state = (size_t)S * p->ny * p->nx * p->rsz;
        for (int b0 = 0; b0 < batch; b0 += chunk) {
            const int g0 = b0 / bpg;
            const int bpg_c = bpg >= chunk ? chunk : bpg;
            const char* in_c = (const char*)in + (size_t)b0 * state;
            char* out_c = (char*)out + (size_t)b0 * state;
            const int* qs_c = p->qslot + (size_t)g0 * p->P;
            const char* lp_c = (const char*)p->lp + (size_t)g0 * 2 * p->nz * p->rsz;
            HFD_HIP(launch_xfwd(p->fp64, p->Lx, in_c, x1, p->nx, p->ny, (long long)p->ny * p->nx,
                                p->nx, chunk * S, p->twx, s, xty));
            HFD_HIP(launch_fused(p->fp64, p->Ly, p->nz, x1, p->ny, p->M, chunk, p->Q, p->qcs, qs_c,
                                 p->QX, p->QY, lp_c, bpg_c, adjoint, p->twy, s,
                                 gen));
            HFD_HIP(launch_xinv(p->fp64, p->Lx, x1, out_c, p->nx, p->ny, (long long)p->ny * p->nx,
                                p->nx, chunk * S, p->twx, s, xty));
        }
        if (nstage) *nstage = 3;
        return HFD_OK;
    }
    if ((path == 2 || path == 3) && !mix_batched_supported(p->nz, batch, p->G)) path = 1;
    int k = 0;
    auto mark = [&]() {
        if (stage_ev) (void)hipEventRecord(stage_ev[k], s);
        ++k;
    };
    auto on = [&]() { return only < 0 || only == k; };
    if (on())
        HFD_HIP(launch_xfwd(p->fp64, p->Lx, in, x1, p->nx, p->ny, (long long)p->ny * p->nx, p->nx,
                            nsig, p->twx, s, xty));
    mark();
    if (path == 0) {
        if (on())
            HFD_HIP(launch_fused(p->fp64, p->Ly, p->nz, x1, p->ny, p->M, batch, p->Q, p->qcs,
                                 p->qslot, p->QX, p->QY, p->lp, bpg, adjoint, p->twy, s,
                                 gen));
        mark();
    } else {
        const long long ncols = (long long)nsig * p->M;
        if (on()) HFD_HIP(launch_yfwd(p->fp64, p->Ly, x1, p->Mh, p->ny, ncols, p->twy, s));
        mark();
        if (on()) {
            if (path == 4) {
                // equidistant: unpack the packed column, z pass, repack
                char* bc = (char*)p->Bc;
                char* hbc = bc + (size_t)p->batch_max * 3 * p->nz * p->Ly * p->csz;
                HFD_HIP(launch_eq3d_mix(p->fp64, p->Lz, p->Mh, bc, p->Hh, hbc, p->nz, p->M, p->Ly,
                                        batch, p->Q, p->QY, p->twz, s));
            } else if (path == 2 || path == 3) {
                // packed column by the generic kernel, the rest batched
                HFD_HIP(launch_mix_generic(p->fp64, p->Mh, p->Hh, p->nz, p->M, p->Ly, batch, p->Q,
                                           p->qcs, p->qslot, p->QX, p->QY, p->lp, bpg, adjoint, 0, 1,
                                           s));
                HFD_HIP(launch_mix_batched(path == 3, p->Mh, p->Hh, p->nz, p->M, p->Ly, batch, p->Q,
                                           p->qcs, p->qslot, p->QY, p->lp, bpg, adjoint, s));
            } else {
                HFD_HIP(launch_mix_generic(p->fp64, p->Mh, p->Hh, p->nz, p->M, p->Ly, batch, p->Q,
                                           p->qcs, p->qslot, p->QX, p->QY, p->lp, bpg, adjoint, 0,
                                           p->M, s));
            }
        }
        mark();
        if (on()) HFD_HIP(launch_yinv(p->fp64, p->Ly, p->Hh, x1, p->ny, ncols, p->twy, s));
        mark();
    }
    if (on())
        HFD_HIP(launch_xinv(p->fp64, p->Lx, x1, out, p->nx, p->ny, (long long)p->ny * p->nx, p->nx,
                            nsig, p->twx, s, xty));
    mark();
    if (nstage) *nstage = k;
    return HFD_OK;
}

std::string stage_names(int path)
{
    switch (path) {
    case 0: return "xfwd;ymix_fused;xinv";
    case 1: return "xfwd;yfwd;mix;yinv;xinv";
    case 2: return "xfwd;yfwd;mix_batched_fp32;yinv;xinv";
    case 3: return "xfwd;yfwd;mix_bf16_mfma;yinv;xinv";
    default: return "xfwd;yfwd;zpass;yinv;xinv";
    }
}

}  // namespace

extern "C" {

const char* hfd_last_error(void) { return g_err.c_str(); }

hfd_status hfd_setup_tensor(hfd_plan* out, int nx, int ny, double dx, double dy, int nz,
                            const double* thickness, const double* z_bottom, int n_geom,
                            int batch_max, unsigned flags, void* stream)
{
    if (!out) return fail(HFD_EINVAL, "out is NULL");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nx > 2048 || ny > 2048)
        return fail(HFD_EINVAL, "nx and ny must be in [1, 2048]");
    if (!std::isfinite(dx) || !std::isfinite(dy) || !(dx > 0) || !(dy > 0))
        return fail(HFD_EINVAL, "dx and dy must be finite and > 0");
    if (nz < 1 || nz > 64) return fail(HFD_EINVAL, "nz must be in [1, 64]");
    if (n_geom < 1 || n_geom > 4096) return fail(HFD_EINVAL, "n_geom must be in [1, 4096]");
    if (batch_max < 1) return fail(HFD_EINVAL, "batch_max must be >= 1");
    if (batch_max < n_geom) return fail(HFD_EINVAL, "batch_max must be >= n_geom");
    if (flags & ~kKnownFlags) return fail(HFD_EINVAL, "unknown flag bits");
    if ((flags & HFD_FP64) && (flags & (HFD_MIX_SPLIT_BF16 | HFD_MIX_BATCHED_FP32)))
        return fail(HFD_EINVAL, "HFD_MIX_SPLIT_BF16 / HFD_MIX_BATCHED_FP32 require the FP32 field path");
    if ((flags & HFD_MIX_SPLIT_BF16) && (flags & HFD_MIX_BATCHED_FP32))
        return fail(HFD_EINVAL, "HFD_MIX_SPLIT_BF16 and HFD_MIX_BATCHED_FP32 are exclusive");
    if ((flags & HFD_EQUIDISTANT) && (flags & ~(HFD_EQUIDISTANT | HFD_FP64)))
        return fail(HFD_EINVAL, "HFD_EQUIDISTANT combines with HFD_FP64 only");

    hfd_plan p = new (std::nothrow) hfd_plan_s();
    if (!p) return fail(HFD_ENOMEM, "host allocation of the plan failed");
    p->nx = nx; p->ny = ny; p->nz = nz; p->G = n_geom; p->batch_max = batch_max;
    p->dx = dx; p->dy = dy; p->flags = flags;
    p->fp64 = flags & HFD_FP64;
    p->bf16 = flags & HFD_MIX_SPLIT_BF16;
    p->batched32 = flags & HFD_MIX_BATCHED_FP32;
    p->rsz = p->fp64 ? 8 : 4;
    p->csz = 2 * p->rsz;
    p->Lx = std::max(kMinL, next_pow2(2LL * nx));
    p->Ly = std::max(kMinL, next_pow2(2LL * ny));
    p->M = p->Lx / 2;
    p->QX = p->M + 1;
    p->QY = p->Ly / 2 + 1;
    p->P = nz * (nz + 1) / 2;
    hfd_status st = validate_geometry(nz, n_geom, thickness, z_bottom, p->thick, p->zbot);
    if (st) { delete p; return st; }
    p->eq3d = flags & HFD_EQUIDISTANT;
    if (p->eq3d) {
        st = check_equidistant(nz, n_geom, p->thick, p->zbot);
        if (st) { delete p; return st; }
        p->Lz = std::max(2, next_pow2(2LL * nz));
    }
    p->fused = !(flags & HFD_SPLIT_PASSES) && !p->bf16 && !p->batched32 && !p->eq3d &&
               fused_supported(p->fp64, p->Ly, nz, nullptr);
    p->path = p->eq3d ? 4 : (p->fused ? 0 : (p->bf16 ? 3 : (p->batched32 ? 2 : 1)));

    // sizes (overflow checked)
    const long long S = 3LL * nz;
    const long long q_per_geom = p->eq3d ? mul_ll(mul_ll((long long)(p->Lz / 2 + 1) * 6, p->QX), p->QY)
                                         : mul_ll(mul_ll((long long)p->P * 5, p->QX), p->QY);
    const long long bc = p->eq3d ? mul_ll(mul_ll(2LL * batch_max, S), (long long)p->Ly * (long long)p->csz) : 0;
    const long long q_elems = mul_ll(q_per_geom, n_geom);
    const long long x1 = mul_ll(mul_ll(mul_ll((long long)batch_max, S), p->M), (long long)ny * (long long)p->csz);
    const long long mh = mul_ll(mul_ll(mul_ll((long long)batch_max, S), p->M), (long long)p->Ly * (long long)p->csz);
    if (q_elems < 0 || x1 < 0 || mh < 0) { delete p; return fail(HFD_ENOMEM, "size overflow"); }
    p->q_geom_stride = q_per_geom;
    if (!p->eq3d) {
        p->nslot = n_geom * p->P;
        p->qcs = (long long)p->nslot * 5 * p->QY;
        // kernels read the slot table through 32-bit byte offsets from the
        // start of a kx row (the packed column: of the first two rows)
        if (2 * p->qcs * (long long)p->rsz >= (1LL << 31)) {
            delete p;
            return fail(HFD_ENOTSUP, "one kx row of the tensor table (n_geom * nz (nz + 1) / 2 pairs) exceeds "
                                     "2 GiB: use fewer stacks per plan");
        }
    }
    p->x1_bytes = (size_t)x1;
    p->mh_bytes = (size_t)mh;

    hipStream_t s = (hipStream_t)stream;
    if (hipGetDevice(&p->dev) != hipSuccess) { delete p; return fail(HFD_EHIP, "hipGetDevice failed"); }
    st = scratch_init(p->dev);
    if (st) { delete p; return st; }
    size_t freeb = 0, totalb = 0;
    if (hipMemGetInfo(&freeb, &totalb) == hipSuccess) {
        const long double need = (long double)q_elems * p->rsz + (long double)x1 + 2.0L * mh + (long double)bc;
        if (need > (long double)freeb) {
            delete p;
            return fail(HFD_ENOMEM, "plan needs " + std::to_string((double)need) + " bytes of device memory, " +
                                        std::to_string(freeb) + " free");
        }
    }
    do {
        st = dev_alloc(&p->Q, (size_t)q_elems * p->rsz, "Fourier tensor");
        if (st) break;
        st = dev_alloc(&p->lp, (size_t)n_geom * 2 * nz * p->rsz, "layer parameters");
        if (st) break;
        if (!p->eq3d) {
            st = dev_alloc(&p->qslot, sizeof(int) * (size_t)p->nslot, "tensor slot map");
            if (st) break;
        }
        st = dev_alloc(&p->X1, p->x1_bytes, "x-pass workspace");
        if (st) break;
        st = dev_alloc(&p->Mh, p->mh_bytes, "spectrum workspace");
        if (st) break;
        st = dev_alloc(&p->Hh, p->mh_bytes, "spectrum workspace");
        if (st) break;
        if (p->eq3d) {
            st = dev_alloc(&p->Bc, (size_t)bc, "split-column workspace");
            if (st) break;
        }
        st = upload_twiddles(p, s);
        if (st) break;
        st = alloc_setup_scratch(p);
        if (st) break;
        if (p->eq3d) {
            st = build_tensor3d(p, s);
            break;
        }
        st = build_tensor(p, s);
        if (st) break;
        st = setup_derivatives(p, s);
        if (st) break;
        if (flags & HFD_STORE_DTENSOR) {
            st = compute_derivatives(p, 0, s);
            if (st == HFD_OK && hipStreamSynchronize(s) != hipSuccess) st = fail(HFD_EHIP, "sync failed");
            p->d_valid = (st == HFD_OK);
        }
    } while (0);
    if (st) {
        free_plan_memory(p);
        delete p;
        return st;
    }
    {
        std::lock_guard<std::mutex> lk(g_plans_mu);
        g_plans.insert(p);
    }
    *out = p;
    return HFD_OK;
}

hfd_status hfd_set_thickness(hfd_plan p, const double* thickness, const double* z_bottom, void* stream)
{
    HFD_TRY(check_plan(p));
    std::vector<double> t, z;
    HFD_TRY(validate_geometry(p->nz, p->G, thickness, z_bottom, t, z));
    if (p->eq3d) HFD_TRY(check_equidistant(p->nz, p->G, t, z));
    DeviceGuard dg;
    HFD_HIP(dg.set(p->dev));
    // from here on the stored tensor is being replaced: the plan is unusable
    // until the rebuild has completed
    p->ready = false;
    p->thick = t;
    p->zbot = z;
    hipStream_t s = (hipStream_t)stream;
    if (p->eq3d) {
        HFD_TRY(build_tensor3d(p, s));
        p->ready = true;
        return HFD_OK;
    }
    HFD_TRY(build_tensor(p, s));
    HFD_TRY(setup_derivatives(p, s));
    if (p->flags & HFD_STORE_DTENSOR) {
        HFD_TRY(compute_derivatives(p, 0, s));
        HFD_HIP(hipStreamSynchronize(s));
        p->d_valid = true;
    }
    p->ready = true;
    return HFD_OK;
}

hfd_status hfd_demag_field(hfd_plan p, const void* m, void* h, int batch, void* stream)
{
    HFD_TRY(check_ready(p));
    HFD_TRY(check_field_args(p, m, h, batch, "m", "h"));
    DeviceGuard dg;
    HFD_HIP(dg.set(p->dev));
    return run_field(p, m, h, batch, 0, (hipStream_t)stream);
}

hfd_status hfd_demag_field_noalloc(hfd_plan p, const void* m, void* h, int batch, void* stream)
{
    HFD_TRY(check_ready(p));
    HFD_TRY(check_field_args(p, m, h, batch, "m", "h"));
    if (p->eq3d || (p->flags & HFD_SPLIT_PASSES) || !fused_supported(p->fp64, p->Ly, p->nz, nullptr))
        return fail(HFD_ENOTSUP, "hfd_demag_field_noalloc runs the fused y-pass, which this plan cannot use");
    const long double need = (long double)batch * 3 * p->nz * p->M * (long double)p->ny * p->csz;
    if (need > (long double)kScratchBytes)
        return fail(HFD_EINVAL, "hfd_demag_field_noalloc: batch " + std::to_string(batch) + " needs " +
                                    std::to_string((double)need) + " bytes of scratch, the limit is " +
                                    std::to_string(kScratchBytes));
    void* x1 = scratch_ptr(p->dev);
    if (!x1) return fail(HFD_EHIP, "device scratch was not initialised for this device");
    DeviceGuard dg;
    HFD_HIP(dg.set(p->dev));
    return run_field(p, m, h, batch, 0, (hipStream_t)stream, nullptr, nullptr, 0, -1, -1, x1);
}

// Fused path of the VJP: per run of states (as run_field chunks them) one x
// pass of grad_h feeds both its y transform into Hh (the spectra G of the
// thickness gradient) and the in-place fused adjoint y pass with the inverse x
// pass (grad_m), instead of a second x pass of grad_h.
static hfd_status adjoint_and_spectra(hfd_plan p, const void* gh, void* gm, int batch, hipStream_t s)
{
    const int S = 3 * p->nz, bpg = batch / p->G;
    int chunk = chunk_for(p, batch);
    if (!(chunk < batch && chunk_ok(p, batch, chunk))) chunk = batch;
    const bool gen = generic_for(p, batch);
    const int xty = xty_for(p, batch);
    const size_t state = (size_t)S * p->ny * p->nx * p->rsz;
    const size_t hstate = (size_t)S * p->M * p->Ly * p->csz;
    const long long sig_stride = (long long)p->ny * p->nx;
    for (int b0 = 0; b0 < batch; b0 += chunk) {
        const int g0 = b0 / bpg;
        const int bpg_c = bpg >= chunk ? chunk : bpg;
        const char* in_c = (const char*)gh + (size_t)b0 * state;
        char* out_c = (char*)gm + (size_t)b0 * state;
        const char* lp_c = (const char*)p->lp + (size_t)g0 * 2 * p->nz * p->rsz;
        HFD_HIP(launch_xfwd(p->fp64, p->Lx, in_c, p->X1, p->nx, p->ny, sig_stride, p->nx, chunk * S,
                            p->twx, s, xty));
        HFD_HIP(launch_yfwd(p->fp64, p->Ly, p->X1, (char*)p->Hh + (size_t)b0 * hstate, p->ny,
                            (long long)chunk * S * p->M, p->twy, s));
        HFD_HIP(launch_fused(p->fp64, p->Ly, p->nz, p->X1, p->ny, p->M, chunk, p->Q, p->qcs,
                             p->qslot + (size_t)g0 * p->P, p->QX, p->QY, lp_c, bpg_c, 1, p->twy, s, gen));
        HFD_HIP(launch_xinv(p->fp64, p->Lx, p->X1, out_c, p->nx, p->ny, sig_stride, p->nx, chunk * S,
                            p->twx, s, xty));
    }
    return HFD_OK;
}

hfd_status hfd_demag_vjp(hfd_plan p, const void* m, const void* grad_h, void* grad_m,
                         double* grad_thickness, int batch, void* stream)
{
    HFD_TRY(check_ready(p));
    if (!grad_m && !grad_thickness) return fail(HFD_EINVAL, "grad_m and grad_thickness are both NULL");
    if (p->eq3d && grad_thickness)
        return fail(HFD_ENOTSUP, "thickness gradients need the non-equidistant plan (no HFD_EQUIDISTANT)");
    if (grad_thickness && (long long)p->nzeta_max * 6 * p->QY * (long long)p->rsz >= (1LL << 31))
        return fail(HFD_ENOTSUP, "one kx row of the thickness-derivative table exceeds 2 GiB (" +
                                     std::to_string(p->nzeta_max) + " offsets): use fewer stacks per "
                                     "plan or leave out HFD_STORE_DTENSOR");
    if (grad_m) HFD_TRY(check_field_args(p, grad_h, grad_m, batch, "grad_h", "grad_m"));
    if (grad_thickness) {
        HFD_TRY(check_field_args(p, m, grad_h, batch, "m", "grad_h"));
        if ((uintptr_t)grad_thickness & 7) return fail(HFD_EINVAL, "grad_thickness must be 8-byte aligned");
    }
    DeviceGuard dg;
    HFD_HIP(dg.set(p->dev));
    hipStream_t s = (hipStream_t)stream;
    // (dh/dm)^T grad_h = T (dh/dm) T^-1 grad_h
    if (!grad_thickness) return run_field(p, grad_h, grad_m, batch, 1, s);
    const int nsig = batch * 3 * p->nz;
    const long long ncols = (long long)nsig * p->M;
    const long long sig_stride = (long long)p->ny * p->nx;
    if (grad_m && path_for(p, batch) == 0) {
        HFD_TRY(adjoint_and_spectra(p, grad_h, grad_m, batch, s));
    } else {
        // (the five-pass paths use Mh and Hh themselves: grad_m first)
        if (grad_m) HFD_TRY(run_field(p, grad_h, grad_m, batch, 1, s));
        HFD_HIP(launch_xfwd(p->fp64, p->Lx, grad_h, p->X1, p->nx, p->ny, sig_stride, p->nx, nsig, p->twx, s));
        HFD_HIP(launch_yfwd(p->fp64, p->Ly, p->X1, p->Hh, p->ny, ncols, p->twy, s));
    }
    HFD_HIP(launch_xfwd(p->fp64, p->Lx, m, p->X1, p->nx, p->ny, sig_stride, p->nx, nsig, p->twx, s));
    HFD_HIP(launch_yfwd(p->fp64, p->Ly, p->X1, p->Mh, p->ny, ncols, p->twy, s));
    const int bpg = batch / p->G;
    const bool stored = (p->flags & HFD_STORE_DTENSOR) != 0;
    if (stored && !p->d_valid) {
        // stored mode whose table is not built yet: build the shared table once
        HFD_TRY(compute_derivatives(p, 0, s));
        p->d_valid = true;
    }
    if (stored) {
        HFD_HIP(launch_tgrad(p->fp64, p->Mh, p->Hh, p->nz, p->M, p->Ly, 0, batch, p->Q, p->qcs,
                             p->qslot, p->D, p->nzeta_max, p->itab, p->itab_stride, p->lp, bpg, p->QX,
                             p->QY, p->partial, s));
    } else {
        // recompute the derivative tensor of one group of stacks at a time
        for (size_t k = 0; k + 1 < p->dgroup.size(); ++k) {
            const int g0 = p->dgroup[k], g1 = p->dgroup[k + 1];
            HFD_TRY(compute_derivatives(p, (int)k, s));
            HFD_HIP(launch_tgrad(p->fp64, p->Mh, p->Hh, p->nz, p->M, p->Ly, g0 * bpg, (g1 - g0) * bpg,
                                 p->Q, p->qcs, p->qslot, p->D, p->nzeta_max, p->itab,
                                 p->itab_stride, p->lp, bpg, p->QX, p->QY, p->partial, s));
        }
    }
    HFD_HIP(launch_tgrad_finish(p->partial, p->ntiles, batch, p->nz, p->itab, p->itab_stride, bpg,
                                grad_thickness, s));
    return HFD_OK;
}

hfd_status hfd_time_stages(hfd_plan p, const void* m, void* h, int batch, int reps, void* stream,
                           double* ms_per_stage, int* n_stages, char* names, int name_len)
{
    HFD_TRY(check_ready(p));
    HFD_TRY(check_field_args(p, m, h, batch, "m", "h"));
    if (reps < 1 || !ms_per_stage || !n_stages) return fail(HFD_EINVAL, "bad timing arguments");
    DeviceGuard dg;
    HFD_HIP(dg.set(p->dev));
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HFD_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(HFD_EHIP, "hipEventCreate failed");
    }
    int ns = 0;
    // one full evaluation fills the intermediate buffers; then each stage's
    // kernels run `reps` times back to back between two events
    // (stages of the whole batch: a chunked configuration is timed unchunked)
    hfd_status st = run_field(p, m, h, batch, 0, s, nullptr, &ns, -1, -1, -1, nullptr, batch);
    for (int k = 0; k < ns && st == HFD_OK; ++k) {
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps && st == HFD_OK; ++r)
            st = run_field(p, m, h, batch, 0, s, nullptr, nullptr, -1, k, -1, nullptr, batch);
        (void)hipEventRecord(e1, s);
        if (st) break;
        if (hipEventSynchronize(e1) != hipSuccess) { st = fail(HFD_EHIP, "event sync failed"); break; }
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        ms_per_stage[k] = (double)ms / reps;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    for (int k = ns; k < 8; ++k) ms_per_stage[k] = 0.0;
    *n_stages = ns;
    if (names && name_len > 0) {
        int path = path_for(p, batch);
        if ((path == 2 || path == 3) && !mix_batched_supported(p->nz, batch, p->G)) path = 1;
        std::string n = stage_names(path);
        std::snprintf(names, (size_t)name_len, "%s", n.c_str());
    }
    return HFD_OK;
}

hfd_status hfd_autotune(hfd_plan p, int batch, void* stream, char* report, int report_len)
{
    HFD_TRY(check_ready(p));
    if (batch < 1 || batch > p->batch_max) return fail(HFD_EBATCH, "batch out of range");
    if (batch % p->G) return fail(HFD_EINVAL, "batch must be a multiple of n_geom");
    DeviceGuard dg;
    HFD_HIP(dg.set(p->dev));
    hipStream_t s = (hipStream_t)stream;
    // candidates: every compiled path valid for this plan; split-BF16 only when
    // the plan was created with it (it changes the rounding of the mixing)
    std::vector<int> cand;
    if (p->eq3d) cand.push_back(4);
    else {
        if (!(p->flags & HFD_SPLIT_PASSES) && fused_supported(p->fp64, p->Ly, p->nz, nullptr))
            cand.push_back(0);
        cand.push_back(1);
    }
    // the batched kernels apply each frequency matrix to 16 states at a time;
    // below that they are not worth timing
    if (!p->eq3d && !p->fp64 && batch >= 16 && mix_batched_supported(p->nz, batch, p->G)) {
        cand.push_back(2);
        if (p->bf16) cand.push_back(3);
    }
    const size_t bytes = (size_t)batch * 3 * p->nz * p->ny * p->nx * p->rsz;
    void *m = nullptr, *h = nullptr;
    HFD_TRY(dev_alloc(&m, bytes, "autotune input"));
    hfd_status st = dev_alloc(&h, bytes, "autotune output");
    if (st) { (void)hipFree(m); return st; }
    hipEvent_t e0, e1;
    std::string rep = "batch=" + std::to_string(batch);
    int best = p->path;
    int best_ty = xty_for(p, batch);
    int best_chunk = 0, best_gen = 0;
    double best_ms = 1e30;
    do {
        if (hipMemsetAsync(m, 0, bytes, s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
            hipEventCreate(&e1) != hipSuccess) {
            st = fail(HFD_EHIP, "autotune setup failed");
            break;
        }
        // time one configuration: two warm-up evaluations, then 10 back to back
        auto time_cfg = [&](int path, int xty, int chunk, double& per, int gen = 0) -> hfd_status {
            hfd_status t = HFD_OK;
            for (int w = 0; w < 2 && t == HFD_OK; ++w)
                t = run_field(p, m, h, batch, 0, s, nullptr, nullptr, path, -1, xty, nullptr, chunk, gen);
            const int reps = 10;
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < reps && t == HFD_OK; ++r)
                t = run_field(p, m, h, batch, 0, s, nullptr, nullptr, path, -1, xty, nullptr, chunk, gen);
            (void)hipEventRecord(e1, s);
            if (t) return t;
            if (hipEventSynchronize(e1) != hipSuccess) return fail(HFD_EHIP, "autotune sync failed");
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            per = ms / reps;
            return HFD_OK;
        };
        // stage 1: the field path, x passes with their default tile
        const int xdef = xty_for(p, batch);
        for (int path : cand) {
            double per = 0;
            st = time_cfg(path, xdef, batch, per);
            if (st) break;
            char buf[96];
            std::snprintf(buf, sizeof buf, " %s=%.4fms", path_name(path), per);
            rep += buf;
            if (per < best_ms) { best_ms = per; best = path; }
        }
        // stage 2: rows per block of the x passes for the chosen path
        if (st == HFD_OK) {
            rep += " | x tile:";
            for (int ty : {0, 4, 8, 12, 16, 24, 32}) {
                if (!x_tile_supported(p->fp64, p->Lx, ty) || ty == xdef) continue;
                double per = 0;
                st = time_cfg(best, ty, batch, per);
                if (st) break;
                char buf[64];
                std::snprintf(buf, sizeof buf, " %d=%.4fms", ty, per);
                rep += buf;
                if (per < best_ms) { best_ms = per; best_ty = ty; }
            }
        }
        // stage 3: the run-time layer-count fused kernel where an exact one exists
        if (st == HFD_OK && best == 0 && fused_exact_supported(p->fp64, p->Ly, p->nz)) {
            double per = 0;
            st = time_cfg(0, best_ty, batch, per, 1);
            if (st == HFD_OK) {
                char buf[64];
                std::snprintf(buf, sizeof buf, " | generic fused=%.4fms", per);
                rep += buf;
                if (per < best_ms) { best_ms = per; best_gen = 1; }
            }
        }
        // stage 4: states per run of the fused path (halving down to 1)
        if (st == HFD_OK && best == 0 && batch > 1) {
            rep += " | chunk:";
            for (int c = batch / 2; c >= 1; c /= 2) {
                if (!chunk_ok(p, batch, c)) continue;
                double per = 0;
                st = time_cfg(0, best_ty, c, per, best_gen);
                if (st) break;
                char buf[64];
                std::snprintf(buf, sizeof buf, " %d=%.4fms", c, per);
                rep += buf;
                if (per < best_ms) { best_ms = per; best_chunk = c; }
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    } while (0);
    (void)hipStreamSynchronize(s);
    (void)hipFree(m);
    (void)hipFree(h);
    if (st) return st;
    p->tuned[batch] = {best, best_ty, best_chunk, best_gen};
    rep += std::string(" -> ") + path_name(best) + " x" + std::to_string(best_ty);
    if (best_gen) rep += " generic";
    if (best_chunk > 0) rep += " chunk" + std::to_string(best_chunk);
    if (report && report_len > 0) std::snprintf(report, (size_t)report_len, "%s", rep.c_str());
    return HFD_OK;
}

hfd_status hfd_set_path(hfd_plan p, int batch, int path, int x_tile)
{
    HFD_TRY(check_plan(p));
    if (batch < 1 || batch > p->batch_max) return fail(HFD_EBATCH, "batch out of range");
    if (batch % p->G) return fail(HFD_EINVAL, "batch must be a multiple of n_geom");
    if (path < 0) {
        p->tuned.erase(batch);
        return HFD_OK;
    }
    bool ok = false;
    if (p->eq3d) ok = path == 4;
    else if (path == 0) ok = !(p->flags & HFD_SPLIT_PASSES) && fused_supported(p->fp64, p->Ly, p->nz, nullptr);
    else if (path == 1) ok = true;
    else if (path == 2) ok = !p->fp64;
    else if (path == 3) ok = p->bf16;
    if (!ok) return fail(HFD_EINVAL, "path " + std::to_string(path) + " is not available for this plan");
    if (!x_tile_supported(p->fp64, p->Lx, x_tile))
        return fail(HFD_EINVAL, "x tile " + std::to_string(x_tile) + " is not compiled for Lx = " +
                                    std::to_string(p->Lx));
    p->tuned[batch] = {path, x_tile};
    return HFD_OK;
}

hfd_status hfd_set_fused(hfd_plan p, int batch, int chunk, int generic)
{
    HFD_TRY(check_plan(p));
    if (batch < 1 || batch > p->batch_max) return fail(HFD_EBATCH, "batch out of range");
    if (batch % p->G) return fail(HFD_EINVAL, "batch must be a multiple of n_geom");
    if (chunk != 0 && !chunk_ok(p, batch, chunk))
        return fail(HFD_EINVAL, "chunk must divide the batch and lie inside one stack or cover whole stacks");
    if (generic != 0 && generic != 1) return fail(HFD_EINVAL, "generic must be 0 or 1");
    auto it = p->tuned.find(batch);
    if (it == p->tuned.end()) {
        p->tuned[batch] = {p->path, xty_for(p, batch), chunk, generic};
    } else {
        it->second.chunk = chunk;
        it->second.generic = generic;
    }
    return HFD_OK;
}

hfd_status hfd_get_info(hfd_plan p, hfd_info* info)
{
    HFD_TRY(check_plan(p));
    if (!info) return fail(HFD_EINVAL, "info is NULL");
    info->nx = p->nx; info->ny = p->ny; info->nz = p->nz; info->n_geom = p->G;
    info->batch_max = p->batch_max; info->Lx = p->Lx; info->Ly = p->Ly;
    info->fused = p->fused; info->fp64 = p->fp64; info->mix_bf16 = p->bf16;
    info->tensor_bytes = p->q_geom_stride * (long long)p->G * (long long)p->rsz;
    info->work_bytes = (long long)(p->x1_bytes + 2 * p->mh_bytes);
    if (p->eq3d) info->work_bytes += 2LL * p->batch_max * 3 * p->nz * p->Ly * (long long)p->csz;
    info->equidistant = p->eq3d;
    info->Lz = p->Lz;
    info->tensor_slots = p->eq3d ? 0 : p->nslot_used;
    return HFD_OK;
}

hfd_status hfd_export_fourier_tensor(hfd_plan p, int geom, void* dst, long long dst_bytes)
{
    HFD_TRY(check_ready(p));
    if (geom < 0 || geom >= p->G) return fail(HFD_EINVAL, "geom out of range");
    const long long bytes = p->q_geom_stride * (long long)p->rsz;
    if (!dst || dst_bytes < bytes) return fail(HFD_EINVAL, "dst too small (need " + std::to_string(bytes) + " bytes)");
    DeviceGuard dg;
    HFD_HIP(dg.set(p->dev));
    HFD_HIP(hipDeviceSynchronize());
    if (p->eq3d) {
        HFD_HIP(hipMemcpy(dst, (char*)p->Q + (size_t)geom * p->q_geom_stride * p->rsz, (size_t)bytes,
                          hipMemcpyDeviceToHost));
        return HFD_OK;
    }
    // gather the stack's pairs from their slots: per pair the table rows kx = 0
    // and M (stored first) and the block of rows 1 .. M - 1
    const size_t w = (size_t)5 * p->QY * p->rsz, drow = (size_t)p->P * w, srow = (size_t)p->qcs * p->rsz;
    for (int u = 0; u < p->P; ++u) {
        const char* src = (const char*)p->Q + (size_t)p->qslot_host[(size_t)geom * p->P + u] * w;
        char* d = (char*)dst + (size_t)u * w;
        HFD_HIP(hipMemcpy(d, src, w, hipMemcpyDeviceToHost));
        HFD_HIP(hipMemcpy(d + (size_t)p->M * drow, src + srow, w, hipMemcpyDeviceToHost));
        if (p->M > 1)
            HFD_HIP(hipMemcpy2D(d + drow, drow, src + 2 * srow, srow, w, (size_t)p->M - 1,
                                hipMemcpyDeviceToHost));
    }
    return HFD_OK;
}

hfd_status hfd_export_real_tensor(hfd_plan p, int geom, int i, int j, double* dst, void* stream)
{
    HFD_TRY(check_plan(p));
    if (geom < 0 || geom >= p->G || i < 0 || j < 0 || i >= p->nz || j >= p->nz)
        return fail(HFD_EINVAL, "geom or pair index out of range");
    if (!dst) return fail(HFD_EINVAL, "dst is NULL");
    DeviceGuard dg;
    HFD_HIP(dg.set(p->dev));
    hipStream_t s = (hipStream_t)stream;
    const size_t n = 6 * (size_t)(2 * p->nx - 1) * (2 * p->ny - 1);
    double* W = nullptr;
    PairGeoH* pg = nullptr;
    HFD_TRY(dev_alloc(&W, n * 8, "export"));
    hfd_status st = dev_alloc(&pg, sizeof(PairGeoH), "export");
    if (st) { (void)hipFree(W); return st; }
    const double* t = &p->thick[(size_t)geom * p->nz];
    const double* z = &p->zbot[(size_t)geom * p->nz];
    PairGeoH h = {t[i], t[j], z[i] - z[j], 0.0};
    hipError_t e = hipMemcpyAsync(pg, &h, sizeof(h), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(W, 0, n * 8, s);
    if (e == hipSuccess)
        e = launch_tensor_real(W, pg, 1, p->nx, p->ny, p->Lx, p->Ly, p->dx, p->dy,
                               std::max(h.ti, h.tj), 1, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dst, W, n * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(W);
    (void)hipFree(pg);
    if (e != hipSuccess) return fail(HFD_EHIP, std::string("export_real_tensor: ") + hipGetErrorString(e));
    return HFD_OK;
}

hfd_status hfd_forward_spectrum(hfd_plan p, const void* m, void* dst, long long dst_bytes, int batch,
                                void* stream)
{
    HFD_TRY(check_plan(p));
    if (!m || !dst) return fail(HFD_EINVAL, "m or dst is NULL");
    if (batch < 1 || batch > p->batch_max) return fail(HFD_EBATCH, "batch out of range");
    const long long need = (long long)batch * 3 * p->nz * p->M * (long long)p->Ly * (long long)p->csz;
    if (dst_bytes < need) return fail(HFD_EINVAL, "dst too small (need " + std::to_string(need) + " bytes)");
    DeviceGuard dg;
    HFD_HIP(dg.set(p->dev));
    hipStream_t s = (hipStream_t)stream;
    const int nsig = batch * 3 * p->nz;
    HFD_HIP(launch_xfwd(p->fp64, p->Lx, m, p->X1, p->nx, p->ny, (long long)p->ny * p->nx, p->nx, nsig, p->twx, s));
    HFD_HIP(launch_yfwd(p->fp64, p->Ly, p->X1, dst, p->ny, (long long)nsig * p->M, p->twy, s));
    return HFD_OK;
}

hfd_status hfd_destroy(hfd_plan p)
{
    HFD_TRY(check_plan(p));
    {
        std::lock_guard<std::mutex> lk(g_plans_mu);
        g_plans.erase(p);
    }
    DeviceGuard dg;
    (void)dg.set(p->dev);
    (void)hipDeviceSynchronize();
    free_plan_memory(p);
    p->magic = kDead;
    delete p;
    return HFD_OK;
}

}  // extern "C"
