/*
 * hfd.h -- C ABI of the MI355X (gfx950) hybrid-FFT demagnetization-field
 * library (Heistracher, Bruckner, Abert, Vogler, Suess, "Hybrid FFT algorithm
 * for fast demagnetization field calculations on non-equidistant magnetic
 * layers", arXiv:1910.07054).
 *
 * Problem (Sec. 3 of the paper, discrete field and its non-equidistant finite
 * difference model): nz layers share a lateral grid of nx x ny cells of size
 * dx x dy; layer l has its own thickness t_l and bottom z_l.  For a
 * magnetization m (unit vectors, M_s = 1) the library returns
 *
 *     h_i(p) = - sum_j sum_q N^{ij}(p - q) m_j(q)
 *
 * where N^{ij} is the cell-averaged demagnetization tensor between a cell of
 * layer i and a cell of layer j (Sec. 2, generalized Newell formulas, with the
 * four-point stencils of appendices A and B).  The sum over the lateral
 * offsets uses the discrete convolution theorem on zero-padded grids; the sum
 * over layers is explicit per lateral frequency (Sec. 3.1, hybrid form).
 *
 * Units: any consistent length unit (N is scale invariant); h is in units of
 * M_s.  Per-layer saturation magnetizations are the caller's: scale m_j by
 * M_s,j / M_s,ref before the call.
 *
 * Memory and layout:
 *   - m, h and the gradient fields are DEVICE pointers owned by the caller,
 *     layout [batch][3][nz][ny][nx] (x fastest, component-major), FP32, or
 *     FP64 for plans created with HFD_FP64.  They must be 16-byte aligned and
 *     must not overlap each other.
 *   - a plan owns its device tensor and all workspace, allocated in
 *     hfd_setup_tensor for up to batch_max states; hfd_demag_field and
 *     hfd_demag_vjp allocate nothing and only enqueue work on the given HIP
 *     stream (NULL = the default stream), so they may be captured in a HIP
 *     graph.  A plan must not be used from two streams at the same time.
 *
 * Errors: every call returns an hfd_status; arguments are validated on the
 * host before any HIP call.  On failure hfd_last_error() returns a message
 * (thread-local, valid until the next call on that thread).
 */
#ifndef HFD_H
#define HFD_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hfd_plan_s *hfd_plan;

typedef enum {
    HFD_OK = 0,
    HFD_EINVAL = -1,   /* invalid argument                                 */
    HFD_ENOMEM = -2,   /* device or host allocation failed / size overflow */
    HFD_EHIP = -3,     /* a HIP runtime call or kernel launch failed       */
    HFD_EBATCH = -4,   /* batch larger than the plan's batch_max           */
    HFD_EHANDLE = -5,  /* NULL, destroyed or corrupted plan                */
    HFD_ENOTSUP = -6   /* size outside the compiled kernel range           */
} hfd_status;

/* Flags for hfd_setup_tensor. */
enum {
    HFD_FP32 = 0,               /* FFTs and z-mixing in FP32 (tensor set up in FP64)   */
    HFD_FP64 = 1,               /* FFTs and z-mixing in FP64                           */
    HFD_MIX_SPLIT_BF16 = 2,     /* five-pass path, z-mixing of 16 states at a time on
                                   MFMA with a three-way BF16 split of tensor and
                                   spectra, FP32 accumulation (nz <= 8)                */
    HFD_SPLIT_PASSES = 4,       /* force the five-pass path (y-FFT, mix and inverse
                                   y-FFT as separate kernels) even where the fused
                                   y-pass fits in LDS                                  */
    HFD_STORE_DTENSOR = 8,      /* keep the thickness-derivative tensors resident
                                   between hfd_demag_vjp calls: one table over the
                                   distinct |interface offsets| of all stacks, built
                                   by setup / hfd_set_thickness (default: rebuilt
                                   inside every call for groups of consecutive
                                   stacks whose shared table holds at most 256 MiB
                                   of spectra, or one stack's table if larger)        */
    HFD_MIX_BATCHED_FP32 = 16,  /* five-pass path with the batched (16 states per
                                   block) FP32 VALU mixing, the FP32 twin of
                                   HFD_MIX_SPLIT_BF16                                 */
    HFD_EQUIDISTANT = 32        /* equidistant stack (all thicknesses equal, uniform
                                   pitch z_bottom[l+1] - z_bottom[l], n_geom = 1):
                                   the layer sum by FFT along z as well (eq. FFT_3D,
                                   Sec. 3.1), the method the paper compares with;
                                   FP32 or FP64, no other flag; hfd_demag_vjp
                                   supports grad_m only                               */
};

/*
 * Create a plan and build the Fourier-space tensor.
 *
 *   nx, ny      lateral cell counts, 1 <= nx, ny <= 2048
 *   dx, dy      lateral cell size, > 0
 *   nz          number of layers, 1 <= nz <= 64
 *   thickness   HOST array [n_geom][nz], every entry > 0 and finite
 *   z_bottom    HOST array [n_geom][nz] of layer bottoms, strictly increasing
 *               with z_bottom[l+1] >= z_bottom[l] + thickness[l] (layers may
 *               touch, not overlap); NULL stacks the layers without gaps
 *               starting at 0
 *   n_geom      number of stacks (thickness candidates) sharing nx, ny, dx,
 *               dy, nz; a batch of B states is split into n_geom equal runs
 *               and run g uses stack g (B must be a multiple of n_geom)
 *   batch_max   largest batch later passed to hfd_demag_field / _vjp
 *   flags       HFD_FP32 or HFD_FP64, optionally | HFD_MIX_SPLIT_BF16 or
 *               HFD_MIX_BATCHED_FP32 (FP32 only) | HFD_SPLIT_PASSES |
 *               HFD_STORE_DTENSOR; or HFD_EQUIDISTANT alone (with FP32/FP64)
 *   stream      HIP stream for the setup kernels; the call returns after the
 *               setup has completed on that stream
 *
 * The tensor of every layer pair (Sec. 2) is computed in FP64 on the GPU:
 * generalized Newell formulas near the diagonal, Gauss-Legendre quadrature
 * of the dipole kernel beyond six cell sizes (where the 64-term Newell sum
 * loses its digits to cancellation); then a 2D FFT per pair (F1 F2 of Sec.
 * 3.1) in FP64, rounded to the plan's precision.  Only the unique pairs
 * i <= j are stored (reciprocity t_i N^{ij}(d) = t_j N^{ji}(-d)), and a pair
 * geometry (both thicknesses and the offset) that occurs several times, in
 * one stack or in several, is computed and stored once (hfd_info.tensor_slots
 * counts them): thickness candidates that differ in one layer share the
 * tensors of all other pairs.  Memory is reserved for n_geom * nz (nz + 1) / 2
 * pair tensors, so hfd_set_thickness never reallocates it; a kx row of that
 * table must stay below 2 GiB (else HFD_ENOTSUP).
 */
hfd_status hfd_setup_tensor(hfd_plan *out, int nx, int ny, double dx, double dy, int nz,
                            const double *thickness, const double *z_bottom, int n_geom,
                            int batch_max, unsigned flags, void *stream);

/*
 * Rebuild the tensor of an existing plan for new thicknesses / bottoms (same
 * nx, ny, dx, dy, nz, n_geom; same conventions as hfd_setup_tensor).  This is
 * the step of the layer-thickness optimisation of Sec. 4 (Newton iteration on
 * one layer thickness until the mean field in the free layer vanishes): the
 * geometry changes, the lateral grid stays.  Blocks until the new tensor is
 * ready on `stream`; allocates nothing (the setup scratch belongs to the
 * plan) except that the thickness-derivative tables grow when the new
 * geometry has more distinct interface offsets than any earlier one.
 *
 * The stored Fourier tensor is rewritten in place, so a HIP graph that
 * captured hfd_demag_field (or hfd_demag_vjp without grad_thickness) stays
 * valid and computes the new geometry on its next replay.  A graph that
 * captured hfd_demag_vjp with grad_thickness must be captured again: its
 * kernels are sized by the per-geometry offset counts.
 *
 * Invalid arguments return HFD_EINVAL with the plan unchanged.  A failure
 * after validation (device allocation or kernel error) leaves the plan
 * unusable: field and vjp calls return HFD_EINVAL until a later
 * hfd_set_thickness succeeds.
 */
hfd_status hfd_set_thickness(hfd_plan plan, const double *thickness, const double *z_bottom,
                             void *stream);

/*
 * h = -N * m  for `batch` states (Sec. 3.1, hybrid 2D FFT + explicit z sum).
 * m and h: device [batch][3][nz][ny][nx]; h is overwritten.  batch must be in
 * [1, batch_max] and a multiple of n_geom.  m == h (or overlap) -> HFD_EINVAL.
 */
hfd_status hfd_demag_field(hfd_plan plan, const void *m, void *h, int batch, void *stream);

/*
 * Same result as hfd_demag_field, for callers that cannot allocate device
 * memory or use per-plan workspace (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): the x-pass spectra live in a
 * device scratch array of the library (32 MiB per GPU, held until the process
 * ends) instead of the plan's workspace, and the call allocates nothing.
 * It runs the fused y-pass: HFD_ENOTSUP for plans that cannot (HFD_EQUIDISTANT,
 * HFD_SPLIT_PASSES, or a column that does not fit in LDS).  HFD_EINVAL when
 * batch * 3 nz * (Lx/2) * ny complex values exceed the 32 MiB (e.g. more than
 * two states of a 256 x 256 x 8 FP32 stack), plus the checks of
 * hfd_demag_field.  Every call on one GPU shares that scratch: calls that
 * overlap in time on the same GPU (other streams, other threads, other plans)
 * race and must be serialized by the caller.
 */
hfd_status hfd_demag_field_noalloc(hfd_plan plan, const void *m, void *h, int batch, void *stream);

/*
 * Vector-Jacobian product of h = h(m, t) for an upstream gradient grad_h.
 * The paper optimises a layer thickness by Newton's method on the mean field
 * in the free layer (Sec. 4) without saying how the derivative is formed;
 * this call supplies it analytically, together with the gradient in m:
 *   grad_m = (dh/dm)^T grad_h           (device [batch][3][nz][ny][nx]), and
 *   grad_thickness[b][k] = d <grad_h_b, h_b> / d t_k   (device FP64
 *                                       [batch][nz]) for a stack whose gaps stay
 *                                       fixed (raising t_k lifts the layers above k).
 * Either output may be NULL.  The transpose uses reciprocity:
 * (dh/dm)^T = T (dh/dm) T^{-1}, T = diag(t_l).  The thickness derivative uses
 * the derivatives of the Newell kernels with respect to the z offset,
 * evaluated in FP64 and transformed like the tensor.  grad_thickness returns
 * HFD_ENOTSUP on equidistant plans and when one kx row of the derivative
 * table (distinct interface offsets x 6 x (Ly/2+1) values) exceeds 2 GiB.
 * m may be NULL when grad_thickness is NULL.  Allocates nothing; the derivative
 * tables are rebuilt inside the call unless the plan has HFD_STORE_DTENSOR.
 */
hfd_status hfd_demag_vjp(hfd_plan plan, const void *m, const void *grad_h, void *grad_m,
                         double *grad_thickness, int batch, void *stream);

/* Time each kernel stage of hfd_demag_field (inputs as for hfd_demag_field):
 * one full evaluation, then the kernels of each stage launched `reps` times
 * back to back between two HIP events on `stream`.  ms_per_stage[k] receives
 * the average time per launch of stage k (host array of length 8); n_stages and
 * names (semicolon separated, host buffer of name_len bytes) describe the
 * stages.  Repeated stages run on their own output, so h holds unspecified
 * values afterwards.  For measurement only; it synchronizes the stream. */
hfd_status hfd_time_stages(hfd_plan plan, const void *m, void *h, int batch, int reps,
                           void *stream, double *ms_per_stage, int *n_stages, char *names,
                           int name_len);

/* Time every field path the plan can run for `batch` states (the fused
 * y-pass where it fits in LDS, the five-pass path with generic mixing, the
 * batched FP32 mixing for nz <= 8 and batch >= 16, the split-BF16 matrix-core
 * mixing when the plan was created with HFD_MIX_SPLIT_BF16) on zero input and
 * keep the fastest for this batch size; later calls with that batch use it.
 * Allocates and frees a scratch input/output pair and synchronizes the stream,
 * so it must not be captured in a graph.  `report` (host buffer) receives the
 * timings and the choice as text, e.g. "batch=1 fused=0.047ms ... -> fused". */
hfd_status hfd_autotune(hfd_plan plan, int batch, void *stream, char *report, int report_len);

/* Pin the field configuration used for `batch` states instead of timing it
 * (hfd_autotune): path 0 fused y-pass, 1 five-pass with per-frequency mixing,
 * 2 five-pass with batched FP32 mixing, 3 five-pass with split-BF16 MFMA
 * mixing (plans created with HFD_MIX_SPLIT_BF16), 4 equidistant plans; x_tile
 * = rows per block of the x passes (0 = default tile, or 4, 8, 12, 16, 24, 32
 * where the block fits).  path < 0 drops the pinned choice.  Host only;
 * HFD_EINVAL for a configuration the plan cannot run. */
hfd_status hfd_set_path(hfd_plan plan, int batch, int path, int x_tile);

/* Pin how the fused path runs `batch` states (hfd_autotune chooses both by
 * timing; host only):
 *   chunk    states per run (0 = the whole batch in one run).  The fused path
 *            launches its three kernels once per run of `chunk` consecutive
 *            states, reusing one x-pass buffer of `chunk` states, so that
 *            between the kernels the spectra of a run can stay in the 256 MB
 *            Infinity Cache instead of travelling through HBM (the batched
 *            evaluation of Sec. 3.1, ordered state by state).  chunk must
 *            divide batch, and a run must lie inside one stack or cover whole
 *            stacks (chunk divides batch / n_geom, or is a multiple of it).
 *   generic  1: the y pass with the layer count read at run time even where a
 *            kernel compiled for the exact layer count exists (FP32; 256- and
 *            512-point columns up to 10 layers, 1024-point columns up to 4);
 *            0: the exact kernel where it exists.
 * HFD_EINVAL for other values. */
hfd_status hfd_set_fused(hfd_plan plan, int batch, int chunk, int generic);

/* Plan description (host). */
typedef struct {
    int nx, ny, nz, n_geom, batch_max;
    int Lx, Ly;             /* padded lateral lengths (powers of two >= 2n)        */
    int fused;              /* 1: three-pass path (fused y-pass), 0: five passes   */
    int fp64;               /* 1 if the field path runs in FP64                    */
    int mix_bf16;           /* 1 if the z-mixing runs on split-BF16 MFMA           */
    long long tensor_bytes; /* bytes allocated for the Fourier tensor (all stacks) */
    long long work_bytes;   /* bytes of the field workspace                        */
    int equidistant;        /* 1 for an HFD_EQUIDISTANT plan                       */
    int Lz;                 /* padded length along z (equidistant plans), else 0   */
    int tensor_slots;       /* distinct pair tensors stored (pairs of equal
                               thicknesses and offset share one, also across
                               stacks); 0 for equidistant plans                   */
} hfd_info;
hfd_status hfd_get_info(hfd_plan plan, hfd_info *info);

/* Copy the stored Fourier tensor of stack `geom` to the HOST buffer `dst`:
 * layout [Lx/2+1][P_u][5][Ly/2+1] (kx, pair, component, ky) in the plan's
 * precision, P_u = nz(nz+1)/2
 * unique pairs i <= j in row-major upper-triangle order, components
 * (xx, yy, xy, xz, yz) of t_i * (-DFT2(N^{ij}) / (Lx Ly)); real parts for
 * xx, yy, xy, imaginary parts for xz, yz (the only non-zero parts by
 * lateral parity); zz follows from the trace of the self-pair block.
 * HFD_EQUIDISTANT plans: layout [Lx/2+1][Lz/2+1][6][Ly/2+1] (kx, kz,
 * component, ky), components (xx, yy, zz, xy, xz, yz) of
 * -DFT3(N) / (Lx Ly Lz), which are real by parity (eq. FFT_3D). */
hfd_status hfd_export_fourier_tensor(hfd_plan plan, int geom, void *dst, long long dst_bytes);

/* Compute the real-space FP64 tensor N^{ij}(p, q) of stack `geom` for one
 * ordered pair (target i, source j), p in [-(nx-1), nx-1], q in
 * [-(ny-1), ny-1], into the HOST buffer dst [6][2ny-1][2nx-1] (components
 * xx, yy, zz, xy, xz, yz), with the same kernels the setup uses. */
hfd_status hfd_export_real_tensor(hfd_plan plan, int geom, int i, int j, double *dst, void *stream);

/* Forward spectra (2D DFT of the zero-padded m, FP32/FP64 complex) on the
 * DEVICE buffer dst: layout [batch][3][nz][Lx/2][Ly], the kx = 0 and
 * kx = Lx/2 columns packed as (Re X(0, ky) + i Re X(Lx/2, ky)) before the
 * y transform (i.e. column 0 holds the y-DFT of that packed sequence).
 * dst_bytes must cover batch * 3 * nz * (Lx/2) * Ly complex values. */
hfd_status hfd_forward_spectrum(hfd_plan plan, const void *m, void *dst, long long dst_bytes,
                                int batch, void *stream);

hfd_status hfd_destroy(hfd_plan plan);

const char *hfd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HFD_H */
