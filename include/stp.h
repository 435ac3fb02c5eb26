/*
 * stp.h -- C ABI of libstp.so: the element-local space-time predictor (STP) of the linear ADER-DG scheme
 * (Gallard, Rannabauer, Reinarz, Bader, arXiv:2003.12787) on AMD Instinct MI355X (gfx950).
 *
 * What one call computes (Sec. II-A, Eqs. (3)-(4) and the recursion below Eq. (4); Sec. II-B output
 * contract). For every element e with DOFs Q_e, element size h_e and time step dt_e:
 *
 *   PDE        q_t + sum_d (A_d q)_{x_d} + B_d dq/dx_d = 0           (Eq. (1), material absorbed in B_d)
 *   operator   V(u) = sum_d V_d(u),
 *              V_d(u) = -(1/h) [ D x_d (A_d o u) + B_d o (D x_d u) ]  (Sec. II-A volume term)
 *              D[i][j] = l_j'(xi_i) on the n = N+1 Gauss-Legendre (or Gauss-Lobatto, stp_plan_desc.nodes)
 *              nodes of [0,1]; "D x_d" contracts
 *              spatial axis d; "o" is the nodewise m x m product.
 *   Taylor     p_0 = Q, p_{o+1} = V p_o (+ S_o), o = 0..N-1          (Cauchy-Kowalewsky, Eq. (4))
 *   outputs    qavg    = sum_{o=0..N} dt^o/(o+1)! p_o                 time AVERAGE (Eq. (4) / dt)
 *              favg[d] = V_d(qavg)                                    time-averaged flux divergence + NCP
 *                                                                     per direction (Fig. 1 favg[d]; computed
 *                                                                     from qavg by linearity as in Fig. 5)
 *              qface[f] = qavg extrapolated to face f                 (Sec. II-B: one product per face)
 *              fface[f] = (A_{d_f} o qavg) extrapolated to face f     (only when A is present)
 *
 * Layouts (element-contiguous, no padding; the node index is (z*n + y)*n + x, the quantity index fastest,
 * i.e. the AoS tensor of Sec. III-A/B):
 *   Q, qavg           [e][z][y][x][s]                 n^3 * m values per element
 *   favg              [e][d][z][y][x][s]              3 * n^3 * m  (n^3 * m with STP_FAVG_SUM)
 *   qface, fface      [e][f][a][b][s]                 6 * n^2 * m; f = x-, x+, y-, y+, z-, z+ (reference
 *                                                     coordinate 0 / 1 along the normal), (a, b) = the two
 *                                                     other axes, slower first: (z,y), (z,x), (y,x)
 *   params (presets)  [e][z][y][x][p] or [e][p] with STP_PARAM_PER_ELEMENT;
 *                     acoustic p = (rho, K), elastic p = (rho, lambda, mu), curvilinear elastic
 *                     p = (rho, lambda, mu, G[0][0], G[0][1], ..., G[2][2]) (12 values, G row-major)
 *   A, B (generic)    [e][d][row s][col r][z][y][x] (node fastest, so that the threads of a workgroup, one
 *                     per node, read consecutive words), or [e][d][s][r] with STP_COEF_PER_ELEMENT
 *   src (point src)   [e][n^3 + m + N]: nodal projection P[node], amplitude a[s], time derivatives
 *                     sigma^(o)(t_n), o = 0..N-1; S_o[node][s] = P[node] a[s] sigma^(o)
 *   dt, h             [e] doubles (device), or host scalars when dt_h_scalar = 1
 *
 * Physics presets (quantity order):
 *   STP_ACOUSTIC  m = 4 (p, v_x, v_y, v_z):   p_t + K div v = 0,  v_t + grad p / rho = 0
 *   STP_ELASTIC   m = 9 (v_x, v_y, v_z, s_xx, s_yy, s_zz, s_xy, s_yz, s_xz):
 *                 rho v_t = div sigma,  sigma_t = lambda (div v) I + mu (grad v + grad v^T)
 *   STP_GENERIC   any 1 <= m <= 16: dense B_d (and optionally A_d) given per node or per element
 *   STP_ELASTIC_CURV  m = 9, the elastic system on a curvilinear element (the benchmark physics of Sec. VI:
 *                 9 wave quantities plus 3 material and 9 geometry parameters per point). The element is
 *                 the image of the reference cube under a map x(xi); by the chain rule the system becomes
 *                 q_t + sum_d B_d dq/dxi_d / h = 0 with B_d = sum_j G[d][j] M_j, M_j the Cartesian elastic
 *                 matrices and G[d][j] = h dxi_d/dx_j the metric terms (the inverse Jacobian of the map
 *                 scaled by the element size h; an undeformed cube of side h has G = I).
 *
 * Precision: STP_FP64 computes and stores in double. STP_FP32 and STP_BF16X3 read and write float. STP_FP32
 * forms its derivative contractions in FP32, on the VALU or (acoustic and elastic presets at N = 7) as FP32
 * matrix-core products. STP_BF16X3 forms them on the matrix cores with the operands split into three BF16 pieces
 * each (D = D0 + D1 + D2 and u = hi + mid + lo; at N = 7 the six products of order up to 2^-16 are formed, at
 * N = 8, 9 all nine) and FP32 accumulation (about FP32 accuracy). An STP_BF16X3 class without such a kernel
 * (orders below 7, FP64 accumulation, point sources, generic physics) runs the FP32 kernels.
 * Classes whose order is >= acc64_min_order (when > 0) accumulate qavg and the face extrapolation in FP64.
 *
 * Ownership: the caller owns every buffer and passes raw pointers; device pointers must be device memory
 * of the plan's device. The library never frees or retains caller buffers after stp_run returns (after
 * stp_submit they must stay valid until stp_poll reports completion). The plan owns its constant tables,
 * streams, events and scratch; its tables are immutable after creation and stp_run may be called from
 * several host threads on different streams (see stp_run for heterogeneous plans).
 *
 * Errors: every entry point returns a stp_status and never throws or aborts. Problems detectable on the
 * host (bad sizes, NULL required pointers, unsupported order/quantity count, h <= 0 or dt < 0 given as host
 * scalars, outputs aliasing inputs) return STP_E_INVAL or STP_E_UNSUPPORTED before any device work is
 * queued. Class ids are device data: out-of-range ids are reported by stp_sync and stp_poll (see stp_run).
 * HIP failures return STP_E_DEVICE. A human-readable
 * message for the last failure on the calling thread is available from stp_last_error().
 */
#ifndef STP_H
#define STP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stp_plan_s* stp_plan_t;

typedef enum {
    STP_OK = 0,
    STP_PENDING = 1,          /* stp_poll: the ticket is queued or running                          */
    STP_E_INVAL = -1,         /* invalid argument                                                   */
    STP_E_UNSUPPORTED = -2,   /* order / quantity count / physics / precision not supported          */
    STP_E_NOMEM = -3,         /* allocation failed, or a submitted batch exceeds the serving budget  */
    STP_E_DEVICE = -4,        /* a HIP runtime call or a kernel launch failed                        */
    STP_E_BUSY = -5,          /* serving queue full                                                  */
    STP_E_TIMEOUT = -6        /* serving: the ticket's deadline passed before its batch was launched */
} stp_status;

typedef enum { STP_ACOUSTIC = 0, STP_ELASTIC = 1, STP_GENERIC = 2, STP_ELASTIC_CURV = 3 } stp_physics;
typedef enum { STP_FP64 = 0, STP_FP32 = 1, STP_BF16X3 = 2 } stp_prec;

/* stp_class.flags */
enum {
    STP_PARAM_PER_ELEMENT = 1u << 0, /* presets: params [e][p] instead of per node                     */
    STP_A_PRESENT = 1u << 1,         /* generic: conservative flux matrices A_d given; fface written    */
    STP_COEF_PER_ELEMENT = 1u << 2,  /* generic: A, B given once per element [e][d][s][r]               */
    STP_FAVG_SUM = 1u << 3,          /* favg holds sum_d favg[d] ([e][n^3][m])                          */
    STP_SRC_POINT = 1u << 4          /* a point source per element (src array)                          */
};

/* One element class: polynomial degree N (order; n = N+1 nodes per axis), quantity count m, physics. */
typedef struct {
    int order;      /* N, 1..9                                                  */
    int nquant;     /* m: 4 (acoustic), 9 (elastic, curvilinear), 1..16 (generic) */
    int physics;    /* stp_physics                                              */
    unsigned flags; /* STP_* class flags                                        */
} stp_class;

typedef struct {
    int nclass;                /* number of classes, 1..64                                              */
    const stp_class* classes;  /* host array [nclass], copied by stp_plan                                */
    int prec;                  /* stp_prec                                                               */
    int acc64_min_order;       /* FP32/BF16X3: FP64 accumulation of qavg and faces when order >= this;
                                  0 = never. Ignored for STP_FP64.                                        */
    int device;                /* HIP device ordinal                                                     */
    int variant;               /* 0 = autotuned choice; otherwise a kernel variant id (STP_VARIANT_*)  */
    size_t serve_mem_budget;   /* bytes of in-flight serving memory for stp_submit; 0 disables serving  */
    int autotune;              /* with variant = STP_VARIANT_AUTO: 0 = take the kernel variant (single-
                                  class plans) and the persistent grid and tile LDS budget (heterogeneous
                                  plans) from the tuning cache, else built-in rules; 1 = also time the
                                  candidates the cache lacks on a synthetic batch (at plan creation, tens
                                  of ms per entry) and store them; 2 = retime everything. Cache: the JSON
                                  file named by STP_TUNE_CACHE, else $HOME/.cache/stp_tune.json, keyed by
                                  architecture, HIP runtime version, CU count and class. STP_E_INVAL
                                  outside 0..2.                                                          */
    int nodes;                 /* interpolation nodes of the nodal basis (Sec. II-A allows both): 0 =
                                  Gauss-Legendre, 1 = Gauss-Lobatto (the faces are then boundary nodes and
                                  the corrector's mass matrix is the Lobatto quadrature). STP_E_INVAL
                                  outside 0..1.                                                          */
} stp_plan_desc;

/* Kernel variants selectable through stp_plan_desc.variant (0 = library choice). */
enum {
    STP_VARIANT_AUTO = 0,
    STP_VARIANT_PLAIN = 1,   /* one element per workgroup, one thread per node, LDS-staged; generic
                                classes with dense per-node B_d and neither A nor a point source, FP32
                                arithmetic (m = 4 at N = 4..9, m = 9 at N = 7..9): the same algorithm
                                with part or all of each node's B_d held in registers and LDS through
                                the Taylor loop (Sec. IV-A's footprint argument on a CU)               */
    STP_VARIANT_FUSED = 2,   /* register-blocked lines, LDS transposes (acoustic and elastic presets,
                                FP32 I/O without FP64 accumulation or point source, N <= 7)            */
    STP_VARIANT_MFMA = 3     /* matrix-core contractions, without FP64 accumulation or point source:
                                STP_FP32 FP32 products (acoustic and elastic presets at N = 7);
                                STP_BF16X3 split-BF16x3 products with FP32 accumulation (acoustic,
                                elastic and curvilinear elastic presets at N = 7; acoustic and elastic
                                at N = 8, 9). The library's choice where such a kernel exists.         */
};

typedef struct {
    int64_t nelem;               /* number of elements (>= 0; 0 is a no-op)                               */
    const int32_t* cls;          /* device [nelem] class index per element; NULL when nclass == 1        */
    const int64_t* off_q;        /* device [nelem] offset (in values) of each element in Q and qavg; favg
                                    uses 3*off_q (off_q with STP_FAVG_SUM). NULL = contiguous (one class) */
    const int64_t* off_coef;     /* device [nelem] offset of each element in params or in A and B.
                                    NULL = contiguous (one class)                                         */
    const int64_t* off_face;     /* device [nelem] offset in qface / fface. NULL = contiguous (one class)  */
    const int64_t* off_src;      /* device [nelem] offset in src. NULL = contiguous (one class)            */
    const double* dt;            /* device [nelem], or host pointer to one value when dt_h_scalar = 1      */
    const double* h;             /* device [nelem], or host pointer to one value when dt_h_scalar = 1      */
    int dt_h_scalar;             /* 1: dt[0], h[0] are host scalars shared by all elements                 */
    const void* Q;               /* device input DOFs                                                      */
    const void* params;          /* device material parameters (presets)                                   */
    const void* A;               /* device A_d (generic with STP_A_PRESENT)                               */
    const void* B;               /* device B_d (generic)                                                  */
    const void* src;             /* device point sources (STP_SRC_POINT)                                  */
    void* qavg;                  /* device outputs                                                         */
    void* favg;
    void* qface;
    void* fface;                 /* only written when the class has STP_A_PRESENT                         */
} stp_batch;

typedef struct {
    double t_submit;  /* host monotonic seconds when stp_submit accepted the batch   */
    double t_start;   /* when the dispatcher queued the launch                        */
    double t_done;    /* when the completion poller observed the end of the launch    */
    int status;       /* STP_OK, STP_PENDING or an error                              */
} stp_ticket_info;

/* Build a plan: host tables (Gauss-Legendre or Gauss-Lobatto nodes, D, face vectors, three-piece BF16 split of D)
 * in FP64, uploaded once to the device; kernel choice per class. Returns STP_E_UNSUPPORTED for an order
 * outside 1..9, a preset with the wrong m, a generic m outside 1..16, or a requested variant that has no
 * kernel for a class. *out is NULL on failure. */
stp_status stp_plan(const stp_plan_desc* desc, stp_plan_t* out);

/* Release a plan (waits for its outstanding serving work). NULL is a no-op. */
void stp_plan_free(stp_plan_t plan);

/* Run the predictor on a batch, asynchronously on the HIP stream `hip_stream` (NULL = the null stream).
 * Returns after the launches are queued.
 * Single-class plan: one launch, no allocation; stream-capturable. Calls may overlap on different streams.
 * Heterogeneous plan (nclass > 1): a bucketing pass sorts the elements by class, then classes of order <= 7
 * in FP32 I/O without FP64 accumulation run in one persistent launch per physics bucket (workgroups take
 * tiles of one class from a queue, most expensive classes first) and the other classes run one launch each.
 * The element lists and tile queues live in the plan's scratch, which the first call that needs more of it
 * allocates synchronously (stp_reserve avoids that, after which the call is stream-capturable). Because the
 * scratch is shared, stp_run calls of one heterogeneous plan must not overlap on the device: queue them on
 * one stream, or use one plan per stream. The class ids live in device memory and are checked there:
 * elements whose id is outside 0..nclass-1 are skipped (their outputs are not written) and flagged, and the
 * next stp_sync of the plan returns STP_E_INVAL. */
stp_status stp_run(stp_plan_t plan, const stp_batch* batch, void* hip_stream);

/* Wait for the work queued on hip_stream (NULL = the null stream), then report what the device found in the
 * plan's heterogeneous batches since the previous stp_sync: STP_E_INVAL if any element of a batch of stp_run
 * or stp_run_noalloc had a class id outside 0..nclass-1 (those elements' outputs were not written; the flag
 * is cleared), else STP_OK. STP_E_DEVICE if the stream reported a failure. Synchronous; not capturable. */
stp_status stp_sync(stp_plan_t plan, void* hip_stream);

/* stp_run for callers that cannot allocate device memory (code under HIP graph capture, serving loops and
 * harnesses that forbid hipMalloc). Same arguments, outputs and kernels as stp_run. A heterogeneous plan's
 * bucketing scratch (per-class element lists, counts, tile queues) comes from a static array of the library
 * (16 MiB of element lists plus a 4 KiB header per device, held until the process ends) instead of the
 * plan's allocated scratch; the call allocates nothing and calls no allocating routine, and the kernels clear
 * what must start at zero. Limit: nclass * nelem <= 4194304 (STP_E_INVAL beyond, before any launch).
 * Classes with their own launch run on hip_stream (no side streams). Every call on one device shares that
 * device's array, which keeps the last call's contents: calls that overlap on one device race, whatever
 * their plan; queue them on one stream. Single-class plans use no scratch and behave exactly as stp_run. */
stp_status stp_run_noalloc(stp_plan_t plan, const stp_batch* batch, void* hip_stream);

/* One corrector step on a periodic Cartesian mesh (the update of Sec. II-A, Eq. (5)): from q(t_n) and the
 * predictor's outputs of every element, q(t_{n+1}) = q(t_n) + dt sum_d favg[d] + dt (face terms). The
 * numerical flux is linear (a Rusanov flux in fluctuation form, upwind for a single wave): at the face of an
 * element with outward normal s e_d and states q-/F- (own face projections of q-bar and A_d q-bar) and q+/F+
 * (the neighbour's), the correction is C = 1/2 alpha (q+ - q-) - 1/2 s (F+ - F-) - 1/2 s Bbar_d (q+ - q-),
 * Bbar_d the mean of both elements' B_d and alpha the larger fastest wave speed (acoustic sqrt(K/rho),
 * elastic sqrt((lambda + 2 mu)/rho), generic max_d ||A_d + B_d||_inf; curvilinear elements with affine
 * geometry, STP_ELASTIC_CURV with STP_PARAM_PER_ELEMENT: B_d = sum_j G[d][j] M_j, the mean taken of the two
 * elements' products, and sqrt((lambda + 2 mu)/rho) max_d |G[d][:]|_2; curved elements, parameters per node:
 * the same with each side's parameters extrapolated to the face point by the face vectors, or read from
 * stp_step.fparams (stp_face_params), so the material must be smooth inside an element). Node k receives
 * dt l_{k_d}(face) / (h w_{k_d}) C at its face node (collocation on the plan's nodes, diagonal mass matrix).
 * Elements e = (iz * ny + iy) * nx + ix, uniform size h, periodic in x, y and z; layouts as in stp_batch,
 * contiguous (element e at e * size). Stability of the full step needs dt <= about 0.2 h / ((2N+1) c_max). */
typedef struct {
    int nx, ny, nz;       /* elements per direction (nx * ny * nz <= 2^31 - 1)                               */
    double dt, h;         /* time step (>= 0) and element size (> 0)                                          */
    const void* Q;        /* q(t_n) [e][n^3][m]                                                               */
    const void* params;   /* presets: [e][np] (np = 2, 3 or 12, STP_PARAM_PER_ELEMENT); curvilinear without
                             STP_PARAM_PER_ELEMENT: [e][n^3][12]                                             */
    const void* A;        /* generic: [e][d][m][m] (STP_COEF_PER_ELEMENT); NULL without STP_A_PRESENT         */
    const void* B;        /* generic: [e][d][m][m]                                                            */
    const void* favg;     /* stp_run outputs of the same elements with the same dt and h                      */
    const void* qface;
    const void* fface;    /* with STP_A_PRESENT only                                                          */
    void* Qnew;           /* q(t_{n+1}) [e][n^3][m]; must not alias Q, favg or qface                          */
    const void* fparams;  /* curved curvilinear elements, optional: params extrapolated to the face points,
                             [e][6][n^2][12] from stp_face_params of the same params (NULL: the corrector
                             extrapolates them at every step, with the same arithmetic); NULL otherwise     */
} stp_step;

/* Queue the corrector of one step on `hip_stream`. Needs a single-class plan with per-element coefficients
 * (curvilinear elements: per element or per node) and no point source (STP_E_UNSUPPORTED otherwise);
 * STP_E_INVAL for NULL or aliasing buffers, a mesh dimension < 1, h <= 0 or dt < 0. I/O precision as the plan's (double for STP_FP64, else float). */
stp_status stp_correct(stp_plan_t plan, const stp_step* step, void* hip_stream);

/* The parameters of curved curvilinear elements (STP_ELASTIC_CURV without STP_PARAM_PER_ELEMENT, params
 * [e][n^3][12]) at the points of their six faces: each of the 12 values extrapolated along the face normal
 * with the face vector l_j(0) or l_j(1) of the plan's nodes, the face projection of Sec. II-A applied to the
 * material and metric fields. fparams [e][6][n^2][12], faces and face nodes ordered as qface. These are the
 * values the corrector forms at every face point; they do not change between steps, so a time loop computes
 * them once and hands them to every stp_correct in stp_step.fparams, which then reads 24 values per face
 * point instead of 24 n. The result is bit-identical to the corrector's own extrapolation. Queued on
 * hip_stream (NULL = the null stream); allocates nothing; stream-capturable. STP_E_UNSUPPORTED unless the
 * plan has a single class, a curved curvilinear one; STP_E_INVAL for NULL buffers, nelem outside
 * 0..2^31-1 or fparams overlapping params. I/O precision as the plan's. */
stp_status stp_face_params(stp_plan_t plan, int64_t nelem, const void* params, void* fparams, void* hip_stream);

/* Describe the plan's choices as a JSON object into buf (NUL-terminated): per class the kernel variant,
 * whether it is tiled in the persistent heterogeneous launch and its elements per tile, FP64 accumulation,
 * and whether its kernel keeps B_d on chip ("on_chip_B"); the persistent grid per CU and the tile LDS
 * budget. STP_E_INVAL for a NULL plan or buffer, or when len
 * is too small (the message states the size needed). */
stp_status stp_plan_describe(stp_plan_t plan, char* buf, size_t len);

/* Reserve the device scratch of heterogeneous plans (per-class element lists and tile queues) for batches of
 * up to max_nelem elements, so that later stp_run calls allocate nothing: with a reservation in place stp_run
 * queues only kernels (no allocation, memset or host synchronisation) and can be captured into a HIP graph.
 * Synchronous; a no-op for single-class plans. STP_E_INVAL for a NULL plan or max_nelem outside
 * 0..2^31-1, STP_E_DEVICE if the allocation fails. */
stp_status stp_reserve(stp_plan_t plan, int64_t max_nelem);

/* Serving: enqueue a batch for the plan's dispatcher thread. The batch descriptor is copied; its device
 * buffers must stay valid until stp_poll reports completion. The serving streams do not wait for any other
 * stream: work that produces the inputs (or touches the outputs) must be complete before stp_submit. With the
 * environment variable STP_SERVE_SPLIT = k > 0 at plan creation, a batch of more than k elements is queued as
 * parts of at most k consecutive elements, which run on different serving lanes (default: not split); the
 * ticket completes when every part has. Admission: each part's output+scratch bytes must fit
 * serve_mem_budget (STP_E_NOMEM if it never can); parts wait while the in-flight total would exceed it.
 * Returns STP_E_BUSY when the queue would hold more than 65536 pending parts. */
stp_status stp_submit(stp_plan_t plan, const stp_batch* batch, uint64_t* ticket);

/* stp_submit with a deadline: every part of the batch must be launched within timeout_s seconds of the
 * submission. Parts still queued when it passes are dropped (their elements' outputs are not written; parts
 * already launched run to completion) and the ticket completes with STP_E_TIMEOUT. timeout_s = HUGE_VAL is
 * stp_submit; STP_E_INVAL for a negative or NaN timeout. */
stp_status stp_submit_deadline(stp_plan_t plan, const stp_batch* batch, double timeout_s, uint64_t* ticket);

/* Query a ticket. Returns STP_PENDING while queued or running, STP_OK once complete (info filled, the
 * ticket retired), STP_E_INVAL for an unknown or already retired ticket, or for a completed batch with class
 * ids outside 0..nclass-1 (those elements' outputs were not written), STP_E_TIMEOUT when its deadline passed
 * before all of it was launched, STP_E_DEVICE if a launch failed. A failed ticket is retired too. info may be
 * NULL; t_start is the launch of its first part, t_done the completion of its last. */
stp_status stp_poll(stp_plan_t plan, uint64_t ticket, stp_ticket_info* info);

/* Wait until every submitted ticket of the plan has completed (completion info stays pollable). */
stp_status stp_drain(stp_plan_t plan);

/* Algorithmic cost of one element of a class: HBM bytes (inputs read once, outputs written once, in the
 * plan's I/O precision) and flops (derivatives of only the quantities B_d reads, pointwise terms, time
 * accumulation, faces). Either pointer may be NULL. */
stp_status stp_class_cost(stp_plan_t plan, int cls, double* bytes, double* flops);

/* Message of the last failure on the calling thread ("" if none). Valid until the next call. */
const char* stp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* STP_H */
