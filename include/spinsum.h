/*
 * spinsum.h -- C-ABI of libspinsum, spin summations on AMD Instinct MI355X
 * (gfx950).
 *
 * The operation (Springer, Matthews, Bientinesi, "Spin Summations: A
 * High-Performance Perspective"):
 *
 *   Def. 1 (Eq. 1-2)  a permutation pi_{phi(1)...phi(d)} maps the index tuple
 *                     (i_1..i_d) to (i_phi(1)..i_phi(d)).  In this API a
 *                     permutation is an array p[0..d-1] of 0-based positions,
 *                     p[m] = phi(m+1) - 1.
 *   Def. 2 (Eq. 3)    B_i <- A_{pi(i)}: a term (p, alpha) adds
 *                     alpha * In[.., i_{p[0]}, .., i_{p[d-1]}, ..] to
 *                     Out[.., i_0, .., i_{d-1}, ..].
 *   Def. 3 (Eq. 4)    a spin summation is Out <- sum_t alpha_t pi_t(In).
 *   Def. 4 (Eq. 5-6)  a factorised summation is a chain of stages
 *                     S_K(...S_1(In)); stage 0 of the arrays below is S_1,
 *                     the innermost factor, applied first.
 *   Sec. 4.6.5        the in-place form In <- sum_t alpha_t pi_t(In) on
 *                     hyper-square groups.
 *
 * Tensor layout: C-contiguous (row-major, last index fastest), extents
 * [outer spectators..., N x d, inner spectators...]: the permuted group is d
 * consecutive dimensions, all of extent N (Sec. 3.1 "hyper-square"); every
 * outer spectator index selects one "cube" of N^d * R contiguous elements,
 * R being the product of the inner spectator extents (1 when the group is
 * trailing).  Inner spectators are not permuted: each group position holds
 * a contiguous run of R elements that moves as a whole.
 *
 * Conventions shared by every entry point:
 *   - every function returns a spinsum_status; no exception crosses the ABI;
 *   - the caller owns all tensor buffers and streams; a plan owns its host
 *     and device tables and frees them in spinsum_plan_destroy;
 *   - `stream` is a hipStream_t (NULL = the default stream);
 *   - tensor pointers are device pointers, 16-byte aligned;
 *   - exec/adjoint calls are asynchronous and stream-ordered, allocate
 *     nothing and never synchronise, so they may be captured in a hipGraph;
 *   - a plan is bound to the device that was current when it was made;
 *   - a plan is not changed by exec/adjoint/exec_batched (they only read
 *     it), so their calls may overlap on several streams and host threads;
 *     spinsum_plan_set_tile, spinsum_autotune
 *     and spinsum_plan_destroy need exclusive use of the plan, and
 *     spinsum_coef_grad calls on one plan must not overlap (they share the
 *     plan's partial-sum buffer);
 *   - HIP failures return SPINSUM_ERR_HIP and the hipError_t is kept on the
 *     plan (spinsum_plan_last_hip_error).
 */
#ifndef SPINSUM_H
#define SPINSUM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SPINSUM_OK = 0,
  SPINSUM_ERR_INVALID_ARG = -1,      /* null pointer, bad count, bad dim, wrong device */
  SPINSUM_ERR_NOT_PERMUTATION = -2,  /* a term is not a bijection of 0..d-1 */
  SPINSUM_ERR_EXTENT_MISMATCH = -3,  /* group extents differ (not hyper-square) */
  SPINSUM_ERR_UNSUPPORTED = -4,      /* d not in {2,3,4}, sizes beyond the limits, tile too big */
  SPINSUM_ERR_ALIASING = -5,         /* out-of-place buffers overlap */
  SPINSUM_ERR_MISALIGNED = -6,       /* tensor pointer not 16-byte aligned */
  SPINSUM_ERR_OUT_OF_MEMORY = -7,    /* host or device allocation failed */
  SPINSUM_ERR_HIP = -8,              /* a HIP runtime call failed */
  SPINSUM_ERR_NO_DEVICE = -9         /* plan made with SPINSUM_FLAG_HOST_ONLY */
} spinsum_status;

typedef enum { SPINSUM_F64 = 0, SPINSUM_F32 = 1 } spinsum_dtype;

/* Plan flags (bitwise or). */
#define SPINSUM_FLAG_HOST_ONLY 0x1u      /* build host tables only, for inspection: exec is
                                            refused and tiles larger than a CU's LDS are kept */
#define SPINSUM_FLAG_NO_NT_STORES 0x2u   /* cached stores instead of non-temporal ones (Sec. 4.6.3
                                            ablation; implies the one-shot kernel) */
#define SPINSUM_FLAG_CHAIN_STAGES 0x4u   /* apply the stages one after another in registers
                                            instead of their pre-multiplied product (Def. 4)  */
#define SPINSUM_FLAG_NO_XCD_REMAP 0x8u   /* plain workgroup order (ablation of XCD grouping) */
#define SPINSUM_FLAG_REVERSE_ORDER 0x10u /* process work items in reverse order (ownership test) */
#define SPINSUM_FLAG_NO_LDS_PAD 0x20u    /* unpadded LDS tiles (bank-conflict ablation) */
#define SPINSUM_FLAG_NO_DIRECT_LDS 0x40u /* never use the direct-LDS variant (ablation)  */
#define SPINSUM_FLAG_NT_STORES 0x100u    /* non-temporal stores even where the planner would
                                            use cached ones (see spinsum_plan_info_t.nt_stores) */
#define SPINSUM_FLAG_MULTI_PASS 0x200u   /* one launch per stage, stage 0 from the input to the
                                            output and every later stage in place on the output:
                                            the two-pass form of Alg. 3 (Sec. 4.3) with the
                                            output as its temporary (ablation of the fused
                                            chain; not with SPINSUM_FLAG_CHAIN_STAGES) */
#define SPINSUM_FLAG_FULL_GROUP 0x400u   /* tile under the whole of S_d even where the operator's
                                            permutations move a smaller run of axes (ablation of
                                            the reduction described at spinsum_plan) */
#define SPINSUM_FLAG_NO_NT_LOADS 0x800u  /* default-policy tile loads where the planner would use
                                            non-temporal ones (see spinsum_plan_info_t.nt_loads) */
#define SPINSUM_FLAG_INDEX_PAIRS 0x80u   /* index-pair form: the d dims right before the group
                                            (the partner indices, extent V each) are permuted
                                            by the same permutation as the group, e.g.
                                            T[a,b,c,i,j,k] with (a,i), (b,j), (c,k) as pairs */

typedef struct spinsum_plan_s* spinsum_plan_t;
typedef struct spinsum_graph_s* spinsum_graph_t;

/* Kernel variants (spinsum_tile_t.variant). */
#define SPINSUM_VARIANT_AUTO 0
#define SPINSUM_VARIANT_DIRECT_LDS 1   /* one item per workgroup, loads straight into LDS
                                          (16-byte rows only; unpadded LDS)               */
#define SPINSUM_VARIANT_REG_PIPELINE 2 /* persistent workgroups, next item prefetched into
                                          registers while the current one is processed   */
#define SPINSUM_VARIANT_REG_ONESHOT 3  /* one item per workgroup, loads through registers */
#define SPINSUM_VARIANT_LDS_PIPELINE 4 /* persistent workgroups, direct LDS loads of the next
                                          item into a second LDS buffer (16-byte rows only;
                                          unpadded LDS)                                  */

/* Tile configuration (the blocking of Alg. 5a/5b, Sec. 4.5).
 * bl: tile edge along every group axis, 1 <= bl <= N; bl == N processes whole
 *     cubes.  cubes_per_wg: whole-cube mode only, spectator cubes per
 *     workgroup (>= 1).  threads: workgroup size, 256, 512 or 1024 for
 *     SPINSUM_VARIANT_DIRECT_LDS (0: chosen so that the workgroups that fit
 *     a CU's LDS hold about 16 waves), always 256 for the other variants.
 *     lds_pad: 1 = odd LDS strides (register variants only).  variant:
 *     SPINSUM_VARIANT_*.  0 in bl / cubes_per_wg / threads / variant means
 *     "choose". */
typedef struct {
  int bl;
  int cubes_per_wg;
  int threads;
  int lds_pad;
  int variant;
  int item_tiles;  /* tile-orbit mode: 0 = one tile orbit per work item; > 0 =
                      runs of consecutive orbits of a cube (in the planner's
                      orbit order, next fit) packed into items of at most
                      max(item_tiles, largest orbit) tiles and 8 orbits.  A
                      tile the planner picks itself (bl == 0) may pack; see
                      spinsum_plan_info_t.items_per_cube */
} spinsum_tile_t;

typedef struct {
  int d;                 /* group size                                   */
  int n;                 /* group extent N                               */
  int64_t ncubes;        /* spectator cubes (sum over blocks if batched) */
  int64_t elems;         /* total elements                               */
  int nstages;           /* stages after canonicalisation                */
  int nterms_expanded;   /* distinct permutations of the expanded sum    */
  int bl, nb, norbits, cubes_per_wg, threads, max_tiles, variant, lds_pad;
  int64_t lds_bytes;     /* LDS per workgroup                            */
  int64_t nitems;        /* workgroup work items per exec                */
  int nblocks;           /* 1, or the batch size                         */
  int dtype, inplace, vector_width, ragged;
  int fits_lds;          /* 1 if the largest work item fits the LDS of a CU */
  int items_per_cube;    /* work items (groups of tile orbits) per cube    */
  int item_tiles;        /* tiles of the largest work item                 */
  int chunks_per_thread; /* 16-byte loads per thread for the largest item */
  int64_t rep_lds_bytes; /* LDS for the element-orbit representatives      */
  int inner;             /* elements of the inner spectator run (1: trailing group) */
  int pair_extent;       /* index-pair form: partner extent V, else 0    */
  int64_t batch_item_bytes; /* batched: whole-cube items are packed up to this size */
  int batch_persistent;  /* batched: 1 = persistent workgroups walk the item list,
                            0 = one workgroup per item */
  int nt_stores;         /* 1: non-temporal stores (default where tile rows are at least
                            64 bytes and a cube has at most 128 tile orbits, and for whole
                            cubes); 0: cached stores, which let the L2 merge the partial
                            128-byte lines that short rows or far-apart items write */
  int exec_d;            /* axes of the group the kernels permute: d, or fewer where the
                            operator's permutations move a smaller run of axes (see
                            spinsum_plan); the tiling fields above describe that group */
  int exec_group_first;  /* its first dim */
  int persistent_per_cu; /* persistent kernel variants and persistent batched plans:
                            workgroups launched per CU (the kernel's occupancy, taken
                            when the tables are built); else 0 */
  int nt_loads;          /* 1: the direct-LDS kernel loads tiles with the non-temporal
                            policy, chosen where every work item owns the 128-byte lines
                            it reads (whole cubes, or tile rows that start and end on line
                            boundaries, for a tensor that starts on a 128-byte boundary as
                            allocations do; an offset view shares some lines between items,
                            which costs speed, not results), and for the whole-cube items
                            of batched plans; 0: default policy, which keeps lines that
                            several items share in the L2 */
  int coef_grad_split;   /* 1: spinsum_coef_grad keeps one tensor in LDS at a time (the
                            upstream gradient waits in registers while x's orbits are
                            gathered), on this plan's tiling; 0: both tensors in LDS */
  int unpack_bl;         /* tile edge of spinsum_unpack: its own tiling of the largest
                            items a CU holds (whole cubes where a cube fits the LDS, else
                            the largest edge whose rows are whole 128-byte lines), or the
                            plan's bl; 0 for index-pair and batched plans */
  int unpack_persistent; /* 1: unpacking runs persistently: each workgroup keeps one item
                            template (a tile orbit or the whole cube), walks its XCD's
                            range of cubes and requests the next cube's packed values
                            before the current item's stores; 0: one item per
                            workgroup */
  int unpack_nt_stores;  /* 1: unpacking stores with the non-temporal policy */
} spinsum_plan_info_t;

/* Create a plan for Out = S_K(...S_1(In)) (Def. 3-4; in-place: Sec. 4.6.5).
 *   ndim, extents : tensor shape, C-contiguous, all extents >= 0.
 *   group_first, d: the permuted group is dims [group_first, group_first+d);
 *                   d in {2,3,4}; dims after it are inner spectators
 *                   (N^d times their product must stay below 2^31
 *                   elements).
 *   nstages >= 1, nterms[k] >= 0 terms in stage k; perms holds sum(nterms)
 *                   rows of d 0-based entries; alpha holds sum(nterms)
 *                   coefficients.  Duplicate permutations within a stage are
 *                   merged (coefficients summed) and zero coefficients are
 *                   dropped.
 *   dtype         : storage and accumulation type (coefficients are rounded
 *                   to it).  inplace: 1 = exec requires in == out.
 *   flags         : SPINSUM_FLAG_*.
 * Index-pair form (SPINSUM_FLAG_INDEX_PAIRS; the paired indices of the
 * coupled-cluster quantities of Sec. 1): dims [group_first - d, group_first)
 * are the partners, all of one extent V (group_first >= d, else
 * SPINSUM_ERR_INVALID_ARG; unequal partner extents give
 * SPINSUM_ERR_EXTENT_MISMATCH), and a term (p, alpha) adds
 *   alpha * In[.., a_{p[0]}..a_{p[d-1]}, i_{p[0]}..i_{p[d-1]}, ..]
 * to Out[.., a_0..a_{d-1}, i_0..i_{d-1}, ..].  Dims before the partners are
 * outer spectators, dims after the group inner spectators.  V <= 1 or
 * N <= 1 reduce to the plain form (over the group, or over the partners).
 * Pair plans run the direct-LDS kernel only, need V * ceil(N / bl) <= 16000,
 * at most 2^26 tile orbits per pair block (their table takes 8 bytes each)
 * and fewer than 2^31 work items, and have no coefficient gradient or
 * autotuner (SPINSUM_ERR_UNSUPPORTED).
 * Subgroup (Sec. 4.6.4, the connected components of Fig. 1b): the terms
 * with nonzero coefficient generate a subgroup H of S_d, and every element
 * (tile) orbit under H lies inside one under S_d.  Where all permutations
 * of the operator (every stage) move only a contiguous run of the group's
 * axes [s, e) with e - s >= 2, the plan executes the summation over those
 * axes alone -- the axes before them become outer spectators, those after
 * them inner spectators that move as whole contiguous runs -- unless
 * SPINSUM_FLAG_FULL_GROUP is set (not for index pairs).  The result is the
 * same; spinsum_plan_info_t.exec_d / exec_group_first report the group the
 * kernels permute.
 * Host arrays are copied; the caller keeps ownership.  On error *plan is set
 * to NULL. */
spinsum_status spinsum_plan(spinsum_plan_t* plan, int ndim, const int64_t* extents,
                            int group_first, int d, int nstages, const int* nterms,
                            const int* perms, const double* alpha, spinsum_dtype dtype,
                            int inplace, unsigned flags);

/* Plan for many tensors ("blocks") that share d, the terms, dtype and the
 * in-place choice but have their own shapes (Def. 3-4 on each block; the
 * blocks form one task list, as the tasks of Alg. 5a): block b has ndims[b]
 * dims with extents extents[b][0..ndims[b]-1] and its permuted group is
 * dims [group_first, group_first + d) -- the same position in every block,
 * with the dims after it as inner spectators -- or, with group_first = -1,
 * the trailing d dims of each block.  Every block must satisfy the limits
 * of spinsum_plan (N^d times the inner run below 2^31 elements).  Arrays
 * are copied.  Executed by one kernel launch (spinsum_exec_batched): one
 * work item per workgroup, or persistent workgroups walking the item list
 * (spinsum_autotune picks; spinsum_plan_info_t.batch_persistent).
 * SPINSUM_FLAG_INDEX_PAIRS is not supported (SPINSUM_ERR_UNSUPPORTED), and
 * SPINSUM_FLAG_CHAIN_STAGES is ignored (the stages are pre-multiplied).
 * On error *plan is set to NULL. */
spinsum_status spinsum_plan_batched(spinsum_plan_t* plan, int nblocks, const int* ndims,
                                    const int64_t* const* extents, int group_first, int d,
                                    int nstages, const int* nterms, const int* perms,
                                    const double* alpha, spinsum_dtype dtype, int inplace,
                                    unsigned flags);

/* Replace the tile configuration of a single-tensor plan and rebuild its
 * tables (used by the autotuner).  Fields equal to 0 are chosen by the
 * planner.  Returns SPINSUM_ERR_UNSUPPORTED if the tile orbit does not fit
 * the 160 KiB LDS of a CU. */
spinsum_status spinsum_plan_set_tile(spinsum_plan_t plan, const spinsum_tile_t* tile);

spinsum_status spinsum_plan_get_info(spinsum_plan_t plan, spinsum_plan_info_t* info);

/* The expanded operator: the distinct permutations of the product of all
 * stages with non-zero coefficient (host arrays of capacity `cap` terms;
 * *nterms receives the count even when it exceeds cap). */
spinsum_status spinsum_plan_expanded(spinsum_plan_t plan, int cap, int* nterms, int* perms,
                                     double* alpha);

/* Host check of the work decomposition of block `block` of the plan: every
 * tile orbit is closed under all permutations of the group, and every
 * element of a cube is owned by exactly one (orbit, representative,
 * permutation) triple up to the repeats of degenerate element orbits.
 * Returns SPINSUM_OK or SPINSUM_ERR_INVALID_ARG with a message in *why. */
spinsum_status spinsum_plan_check_ownership(spinsum_plan_t plan, int block, const char** why);

/* Out = S(In) on `stream` (Def. 3-4).  In-place plans need in == out;
 * out-of-place plans reject overlapping buffers (SPINSUM_ERR_ALIASING). */
spinsum_status spinsum_exec(spinsum_plan_t plan, const void* in, void* out, void* stream);

/* Batched form of spinsum_exec (Def. 3-4 on every block of the plan, as one
 * task list, Alg. 5a): in/out are DEVICE arrays of nblocks device pointers
 * (8-byte aligned arrays; every block pointer 16-byte aligned, each block
 * in place or not overlapping its output, as for spinsum_exec -- the
 * pointers are read by the kernel, so these are not checked here).  The
 * caller owns the arrays and the block buffers.  Asynchronous on `stream`,
 * allocates nothing; SPINSUM_ERR_INVALID_ARG for a plan that is not
 * batched or NULL arrays, SPINSUM_ERR_MISALIGNED for misaligned arrays. */
spinsum_status spinsum_exec_batched(spinsum_plan_t plan, const void* const* in,
                                    void* const* out, void* stream);

/* grad_in = S^T grad_out, the adjoint of the linear map (the transpose of
 * the permutation matrices of Def. 2: every permutation replaced by its
 * inverse, stages in reverse order).  In-place plans need grad_out ==
 * grad_in. */
spinsum_status spinsum_adjoint(spinsum_plan_t plan, const void* grad_out, void* grad_in,
                               void* stream);

/* Coefficient gradient (not in the paper; the derivative of <g, S(x)> with
 * respect to the coefficient of each permutation, Def. 2-3): grad[r] =
 * <g, pi_r(x)> for the r-th permutation of the group in lexicographic order
 * (d! values, r = 0 the identity), for the plan's tensor shape.  x and g are
 * device tensors of the plan's shape and dtype (16-byte aligned); grad is a
 * device array of d! doubles (8-byte aligned), overwritten.  The sums are
 * accumulated in double (per workgroup, then atomically into 2048 partial
 * sums per permutation held by the plan, then one reduction), so the last
 * bits may differ from run to run; calls on one plan must not overlap.
 * Needs the direct-LDS tile layout (whole cubes, or tile rows of whole
 * 16-byte chunks) and a plan without SPINSUM_FLAG_INDEX_PAIRS:
 * SPINSUM_ERR_UNSUPPORTED otherwise.  Where the plan's whole cubes are too
 * large for both tensors in one CU's LDS, the gradient runs on tiles of its
 * own, made with the plan.  Asynchronous on `stream`. */
spinsum_status spinsum_coef_grad(spinsum_plan_t plan, const void* x, const void* g,
                                 double* grad, void* stream);

/* Unpacking (the paper names tensor unpacking, Sec. 1 and Sec. 7, as another
 * sum of permutations; its layout is not fixed there).  A packed tensor
 * holds one value per strictly increasing tuple i_0 < ... < i_{d-1} of the
 * group, in lexicographic order, for every outer spectator index and inner
 * run: shape [outer..., C(N, d), inner...], C-contiguous.
 *   spinsum_unpack: full = S(E(packed)), E putting the packed values at the
 *     strictly increasing positions of a zero tensor and S the plan's
 *     operator (Def. 3; its pre-multiplied form).  With S the
 *     antisymmetriser (every permutation weighted by its sign) this is the
 *     unpacking of an antisymmetric tensor: full[sigma . x] = sgn(sigma) *
 *     packed[x] for increasing x, zero where indices repeat.
 *   spinsum_pack: the adjoint, packed = E^T S^T full: for every strictly
 *     increasing x, sum over sigma of a(sigma^-1) full[sigma . x].
 * The plan is an ordinary plan of the full tensor's shape (not batched, not
 * index pairs), run on the whole group's tiles in the direct-LDS layout
 * (SPINSUM_ERR_UNSUPPORTED otherwise, and for N >= 65536).  full: device
 * pointer, 16-byte aligned; packed: device pointer aligned to the element
 * size; the two must not overlap (SPINSUM_ERR_ALIASING).  Out-of-place,
 * asynchronous on `stream`, allocates nothing. */
spinsum_status spinsum_unpack(spinsum_plan_t plan, const void* packed, void* full, void* stream);
spinsum_status spinsum_pack(spinsum_plan_t plan, const void* full, void* packed, void* stream);

/* Gradients with respect to the coefficients of every stage of a chain
 * (Def. 4; not in the paper): S = S_K ... S_1 is linear in the coefficients
 * of each stage, so for L = <g, S(x)> and stage k
 *   dL / d alpha_{k,p} = < (S_K ... S_{k+1})^T g , pi_p (S_{k-1} ... S_1 x) >,
 * the inner stages applied forward and the outer ones as adjoints, one
 * launch per stage (as SPINSUM_FLAG_MULTI_PASS), then the kernels of
 * spinsum_coef_grad.  grad[k * d! + r] receives that value for the r-th
 * permutation of the group in lexicographic order and stage k (stage 0 =
 * S_1, applied first); grad is a device array of nstages * d! doubles.
 * work_u, work_h: device buffers of the plan's shape and dtype that are
 * overwritten (caller-owned; NULL allowed when the plan has one stage).
 * x, g as for spinsum_coef_grad; same restrictions and errors.  Calls on
 * one plan must not overlap.  Asynchronous on `stream`. */
spinsum_status spinsum_coef_grad_stages(spinsum_plan_t plan, const void* x, const void* g,
                                        double* grad, void* work_u, void* work_h, void* stream);

/* spinsum_coef_grad for callers that cannot allocate device memory (code
 * under hipGraph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, but the partial sums go to a
 * static array of the library (kGradSlots x d! doubles, at most 384 KiB per
 * GPU, held until the process ends) instead of the plan's buffer.  Calls no
 * hipMalloc/hipFree; the first call on a device looks up that device's
 * copy of the array (hipGetSymbolAddress).  Every call on one GPU shares
 * the array: calls that overlap on one GPU (any plans, any streams) race
 * and must be serialised by the caller.  Sizes beyond the array
 * (SPINSUM_ERR_UNSUPPORTED) cannot occur for d <= 4.  Arguments, layout and
 * errors as spinsum_coef_grad. */
spinsum_status spinsum_coef_grad_noalloc(spinsum_plan_t plan, const void* x, const void* g,
                                         double* grad, void* stream);

/* Capture one spinsum_exec_batched launch into a hipGraph (captured on a
 * private stream) and instantiate it.  The pointer arrays must stay valid
 * for the life of the graph, and so must the plan's device tables: create
 * the graph again after spinsum_plan_set_tile or spinsum_autotune. */
spinsum_status spinsum_graph_create(spinsum_plan_t plan, const void* const* in,
                                    void* const* out, spinsum_graph_t* graph);
spinsum_status spinsum_graph_launch(spinsum_graph_t graph, void* stream);
void spinsum_graph_destroy(spinsum_graph_t graph);

/* Time candidate tile configurations of a single-tensor plan on the given
 * buffers (their contents are overwritten with unspecified values), keep
 * the fastest in the plan and, if cache_path is not NULL, record it in that
 * cache file (one "key value" line per configuration).  *best_ms receives
 * the best time of one exec.  Synchronises the stream.  Index-pair plans:
 * SPINSUM_ERR_UNSUPPORTED.  Batched plans: in/out are the DEVICE arrays of
 * block pointers of spinsum_exec_batched; the candidates are the size up to
 * which whole cubes are packed into one work item (8 to 64 KiB) and one
 * workgroup per item against persistent workgroups walking the item list;
 * best->cubes_per_wg receives the item size in KiB and best->variant 1 for
 * the persistent launch, 0 otherwise. */
spinsum_status spinsum_autotune(spinsum_plan_t plan, void* in, void* out, void* stream,
                                const char* cache_path, spinsum_tile_t* best,
                                float* best_ms);

/* Copy nbytes (multiple of 16) from in to out with the same load/store
 * instructions as the spin-summation kernels: the achievable HBM ceiling. */
spinsum_status spinsum_stream_copy(const void* in, void* out, int64_t nbytes, void* stream);

/* The hipError_t of the last failed HIP call made for this plan (0 if none). */
int spinsum_plan_last_hip_error(spinsum_plan_t plan);

void spinsum_plan_destroy(spinsum_plan_t plan);
const char* spinsum_status_string(spinsum_status s);
const char* spinsum_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPINSUM_H */
