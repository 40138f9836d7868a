/*
 * famlies.h -- C ABI of the MI355X (gfx950) strided tensor-contraction library.
 *
 * Operation (Approach, "Supporting tensor computations": the block-scatter
 * tensor-to-matrix mapping applies matrix algorithms directly to tensors
 * through indexing vectors; Introduction, "Challenges": tensor work fused
 * with the matrix multiplication instead of explicit tensor/matrix
 * conversion; Approach, "Variations on functionality": transposition by
 * swapping strides):
 *
 *     C[c] <- alpha * sum_p A[a(c,p)] * B[b(c,p)] + beta * C[c]
 *
 * over labelled modes (einsum semantics).  A label in A and C is a row ("I")
 * mode, in B and C a column ("J") mode, in A and B a contracted ("P") mode;
 * a label in all three is a batch mode (one independent product per batch
 * index); a label in only A or only B is summed inside that operand; a label
 * repeated within A or B selects a diagonal.  The element with multi-index idx of a
 * tensor lives at  base + sum_d idx[d] * strides[d]  (strides in elements,
 * any sign; zero allowed for A and B).  The descriptor shape follows the
 * labelled-mode tensor interfaces the paper points to (TAPP, Approach,
 * "Supporting tensor computations"; Girder 4 project plans).
 *
 * Conventions:
 *   - beta == 0: C is not read (NaN in C0 does not propagate).
 *     alpha == 0: A and B are not read.
 *   - An extent of 0 in C makes the call a no-op; an extent of 0 in a
 *     contracted mode gives C = beta * C.
 *   - Rank-0 tensors (scalars) are allowed.
 *   - FAMLIES_F32 rounds alpha and beta to float once.  The bf16x3 compute
 *     mode keeps them in double and applies them in double.
 *   - Results are deterministic run to run (no floating-point atomics).
 *
 * Errors: every call returns a famlies_status; nothing aborts or throws
 * across the ABI (a host allocation failure during planning is reported as
 * FAMLIES_ERR_ALLOC).  famlies_last_error() returns a thread-local message
 * for the last failing call on the calling thread (valid until the next
 * call).
 *
 * Handles, plans and networks are opaque, generation-counted tokens, not
 * addresses: a destroyed object's token, a token of another kind or a
 * made-up value is rejected with FAMLIES_ERR_INVALID_ARG (code safety and
 * graceful errors: Girder 1, "Code safety").
 *
 * Logging: with the environment variable FAMLIES_LOG set (not "0"), every
 * plan and planner dry run writes one line to stderr with what the planner
 * decided (sizes, orientation, loaders, tile, split-K, index width,
 * workspace).
 *
 * Ownership: the caller owns all tensor memory (device memory for data,
 * host memory for descriptors).  Descriptor arrays are copied during
 * planning and may be freed afterwards.  A plan owns its device copies of
 * the indexing vectors and any split-K workspace; famlies_execute and
 * famlies_batch_execute allocate nothing and never synchronise, so they may
 * be captured into a HIP graph.  A handle must outlive its plans.  Launches
 * of one plan share its workspace (split-K partial sums, the batched work
 * queues): they must not overlap in time (one stream, or ordered streams).
 *
 * Streams are passed as void* (a hipStream_t; NULL = the default stream).
 */
#ifndef FAMLIES_H
#define FAMLIES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t famlies_status;

#define FAMLIES_OK 0
#define FAMLIES_ERR_INVALID_ARG (-1)    /* null pointer, rank < 0 or > 8, negative extent, bad enum */
#define FAMLIES_ERR_SHAPE_MISMATCH (-2) /* one label with two different extents */
#define FAMLIES_ERR_LABEL (-3)          /* C label in neither A nor B, or repeated in C */
#define FAMLIES_ERR_UNSUPPORTED (-4)    /* valid input the library does not run (see each call) */
#define FAMLIES_ERR_ALIAS (-5)          /* C not injective, or C's span overlaps A's/B's */
#define FAMLIES_ERR_ALIGN (-6)          /* data pointer not aligned to its element size */
#define FAMLIES_ERR_ALLOC (-7)          /* device allocation failed */
#define FAMLIES_ERR_DEVICE (-8)         /* a HIP error (pending errors are reported, not cleared) */
#define FAMLIES_ERR_BOUNDS (-9)         /* planner self-check: an indexing vector would address outside
                                           its tensor's span (host-side, before any upload) */

#define FAMLIES_MAX_RANK 8

/* Element types of A, B and C (all three share one type). */
#define FAMLIES_F64 1
#define FAMLIES_F32 2

/* Compute modes.  NATIVE computes in the element type (FP64 or FP32 MFMA).
 * BF16X3 (FAMLIES_F32 only) splits every operand x into hi = RNE_bf16(x) and
 * lo = RNE_bf16(x - hi) while staging tiles, accumulates hi*hi and
 * hi*lo + lo*hi on BF16 MFMA in FP32, and combines them with alpha, beta
 * and C in FP64 before storing FP32 (mixed precision: Introduction,
 * "Challenges"; "Supporting new and mixed precisions"; the split sits in
 * the packing step as the paper's footnote on forming T*A^T inside the
 * packing of B does for another transform).  BF16X6 (FAMLIES_F32 only)
 * splits three ways (h, m = RNE_bf16(x - h), l = RNE_bf16(x - h - m)) and
 * keeps the six products hh, hm + mh, hl + mm + lh: FP32-level accuracy. */
#define FAMLIES_NATIVE 0
#define FAMLIES_BF16X3 1
#define FAMLIES_BF16X6 2
/* FP64 emulated on INT8 MFMA (FAMLIES_F64 only; new precisions, "Supporting
 * new and mixed precisions"): every row of the left operand's GEMM view and
 * every column of the right one is scaled by a power of two 2^-e (e the
 * smallest integer with max|v| <= (127/128) 2^e), the scaled values are cut
 * into s signed base-2^7 digits by exact rounding to nearest (|first digit|
 * <= 127, the others <= 64), the digit products of the pairs (t, u) with
 * t + u <= s + 1 are summed exactly in int32 on v_mfma_i32_32x32x32_i8
 * (s(s+1)/2 INT8 products per FP64 product), and the sums are recombined
 * with alpha, beta and C in FP64 (the error-free splitting of Ozaki, Ogita,
 * Oishi and Rump in the integer form of Ootomo, Ozaki and Yokota).  Error
 * against the exact result: at most K (s+4)/4 2^-7s 2^(ex+ey) |alpha| per
 * entry (ex, ey the scales of its row and column) plus FP64 rounding; a row
 * or column holding Inf or NaN gives NaN.  FAMLIES_INT8X6: s = 6 (21 INT8
 * products, about 2^-43 of the row and column scales per product);
 * FAMLIES_INT8X7: s = 7 (28 products, about 2^-50). */
#define FAMLIES_INT8X3 19
#define FAMLIES_INT8X4 20
#define FAMLIES_INT8X5 21
#define FAMLIES_INT8X6 22
#define FAMLIES_INT8X7 23

typedef struct famlies_handle_s *famlies_handle;
typedef struct famlies_plan_s *famlies_plan;

/* A labelled strided tensor.  extents, strides and labels each hold `rank`
 * entries (they may be NULL when rank == 0). */
typedef struct {
  int32_t rank;
  const int64_t *extents;
  const int64_t *strides;
  const int32_t *labels;
} famlies_tensor;

/* What the planner decided (host-side summary of a plan). */
typedef struct {
  int64_t m, n, k;          /* GEMM sizes: products of I, J and P extents */
  int64_t batch;            /* product of the batch-mode extents (1 if none) */
  int32_t swapped;          /* 1 when the kernel runs C^T = B^T A^T, so that C's
                               smallest-stride mode lies along the kernel's N */
  int32_t x_kfast, y_kfast; /* 1 when the kernel's left (X) / right (Y) operand
                               is gathered along its contracted modes */
  int32_t n_i, n_j, n_p;    /* mode groups after dropping extent-1 modes and fusing */
  int32_t n_batch;          /* batch modes (extent > 1) */
  int32_t n_trace, n_diag;  /* labels summed inside one input; labels repeated in an input */
  int32_t tile_m, tile_n, tile_k;
  int32_t split_k;          /* number of K slices (1 = none) */
  int32_t index_bits;       /* 32 or 64: width of the indexing vectors (32: every operand spans
                               under 4 GiB -- byte offsets -- or under 2^31 elements -- element
                               offsets, see index_elements; 64: element offsets) */
  int32_t kernel;           /* 1 plain, 3 bf16x3, 4 bf16x6 (1 + bf16 parts per operand), 8 + s FP64 on INT8 with s
                               slices; +16 / +32 when the kernel reads X / Y from affine unit-stride K blocks with
                               16-byte loads (block strides) */
  int32_t split_tiles;      /* split_k > 1: how many tiles run as K slices (the last ones in
                               tile order; the others run whole first); 0 without split-K */
  double flops;             /* 2*batch*m*n*k */
  int32_t index_elements;   /* 1 when the indexing vectors count elements, 0 when bytes */
} famlies_plan_info;

/* Create a handle bound to HIP device `device` (reads the tile table named by
 * the FAMLIES_TUNE_TABLE environment variable if set). */
famlies_status famlies_create(famlies_handle *out, int device);
famlies_status famlies_destroy(famlies_handle h);

/* Plan C = alpha*A.B + beta*C for one contraction (steps: validate and
 * classify labels; drop extent-1 modes, order and fuse mode groups; choose
 * the orientation and gather directions; build the block-scatter indexing
 * vectors -- the "indexing vectors" of the paper's block-scatter mapping --
 * and upload them; choose tile shape and split-K).  UNSUPPORTED when a GEMM
 * dimension reaches 2^31 - 1024.  dtype is FAMLIES_F64 or
 * FAMLIES_F32; compute is FAMLIES_NATIVE, (F32 only) FAMLIES_BF16X3 or
 * FAMLIES_BF16X6, or (F64 only) FAMLIES_INT8X3 .. FAMLIES_INT8X7.  An INT8
 * plan owns a workspace for the digit planes of both operands (s bytes per
 * element of each GEMM view, padded to its tiles) and their exponents.
 * A label summed inside one input is contracted against a zero stride in
 * the other operand (the product runs over it), so it costs MFMA work. */
famlies_status famlies_plan_contract(famlies_handle h, famlies_plan *out, int dtype, int compute,
                                     const famlies_tensor *A, const famlies_tensor *B,
                                     const famlies_tensor *C);

/* Run a plan on device pointers A, B, C (each the address of the element
 * with all-zero multi-index) on `stream`.  Checks pointer alignment and that
 * C's address span does not overlap A's or B's.  Asynchronous. */
famlies_status famlies_execute(famlies_plan p, double alpha, const void *A, const void *B,
                               double beta, void *C, void *stream);

famlies_status famlies_plan_destroy(famlies_plan p);
famlies_status famlies_plan_get_info(famlies_plan p, famlies_plan_info *out);

/* Host-only dry run of the planner: fills *info and, if offsets != NULL,
 * writes the indexing vectors of the kernel view, unpadded and in this
 * order: X rows (m entries), X contracted (k), Y contracted (k), Y columns
 * (n), C rows (m), C columns (n), then the batch offsets of X, Y and C
 * (batch entries each); element (m,k) of batch l of X is at
 * X + xbatch[l] + xrow[m] + xk[k] and so on, where X is A (or B when
 * swapped).  offsets_len must be at least 2m + 2k + 2n + 3 batch.  Touches
 * no device. */
famlies_status famlies_analyze(int dtype, int compute, const famlies_tensor *A,
                               const famlies_tensor *B, const famlies_tensor *C,
                               famlies_plan_info *info, int64_t *offsets, int64_t offsets_len);

/* Batched: n independent contractions (descriptor arrays of length n) of one
 * dtype, run by one persistent kernel over device work queues of
 * (problem, tile) items (one queue per XCD, drawn with an atomic counter
 * that the kernel clears again before it ends).  Each problem's tile is
 * BM x BN with BM, BN in {64, 128}: the batch entry of the handle's tile
 * table for its size class (written by famlies_tune from timed batched
 * launches), else 128 along each of M and N that fills it and 64 otherwise.
 * Orientation as in famlies_plan_contract; each descriptor obeys the same
 * rules.  Tensors of different problems may share memory for A and B; C
 * outputs must be disjoint (not checked).  Batch modes are UNSUPPORTED in
 * batched plans.  famlies_plan_get_info on a batched plan gives batch = n,
 * flops = the total, everything else zero. */
famlies_status famlies_batch_plan(famlies_handle h, famlies_plan *out, int dtype, int64_t n,
                                  const famlies_tensor *A, const famlies_tensor *B,
                                  const famlies_tensor *C);

/* The tile chosen for each problem of a batched plan: tile_m[i] x tile_n[i]
 * of the kernel view of problem i (after any operand exchange), 0 x 0 for a
 * problem with nothing to multiply (M, N or K zero).  Both arrays are host
 * memory of n entries, n equal to the plan's problem count (else
 * INVALID_ARG). */
famlies_status famlies_batch_plan_tiles(famlies_plan p, int32_t *tile_m, int32_t *tile_n, int64_t n);

/* A_dev, B_dev, C_dev: device arrays of n device pointers each.  One kernel
 * launch; graph-capturable. */
famlies_status famlies_batch_execute(famlies_plan p, double alpha, double beta,
                                     const void *const *A_dev, const void *const *B_dev,
                                     void *const *C_dev, void *stream);

/* Pre-packing (the packing step hoisted out of repeated calls, for an
 * operand that many contractions read: Girder 2, "Enabling optimizations
 * across layers").  famlies_pack writes user operand `operand` (0 = A,
 * 1 = B; src is its base pointer as for famlies_execute) into dst in the
 * plan's tile order -- blocks of tile rows x tile_k contracted indices,
 * [row][k], zero-filled past the edges, and for the split-bf16 modes already
 * split into bf16 parts -- so that famlies_execute_packed copies whole tiles
 * instead of gathering and splitting.  dst must hold famlies_pack_size bytes
 * and be 16-byte aligned; it is owned by the caller and valid for this plan
 * only.  UNSUPPORTED for plans whose offsets are not byte offsets (an
 * operand spanning 4 GiB or more).  Asynchronous on `stream`. */
famlies_status famlies_pack_size(famlies_plan p, int operand, size_t *bytes);
famlies_status famlies_pack(famlies_plan p, int operand, const void *src, void *dst, void *stream);
/* As famlies_execute, where bit 0 of `packed` says A points to a buffer
 * written by famlies_pack (operand 0) and bit 1 the same for B. */
famlies_status famlies_execute_packed(famlies_plan p, double alpha, const void *A, const void *B,
                                      double beta, void *C, int packed, void *stream);

/* Contraction networks: an ordered sequence of contractions over tensors
 * that are either bound by the caller or intermediates owned by the network
 * (sequences of contractions, Girder 5; packing hoisted out of repeated
 * calls, Girder 2).  Build: famlies_network_add_tensor (descriptor; an
 * intermediate gets a zeroed device allocation of its address span at
 * compile time), famlies_network_add_contraction (tensor ids; flags may ask
 * to keep A and/or B pre-packed: a bound operand is packed on the first run
 * after each bind, an intermediate on every run), famlies_network_compile
 * (plans every step).  famlies_network_bind sets a caller tensor's base
 * pointer; famlies_network_execute runs the steps in order on `stream`
 * (after the first run per binding it allocates nothing and does not
 * synchronise).  famlies_network_tensor_ptr returns a tensor's base pointer
 * (an intermediate's after compile). */
typedef struct famlies_network_s *famlies_network;
#define FAMLIES_NET_PACK_A 1
#define FAMLIES_NET_PACK_B 2
famlies_status famlies_network_create(famlies_handle h, famlies_network *out, int dtype, int compute);
famlies_status famlies_network_add_tensor(famlies_network n, const famlies_tensor *desc, int intermediate,
                                          int32_t *id);
famlies_status famlies_network_add_contraction(famlies_network n, double alpha, int32_t a, int32_t b,
                                               double beta, int32_t c, int flags);
famlies_status famlies_network_compile(famlies_network n);
famlies_status famlies_network_bind(famlies_network n, int32_t id, void *ptr);
famlies_status famlies_network_tensor_ptr(famlies_network n, int32_t id, void **ptr);
famlies_status famlies_network_execute(famlies_network n, void *stream);
famlies_status famlies_network_destroy(famlies_network n);

/* Autotune (the measured counterpart of the block-size choices that the
 * paper's control tree encodes per level, Section "Building on important
 * advances", "Nesting of algorithms and blockings"): time the candidates on
 * the handle's device for each size class (ceil(log2) of M, N, K) and write
 * the winners to table_path (text, one line per class, as read by
 * famlies_load_tune_table); the handle then uses them.
 *   plain entries: tile shape and split-K of the single-contraction kernels
 *     (FP64, FP32 and bf16x3), timed on one GEMM-shaped contraction;
 *   batch entries: tile class (BM, BN in {64, 128}) of the persistent
 *     batched kernel (FP64 and FP32), timed on batched launches of that
 *     kernel with enough identical problems to fill the device.
 * flags: FAMLIES_TUNE_QUICK (a coarse grid, fewer repetitions),
 * FAMLIES_TUNE_BATCH_ONLY or FAMLIES_TUNE_PLAIN_ONLY (one kind of entry;
 * both: INVALID_ARG).  Allocates about 1.6 GB of scratch device memory for
 * the call.  Errors: INVALID_ARG, ALLOC, DEVICE; on error nothing is
 * written and the handle's table is unchanged. */
#define FAMLIES_TUNE_QUICK 1
#define FAMLIES_TUNE_BATCH_ONLY 2
#define FAMLIES_TUNE_PLAIN_ONLY 4
famlies_status famlies_tune(famlies_handle h, const char *table_path, int flags);
/* Load a table written by famlies_tune (or by hand).  Text, '#' comments,
 * one entry per line:
 *   <plain|batch> <dtype> <compute> <log2 M> <log2 N> <log2 K> <bm> <bn> <bk> <split> [<index bits> [<split tiles>]]
 * A plan takes the entry of its size class (or the nearest one within two
 * classes).  The optional index bits 64 makes such plans use 64-bit indexing
 * vectors even when 32 bits reach every element, e32 makes them use 32-bit
 * element offsets wherever those reach (0 or 32: automatic).  The optional
 * split tiles n > 0 (plain FP64/FP32 plans with split > 1) cuts only the last
 * n tiles in tile order into K slices; the others run over all of K first.
 * Errors: INVALID_ARG for an unreadable or malformed file (the handle's table
 * is then unchanged). */
famlies_status famlies_load_tune_table(famlies_handle h, const char *table_path);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * famlies_plan_contract and famlies_execute in one call that allocates
 * nothing on the device.  The plan is made on the host and its device data
 * -- the indexing vectors and any split-K partial sums -- are placed in one
 * static device array of the library (64 MiB per device, held until the
 * process ends) instead of plan-owned allocations.  Arguments as for the two
 * calls it combines (h from famlies_create; A, B, C descriptors; a, b, c
 * device pointers to the elements with all-zero multi-index).
 * The call copies the indexing vectors into the array on `stream` and waits
 * for that stream (so earlier work on it has finished), then launches the
 * contraction asynchronously; it is not capturable into a graph.  Every call
 * on a device shares that device's array: calls on one stream are ordered,
 * calls that overlap in time on one device (other streams, other threads)
 * race and must not be made.  UNSUPPORTED when the indexing vectors and the
 * partial sums need more than 64 MiB (the message gives the size); other
 * errors as for the two calls. */
famlies_status famlies_contract_noalloc(famlies_handle h, int dtype, int compute, double alpha,
                                        const famlies_tensor *A, const void *a, const famlies_tensor *B,
                                        const void *b, double beta, const famlies_tensor *C, void *c,
                                        void *stream);

const char *famlies_last_error(void);
const char *famlies_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FAMLIES_H */
