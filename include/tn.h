/*
 * tn.h -- C ABI of the MI355X (gfx950) tensor-network contraction library.
 *
 * Operations follow "TensorNetwork: A Library for Physics and Machine
 * Learning" (arXiv:1905.01330): pairwise contraction of connected edges
 * (section III.A "Standard Edges", III.B "Edge Contraction", "Edge
 * Flattening"), trace edges (III.A "Trace Edges"), outer products (III.B,
 * the outer-product equation), ncon networks with a contraction order
 * (Appendix B), and the chain networks of section IV (MPS inner products,
 * operator environments, and the MPS classifier of section IV.A).
 *
 * Conventions for every call
 *  - Tensor data pointers are DEVICE pointers owned by the caller.  The
 *    library never allocates device memory: scratch comes from a caller
 *    workspace whose size the matching *_workspace query returns.  Host
 *    pointers (descriptors, axis lists, label lists) are read during the
 *    call only.
 *  - Every call is asynchronous on `stream` (a hipStream_t passed as void*,
 *    NULL = the default stream).  Outputs are valid once the stream reaches
 *    the point after the call.
 *  - Arguments are validated on the host before anything is launched.  An
 *    invalid call returns a negative tn_status and has no side effects;
 *    tn_last_error() then holds a one-line description (thread-local).
 *  - NaN and Inf propagate through arithmetic; they are not errors.
 *  - Real arithmetic unless a call says otherwise (the *_c64 calls take
 *    complex tensors and conjugation flags).
 *  - Calls on different streams may run concurrently; calls that write the
 *    same workspace or output on overlapping streams race.  Calls that fork
 *    part of their work to a library side stream (the two-ended inner
 *    product, the two-direction sweep, canonicalisation) take the side
 *    stream assigned to their own stream: each device has four, given to
 *    caller streams in turn.
 */
#ifndef TN_H
#define TN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TN_MAX_RANK 8

/* TN_C64: complex, interleaved (real, imaginary) FP32 pairs; strides count
 * complex elements. */
typedef enum { TN_F32 = 0, TN_F64 = 1, TN_C64 = 2 } tn_dtype;

/* Arithmetic used for the contracted-index products.
 *  FP32          FP32 operands, FP32 accumulation (matrix cores, fp32 MFMA).
 *  BF16          operands rounded to BF16 (nearest-even), FP32 accumulation.
 *  SPLIT_BF16    each FP32 operand written exactly as x0 + x1 + x2 (three
 *                BF16 terms); the six products x_i*y_j with i + j <= 2 are
 *                accumulated into one FP32 accumulator per output.
 *  SPLIT_BF16_3P two-term split, three products (error reported only). */
typedef enum {
  TN_PREC_FP32 = 0,
  TN_PREC_BF16 = 1,
  TN_PREC_SPLIT_BF16 = 2,
  TN_PREC_SPLIT_BF16_3P = 3
} tn_precision;

/* A strided view: element (i_0..i_{r-1}) lives at data + sum_k i_k*stride[k]
 * elements.  rank 0 is a scalar (one element).  Every shape[k] >= 1 and
 * every stride[k] >= 0.  dtype: TN_F32 for contractions, TN_F64 where stated. */
typedef struct {
  void* data;
  int32_t dtype;
  int32_t rank;
  int64_t shape[TN_MAX_RANK];
  int64_t stride[TN_MAX_RANK];
} tn_tensor;

typedef enum {
  TN_OK = 0,
  TN_ERR_INVALID_ARGUMENT = -1,   /* NULL pointer, rank or axis out of range, repeated axis */
  TN_ERR_SHAPE_MISMATCH = -2,     /* connected dimensions differ, or output shape is wrong */
  TN_ERR_UNSUPPORTED = -3,        /* dtype / precision / size not handled */
  TN_ERR_WORKSPACE_TOO_SMALL = -4,
  TN_ERR_ALIASING = -5,           /* output memory overlaps an input */
  TN_ERR_DEVICE = -6              /* a HIP runtime call failed (also earlier asynchronous faults) */
} tn_status;

const char* tn_status_string(int32_t status);
const char* tn_last_error(void);
/* Library version string, e.g. "tn-mi355x 0.1 gfx950". */
const char* tn_version(void);

/* ---------------------------------------------------------------------
 * Pairwise contraction (III.A "Standard Edges": a tensordot over the
 * connected axes; III.B "Edge Flattening": all edges between the two nodes
 * contracted at once, so the pairs form one flattened contracted index).
 *
 * out[free_a..., free_b...] = sum_k a[...] * b[...], with axes_a[i] of `a`
 * connected to axes_b[i] of `b` for i < n_pairs.  out's axes are the free
 * axes of a in ascending order, then those of b; out->shape must equal
 * that exactly.  out->stride may be any permutation view, which is how a
 * final reorder_edges is fused into the store.  n_pairs == 0 is an outer
 * product.  a, b, out: TN_F32, and `out` may not overlap `a` or `b`.
 * Rank-0 and rank-1 results use wavefront reductions (FP64 sums); the rest
 * is a tiled matrix-core GEMM whose operand gathers perform the index
 * permutation.
 * workspace (DEVICE, caller-owned, nullable): scratch for results with few
 * long sums (a dot product, a matrix-vector product with few rows): with at
 * least TN_REDUCE_WORKSPACE_BYTES the k range of each sum is cut over many
 * workgroups whose partials are added in a fixed order (deterministic);
 * with NULL / 0 bytes such a sum runs on one workgroup (same result, slower).
 * Calls that share one workspace must not overlap in time.
 * ------------------------------------------------------------------- */
#define TN_REDUCE_WORKSPACE_BYTES 32768
int32_t tn_contract_between(const tn_tensor* a, const tn_tensor* b, int32_t n_pairs,
                            const int32_t* axes_a, const int32_t* axes_b, tn_tensor* out,
                            void* workspace, size_t ws_bytes, int32_t prec, void* stream);

/* Complex pairwise contraction (the V^dagger of III.B: complex nodes):
 * out = op_a(a) . op_b(b) over the paired axes, op = complex conjugation
 * when conj_a / conj_b is nonzero.  a, b, out: TN_C64 (a, out of rank <= 7,
 * b of rank <= 6).  The right operand is expanded once into a real tensor
 * holding (Re b, -Im b; Im b, Re b) with the conjugation signs folded in,
 * in the workspace; one real contraction over (k, real/imaginary) then
 * writes the interleaved complex result (four real products per complex
 * product) on the real path, in precision `prec`.  workspace: at least
 * tn_contract_between_c64_workspace(b) bytes.  Errors as
 * tn_contract_between. */
int32_t tn_contract_between_c64_workspace(const tn_tensor* b, size_t* bytes);
int32_t tn_contract_between_c64(const tn_tensor* a, const tn_tensor* b, int32_t n_pairs,
                                const int32_t* axes_a, const int32_t* axes_b, int32_t conj_a,
                                int32_t conj_b, tn_tensor* out, void* workspace, size_t ws_bytes,
                                int32_t prec, void* stream);

/* Trace edge (III.A "Trace Edges"; the trace of Fig. 2):
 * out[rest] = sum_i a[.. i .. i ..] over axis1 and axis2 (equal dims),
 * rest in ascending axis order.  TN_F32. */
int32_t tn_trace_edge(const tn_tensor* a, int32_t axis1, int32_t axis2, tn_tensor* out,
                      void* stream);

/* Outer product (III.B, the outer-product equation):
 * out[i..., j...] = a[i...] * b[j...]; out shape = a.shape ++ b.shape.  TN_F32. */
int32_t tn_outer_product(const tn_tensor* a, const tn_tensor* b, tn_tensor* out, void* stream);

/* ---------------------------------------------------------------------
 * ncon network (Appendix B).  Node i has labels[offsets[i] .. offsets[i+1]),
 * one per axis.  A label >= 0 is a connected edge and appears exactly twice
 * (twice on one node = a trace edge); a label < 0 is dangling and the
 * output axes are ordered -1, -2, -3, ...  `order` lists the connected
 * labels in contraction order (n_order = 0 or order = NULL: ascending).
 * Contracting a label between two nodes contracts every edge they share
 * (flattening).  Nodes still unconnected at the end are joined by outer
 * products in node order.  The final permutation is fused into the last
 * step's store.  Intermediates, the scratch of the rank-0/1 sums (see
 * tn_contract_between) and the partial results of k-sliced steps live in
 * `workspace` (caller-owned); tn_contract_network_workspace returns the bytes
 * needed.  A step whose result spans few tiles and whose contracted extent
 * is long may run as up to 64 k-slices (one batched launch into partials,
 * then a sum in slice order; the tile tuner times the slice counts); the
 * partials take up to 64x the largest step's result, at most 16 MiB.
 * ------------------------------------------------------------------- */
int32_t tn_contract_network_workspace(int32_t n_nodes, const tn_tensor* nodes,
                                      const int32_t* labels, const int32_t* offsets,
                                      int32_t n_order, const int32_t* order, size_t* bytes);
int32_t tn_contract_network(int32_t n_nodes, const tn_tensor* nodes, const int32_t* labels,
                            const int32_t* offsets, int32_t n_order, const int32_t* order,
                            tn_tensor* out, void* workspace, size_t ws_bytes, int32_t prec,
                            void* stream);

/* The same network contraction for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): no workspace argument, no allocation of any kind.  The
 * intermediates and the split-sum scratch live in a static device array of
 * TN_NOALLOC_SCRATCH_BYTES per GPU (128 MiB), held by every GPU the library
 * runs on until the process ends; its address is looked up once per device
 * on the first call there.  Networks whose workspace query
 * (tn_contract_network_workspace) exceeds that size run their steps whole
 * (no k-slice partials) when the rest fits, and are otherwise rejected with
 * TN_ERR_UNSUPPORTED before anything runs.  The tile tuner never times
 * candidates inside this call.  Every call on one GPU shares that GPU's
 * array: calls that overlap in time on one GPU (other streams, other host
 * threads) race and must be serialised by the caller.  Otherwise the
 * arguments, results and errors are those of tn_contract_network. */
#define TN_NOALLOC_SCRATCH_BYTES (128u << 20)
int32_t tn_contract_network_noalloc(int32_t n_nodes, const tn_tensor* nodes, const int32_t* labels,
                                    const int32_t* offsets, int32_t n_order, const int32_t* order,
                                    tn_tensor* out, int32_t prec, void* stream);

/* Contraction order for the same network description (host only: reads
 * shapes, never data).  method TN_ORDER_GREEDY: repeatedly contract the
 * connected pair of nodes that is best by one criterion (fewest flops;
 * largest shrink of the network, i.e. result size minus operand sizes;
 * smallest result), one pass per criterion, keeping the pass with the
 * fewest total flops; TN_ORDER_OPTIMAL: the
 * exact minimum total flops over all pairwise contraction trees (dynamic
 * programming over node subsets, at most 12 nodes per connected component,
 * else TN_ERR_UNSUPPORTED).  Cost of a pairwise step: 2 x the product of the
 * extents of all labels on the two nodes.  Trace labels come first.
 * order (caller-owned, capacity >= number of connected labels) receives a
 * label order for tn_contract_network, *n_order its length, *flops the
 * total pairwise flops (traces excluded). */
#define TN_ORDER_GREEDY 0
#define TN_ORDER_OPTIMAL 1
int32_t tn_network_order(int32_t n_nodes, const tn_tensor* nodes, const int32_t* labels,
                         const int32_t* offsets, int32_t method, int32_t* order, int32_t* n_order,
                         double* flops);

/* ---------------------------------------------------------------------
 * MPS inner product <psi|phi> (the chain network of Fig. 3a, contracted
 * site by site).  psi[k], phi[k] are TN_F32 [D_k, d, D_{k+1}] with
 * D_0 = D_N = 1 (the two chains may have different bond dims but the same
 * d).  Result written to out2 (DEVICE, 2 doubles): out2[0] = mantissa m,
 * out2[1] = log-scale s, value = m * exp(s).  After every site the
 * environment is rescaled by a power of two (exact) and the exponent is
 * summed in FP64.  Chains of 4 or more sites are contracted from both ends
 * at once: the right half runs on a library-owned side stream (one per
 * device, default priority) forked from and joined back into `stream`, so
 * the call stays ordered on `stream` and can be recorded in a HIP graph;
 * the halves meet in an FP64 sum over the middle bond (m then in [0.5, 1)).
 * ------------------------------------------------------------------- */
int32_t tn_mps_inner_workspace(int32_t n_sites, const tn_tensor* psi, const tn_tensor* phi,
                               size_t* bytes);
int32_t tn_mps_inner(int32_t n_sites, const tn_tensor* psi, const tn_tensor* phi, double* out2,
                     void* workspace, size_t ws_bytes, int32_t prec, void* stream);

/* Complex MPS inner product <psi|phi> = sum conj(psi(s)) phi(s): psi[k],
 * phi[k] TN_C64 [D_k, d, D_{k+1}]; out4 (DEVICE, 4 doubles) = [Re m, Im m,
 * s, 0] with value m * exp(s).  Each site is two complex contractions
 * (E . phi_k, then conj(psi_k) over (a', s)) and an exact power-of-two
 * rescale of E by its largest component.  Workspace from
 * tn_mps_inner_c64_workspace. */
int32_t tn_mps_inner_c64_workspace(int32_t n_sites, const tn_tensor* psi, const tn_tensor* phi,
                                   size_t* bytes);
int32_t tn_mps_inner_c64(int32_t n_sites, const tn_tensor* psi, const tn_tensor* phi, double* out4,
                         void* workspace, size_t ws_bytes, int32_t prec, void* stream);

/* Many independent inner products in one call (chains of uneven length and
 * bond dimension).  psi_sites/phi_sites hold all chains' sites back to back;
 * chain c owns sites [site_offsets[c], site_offsets[c+1]).  out2 is DEVICE,
 * 2 doubles per chain (mantissa, log scale, as for tn_mps_inner).  Chains
 * of 4 or more sites are contracted from both ends at once; all chains
 * advance together, one site per step and end, as grouped GEMMs over every
 * half still active, and each chain's halves meet in an FP64 sum over its
 * middle bond.  Each step's grouped tile comes from the tile autotuner
 * (tn_tune: timed on the first launch per step signature and precision
 * when tuning is on and the stream is not capturing), else from a work
 * estimate. */
int32_t tn_mps_inner_batched_workspace(int32_t n_chains, const int32_t* site_offsets,
                                       const tn_tensor* psi_sites, const tn_tensor* phi_sites,
                                       size_t* bytes);
int32_t tn_mps_inner_batched(int32_t n_chains, const int32_t* site_offsets,
                             const tn_tensor* psi_sites, const tn_tensor* phi_sites, double* out2,
                             void* workspace, size_t ws_bytes, int32_t prec, void* stream);
/* The same call in two parts, so that the launches can be recorded in a
 * HIP graph and replayed.  _upload writes the work tables (chain records,
 * grouped-GEMM problems) into the workspace and waits for the copy to
 * finish on `stream` (not capturable).  _launch only launches kernels on
 * `stream` (capturable; while capturing it takes cached or estimated tiles
 * and times nothing); it uses the tables of the last _upload into the same
 * workspace, which must have been made with the same chains, tensors and
 * workspace.  Errors as tn_mps_inner_batched. */
int32_t tn_mps_inner_batched_upload(int32_t n_chains, const int32_t* site_offsets,
                                    const tn_tensor* psi_sites, const tn_tensor* phi_sites,
                                    void* workspace, size_t ws_bytes, void* stream);
int32_t tn_mps_inner_batched_launch(int32_t n_chains, const int32_t* site_offsets,
                                    const tn_tensor* psi_sites, const tn_tensor* phi_sites, double* out2,
                                    void* workspace, size_t ws_bytes, int32_t prec, void* stream);

/* ---------------------------------------------------------------------
 * Operator environments of <psi|H|psi> for an MPO H.  psi[k]: TN_F32
 * [D_k, d, D_{k+1}]; mpo[k]: TN_F32 [w_k, w_{k+1}, t, s] = <t|O|s> with
 * w_0 = w_N = 1.
 *   L_0 = 1, L_{k+1}[b', v, b] = sum A_k[a',t,b'] W_k[u,v,t,s] L_k[a',u,a] A_k[a,s,b]
 *   R_N = 1, R_k[a', u, a]     = sum A_k[a',t,b'] W_k[u,v,t,s] R_{k+1}[b',v,b] A_k[a,s,b]
 * L_out / R_out: arrays of N+1 TN_F32 tensors [D_k, w_k, D_k] (any strides),
 * or NULL to skip that direction's stores (the sweep still runs when energy
 * is requested).  energy2 (DEVICE, 2 doubles, nullable): [L_N, R_0].
 * which: bit 0 = left sweep, bit 1 = right sweep.
 * Each site is three steps: ket-site GEMM, MPO step, bra-site GEMM.  A
 * GEMM that fills few compute units (small bond dimensions) may run as
 * k-slices into the workspace, added in slice order by a second kernel
 * (the tuner's choice, deterministic for a given choice).
 * With both bits set the right sweep runs on a second stream that the
 * library owns (one per device, default priority), forked from `stream`
 * by an event before its first launch and joined back into `stream`
 * after its last, so all work stays ordered after earlier and before
 * later work on `stream` and the call can be captured in a graph.
 * ------------------------------------------------------------------- */
int32_t tn_mps_env_sweep_workspace(int32_t n_sites, const tn_tensor* psi, const tn_tensor* mpo,
                                   size_t* bytes);
int32_t tn_mps_env_sweep(int32_t n_sites, const tn_tensor* psi, const tn_tensor* mpo,
                         tn_tensor* L_out, tn_tensor* R_out, double* energy2, int32_t which,
                         void* workspace, size_t ws_bytes, int32_t prec, void* stream);

/* ---------------------------------------------------------------------
 * Left-canonical gauge in FP64 on the GPU (support step for the operator
 * sweeps): A_k reshaped (D_k d, D_{k+1}) = Q R by Householder QR with
 * diag(R) >= 0; Q replaces A_k, R is absorbed into A_{k+1}; the final 1x1 R
 * is the state's norm, written as its logarithm to *lognorm (DEVICE) and
 * divided out.  sites: TN_F64, contiguous, modified in place.  Requires
 * D_{k+1} <= d * D_k.  Each site's Q is formed on the library-owned side
 * stream (one per device, default priority) while the next site is
 * factorised; the call joins it back into `stream` before it returns, so all
 * of its work stays ordered on `stream`.
 * ------------------------------------------------------------------- */
int32_t tn_mps_left_canonicalize_workspace(int32_t n_sites, const tn_tensor* sites, size_t* bytes);
int32_t tn_mps_left_canonicalize(int32_t n_sites, tn_tensor* sites, double* lognorm,
                                 void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * MPS classifier (section IV.A).  sites[k]: TN_F32 contiguous
 * [D_k, 2, D_{k+1}] except sites[label_site] = [D_c, 2, n_labels, D_{c+1}];
 * D_0 = D_N = 1 and all inner bonds equal (chi).  pixels: TN_F32 [B, N] in
 * [0, 1], encoded by Phi(p) = (cos(pi p/2), sin(pi p/2)).
 * logits: TN_F32 [B, n_labels], f[b, l] = <W^l, Phi(x_b)>.
 * Forward keeps every left/right environment vector of each sample on chip
 * and stores one of every `ckpt_every` of them to ckpt (nullable; an opaque
 * buffer of the 4-byte words that tn_mps_classifier_ckpt_shape counts: per
 * checkpoint the B vectors as FP32 high parts, B power-of-two exponents and
 * the FP32 low parts, so a stored vector keeps about 48 significant bits)
 * for the backward.  The running vectors handed from one chain launch to
 * the next keep the same two-part form.
 * Backward: dlogits [B, n_labels] -> dsites (same shapes as sites); it
 * recomputes the vectors between checkpoints (ckpt is required there).
 * prec: FP32 or SPLIT_BF16; it applies to the label-site and weight-gradient
 * contractions.  The chain steps themselves (one site after another for
 * every sample) run on the FP64 matrix cores with FP64 running vectors,
 * stored as FP32 between kernel runs: FP32 chain steps compounded over 784
 * sites to about 3e-5 relative on the scores.
 * Requirements: 1 <= label_site <= n_sites - 2, chi <= 256, every site
 * contiguous, 1 <= ckpt_every <= 64.
 * ------------------------------------------------------------------- */
/* n_floats: 4-byte words of the checkpoint buffer for this geometry. */
int32_t tn_mps_classifier_ckpt_shape(int32_t n_sites, int32_t label_site, int32_t batch,
                                     int32_t chi, int32_t ckpt_every, int64_t* n_floats);
int32_t tn_mps_classifier_workspace(int32_t n_sites, int32_t label_site, int32_t n_labels,
                                    int32_t batch, int32_t chi, int32_t ckpt_every,
                                    size_t* bytes);
int32_t tn_mps_classifier_forward(int32_t n_sites, int32_t label_site, int32_t n_labels,
                                  const tn_tensor* sites, const tn_tensor* pixels,
                                  tn_tensor* logits, float* ckpt, int32_t ckpt_every,
                                  void* workspace, size_t ws_bytes, int32_t prec, void* stream);
int32_t tn_mps_classifier_backward(int32_t n_sites, int32_t label_site, int32_t n_labels,
                                   const tn_tensor* sites, const tn_tensor* pixels,
                                   const float* ckpt, int32_t ckpt_every,
                                   const tn_tensor* dlogits, tn_tensor* dsites, void* workspace,
                                   size_t ws_bytes, int32_t prec, void* stream);

/* Softmax cross-entropy of the scores against integer labels (the loss the
 * classifier is trained with): loss (DEVICE double) = mean_b [logsumexp(f_b)
 * - f_b[y_b]], dlogits[b, l] = (softmax(f_b)_l - [l == y_b]) / batch.
 * labels: DEVICE int64 [batch].  workspace >= 8 * batch bytes. */
int32_t tn_softmax_xent(const tn_tensor* logits, const int64_t* labels, int32_t batch, double* loss,
                        tn_tensor* dlogits, void* workspace, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------
 * Node splitting (III.B "Node Splitting"; Appendix A "Saving Memory").
 * The node `a` (TN_F32 or TN_F64, any strides) is read as the matrix
 * A[(axes 0 .. n_left-1), (axes n_left .. rank-1)] (permute the view to
 * choose the left and right edges) and decomposed as A = U S V^T in FP64 on
 * the GPU (one-sided block Jacobi; when the longer leg is at most 2048 and
 * the shorter at least 32, on R^T of a Householder QR of the matrix, whose
 * columns are closer to orthogonal, with both factors recovered through Q).
 * The new bond has at most
 * kmax = min(prod left dims, prod right dims) values.
 *
 * tn_split_node_decompose runs the decomposition into `workspace` (size
 * from tn_split_node_workspace) and applies the truncation rule: keep
 * k = max(1, min(k_count, k_err)) singular values, with
 * k_count = min(kmax, max_singular_values) (<= 0: no count limit) and k_err
 * the smallest k whose dropped values s_k .. s_{kmax-1} add up to at most
 * max_truncation_err (< 0: no error limit).  It synchronises `stream` once
 * per Jacobi sweep and at the end, and returns k (and, if `sweeps` is not
 * NULL, the sweeps run) on the host.  The workspace then holds the
 * decomposition until it is reused; the writers below read it.
 *
 * tn_split_node writes left = U sqrt(S) [left dims..., k] and right =
 * sqrt(S) V^T [k, right dims...]; tn_split_node_full_svd writes u = U,
 * s = S ([k] or a [k, k] diagonal matrix) and vh = V^T.  Outputs are
 * strided views in a's dtype; k may be any value in 1..kmax (normally the
 * decomposition's).  trun_err (nullable; [kmax - k]) receives the dropped
 * singular values, largest first.  Singular values are in descending
 * order (equal values: the order is unspecified); singular vectors of
 * zero singular values are written as zero.  Asynchronous on `stream`.
 * Errors: TN_ERR_INVALID_ARGUMENT (n_left outside 1..rank-1, k out of
 * range), TN_ERR_SHAPE_MISMATCH (an output's extents), TN_ERR_ALIASING
 * (outputs overlap each other or the node), TN_ERR_UNSUPPORTED (the
 * shorter effective leg above 16384).
 * ------------------------------------------------------------------- */
int32_t tn_split_node_workspace(const tn_tensor* a, int32_t n_left, size_t* bytes);
int32_t tn_split_node_decompose(const tn_tensor* a, int32_t n_left, int32_t max_singular_values,
                                double max_truncation_err, int32_t* k, int32_t* sweeps,
                                void* workspace, size_t ws_bytes, void* stream);
int32_t tn_split_node(const tn_tensor* a, int32_t n_left, int32_t k, tn_tensor* left, tn_tensor* right,
                      tn_tensor* trun_err, void* workspace, size_t ws_bytes, void* stream);
int32_t tn_split_node_full_svd(const tn_tensor* a, int32_t n_left, int32_t k, tn_tensor* u, tn_tensor* s,
                               tn_tensor* vh, tn_tensor* trun_err, void* workspace, size_t ws_bytes,
                               void* stream);

/* ---------------------------------------------------------------------
 * Two-site DMRG update (the algorithm section III.B "Node Splitting" names
 * as the user of node splitting).  For the two-site tensor theta[a, s1, s2,
 * b] (TN_F32 [Dl, d1, d2, Dr]) between the left environment L (TN_F32
 * [Dl, wl, Dl], layout of tn_mps_env_sweep) and the right environment R
 * ([Dr, wr, Dr]), with the operator sites w1 [wl, wm, d1, d1] and w2
 * [wm, wr, d2, d2]:
 *   (H_eff theta)[a', t1, t2, b'] =
 *     sum L[a', u, a] w1[u, v, t1, s1] w2[v, x, t2, s2] R[b', x, b] theta[a, s1, s2, b]
 * contracted as one network (L-theta, w1, w2, R) on the contraction kernels
 * in precision `prec`.
 * tn_dmrg_apply_heff: out = H_eff theta (out: theta's shape, any strides).
 * tn_dmrg_eigensolve: the lowest eigenpair of H_eff by Lanczos with full
 * reorthogonalisation, `krylov` (2..32) vectors per restart, `restarts`
 * restarts from the Ritz vector; theta (contiguous) is the starting vector
 * on entry and the normalised eigenvector on return; out2 (DEVICE, 2
 * doubles) = [energy, |H_eff theta - energy theta|].  No host
 * synchronisation.  The split of theta into two sites is tn_split_node.
 * Workspace from tn_dmrg_workspace (it also serves tn_dmrg_apply_heff).
 * ------------------------------------------------------------------- */
int32_t tn_dmrg_workspace(const tn_tensor* L, const tn_tensor* R, const tn_tensor* w1, const tn_tensor* w2,
                          const tn_tensor* theta, int32_t krylov, size_t* bytes);
int32_t tn_dmrg_apply_heff(const tn_tensor* L, const tn_tensor* R, const tn_tensor* w1, const tn_tensor* w2,
                           const tn_tensor* theta, tn_tensor* out, void* workspace, size_t ws_bytes, int32_t prec,
                           void* stream);
int32_t tn_dmrg_eigensolve(const tn_tensor* L, const tn_tensor* R, const tn_tensor* w1, const tn_tensor* w2,
                           tn_tensor* theta, int32_t krylov, int32_t restarts, double* out2, void* workspace,
                           size_t ws_bytes, int32_t prec, void* stream);

/* ---------------------------------------------------------------------
 * Tile autotuner for the contraction GEMM.
 * level 0: heuristic tiles only;
 *       1: on the first contraction of each new (shape, layout, precision)
 *          signature, time every candidate tile 3 times and keep the fastest;
 *       2: the same with 10 timed launches per candidate (less noise).
 * The uneven batched inner product is tuned the same way per site step:
 * the first launch of each (step signature, precision) times its
 * grouped tiles, re-running the step on its real inputs, and keeps the
 * fastest.
 * The GEMMs of a two-direction environment sweep and of a two-ended inner
 * product share the chip with the other direction's stream: they are
 * chosen apart from the same GEMMs issued alone (their cache lines carry
 * 1000 added to the groups field), estimated for half the compute units
 * and timed as two copies issued together on two streams.
 * Tile choices are cached per process; the cache is mutex-guarded, so
 * concurrent calls from several threads are safe.  Timing is skipped while
 * the stream is being captured into a graph (the heuristic is used then).
 *
 * tn_tune(cache_path, level): sets the level and, when cache_path is not
 * NULL, persists the choices in that text file: entries already in it are
 * loaded now (lines "M N K batch amode bmode cmode prec groups -> choice",
 * choice = tile + 100 log2(k-slices) (k-slices only inside the calls that
 * hold their scratch: up to 4 in the environment sweeps and inner products,
 * up to 64 in network steps), and
 * "G step-signature prec -> grouped tile", malformed lines are skipped) and
 * every timed choice made later is appended.
 * NULL keeps the choices in memory only.  Changing the level clears the
 * in-memory choices (the file is reloaded).  The environment variables
 * TN_TUNE=off|quick|full and TN_TUNE_CACHE=<path> give the starting state
 * when the library loads.  Errors: TN_ERR_INVALID_ARGUMENT for a level
 * outside 0..2, TN_ERR_DEVICE if the file cannot be opened for appending.
 * ------------------------------------------------------------------- */
int32_t tn_tune(const char* cache_path, int32_t level);
/* The same as tn_tune(NULL, level) without touching the cache file setting
 * (level 0 or 1). */
int32_t tn_tune_set_level(int32_t level);
/* Tile id chosen for the last contraction GEMM on this thread (-1: none
 * yet; calls served by the reduction or small-extent paths do not change
 * it).  For logging and tests. */
int32_t tn_tune_last_choice(void);
/* Pin one tile configuration (0 .. tn_tune_num_configs()-1) for every
 * subsequent contraction GEMM in the process; -1 restores automatic choice.
 * Meant for measurement. */
int32_t tn_tune_force_config(int32_t cfg);
int32_t tn_tune_num_configs(void);
/* Measurement: the matrix-core rate of the split-BF16 term products alone.
 * One launch runs 256 x 8 waves, each wave five 32 x 32 blocks over n_steps
 * k-steps of 16 with the six BF16 term products per block and step chained
 * from zero and added to the FP32 accumulator every two steps, as the
 * contraction kernels do, with register operands: no loads, no LDS.  For
 * reading the contraction GEMM's matrix-core fraction against what the
 * chip sustains for the same products.  At
 * n_steps = 64 it issues the same 1.288e11 flops as the split-BF16 product
 * of the bulk-site contraction M = 5120, K = 1024, N = 2048.  zero_operands
 * = 0 fills the operands with hashed bits (random mantissas), 1 with zeros:
 * the chip's clock under this load depends on the bits the matrix cores
 * toggle.  out: DEVICE, 131072 floats (one per lane; overwritten).
 * TN_ERR_INVALID_ARGUMENT for a NULL out or an odd or non-positive
 * n_steps. */
int32_t tn_measure_split_mfma_rate(int32_t n_steps, int32_t zero_operands, float* out, void* stream);

/* Pin the tile of every site step of the uneven batched inner product:
 * 0: 128 x 128, 1: 64 x 64, 2: 32 x 32, 3: 64 x 64 in two k-slices,
 * 4: 160 x 256 on eight waves (launches whose problems need the run-time
 * gathers take 0 instead); -1 restores the per-step choice (tuned or
 * estimated).  The upload writes the tile tables of all five tiles, so the
 * setting may change between an upload and its launches.  Meant for
 * measurement and tests.  TN_ERR_INVALID_ARGUMENT outside -1 .. 4. */
int32_t tn_tune_force_grouped_config(int32_t cfg);

#ifdef __cplusplus
}
#endif
#endif /* TN_H */
