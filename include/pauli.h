/*
 * pauli.h -- C ABI of libpauli, a gfx950 (MI355X) library for the dense Pauli
 * decomposition of T. Jones, "Decomposing dense matrices into dense Pauli
 * tensors" (2024).
 *
 * Operation (paper, section 1, Eq. (1) and Eq. (cn_compact)): a complex
 * 2^N x 2^N matrix G is written as G = sum_n c_n P_n over the 4^N Pauli
 * strings P_n, with c_n = 2^-N Tr(P_n G).
 *
 * Conventions fixed by the paper and used by every entry point:
 *   - Matrices are row-major, G[r][c] at element r * 2^N + c, complex values
 *     stored as interleaved (re, im) pairs: float pairs for PAULI_C64,
 *     double pairs for PAULI_C128.
 *   - Bit t of a row or column index belongs to qubit t, the t-th Kronecker
 *     factor counted from the RIGHT (section 2, notation paragraph).
 *   - Coefficient n takes operator t from bits (2t+1, 2t) of n:
 *     0 = identity, 1 = X, 2 = Y, 3 = Z (section 2, last paragraph), so
 *     c_1 multiplies I (x) X and c_4 multiplies X (x) I for N = 2 (Eq. (2)).
 *   - The Pauli matrices are those of Eq. (3), Y = [[0, -i], [i, 0]].
 *
 * Memory: every data pointer (G, coefficients, gradients, workspace) is a
 * DEVICE pointer, allocated and owned by the caller, aligned to 16 bytes
 * (256 for a workspace).  Input, output and workspace must not overlap.
 * The matrix-core algorithms need a scratch buffer for their packed operand
 * (pauli_workspace_bytes); when opts->workspace is NULL the library takes it
 * from a stream-ordered memory pool of its own (one per device, kept for
 * reuse until the process ends) and returns it on the same stream.
 *
 * Execution: work is enqueued on opts->stream (a hipStream_t passed as
 * void*, NULL = the null stream) and the call returns without waiting.  The
 * caller synchronises before reading results.  No C++ exception crosses this
 * interface.  With opts->workspace set, pauli_decompose, pauli_reconstruct,
 * pauli_decompose_backward, pauli_pack and pauli_contract enqueue kernels
 * only, so they may be captured in a HIP graph and replayed; the list and
 * batched entry points copy a host-built plan on every call and must not be
 * captured by the caller (the batched one replays a graph of its own).
 *
 * Errors: every function returns a pauli_status.  On failure nothing has been
 * enqueued and pauli_last_error() returns a message for the calling thread.
 */
#ifndef PAULI_H
#define PAULI_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pauli_status {
    PAULI_OK = 0,
    PAULI_EINVAL = 1,       /* bad argument: N out of range, NULL, misaligned, overlap, count */
    PAULI_EUNSUPPORTED = 2, /* valid request the library does not implement */
    PAULI_EHIP = 3,         /* HIP runtime error; message carries hipGetErrorString */
    PAULI_ENOMEM = 4        /* caller workspace smaller than required */
} pauli_status;

typedef enum pauli_dtype {
    PAULI_C64 = 0,  /* complex float: (float re, float im) */
    PAULI_C128 = 1  /* complex double: (double re, double im) */
} pauli_dtype;

typedef enum pauli_algo {
    /* Binary64 VALU kernel that sums every coefficient in Gray-code order
     * with the one-sign recurrence of section 2, Eq. (lambda_recurrence_over_i),
     * as the paper's algorithm (section 3, Fig. 1b) does. */
    PAULI_ALGO_FP64_GRAY = 0,
    /* Binary32 matrix-core (MFMA) contraction of the gathered XOR diagonals
     * against the +-1 sign matrix, FP32 accumulation. */
    PAULI_ALGO_FP32 = 1,
    /* Each binary32 input component split exactly into three bfloat16 parts
     * (hi, mid, lo); bf16 MFMA with two FP32 accumulators (hi; mid+lo),
     * recombined in binary64 before the phase and 2^-N scaling. */
    PAULI_ALGO_SPLIT_BF16 = 2,
    /* Not the paper's O(8^N) evaluation: for every flip mask the coefficients
     * are a Sylvester-Hadamard transform of the gathered XOR diagonal
     * (section 2, Eq. (c_def_in_terms_of_fn)), done by fast Walsh-Hadamard
     * butterflies in O(N 4^N), binary64 throughout: two passes over HBM
     * through a workspace of 16 bytes per matrix element (N >= 9; up to
     * N = 8 one kernel works in LDS and needs none).  All three directions
     * (decompose, reconstruct, backward), 0 <= N <= 16. */
    PAULI_ALGO_FWHT = 3,
    /* The matrix-core contraction of FP32 and SPLIT_BF16 on two fp16 planes:
     * a reduction pass finds the largest |re|, |im| of each input and a
     * power of two 2^pe brings it just below 2^15; each scaled binary32
     * component g is then split as g = hi + 2^-11 lo + r, hi with at most 11
     * significant bits on a power-of-two grid shared by a 4x4 block of G, lo
     * the fp16 rounding of 2^11 (g - hi), |r| <= 2^-24 of the block's
     * largest component; fp16 MFMA with one FP32 accumulator per plane,
     * recombined in binary64 (hi + 2^-11 lo) with 2^-pe folded into the
     * output scale.  Two thirds of SPLIT_BF16's matrix-core work; finite
     * inputs only (an infinite or NaN component gives unspecified output). */
    PAULI_ALGO_SPLIT_FP16 = 4,
    /* FWHT with a binary32 intermediate (8 bytes per matrix element of
     * workspace, N >= 9): every butterfly still adds in binary64, but the
     * partial transforms between the two passes are rounded to binary32
     * (once more after each extra top pass at N = 15, 16), so each
     * coefficient c(x, 32 z_h + z_l) is off by at most 2^-24 times the
     * 2-norm of the 2^(N-5) coefficients c(x, 32 k + z_l), k < 2^(N-5), per
     * rounding (plus the output's own rounding): at most 2^-24 2^((N-5)/2)
     * max|c|; 2.6e-8 of max|c| measured at N = 14.  Up to N = 8
     * it is the binary64 one-kernel path.  Same directions and range as
     * PAULI_ALGO_FWHT. */
    PAULI_ALGO_FWHT_F32 = 5,
    /* Fixed point on int8 matrix cores, the same contraction as the splits
     * (section 2, Eq. (c_def_in_terms_of_fn)): a reduction pass finds the
     * largest |re|, |im| of each input, m = mm 2^e (1 <= mm < 2); every
     * component g becomes the integer q = rint(g 2^-e 8355711 / mm),
     * |q| <= 8355711, split into three balanced base-256 digits (the top one
     * at most 127 in magnitude); int8 MFMA sums +-1 times each digit exactly
     * in int32 (two walks over K: the two upper digit planes, then the
     * lowest), and the digit sums are combined exactly in binary64 and
     * scaled by 2^(e-N) mm / 8355711.  The contraction rounds nothing: each
     * coefficient is off by at most m / (2 * 8355711) (6.0e-8 m) per
     * component from the quantisation, plus the output's own rounding.
     * The bound is relative to the largest entry of the matrix, not to each
     * entry (fixed point); for iid inputs the error is about 2e-7 of
     * max|c| (2.2e-7 at N = 14).  Three quarters of SPLIT_FP16's
     * matrix-core time at int8's doubled rate.  pauli_decompose,
     * pauli_decompose_noalloc, pauli_decompose_hermitian (on Hermitian
     * input it equals pauli_decompose bit for bit, the sums being exact),
     * pauli_reconstruct and pauli_decompose_backward (the coefficient vector
     * quantised the same way from its own largest component m_c: each entry
     * of G off by at most 2^N m_c / (2 * 8355711) per component, times the
     * gradient's 2^-N), equal-order batches, one tile shape, also split into
     * pauli_pack / pauli_contract (every mode); the batched and tuning entry
     * points return PAULI_EUNSUPPORTED.  An infinite or NaN component makes
     * every output of that matrix NaN; an all-zero input gives zeros. */
    PAULI_ALGO_SPLIT_I8 = 6
} pauli_algo;

typedef struct pauli_opts {
    int algo;               /* pauli_algo */
    int in_dtype;           /* pauli_dtype of the input */
    int out_dtype;          /* pauli_dtype of the output */
    int tile;               /* 0 = tuned/default tile; >0 forces a tile id (pauli_tile_valid) */
    void* stream;           /* hipStream_t, NULL = null stream */
    void* workspace;        /* optional device scratch, see pauli_workspace_bytes */
    size_t workspace_bytes; /* its size in bytes */
} pauli_opts;

/* Fill *o with the defaults: SPLIT_BF16, C64 in, C64 out, tile 0, null stream,
 * no workspace. */
void pauli_opts_default(pauli_opts* o);

/*
 * Decompose `batch` matrices of order 2^N stored back to back in G
 * (batch * 4^N elements) into out (batch * 4^N coefficients):
 *     out[b * 4^N + n] = 2^-N Tr(P_n G_b)                (Eq. (cn_compact))
 * evaluated as in section 2, Eq. (c_def_in_terms_of_fn):
 *     c_n = 2^-N sum_i lambda_i^(n) G[i xor m^(n)][i].
 * 0 <= N <= 16 (the coefficient index needs 2N bits, section 2); batch >= 1.
 * The MFMA algorithms read C128 input rounded to binary32.
 * Input range: FP32 and SPLIT_BF16 accumulate unscaled binary32 partial sums
 * of up to 2^N terms, so their results are finite for components of
 * magnitude below 2^(127 - N); SPLIT_FP16 rescales each matrix by a power of
 * two first and has no limit beyond finite binary32 components; FP64_GRAY
 * and both FWHT algorithms sum in binary64.  For such inputs every path scales exactly:
 * c(2^k G) = 2^k c(G) bit for bit while all operands, split parts and
 * partial sums stay normal numbers.  Infinite or NaN components give
 * non-finite outputs (no error is reported).
 * opts may be NULL (defaults).
 */
int pauli_decompose(const void* G, int N, int batch, void* out, const pauli_opts* opts);

/*
 * pauli_decompose for Hermitian G (G[j][i] = conj(G[i][j])), whose
 * coefficients are real (every Pauli string is Hermitian, so Tr(P_n G) is
 * real).  Not the paper's method: it uses what the paper sets aside (its
 * algorithm is for arbitrary dense matrices, Abstract).  For a flip mask x,
 * v_x[i xor x] = conj(v_x[i]) in Eq. (c_def_in_terms_of_fn), so the sum over
 * half of the i, doubled, gives the sum over all: the matrix-core contraction
 * walks half of its K range for every block of 32 flip masks whose common
 * high bits are large enough (all blocks but the first few).  That half sum
 * does not see bit b of z either (b = the block's top flip-mask bit), so
 * rows z and z xor 2^b share it: one gives the real part (popc(x&z) even),
 * the other the imaginary part, and where 2^b spans whole workgroup tiles
 * only one of the two row tiles is computed (a quarter of the general
 * work).  Every coefficient's imaginary part is written as exactly zero.
 * algo SPLIT_FP16, SPLIT_BF16, FP32 or SPLIT_I8 (others:
 * PAULI_EUNSUPPORTED); register-ring tiles only (pauli_tile_valid_hermitian;
 * a forced LDS-staged tile fails with PAULI_EINVAL); pauli_tile_selected_hermitian
 * gives the tile it uses (0 for SPLIT_I8, which has one shape: blocks of
 * flip masks from 512 on take the half walk, and its exact integer sums make
 * the result equal pauli_decompose's bit for bit).  Limits, layouts, workspace and stream as pauli_decompose.
 * The Hermitian property is the caller's promise and is not checked: the
 * kernel reads only one entry of most pairs (G[i xor x][i], G[i][i xor x]),
 * so for a non-Hermitian G the result is unspecified (finite input still
 * gives finite output, and no memory outside G, out and the workspace is
 * touched).
 */
int pauli_decompose_hermitian(const void* G, int N, int batch, void* out, const pauli_opts* opts);

/*
 * Recompose matrices from coefficients, G = sum_n c_n P_n (Eq. (1)), for
 * `batch` coefficient vectors of length 4^N stored back to back.  Exact
 * inverse of pauli_decompose up to rounding.  Same limits as above.
 */
int pauli_reconstruct(const void* c, int N, int batch, void* G, const pauli_opts* opts);

/*
 * Adjoint of pauli_decompose, used for reverse-mode differentiation: given
 * grad_c = dL/dRe(c) + i dL/dIm(c) for a real loss L, write
 *     grad_G = dL/dRe(G) + i dL/dIm(G) = 2^-N sum_n grad_c[n] P_n,
 * which follows from the linear form Eq. (cn_compact) and the Hermiticity of
 * every Pauli string.  Layout, limits and batching as pauli_reconstruct.
 */
int pauli_decompose_backward(const void* grad_c, int N, int batch, void* grad_G,
                             const pauli_opts* opts);

/*
 * Decompose `count` matrices of uneven sizes (section 3: coefficients are
 * independent, here also across matrices): G[k] (device pointer) holds a
 * 2^N[k] x 2^N[k] matrix, out[k] receives its 4^N[k] coefficients.  G, N and
 * out are HOST arrays of length count.  1 <= N[k] <= 12, count >= 1; algo
 * SPLIT_BF16, SPLIT_FP16 or FP32, C64 in and out (SPLIT_FP16 first finds
 * every matrix's prescale with two more kernels in the same graph).
 * opts->workspace (required) must hold pauli_batched_workspace_bytes(count,
 * N, algo) bytes of device memory that stays untouched while the work runs.
 * The work is one batched pack launch and one persistent contraction launch
 * whose workgroups take output tiles (largest matrices first) from a counter
 * in the workspace.  Both are captured once per (stream, workspace, algo,
 * tile, N list) in a HIP graph that later calls replay; the descriptor table
 * (pointers) and the pack-tile and output-tile to matrix tables are copied
 * into the workspace on every call, so new buffers are honoured.  The library keeps at most 64 such
 * captures (with their pinned host staging) and releases the least recently
 * used one, after its last replay has finished, to make room for a new one.
 * opts->tile: 0 = the tuned or default shape, 1..
 * pauli_batched_tile_count() forces one.  Shapes 1-5 read an operand packed
 * by a separate kernel; shapes 6-9 gather and split it from G inside the
 * contraction (no pack kernel); the default is shape 8 (9 for SPLIT_BF16).
 * Every shape gives the same result bit for bit.  Calls sharing a workspace
 * must be ordered on one stream.
 */
int pauli_decompose_batched(int count, const void* const* G, const int* N, void* const* out,
                            const pauli_opts* opts);

/* Workspace bytes pauli_decompose_batched needs (0 for invalid arguments). */
size_t pauli_batched_workspace_bytes(int count, const int* N, int algo);

/* Number of persistent-kernel tile shapes for the uneven batch. */
int pauli_batched_tile_count(void);

/* 1 if batched tile shape `tile` can run `algo` (shape 7, 512 rows fused, runs SPLIT_FP16 only). */
int pauli_batched_tile_valid(int algo, int tile);

/*
 * Run pauli_decompose_batched with every tile shape on the given buffers
 * (outputs are overwritten with the same correct result), time each and keep
 * the fastest for this list of N values (in the process-wide table, and in
 * the PAULI_TUNE_CACHE file if that variable is set, see pauli_autotune).
 * Blocking.
 */
int pauli_autotune_batched(int count, const void* const* G, const int* N, void* const* out,
                           const pauli_opts* opts);

/* Tile shape pauli_decompose_batched would use for this N list and algo. */
int pauli_batched_tile_selected(int count, const int* N, int algo);

/*
 * Device scratch bytes pauli_decompose, pauli_reconstruct and
 * pauli_decompose_backward need for (algo, N, batch) when the caller supplies
 * opts->workspace: 12 bytes per matrix element for SPLIT_BF16 (six bf16
 * planes), 8 for SPLIT_FP16 (four fp16 planes) plus its prescale exponent and
 * partial maxima, 8 for FP32, 6 for SPLIT_I8 (six int8 planes) plus its
 * scale record and partial maxima (N < 5 counts as N = 5 for these four);
 * 16 for FWHT and 8 for FWHT_F32 from N = 9 on, none below; 0 for FP64_GRAY.
 * A smaller workspace fails with PAULI_ENOMEM.  Returns 0 for invalid
 * arguments.
 */
size_t pauli_workspace_bytes(int algo, int N, int batch);

/*
 * Time every tile configuration of `algo` for N_min <= N <= N_max on the
 * current device (allocating and freeing its own scratch matrices, timed on
 * a fixed pseudo-random matrix with components uniform on [-1, 1), since
 * the power drawn by the matrix cores, and so the clock, depends on the
 * operand values), keep the
 * fastest per N in the process-wide tune table, and write the table to the
 * file named by the PAULI_TUNE_CACHE environment variable if it is set.
 * Blocking.  opts supplies algo and stream (may be NULL: SPLIT_BF16).
 * The file, read once per process before the first tile choice, holds one
 * entry per line: "algo N tile" for single matrices and
 * "B planes tile c_1 ... c_12" for a batch of c_n matrices of order n
 * (planes 3 = SPLIT_BF16, 2 = SPLIT_FP16, 1 = FP32); lines that do not parse
 * are ignored.  The table applies to pauli_decompose, pauli_reconstruct,
 * pauli_decompose_backward and the two-pass entry points;
 * pauli_decompose_hermitian keeps its own defaults (its tiles do a quarter
 * of the work with twice the stores, so the general timings do not carry
 * over).
 */
int pauli_autotune(int N_min, int N_max, const pauli_opts* opts);

/* Number of tile configurations for `algo` (ids 1..count; 1 for FP64_GRAY,
 * FWHT, FWHT_F32 and SPLIT_I8, which have one shape each). */
int pauli_tile_count(int algo);

/*
 * 1 if tile id `tile` can run `algo` at order N, else 0.  A tile needs at
 * least as many (padded) matrix rows as one workgroup covers, and FP32 does
 * not offer the register-ring tiles of 4 x 32 rows per wave (ids 1, 2, 7, 10,
 * 11); a forced invalid tile fails with PAULI_EINVAL.
 */
int pauli_tile_valid(int algo, int tile, int N);

/* 1 if tile id `tile` can run pauli_decompose_hermitian for `algo` at order
 * N: a valid tile of pauli_tile_valid that is not LDS-staged (ids 1..12). */
int pauli_tile_valid_hermitian(int algo, int tile, int N);

/* Tile id pauli_decompose would use for (algo, N) right now; 0 for the
 * algorithms without a tile choice (FP64_GRAY, FWHT, FWHT_F32, SPLIT_I8). */
int pauli_tile_selected(int algo, int N);

/* Tile id pauli_decompose_hermitian would use for (algo, N) right now (0 if
 * the algorithm has no Hermitian variant or N is out of range). */
int pauli_tile_selected_hermitian(int algo, int N);

/*
 * Coefficients of a caller-chosen list of Pauli strings (the paper's inner
 * product of a matrix with a single Pauli string, O(2^N) each; sections 3
 * and 4):
 *     out[k] = 2^-N Tr(P_{strings[k]} G),   k = 0 .. count-1,
 * the same value pauli_decompose gives for that n (section 2,
 * Eq. (c_def_in_terms_of_fn)), summed in binary64 whatever the dtypes.
 * G: DEVICE, one 2^N x 2^N matrix (opts->in_dtype).  strings: HOST array of
 * count string indices, each below 4^N (else PAULI_EINVAL); repeats allowed.
 * out: DEVICE, count coefficients (opts->out_dtype), in the order of strings.
 * 0 <= N <= 16, count >= 1.  opts->algo and opts->tile are ignored.
 * The library sorts the list by flip mask on the host (strings whose flip
 * masks agree above bit 3 share one pass over their 16 XOR-diagonals of G)
 * and copies that plan into opts->workspace (at least
 * pauli_coeffs_at_workspace_bytes(count) bytes) or, when it is NULL, into
 * memory from the library's pool.  The strings array may be reused as soon
 * as the call returns.
 */
int pauli_coeffs_at(const void* G, int N, const unsigned int* strings, int count, void* out,
                    const pauli_opts* opts);

/*
 * Adjoint of pauli_coeffs_at, for reverse-mode differentiation: given
 * grad_c[k] = dL/dRe(c_k) + i dL/dIm(c_k) for the listed strings (DEVICE,
 * count values, opts->in_dtype), write the dense
 *     grad_G = 2^-N sum_k grad_c[k] P_{strings[k]}
 * (DEVICE, 2^N x 2^N, opts->out_dtype), zero away from the listed strings'
 * XOR diagonals; repeated strings add.  This is the linear map's adjoint
 * (Eq. (cn_compact) with Hermitian P_n), as for pauli_decompose_backward.
 * strings is a HOST array as in pauli_coeffs_at; limits and workspace as
 * there.  Summed in binary64.
 */
int pauli_coeffs_at_backward(const void* grad_c, int N, const unsigned int* strings, int count, void* grad_G,
                             const pauli_opts* opts);

/*
 * Workspace bytes that suffice for pauli_coeffs_at and
 * pauli_coeffs_at_backward with any list of `count` strings at order N (the plan plus, for short lists whose columns are split
 * over several workgroups, binary64 partial sums); 0 for invalid arguments.
 */
size_t pauli_coeffs_at_workspace_bytes(int N, int count);

/* Message describing the calling thread's most recent failure ("" if none). */
const char* pauli_last_error(void);

/*
 * The two passes of the matrix-core algorithms (SPLIT_BF16, SPLIT_FP16,
 * FP32, and SPLIT_I8 for modes 0 and 3: its pack is the scale reduction, the
 * quantisation and the digit split), for callers that schedule or time them
 * separately; opts->workspace is required (pauli_workspace_bytes).  mode:
 * 0 = decompose, 1 = reconstruct,
 * 2 = backward, 3 = decompose a Hermitian matrix (pauli_decompose_hermitian;
 * its pack writes only the parts of the operand that the half walk of any
 * tile reads, its contraction takes the register-ring tiles of
 * pauli_tile_valid_hermitian; a mode-3 contraction therefore needs a mode-3
 * pack).
 *   pauli_pack: gather the input of the contraction (for mode 0 the XOR
 *     diagonals G[i ^ x][i] of section 2, Eq. (c_def_in_terms_of_fn); for
 *     modes 1 and 2 the coefficient blocks) and store it, converted to the
 *     matrix-core operand format, in the workspace.
 *   pauli_contract: contract the packed operand against the +-1 sign matrix
 *     and write the output of pauli_decompose / pauli_reconstruct /
 *     pauli_decompose_backward / pauli_decompose_hermitian.
 * pauli_pack followed by pauli_contract on the same stream, workspace and
 * arguments equals the one-call entry point bit for bit.
 */
int pauli_pack(const void* in, int N, int batch, int mode, const pauli_opts* opts);
int pauli_contract(int N, int batch, int mode, void* out, const pauli_opts* opts);

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * pauli_decompose with every argument, limit and result as there, except
 * that the device scratch of the algorithm (the packed operand of the
 * matrix-core algorithms, the intermediate of the two FWHT algorithms;
 * FP64_GRAY needs none) is a
 * fixed array of pauli_noalloc_scratch_bytes() bytes (64 MiB) that the
 * library holds on each GPU it runs on until the process ends, so the call
 * itself allocates nothing (no hipMalloc, no pool, no host allocation of
 * device memory).  opts->workspace and opts->workspace_bytes are ignored.
 * A request whose scratch exceeds the array (pauli_workspace_bytes(algo, N,
 * batch) > 64 MiB, e.g. SPLIT_BF16 at N >= 12, or batch > 1 at N = 11)
 * fails with PAULI_ENOMEM before any launch.  All calls on one GPU share its
 * array: calls that overlap in time on one GPU (different streams or host
 * threads without ordering) race and give undefined results; calls ordered
 * on one stream are safe.  Nothing in the array needs to start at zero:
 * each call writes every byte it later reads.
 */
int pauli_decompose_noalloc(const void* G, int N, int batch, void* out, const pauli_opts* opts);

/* Size in bytes of the fixed per-GPU scratch of pauli_decompose_noalloc. */
size_t pauli_noalloc_scratch_bytes(void);

/* Library ABI version, currently 1. */
int pauli_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PAULI_H */
