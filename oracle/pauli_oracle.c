/*
 * Plain CPU oracle for the dense Pauli decomposition of
 * T. Jones, "Decomposing dense matrices into dense Pauli tensors" (2024).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  The GPU library
 * shares no code, header, table or helper with it.
 *
 * Everything is IEEE binary64, single-threaded, built with -O2
 * -ffp-contract=off and no fast-math, so every addition rounds once.
 *
 * Conventions (all from the paper):
 *   - G is a 2^N x 2^N complex matrix, row-major, entries stored as
 *     interleaved (re, im) doubles: G[r][c] -> G[2*(r*D + c) + {0,1}].
 *   - Matrix indices start at zero; bit 0 of an index is the rightmost bit
 *     and belongs to the rightmost (zero-th) Pauli factor (section 2,
 *     notation paragraph).
 *   - The n-th Pauli string takes its t-th operator from the t-th pair of
 *     bits of n: flag = 2*bit(2t+1) + bit(2t), with 0 = identity, 1 = X,
 *     2 = Y, 3 = Z (section 2, last paragraph; Fig. 1a getPauliFlag), which
 *     gives the ordering of Eq. (2).
 *   - The Pauli matrices are those of Eq. (3), Y = [[0,-i],[i,0]].
 *
 * Parity pins (see the test-suite): brute-force Tr(P_n G) for small N, the
 * Eq. (2) ordering, one-hot strings, closed forms, Kronecker factorisation,
 * Parseval, Hermitian => real, reconstruction and adjoint identities.
 */
#include <stdint.h>

typedef struct { double re, im; } cplx;

static cplx cmul(cplx a, cplx b) {
    cplx r;
    r.re = a.re * b.re - a.im * b.im;
    r.im = a.re * b.im + a.im * b.re;
    return r;
}

static cplx cadd(cplx a, cplx b) {
    cplx r;
    r.re = a.re + b.re;
    r.im = a.im + b.im;
    return r;
}

/* Division by a value of unit modulus, written as multiplication by its
 * conjugate.  The paper's beta factors all lie in {+-1, +-i} (section 2,
 * definition of beta), so this equals the quotient exactly. */
static cplx cdiv_unit(cplx a, cplx b) {
    cplx bc;
    bc.re = b.re;
    bc.im = -b.im;
    return cmul(a, bc);
}

/* Elements of the four Pauli matrices, Eq. (3), indexed [flag][row][col]. */
static const cplx PAULI[4][2][2] = {
    { { {1, 0}, {0, 0} }, { {0, 0}, { 1, 0} } },   /* identity */
    { { {0, 0}, {1, 0} }, { {1, 0}, { 0, 0} } },   /* X */
    { { {0, 0}, {0,-1} }, { {0, 1}, { 0, 0} } },   /* Y */
    { { {1, 0}, {0, 0} }, { {0, 0}, {-1, 0} } },   /* Z */
};

static int get_bit(uint64_t v, int t) { return (int)((v >> t) & 1u); }

/* Base-4 digit t of n: which Pauli sits at position t (section 2, last
 * paragraph; Fig. 1a getPauliFlag). */
int oracle_pauli_flag(uint64_t n, int t) {
    return (get_bit(n, 2 * t + 1) << 1) | get_bit(n, 2 * t);
}

/* Bitmask m^(n): bit t set iff operator t is X or Y (section 2, definition
 * of f_n and its mask; Fig. 1a getMaskOfXY). */
uint64_t oracle_xy_mask(uint64_t n, int N) {
    uint64_t m = 0;
    for (int t = 0; t < N; t++) {
        int p = oracle_pauli_flag(n, t);
        uint64_t b = (p > 0 && p < 3) ? 1u : 0u;
        m |= b << t;
    }
    return m;
}

/* beta^(n,t) for row bit i_[t] and column bit i_[t] xor m_[t] (section 2,
 * beta labelling; Fig. 1a getBeta). */
static cplx get_beta(uint64_t n, int t, uint64_t i, uint64_t m) {
    int p = oracle_pauli_flag(n, t);
    int a = get_bit(i, t);
    int b = a ^ get_bit(m, t);
    return PAULI[p][a][b];
}

/* lambda_i^(n) as the full N-term product, Eq. (lambda_def). */
static cplx get_lambda(uint64_t n, uint64_t i, uint64_t m, int N) {
    cplx l = {1.0, 0.0};
    for (int t = 0; t < N; t++) l = cmul(l, get_beta(n, t, i, m));
    return l;
}

static uint64_t gray_code(uint64_t k) { return k ^ (k >> 1); }

/* Position of the single set bit of a power of two (the changed bit between
 * consecutive Gray codes, section 2 on constant-time bit position). */
static int changed_bit(uint64_t i, uint64_t j) {
    uint64_t d = i ^ j;
    int t = 0;
    while ((d >> t) != 1u) t++;
    return t;
}

static cplx load(const double* G, uint64_t D, uint64_t r, uint64_t c) {
    cplx v;
    v.re = G[2 * (r * D + c)];
    v.im = G[2 * (r * D + c) + 1];
    return v;
}

/*
 * Eq. (c_def_in_terms_of_fn) for string n with XY mask m, given lambda_0^(n):
 * i enumerated in Gray-code order, every later lambda obtained from the
 * previous one by the one-beta recurrence of Eq. (lambda_recurrence_over_i),
 * the sum divided by 2^N at the end.  The paper's first accumulation names
 * an undefined "matrix"; it is read as G, i.e. the term G[m][0].
 */
static void gray_sum(const double* G, int N, uint64_t n, uint64_t m, cplx l, double* out) {
    uint64_t dim = (uint64_t)1 << N;
    cplx c = cmul(l, load(G, dim, m, 0));
    for (uint64_t k = 1; k < dim; k++) {
        uint64_t i = gray_code(k);
        uint64_t j = gray_code(k - 1);
        int t = changed_bit(i, j);
        cplx bi = get_beta(n, t, i, m);
        cplx bj = get_beta(n, t, j, m);
        l = cmul(l, cdiv_unit(bi, bj));
        c = cadd(c, cmul(l, load(G, dim, i ^ m, i)));
    }
    out[0] = c.re / (double)dim;
    out[1] = c.im / (double)dim;
}

/*
 * One coefficient by the paper's algorithm (section 3, Fig. 1b, "Fast"):
 * lambda_0 computed in full as the N-term product, then the Gray-order sum.
 */
void oracle_coeff_fast(const double* G, int N, uint64_t n, double* out) {
    uint64_t m = oracle_xy_mask(n, N);
    gray_sum(G, N, n, m, get_lambda(n, 0, m, N), out);
}

/*
 * k-th string of the reflected quaternary Gray code over N base-4 digits
 * (section 2, enumeration of the P_n by the quaternary Gray code): the
 * sequence runs the lowest digit 0,1,2,3 and then back 3,2,1,0 each time
 * the digit above advances, so digit t of the code is digit t of k when
 * digit t+1 of k is even and 3 minus it when that digit is odd.  Consecutive
 * codes differ in one digit, by one step (I-X, X-Y or Y-Z).
 */
uint64_t oracle_quaternary_gray(uint64_t k, int N) {
    uint64_t g = 0;
    for (int t = 0; t < N; t++) {
        int d = oracle_pauli_flag(k, t);
        int up = t + 1 < N ? oracle_pauli_flag(k, t + 1) : 0;
        int e = (up & 1) ? 3 - d : d;
        g |= (uint64_t)e << (2 * t);
    }
    return g;
}

/*
 * All 4^N coefficients with the strings enumerated in quaternary Gray order
 * and the recurrence across n of section 2: from string n to the next
 * string n', which differs at one operator position t, the XY mask keeps
 * bit t when that operator changes between identity and Z or between X
 * and Y and flips it otherwise, and
 *     lambda_0^(n') = lambda_0^(n) beta^(n',t)_{0, m'_[t]} / beta^(n,t)_{0, m_[t]},
 * so lambda_0 is never formed as an N-term product (the serial saving the
 * paper notes).  Each coefficient's sum over i is the Gray-order sum of
 * oracle_coeff_fast; since every lambda is exactly one of +-1, +-i, the
 * result equals oracle_decompose bit for bit.  out is indexed by n.
 */
void oracle_decompose_qgray(const double* G, int N, double* out) {
    uint64_t total = (uint64_t)1 << (2 * N);
    uint64_t n = 0, m = 0;          /* the identity string: no X/Y, lambda_0 = 1 */
    cplx l = {1.0, 0.0};
    gray_sum(G, N, n, m, l, out);
    for (uint64_t k = 1; k < total; k++) {
        uint64_t nn = oracle_quaternary_gray(k, N);
        int t = 0;
        while (oracle_pauli_flag(n, t) == oracle_pauli_flag(nn, t)) t++;
        int fo = oracle_pauli_flag(n, t), fn = oracle_pauli_flag(nn, t);
        int same_mask = (fo == 0 && fn == 3) || (fo == 3 && fn == 0) || (fo == 1 && fn == 2) ||
                        (fo == 2 && fn == 1);
        uint64_t mm = same_mask ? m : (m ^ ((uint64_t)1 << t));
        cplx bnew = PAULI[fn][0][get_bit(mm, t)];
        cplx bold = PAULI[fo][0][get_bit(m, t)];
        l = cmul(l, cdiv_unit(bnew, bold));
        n = nn;
        m = mm;
        gray_sum(G, N, n, m, l, out + 2 * n);
    }
}

/* The paper's comparison algorithm (Fig. 1b, "Slow"): natural order of i,
 * lambda_i evaluated in full for every term. */
void oracle_coeff_slow(const double* G, int N, uint64_t n, double* out) {
    uint64_t dim = (uint64_t)1 << N;
    uint64_t m = oracle_xy_mask(n, N);
    cplx c = {0.0, 0.0};
    for (uint64_t i = 0; i < dim; i++) {
        cplx l = get_lambda(n, i, m, N);
        c = cadd(c, cmul(l, load(G, dim, i ^ m, i)));
    }
    out[0] = c.re / (double)dim;
    out[1] = c.im / (double)dim;
}

/* Coefficients n0 <= n < n1 (out holds (n1-n0) interleaved complex values).
 * Evaluation over n is independent per coefficient (section 3, closing
 * remarks on parallelism), so disjoint ranges may run on separate threads. */
void oracle_decompose_range(const double* G, int N, uint64_t n0, uint64_t n1,
                            double* out) {
    for (uint64_t n = n0; n < n1; n++) oracle_coeff_fast(G, N, n, out + 2 * (n - n0));
}

/* Full decomposition, Eq. (1): all 4^N coefficients. */
void oracle_decompose(const double* G, int N, double* out) {
    oracle_decompose_range(G, N, 0, (uint64_t)1 << (2 * N), out);
}

/* Selected coefficients ns[0..count). */
void oracle_coeffs_at(const double* G, int N, const uint64_t* ns, int64_t count,
                      double* out) {
    for (int64_t q = 0; q < count; q++) oracle_coeff_fast(G, N, ns[q], out + 2 * q);
}

/* One element [P_n]_{ij} as the product of single-qubit elements,
 * Eq. (pauli_tensor_elems_bitwise). */
void oracle_pauli_element(uint64_t n, int N, uint64_t i, uint64_t j, double* out) {
    cplx e = {1.0, 0.0};
    for (int t = 0; t < N; t++) {
        int p = oracle_pauli_flag(n, t);
        e = cmul(e, PAULI[p][get_bit(i, t)][get_bit(j, t)]);
    }
    out[0] = e.re;
    out[1] = e.im;
}

/*
 * Entries of the recomposed matrix sum_n c_n P_n (Eq. (1)) at positions
 * (rows[q], cols[q]).  Every Pauli matrix is diagonal or anti-diagonal
 * (section 2, beta labelling), so [P_n]_{ab} vanishes unless operator t is
 * identity/Z where a and b agree on bit t, and X/Y where they differ; the
 * sum therefore runs over the 2^N strings allowed by that rule, each term
 * weighted by the element of Eq. (pauli_tensor_elems_bitwise).  The strings
 * are visited in increasing order of n.  scale multiplies the result.
 */
void oracle_recompose_entries(const double* c, int N, const uint64_t* rows,
                              const uint64_t* cols, int64_t count, double scale,
                              double* out) {
    uint64_t dim = (uint64_t)1 << N;
    for (int64_t q = 0; q < count; q++) {
        uint64_t a = rows[q], b = cols[q];
        cplx acc = {0.0, 0.0};
        for (uint64_t s = 0; s < dim; s++) {
            uint64_t n = 0;
            for (int t = 0; t < N; t++) {
                int differ = get_bit(a, t) ^ get_bit(b, t);
                int choice = get_bit(s, t);
                /* agree: identity (0) or Z (3); differ: X (1) or Y (2) */
                uint64_t flag = differ ? (uint64_t)(1 + choice) : (uint64_t)(3 * choice);
                n |= flag << (2 * t);
            }
            double e[2];
            oracle_pauli_element(n, N, a, b, e);
            cplx pe = {e[0], e[1]};
            cplx cn = {c[2 * n], c[2 * n + 1]};
            acc = cadd(acc, cmul(cn, pe));
        }
        out[2 * q] = acc.re * scale;
        out[2 * q + 1] = acc.im * scale;
    }
}

/* The whole recomposed matrix G = sum_n c_n P_n, Eq. (1). */
void oracle_recompose(const double* c, int N, double* G) {
    uint64_t dim = (uint64_t)1 << N;
    for (uint64_t a = 0; a < dim; a++) {
        for (uint64_t b = 0; b < dim; b++) {
            oracle_recompose_entries(c, N, &a, &b, 1, 1.0, G + 2 * (a * dim + b));
        }
    }
}

/*
 * Gradient of a real loss L(c) with respect to G, at entries (rows, cols),
 * given gc = dL/dRe(c) + i dL/dIm(c).  c = 2^-N Tr(P_n G) is linear in G
 * (Eq. (cn_compact)); its adjoint maps gc to 2^-N sum_n gc_n P_n^dagger, and
 * every Pauli string is Hermitian, so the gradient is the recomposition of
 * gc scaled by 2^-N.
 */
void oracle_grad_entries(const double* gc, int N, const uint64_t* rows,
                         const uint64_t* cols, int64_t count, double* out) {
    oracle_recompose_entries(gc, N, rows, cols, count, 1.0 / (double)((uint64_t)1 << N), out);
}
