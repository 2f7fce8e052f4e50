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
 *   - String n carries its operator on qubit t in its t-th base-4 digit
 *     (the bit pair 2t+1, 2t), with 0 = identity, 1 = X, 2 = Y, 3 = Z
 *     (section 2, closing paragraph), which gives the ordering of Eq. (2).
 *   - The single-qubit matrices are those of Eq. (3), Y = [[0,-i],[i,0]].
 *
 * Representation used throughout: every nonzero element of the matrices of
 * Eq. (3) is a power of the imaginary unit, so every beta of section 2 and
 * every lambda of Eq. (lambda_def) is i^q for an integer q taken mod 4.
 * The oracle carries lambda as that quarter-turn count q, multiplies a
 * matrix entry by i^q as an exact rotation of its two parts, and rounds only
 * in the running sum.
 *
 * Parity pins (see the test-suite): brute-force Tr(P_n G) for small N, the
 * Eq. (2) ordering, one-hot strings, closed forms, Kronecker factorisation,
 * Parseval, Hermitian => real, recomposition and adjoint identities.
 */
#include <math.h>
#include <stdint.h>

#define MAX_QUBITS 64

/*
 * Eq. (3) written row by row.  Each of the four matrices has exactly one
 * nonzero element per row (section 2: identity and Z are diagonal, X and Y
 * anti-diagonal).  Row a holds its nonzero element in column a when the
 * matrix is diagonal and in column 1-a when it is anti-diagonal; that
 * element is i^quarter[a].
 *     identity  [[1, 0], [0,  1]]   diagonal       1 = i^0, 1 = i^0
 *     X         [[0, 1], [1,  0]]   anti-diagonal  1 = i^0, 1 = i^0
 *     Y         [[0,-i], [i,  0]]   anti-diagonal -i = i^3, i = i^1
 *     Z         [[1, 0], [0, -1]]   diagonal       1 = i^0,-1 = i^2
 */
typedef struct {
    int antidiagonal;
    int quarter[2];
} eq3_matrix;

static const eq3_matrix EQ3[4] = {
    {0, {0, 0}},
    {1, {0, 0}},
    {1, {3, 1}},
    {0, {0, 2}},
};

/* The operator string n acts with on qubit t: its t-th base-4 digit
 * (section 2, closing paragraph). */
int oracle_operator_at(uint64_t n, int t) {
    return (int)((n >> (2 * t)) & 3u);
}

/* Flip mask m^(n) of section 2: f_n(i) = i xor m^(n) flips the bits of the
 * qubits whose operator is X or Y, i.e. whose matrix is anti-diagonal. */
uint64_t oracle_flip_mask(uint64_t n, int N) {
    uint64_t m = 0;
    for (int q = N - 1; q >= 0; q--) {
        m = (m << 1) | (uint64_t)EQ3[oracle_operator_at(n, q)].antidiagonal;
    }
    return m;
}

/* acc += i^q * g, exactly (a rotation by quarter turns), rounding only in
 * the two additions. */
static void accumulate_rotated(double acc[2], const double* g, int q) {
    switch (q & 3) {
        case 0: acc[0] += g[0]; acc[1] += g[1]; break;
        case 1: acc[0] -= g[1]; acc[1] += g[0]; break;
        case 2: acc[0] -= g[0]; acc[1] -= g[1]; break;
        default: acc[0] += g[1]; acc[1] -= g[0]; break;
    }
}

static const double* entry(const double* G, int N, uint64_t row, uint64_t col) {
    return G + 2 * ((row << N) + col);
}

/* Lowest set bit of k > 0: the Gray codes of k-1 and k differ exactly
 * there (section 2, enumeration of i by Gray codes). */
static int lowest_set_bit(uint64_t k) {
    int t = 0;
    while (!((k >> t) & 1u)) t++;
    return t;
}

/*
 * The sum of Eq. (c_def_in_terms_of_fn) for a string with operators op[],
 * flip mask m and lambda_0 = i^q0, with i visited in Gray-code order
 * (section 3): i starts at 0 and at step k flips its lowest-set bit of k.
 * When bit t of i changes from a to 1-a, only the factor of qubit t in
 * Eq. (lambda_def) changes, and Eq. (lambda_recurrence_over_i) multiplies
 * lambda by the new beta and divides by the old one: in quarter turns, adds
 * quarter[1-a] - quarter[a] of that qubit's matrix.  The sum is scaled by
 * 2^-N once it is complete.
 */
static void gray_walk(const double* G, int N, const int* op, uint64_t m, int q0, double* out) {
    const uint64_t terms = (uint64_t)1 << N;
    double acc[2] = {0.0, 0.0};
    uint64_t i = 0;
    int q = q0;
    accumulate_rotated(acc, entry(G, N, m, 0), q);
    for (uint64_t k = 1; k < terms; k++) {
        int t = lowest_set_bit(k);
        int a = (int)((i >> t) & 1u);
        const eq3_matrix* s = &EQ3[op[t]];
        q += s->quarter[1 - a] - s->quarter[a];
        i ^= (uint64_t)1 << t;
        accumulate_rotated(acc, entry(G, N, i ^ m, i), q);
    }
    out[0] = ldexp(acc[0], -N);
    out[1] = ldexp(acc[1], -N);
}

static void operators_of(uint64_t n, int N, int* op) {
    for (int t = 0; t < N; t++) op[t] = oracle_operator_at(n, t);
}

/*
 * One coefficient c_n by the paper's algorithm (section 3): the flip mask,
 * lambda_0 as the full product of Eq. (lambda_def) at i = 0 (row 0 of every
 * qubit's matrix), then the Gray-order sum with the one-factor recurrence.
 */
void oracle_coefficient(const double* G, int N, uint64_t n, double* out) {
    int op[MAX_QUBITS];
    operators_of(n, N, op);
    int q0 = 0;
    for (int t = 0; t < N; t++) q0 += EQ3[op[t]].quarter[0];
    gray_walk(G, N, op, oracle_flip_mask(n, N), q0, out);
}

/*
 * The same sum in natural order of i with every lambda_i formed in full
 * from Eq. (lambda_def) (the slower scheme of section 3).
 */
void oracle_coefficient_natural(const double* G, int N, uint64_t n, double* out) {
    int op[MAX_QUBITS];
    operators_of(n, N, op);
    const uint64_t m = oracle_flip_mask(n, N);
    double acc[2] = {0.0, 0.0};
    for (uint64_t i = 0; i < ((uint64_t)1 << N); i++) {
        int q = 0;
        for (int t = 0; t < N; t++) q += EQ3[op[t]].quarter[(i >> t) & 1u];
        accumulate_rotated(acc, entry(G, N, i ^ m, i), q);
    }
    out[0] = ldexp(acc[0], -N);
    out[1] = ldexp(acc[1], -N);
}

/*
 * String of rank k in the reflected quaternary Gray order over N base-4
 * digits (section 2, enumeration of the P_n by the quaternary Gray code):
 * the lowest digit runs 0,1,2,3 and then back 3,2,1,0 each time the digit
 * above it advances, so digit t of the code is digit t of k while digit
 * t+1 of k is even and 3 minus it while that digit is odd.  Consecutive
 * codes differ in one digit, by one step (I-X, X-Y or Y-Z).
 */
uint64_t oracle_quaternary_gray(uint64_t k, int N) {
    uint64_t code = 0;
    for (int t = N - 1; t >= 0; t--) {
        uint64_t d = (k >> (2 * t)) & 3u;
        uint64_t above = t + 1 < N ? (k >> (2 * t + 2)) & 1u : 0u;
        code = (code << 2) | (above ? 3u - d : d);
    }
    return code;
}

/*
 * All 4^N coefficients with the strings taken in quaternary Gray order and
 * lambda_0 and the flip mask carried across strings (section 2): when the
 * operator of qubit t changes from s to s', the mask keeps bit t for an
 * identity-Z or X-Y change and flips it otherwise, and lambda_0 gains the
 * factor beta' / beta of row 0 of qubit t (in quarter turns,
 * quarter'[0] - quarter[0]).  lambda_0 is thus never formed as an N-term
 * product.  Each coefficient's sum over i is the same Gray-order sum as in
 * oracle_coefficient; lambda stays exactly a power of i, so the results
 * equal oracle_decompose bit for bit.  out is indexed by n.
 */
void oracle_decompose_qgray(const double* G, int N, double* out) {
    int op[MAX_QUBITS] = {0};     /* the identity string: no X/Y, lambda_0 = 1 */
    uint64_t n = 0, m = 0;
    int q0 = 0;
    gray_walk(G, N, op, m, q0, out);
    const uint64_t strings = (uint64_t)1 << (2 * N);
    for (uint64_t k = 1; k < strings; k++) {
        uint64_t next = oracle_quaternary_gray(k, N);
        uint64_t changed = n ^ next;
        int t = 0;
        while (!((changed >> (2 * t)) & 3u)) t++;
        int from = op[t], to = oracle_operator_at(next, t);
        int keep = (from == 0 && to == 3) || (from == 3 && to == 0) || (from == 1 && to == 2) ||
                   (from == 2 && to == 1);
        if (!keep) m ^= (uint64_t)1 << t;
        q0 += EQ3[to].quarter[0] - EQ3[from].quarter[0];
        op[t] = to;
        n = next;
        gray_walk(G, N, op, m, q0, out + 2 * n);
    }
}

/* Coefficients n0 <= n < n1 (out holds (n1-n0) interleaved complex values).
 * Evaluation over n is independent per coefficient (section 3, closing
 * remarks on parallelism), so disjoint ranges may run on separate threads. */
void oracle_decompose_range(const double* G, int N, uint64_t n0, uint64_t n1, double* out) {
    for (uint64_t n = n0; n < n1; n++) oracle_coefficient(G, N, n, out + 2 * (n - n0));
}

/* Full decomposition, Eq. (1): all 4^N coefficients. */
void oracle_decompose(const double* G, int N, double* out) {
    oracle_decompose_range(G, N, 0, (uint64_t)1 << (2 * N), out);
}

/* Selected coefficients ns[0..count). */
void oracle_coeffs_at(const double* G, int N, const uint64_t* ns, int64_t count, double* out) {
    for (int64_t q = 0; q < count; q++) oracle_coefficient(G, N, ns[q], out + 2 * q);
}

/*
 * One element [P_n]_{ij}, Eq. (pauli_tensor_elems_bitwise): the product
 * over qubits of [sigma_t]_{i_t, j_t}, which vanishes unless j_t is the
 * column of row i_t's nonzero element, and is otherwise i^(sum of the
 * quarter turns).
 */
static int string_element(uint64_t n, int N, uint64_t i, uint64_t j, int* quarter) {
    int q = 0;
    for (int t = 0; t < N; t++) {
        const eq3_matrix* s = &EQ3[oracle_operator_at(n, t)];
        int a = (int)((i >> t) & 1u), b = (int)((j >> t) & 1u);
        if ((a ^ b) != s->antidiagonal) return 0;
        q += s->quarter[a];
    }
    *quarter = q;
    return 1;
}

void oracle_pauli_element(uint64_t n, int N, uint64_t i, uint64_t j, double* out) {
    static const double one[2] = {1.0, 0.0};
    int q;
    out[0] = 0.0;
    out[1] = 0.0;
    if (string_element(n, N, i, j, &q)) accumulate_rotated(out, one, q);
}

/*
 * Entries of the recomposed matrix sum_n c_n P_n (Eq. (1)) at positions
 * (rows[q], cols[q]).  [P_n]_{ab} vanishes unless every qubit where a and b
 * differ carries an anti-diagonal operator (X or Y) and every other qubit a
 * diagonal one (identity or Z), so only 2^N strings contribute: one binary
 * choice per qubit.  They are visited in increasing order of n, each term
 * c_n * [P_n]_{ab} formed as an exact rotation.  scale multiplies the result.
 */
void oracle_recompose_entries(const double* c, int N, const uint64_t* rows, const uint64_t* cols,
                              int64_t count, double scale, double* out) {
    for (int64_t e = 0; e < count; e++) {
        uint64_t a = rows[e], b = cols[e];
        double acc[2] = {0.0, 0.0};
        for (uint64_t s = 0; s < ((uint64_t)1 << N); s++) {
            uint64_t n = 0;
            for (int t = N - 1; t >= 0; t--) {
                int differ = (int)(((a ^ b) >> t) & 1u);
                int choice = (int)((s >> t) & 1u);
                /* agree: identity (0) or Z (3); differ: X (1) or Y (2) */
                n = (n << 2) | (uint64_t)(differ ? 1 + choice : 3 * choice);
            }
            int q;
            if (string_element(n, N, a, b, &q)) accumulate_rotated(acc, c + 2 * n, q);
        }
        out[2 * e] = acc[0] * scale;
        out[2 * e + 1] = acc[1] * scale;
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
void oracle_grad_entries(const double* gc, int N, const uint64_t* rows, const uint64_t* cols,
                         int64_t count, double* out) {
    oracle_recompose_entries(gc, N, rows, cols, count, ldexp(1.0, -N), out);
}
