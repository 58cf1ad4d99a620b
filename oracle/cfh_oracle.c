/*
 * CPU oracle for the Clifford-fullstate hybrid rotation path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or table with the HIP library.
 *
 * What it computes, and from which passage of the paper:
 *   - textbook one- and two-qubit gates on a dense 2^n complex128 vector
 *     (Sec. 2.1: Pauli matrices, H, S, CNOT; qubit j = bit j of the index,
 *     Sec. 3);
 *   - a multi-qubit rotation exp(-i theta/2 P) decomposed the textbook way
 *     (Sec. 5.1, CNOT staircase): a per-letter basis change into Z, a CNOT
 *     ladder collecting the parity on the last support qubit, RZ(theta) there,
 *     then the ladder and the basis change undone;
 *   - the same rotation by its definition, cos(theta/2) I - i sin(theta/2) P
 *     with P acting letter by letter on basis states (Sec. 3), on a sparse
 *     state for large n with small support;
 *   - Heisenberg conjugation C^dag Q C of a Pauli string through a Clifford
 *     gate list, one gate at a time, using per-gate letter tables that are
 *     derived at start-up by multiplying the textbook gate matrices
 *     (Sec. 4.1, backward interpretation; Eq. single_to_multirot);
 *   - <psi|P|psi> with P applied letter by letter (Sec. 4.4, Eq. chfsexp).
 *
 * Letter codes: 0=I 1=X 2=Y 3=Z.  Gate codes: 0=H 1=S 2=Sdg 3=X 4=Y 5=Z
 * 6=CNOT(q0 control, q1 target) 7=CZ 8=SWAP.  All floating point is double.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define PAR_MIN_QUBITS 14

/* ---------------------------------------------------------------- matrices */

static void pauli_matrix(int l, cplx m[4])
{
    /* row-major 2x2: m[0]=<0|.|0>, m[1]=<0|.|1>, m[2]=<1|.|0>, m[3]=<1|.|1> */
    switch (l) {
    case 0: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = 1; break;
    case 1: m[0] = 0; m[1] = 1; m[2] = 1; m[3] = 0; break;
    case 2: m[0] = 0; m[1] = -I; m[2] = I; m[3] = 0; break;
    default: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = -1; break;
    }
}

/* Textbook one-qubit gate matrices; returns 0 for a two-qubit code. */
static int gate1_matrix(int g, cplx m[4])
{
    const double r = 1.0 / sqrt(2.0);
    switch (g) {
    case 0: m[0] = r; m[1] = r; m[2] = r; m[3] = -r; return 1;   /* H */
    case 1: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = I; return 1;    /* S */
    case 2: m[0] = 1; m[1] = 0; m[2] = 0; m[3] = -I; return 1;   /* S^dag */
    case 3: pauli_matrix(1, m); return 1;
    case 4: pauli_matrix(2, m); return 1;
    case 5: pauli_matrix(3, m); return 1;
    default: return 0;
    }
}

/* Two-qubit gate as a 4x4 on local index r = b0 + 2*b1 (b0 = qubit q0). */
static void gate2_matrix(int g, cplx m[16])
{
    memset(m, 0, 16 * sizeof(cplx));
    for (int c = 0; c < 4; ++c) {
        int b0 = c & 1, b1 = c >> 1, r = c;
        if (g == 6) r = b0 | ((b1 ^ b0) << 1);           /* CNOT q0 -> q1 */
        else if (g == 8) r = b1 | (b0 << 1);             /* SWAP */
        m[r * 4 + c] = (g == 7 && b0 && b1) ? -1 : 1;    /* CZ phase */
    }
}

/* ---------------------------------------------------- Heisenberg tables */
/* t1[g][l] = (l', k) with G^dag sigma_l G = i^k sigma_l'.               */
/* t2[g][l0][l1] = (l0', l1', k) for the 4x4 two-qubit gates.             */
static int t1_letter[6][4], t1_phase[6][4];
static int t2_l0[3][4][4], t2_l1[3][4][4], t2_phase[3][4][4];
static int tables_ready = 0;

static cplx ipow(int k) { k &= 3; return k == 0 ? 1 : k == 1 ? I : k == 2 ? -1 : -I; }

static void mat_mul(const cplx *a, const cplx *b, cplx *c, int d)
{
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) {
            cplx s = 0;
            for (int k = 0; k < d; ++k) s += a[i * d + k] * b[k * d + j];
            c[i * d + j] = s;
        }
}

static void mat_dag(const cplx *a, cplx *c, int d)
{
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) c[j * d + i] = conj(a[i * d + j]);
}

static int mat_close(const cplx *a, const cplx *b, int d)
{
    for (int i = 0; i < d * d; ++i)
        if (cabs(a[i] - b[i]) > 1e-12) return 0;
    return 1;
}

static void pauli2(int l0, int l1, cplx m[16])
{
    cplx a[4], b[4];
    pauli_matrix(l0, a);
    pauli_matrix(l1, b);
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c)
            m[r * 4 + c] = a[(r & 1) * 2 + (c & 1)] * b[(r >> 1) * 2 + (c >> 1)];
}

static void build_tables(void)
{
    if (tables_ready) return;
    for (int g = 0; g < 6; ++g) {
        cplx G[4], Gd[4], P[4], T[4], R[4];
        gate1_matrix(g, G);
        mat_dag(G, Gd, 2);
        for (int l = 0; l < 4; ++l) {
            pauli_matrix(l, P);
            mat_mul(Gd, P, T, 2);
            mat_mul(T, G, R, 2);
            t1_letter[g][l] = -1;
            for (int l2 = 0; l2 < 4 && t1_letter[g][l] < 0; ++l2)
                for (int k = 0; k < 4; ++k) {
                    cplx Q[4];
                    pauli_matrix(l2, Q);
                    for (int i = 0; i < 4; ++i) Q[i] *= ipow(k);
                    if (mat_close(Q, R, 2)) { t1_letter[g][l] = l2; t1_phase[g][l] = k; break; }
                }
        }
    }
    for (int g = 6; g < 9; ++g) {
        cplx G[16], Gd[16], P[16], T[16], R[16];
        gate2_matrix(g, G);
        mat_dag(G, Gd, 4);
        for (int l0 = 0; l0 < 4; ++l0)
            for (int l1 = 0; l1 < 4; ++l1) {
                pauli2(l0, l1, P);
                mat_mul(Gd, P, T, 4);
                mat_mul(T, G, R, 4);
                int found = 0;
                for (int a = 0; a < 4 && !found; ++a)
                    for (int b = 0; b < 4 && !found; ++b)
                        for (int k = 0; k < 4 && !found; ++k) {
                            cplx Q[16];
                            pauli2(a, b, Q);
                            for (int i = 0; i < 16; ++i) Q[i] *= ipow(k);
                            if (mat_close(Q, R, 4)) {
                                t2_l0[g - 6][l0][l1] = a;
                                t2_l1[g - 6][l0][l1] = b;
                                t2_phase[g - 6][l0][l1] = k;
                                found = 1;
                            }
                        }
            }
    }
    tables_ready = 1;
}

/* Returns the table entry so tests can compare it with hand-written values. */
int orc_conj_table1(int g, int l, int *phase)
{
    build_tables();
    if (g < 0 || g > 5 || l < 0 || l > 3) return -1;
    *phase = t1_phase[g][l];
    return t1_letter[g][l];
}

/*
 * Q <- C^dag Q C for C = G_{m-1} ... G_0 (gate 0 acts first on the state).
 * letters: n codes, modified in place; *phase: exponent of i, modified.
 */
int orc_heisenberg(const int32_t *gates, int64_t m, uint8_t *letters, int n, int *phase)
{
    build_tables();
    int k = *phase & 3;
    for (int64_t r = m - 1; r >= 0; --r) {
        int g = gates[3 * r], q0 = gates[3 * r + 1], q1 = gates[3 * r + 2];
        if (q0 < 0 || q0 >= n) return -1;
        if (g <= 5) {
            int l = letters[q0];
            letters[q0] = (uint8_t)t1_letter[g][l];
            k += t1_phase[g][l];
        } else if (g <= 8) {
            if (q1 < 0 || q1 >= n || q1 == q0) return -1;
            int a = letters[q0], b = letters[q1];
            letters[q0] = (uint8_t)t2_l0[g - 6][a][b];
            letters[q1] = (uint8_t)t2_l1[g - 6][a][b];
            k += t2_phase[g - 6][a][b];
        } else {
            return -1;
        }
    }
    *phase = k & 3;
    return 0;
}

/* ------------------------------------------------------ dense state ops */

static void apply_mat1(cplx *psi, int n, int q, const cplx m[4])
{
    const int64_t half = (int64_t)1 << (n - 1);
    const int64_t low = ((int64_t)1 << q) - 1;
#pragma omp parallel for schedule(static) if (n >= PAR_MIN_QUBITS)
    for (int64_t i = 0; i < half; ++i) {
        int64_t y0 = ((i & ~low) << 1) | (i & low);
        int64_t y1 = y0 | ((int64_t)1 << q);
        cplx a = psi[y0], b = psi[y1];
        psi[y0] = m[0] * a + m[1] * b;
        psi[y1] = m[2] * a + m[3] * b;
    }
}

static int64_t insert_zero(int64_t i, int bit)
{
    int64_t low = ((int64_t)1 << bit) - 1;
    return ((i & ~low) << 1) | (i & low);
}

static void apply_gate2(cplx *psi, int n, int g, int q0, int q1)
{
    const int64_t quarter = (int64_t)1 << (n - 2);
    const int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
    const int64_t b0 = (int64_t)1 << q0, b1 = (int64_t)1 << q1;
#pragma omp parallel for schedule(static) if (n >= PAR_MIN_QUBITS)
    for (int64_t i = 0; i < quarter; ++i) {
        int64_t y = insert_zero(insert_zero(i, lo), hi);  /* bits q0 = q1 = 0 */
        if (g == 6) {                                     /* CNOT: swap |1,0> <-> |1,1> */
            cplx t = psi[y | b0];
            psi[y | b0] = psi[y | b0 | b1];
            psi[y | b0 | b1] = t;
        } else if (g == 7) {                              /* CZ */
            psi[y | b0 | b1] = -psi[y | b0 | b1];
        } else {                                          /* SWAP: |1,0> <-> |0,1> */
            cplx t = psi[y | b0];
            psi[y | b0] = psi[y | b1];
            psi[y | b1] = t;
        }
    }
}

int orc_apply_gate(cplx *psi, int n, int g, int q0, int q1)
{
    if (n < 1 || q0 < 0 || q0 >= n) return -1;
    cplx m[4];
    if (gate1_matrix(g, m)) {
        apply_mat1(psi, n, q0, m);
        return 0;
    }
    if (g < 6 || g > 8 || q1 < 0 || q1 >= n || q1 == q0 || n < 2) return -1;
    apply_gate2(psi, n, g, q0, q1);
    return 0;
}

/* The inverse of a gate list: inverse gates in reverse order. */
int orc_apply_gates(cplx *psi, int n, const int32_t *gates, int64_t m, int inverse)
{
    for (int64_t r = 0; r < m; ++r) {
        int64_t idx = inverse ? m - 1 - r : r;
        int g = gates[3 * idx];
        if (inverse && g == 1) g = 2;
        else if (inverse && g == 2) g = 1;
        if (orc_apply_gate(psi, n, g, gates[3 * idx + 1], gates[3 * idx + 2])) return -1;
    }
    return 0;
}

static void apply_rz(cplx *psi, int n, int q, double theta)
{
    cplx m[4] = {cexp(-I * theta / 2), 0, 0, cexp(I * theta / 2)};
    apply_mat1(psi, n, q, m);
}

/*
 * exp(-i theta/2 * s * P) with P the letter string and s = +1 or -1 its sign,
 * through basis change + CNOT ladder + RZ.
 */
int orc_rotation_ladder(cplx *psi, int n, const uint8_t *letters, int sign, double theta)
{
    int supp[64], w = 0;
    if (n < 1 || n > 40) return -1;
    for (int j = 0; j < n; ++j) {
        if (letters[j] > 3) return -1;
        if (letters[j]) supp[w++] = j;
    }
    double th = sign < 0 ? -theta : theta;
    if (w == 0) {                         /* identity string: global phase */
        cplx ph = cexp(-I * th / 2);
        const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static) if (n >= PAR_MIN_QUBITS)
        for (int64_t y = 0; y < N; ++y) psi[y] *= ph;
        return 0;
    }
    /* basis change V with V sigma V^dag = Z: X -> H; Y -> S^dag then H */
    for (int i = 0; i < w; ++i) {
        int q = supp[i];
        if (letters[q] == 2) orc_apply_gate(psi, n, 2, q, -1);
        if (letters[q] == 1 || letters[q] == 2) orc_apply_gate(psi, n, 0, q, -1);
    }
    for (int i = 0; i + 1 < w; ++i) orc_apply_gate(psi, n, 6, supp[i], supp[i + 1]);
    apply_rz(psi, n, supp[w - 1], th);
    for (int i = w - 2; i >= 0; --i) orc_apply_gate(psi, n, 6, supp[i], supp[i + 1]);
    for (int i = 0; i < w; ++i) {
        int q = supp[i];
        if (letters[q] == 1 || letters[q] == 2) orc_apply_gate(psi, n, 0, q, -1);
        if (letters[q] == 2) orc_apply_gate(psi, n, 1, q, -1);
    }
    return 0;
}

/* Rotations k = 0..K-1 in order; rows of K x n letters; signs may be NULL. */
int orc_rotations_ladder(cplx *psi, int n, const uint8_t *letters, const int32_t *signs,
                         const double *theta, int64_t K)
{
    for (int64_t k = 0; k < K; ++k)
        if (orc_rotation_ladder(psi, n, letters + k * n, signs ? signs[k] : 1, theta[k])) return -1;
    return 0;
}

/* P|y> letter by letter: returns the image index and multiplies *amp. */
static uint64_t pauli_on_basis(const uint8_t *letters, int n, uint64_t y, cplx *amp)
{
    cplx a = *amp;
    for (int j = 0; j < n; ++j) {
        int b = (int)((y >> j) & 1);
        switch (letters[j]) {
        case 1: y ^= (uint64_t)1 << j; break;                          /* X|b> = |1-b> */
        case 2: a *= b ? -I : I; y ^= (uint64_t)1 << j; break;         /* Y|0> = i|1>, Y|1> = -i|0> */
        case 3: if (b) a = -a; break;                                  /* Z|b> = (-1)^b |b> */
        default: break;
        }
    }
    *amp = a;
    return y;
}

/* <psi| i^phase P |psi> with P applied letter by letter to a copy of psi. */
int orc_expval(const cplx *psi, int n, const uint8_t *letters, int phase, double *re, double *im)
{
    const int64_t N = (int64_t)1 << n;
    double sr = 0, si = 0;
#pragma omp parallel for schedule(static) reduction(+ : sr, si) if (n >= PAR_MIN_QUBITS)
    for (int64_t y = 0; y < N; ++y) {
        cplx a = psi[y];
        uint64_t t = pauli_on_basis(letters, n, (uint64_t)y, &a);
        cplx v = conj(psi[t]) * a;
        sr += creal(v);
        si += cimag(v);
    }
    cplx r = (sr + I * si) * ipow(phase);
    *re = creal(r);
    *im = cimag(r);
    return 0;
}

/* E = sum_j coeff_j Re <psi| i^phase_j P_j |psi>. */
double orc_energy(const cplx *psi, int n, const uint8_t *letters, const int32_t *phases,
                  const double *coeff, int64_t m)
{
    double e = 0;
    for (int64_t j = 0; j < m; ++j) {
        double re, im;
        orc_expval(psi, n, letters + j * n, phases ? phases[j] : 0, &re, &im);
        e += coeff[j] * re;
    }
    return e;
}

/* out = sum_j coeff_j i^phase_j P_j psi, each P_j applied letter by letter. */
int orc_apply_pauli_sum(const cplx *psi, int n, const uint8_t *letters, const int32_t *phases,
                        const double *coeff, int64_t m, cplx *out)
{
    const int64_t N = (int64_t)1 << n;
    memset(out, 0, (size_t)N * sizeof(cplx));
    for (int64_t j = 0; j < m; ++j) {
        const uint8_t *P = letters + j * n;
        cplx f = coeff[j] * ipow(phases ? phases[j] : 0);
        /* out[t] += f * (P psi)[t]; P maps basis y to t = P(y) bijectively */
#pragma omp parallel for schedule(static) if (n >= PAR_MIN_QUBITS)
        for (int64_t y = 0; y < N; ++y) {
            cplx a = psi[y];
            uint64_t t = pauli_on_basis(P, n, (uint64_t)y, &a);
            out[t] += f * a;
        }
    }
    return 0;
}

/* ------------------------------------------------ sparse definition path */
/* Open-addressing hash map uint64 index -> complex amplitude. */

typedef struct {
    uint64_t *key;
    cplx *val;
    int64_t cap, size;
} smap;

static const uint64_t EMPTY = ~(uint64_t)0;

static int smap_init(smap *s, int64_t cap)
{
    int64_t c = 16;
    while (c < 2 * cap) c <<= 1;
    s->key = (uint64_t *)malloc((size_t)c * sizeof(uint64_t));
    s->val = (cplx *)calloc((size_t)c, sizeof(cplx));
    if (!s->key || !s->val) return -1;
    for (int64_t i = 0; i < c; ++i) s->key[i] = EMPTY;
    s->cap = c;
    s->size = 0;
    return 0;
}

static void smap_free(smap *s) { free(s->key); free(s->val); }

static cplx *smap_slot(smap *s, uint64_t k)
{
    uint64_t h = k * 0x9E3779B97F4A7C15ull;
    int64_t i = (int64_t)(h & (uint64_t)(s->cap - 1));
    while (s->key[i] != EMPTY && s->key[i] != k) i = (i + 1) & (s->cap - 1);
    if (s->key[i] == EMPTY) { s->key[i] = k; s->size++; }
    return &s->val[i];
}

/*
 * Sparse simulation by definition: R = cos(theta/2) I - i sin(theta/2) s P.
 * Input: nnz (index, amplitude) pairs; output arrays must hold max_out pairs.
 * Returns the output count, or -1 on overflow/invalid input.
 */
int64_t orc_sparse_rotations(int n, const uint64_t *idx_in, const cplx *amp_in, int64_t nnz,
                             const uint8_t *letters, const int32_t *signs, const double *theta,
                             int64_t K, uint64_t *idx_out, cplx *amp_out, int64_t max_out)
{
    smap cur;
    if (n < 1 || n > 63 || smap_init(&cur, nnz > max_out ? nnz : max_out)) return -1;
    for (int64_t i = 0; i < nnz; ++i) *smap_slot(&cur, idx_in[i]) += amp_in[i];
    for (int64_t k = 0; k < K; ++k) {
        const uint8_t *P = letters + k * n;
        double th = (signs && signs[k] < 0) ? -theta[k] : theta[k];
        double c = cos(th / 2), s = sin(th / 2);
        smap nxt;
        if (smap_init(&nxt, 2 * cur.size + 1)) { smap_free(&cur); return -1; }
        for (int64_t i = 0; i < cur.cap; ++i) {
            if (cur.key[i] == EMPTY) continue;
            uint64_t y = cur.key[i];
            cplx a = cur.val[i];
            *smap_slot(&nxt, y) += c * a;
            cplx pa = a;
            uint64_t t = pauli_on_basis(P, n, y, &pa);
            *smap_slot(&nxt, t) += -I * s * pa;
        }
        smap_free(&cur);
        cur = nxt;
        if (cur.size > max_out) { smap_free(&cur); return -1; }
    }
    int64_t o = 0;
    for (int64_t i = 0; i < cur.cap; ++i)
        if (cur.key[i] != EMPTY) { idx_out[o] = cur.key[i]; amp_out[o] = cur.val[i]; ++o; }
    smap_free(&cur);
    return o;
}

void orc_set_num_threads(int k)
{
#ifdef _OPENMP
    if (k > 0) omp_set_num_threads(k);
#else
    (void)k;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
