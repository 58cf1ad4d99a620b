// Host side of libcfh: error reporting, Pauli encoding and the bit-packed
// Pauli frame tracker in the backward interpretation (Sec. 4.1).
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "cfh_internal.hpp"

namespace cfh {

static thread_local std::string g_last_error;

cfh_status set_error(cfh_status code, const std::string &msg)
{
    g_last_error = msg;
    return code;
}

void clear_error() { g_last_error.clear(); }

cfh_status check_pauli(const cfh_pauli &p, int n, bool need_hermitian, const char *what)
{
    const uint64_t lim = n >= 64 ? ~0ull : ((1ull << n) - 1);
    if ((p.x & ~lim) || (p.z & ~lim))
        return set_error(CFH_E_RANGE, std::string(what) + ": mask bit at or above n");
    if (need_hermitian && (p.e & 1))
        return set_error(CFH_E_NOT_HERMITIAN, std::string(what) + ": odd phase exponent (not Hermitian)");
    return CFH_OK;
}

// P conjugated by the Clifford rotation exp(-i theta/2 Q): a P that commutes
// with Q is left as it is; otherwise theta = pi/2 gives -i Q P and theta = pi
// (exp(-i pi/2 Q) = -i Q) gives -P (App. A, note on pi/4 conjugation).
static Pauli conj_by_rotation(const Pauli &P, const Pauli &Q, bool half_turn)
{
    if (!anticommute(P.x, P.z, Q.x, Q.z)) return P;
    if (half_turn) {
        Pauli r = P;
        r.e = (r.e + 2) & 3;
        return r;
    }
    Pauli r = pauli_mul(Q, P);
    r.e = (r.e + 3) & 3;
    return r;
}

// Rotations R_1..R_m (angles pi/2 or pi) with R_m...R_1 U^dag = phase * I for
// the Clifford U of the frame, so that U Phi = phase * R_m...R_1 Phi: applying
// them to Phi, in order, flushes the frame into the state (Sec. 4.3, App. A).
// Conjugating the rows by each rotation tracks U^dag; the rows end as the
// identity frame, which is checked.
//  1. For each qubit q, a row i not yet placed whose effZ_i acts on q is
//     brought to a one-qubit s1 on q by Q = i s1 effZ_i (s1 anticommuting
//     with effZ_i's letter on q), then its effX_i to a one-qubit s2 on q by
//     Q' = i s2 effX_i (s2 neither s1 nor effX_i's letter on q); Q' commutes
//     with s1.  The other rows commute with both, so they no longer act on q,
//     and later rotations (which do not act on q) leave row i alone.
//  2. Each row's one-qubit pair is turned into (+Z, +X) by pi/2 rotations
//     about one-qubit Paulis and pi rotations for the signs.
//  3. Rows are moved to their own qubits by SWAPs, each the product of the
//     commuting pi/2 rotations about X_a X_b, Y_a Y_b and Z_a Z_b (a SWAP up
//     to a global phase).
cfh_status frame_flush_rotations(const cfh_frame_s &f, std::vector<Pauli> &rot, std::vector<double> &theta)
{
    const int n = f.n;
    std::vector<Pauli> zf = f.zf, xf = f.xf;
    rot.clear();
    theta.clear();
    auto apply = [&](const Pauli &Q, bool half_turn) {
        for (int i = 0; i < n; ++i) {
            zf[i] = conj_by_rotation(zf[i], Q, half_turn);
            xf[i] = conj_by_rotation(xf[i], Q, half_turn);
        }
        rot.push_back(Q);
        theta.push_back(half_turn ? 3.14159265358979323846 : 1.57079632679489661923);
    };
    auto single = [](int q, int letter) {  // letters 1 = X, 2 = Y, 3 = Z
        Pauli p;
        p.x = (letter == 1 || letter == 2) ? 1ull << q : 0;
        p.z = (letter == 3 || letter == 2) ? 1ull << q : 0;
        return p;
    };
    auto letter_at = [](const Pauli &p, int q) {
        const int xb = (int)((p.x >> q) & 1), zb = (int)((p.z >> q) & 1);
        return xb ? (zb ? 2 : 1) : (zb ? 3 : 0);
    };
    auto only_on = [](const Pauli &p, int q) { return ((p.x | p.z) & ~(1ull << q)) == 0; };
    // Q = i s P for anticommuting s and P: Hermitian, and conjugation maps P to s
    auto mover = [](const Pauli &s, const Pauli &P) {
        Pauli Q = pauli_mul(s, P);
        Q.e = (Q.e + 1) & 3;
        return Q;
    };
    std::vector<int> pos(n, -1);
    std::vector<char> placed(n, 0);
    for (int q = 0; q < n; ++q) {
        int i = -1;
        for (int k = 0; k < n && i < 0; ++k)
            if (!placed[k] && (((zf[k].x | zf[k].z) >> q) & 1)) i = k;
        if (i < 0) return set_error(CFH_E_INVAL, "cfh_frame_flush: the frame rows are not a symplectic basis");
        const int sig = letter_at(zf[i], q);
        int s1 = sig;
        if (!only_on(zf[i], q)) {
            s1 = sig == 3 ? 1 : 3;
            apply(mover(single(q, s1), zf[i]), false);
        }
        if (!only_on(xf[i], q)) {
            const int s2 = 6 - s1 - letter_at(xf[i], q);
            apply(mover(single(q, s2), xf[i]), false);
        }
        placed[i] = 1;
        pos[i] = q;
    }
    for (int i = 0; i < n; ++i) {
        const int q = pos[i];
        const int zl = letter_at(zf[i], q);
        if (zl == 1) apply(single(q, 2), false);       // X -> -i Y X = -Z
        else if (zl == 2) apply(single(q, 1), false);  // Y -> -i X Y = Z
        if (letter_at(xf[i], q) == 2) apply(single(q, 3), false);  // Y -> -i Z Y = -X
        if (zf[i].e == 2) apply(single(q, 1), true);   // -Z -> X (-Z) X = Z
        if (xf[i].e == 2) apply(single(q, 3), true);   // -X -> Z (-X) Z = X
    }
    for (int i = 0; i < n; ++i) {
        const int q = pos[i];
        if (q == i) continue;
        const uint64_t m = (1ull << q) | (1ull << i);
        Pauli xx, yy, zz;
        xx.x = m;
        yy.x = m;
        yy.z = m;
        zz.z = m;
        apply(xx, false);
        apply(yy, false);
        apply(zz, false);
        for (int k = 0; k < n; ++k)
            if (pos[k] == i) {
                pos[k] = q;
                break;
            }
        pos[i] = i;
    }
    for (int i = 0; i < n; ++i)
        if (zf[i].x || zf[i].z != (1ull << i) || zf[i].e || xf[i].x != (1ull << i) || xf[i].z || xf[i].e)
            return set_error(CFH_E_INVAL, "cfh_frame_flush: the frame did not reduce to the identity");
    for (const Pauli &Q : rot)
        if (Q.e & 1) return set_error(CFH_E_INVAL, "cfh_frame_flush: a flush rotation is not Hermitian");
    return CFH_OK;
}

cfh_status circuit_translate(cfh_frame_s &f, const int32_t *gates, const double *angles, size_t begin, size_t m,
                             std::vector<cfh_pauli> &rot, std::vector<double> &theta, size_t *stop)
{
    rot.clear();
    theta.clear();
    *stop = m;
    for (size_t i = begin; i < m; ++i) {
        const int code = gates[3 * i], q0 = gates[3 * i + 1], q1 = gates[3 * i + 2];
        if (code == CFH_GATE_MEASURE || code == CFH_GATE_RESET) {
            *stop = i;
            return CFH_OK;
        }
        if (code == CFH_GATE_RX || code == CFH_GATE_RY || code == CFH_GATE_RZ) {
            if (q0 < 0 || q0 >= f.n || q1 != -1)
                return set_error(CFH_E_INVAL, "cfh_circuit_translate: a rotation needs q0 in range and q1 = -1");
            if (!angles) return set_error(CFH_E_INVAL, "cfh_circuit_translate: rotation gate without angles");
            // R_sigma(theta) U = U R_{F(sigma)}(theta), F(sigma) = U^dag sigma U
            const uint64_t b = 1ull << q0;
            const cfh_pauli s{code == CFH_GATE_RZ ? 0 : b, code == CFH_GATE_RX ? 0 : b, 0, 0};
            cfh_pauli a{};
            cfh_status st = cfh_frame_conjugate(&f, &s, &a);
            if (st) return st;
            rot.push_back(a);
            theta.push_back(angles[i]);
        } else {
            cfh_status st = cfh_frame_apply_clifford(&f, code, q0, q1);
            if (st) return st;
        }
    }
    return CFH_OK;
}

void frame_reset(cfh_frame_s &f)
{
    for (int q = 0; q < f.n; ++q) {
        f.zf[q] = Pauli{0, 1ull << q, 0};
        f.xf[q] = Pauli{1ull << q, 0, 0};
    }
}

} // namespace cfh

using namespace cfh;

extern "C" {

int cfh_version(void) { return CFH_API_VERSION; }

const char *cfh_last_error(void) { return g_last_error.c_str(); }

cfh_status cfh_pauli_encode(const uint8_t *letters, int n, size_t m, cfh_pauli *out)
{
    if (!out || (m && !letters) || n < 1 || n > kMaxFrameQubits)
        return set_error(CFH_E_INVAL, "cfh_pauli_encode: bad arguments");
    for (size_t i = 0; i < m; ++i) {
        uint64_t x = 0, z = 0;
        for (int j = 0; j < n; ++j) {
            const uint8_t l = letters[i * (size_t)n + j];
            if (l > 3) return set_error(CFH_E_INVAL, "cfh_pauli_encode: letter code > 3");
            // masks of Sec. 2.2: x = m_X | m_Y, z = m_Z | m_Y
            if (l == 1 || l == 2) x |= 1ull << j;
            if (l == 3 || l == 2) z |= 1ull << j;
        }
        out[i].x = x;
        out[i].z = z;
        out[i].e = 0;
        out[i].reserved = 0;
    }
    return CFH_OK;
}

cfh_status cfh_frame_create(int n, cfh_frame *out)
{
    if (!out || n < 1 || n > kMaxFrameQubits)
        return set_error(CFH_E_INVAL, "cfh_frame_create: n must be in 1..63");
    cfh_frame f = new (std::nothrow) cfh_frame_s;
    if (!f) return set_error(CFH_E_NOMEM, "cfh_frame_create: out of host memory");
    f->n = n;
    f->zf.resize(n);
    f->xf.resize(n);
    for (int q = 0; q < n; ++q) {
        f->zf[q].z = 1ull << q;  // effZ_q = Z_q
        f->xf[q].x = 1ull << q;  // effX_q = X_q
    }
    *out = f;
    return CFH_OK;
}

cfh_status cfh_frame_destroy(cfh_frame f)
{
    delete f;
    return CFH_OK;
}

// Row updates for U <- G U.  New rows are U^dag G^dag sigma G U; each line
// states G^dag sigma G for the changed rows (S^dag X S = -Y = -i X Z, etc.).
cfh_status cfh_frame_apply_clifford(cfh_frame f, int gate, int q0, int q1)
{
    if (!f) return set_error(CFH_E_INVAL, "cfh_frame_apply_clifford: null frame");
    const int n = f->n;
    if (q0 < 0 || q0 >= n) return set_error(CFH_E_INVAL, "cfh_frame_apply_clifford: bad qubit q0");
    const bool two = gate == CFH_GATE_CNOT || gate == CFH_GATE_CZ || gate == CFH_GATE_SWAP;
    if (two) {
        if (q1 < 0 || q1 >= n || q1 == q0)
            return set_error(CFH_E_INVAL, "cfh_frame_apply_clifford: bad qubit q1");
    } else if (q1 != -1) {
        return set_error(CFH_E_INVAL, "cfh_frame_apply_clifford: q1 must be -1 for a one-qubit gate");
    }
    Pauli &Zq = f->zf[q0], &Xq = f->xf[q0];
    switch (gate) {
    case CFH_GATE_H:   // H Z H = X, H X H = Z
        std::swap(Zq, Xq);
        break;
    case CFH_GATE_S: { // S^dag X S = -Y = -i X Z = i Z X
        Pauli t = pauli_mul(Zq, Xq);
        t.e = (t.e + 1) & 3;
        Xq = t;
        break;
    }
    case CFH_GATE_SDG: { // S X S^dag = Y = i X Z = -i Z X
        Pauli t = pauli_mul(Zq, Xq);
        t.e = (t.e + 3) & 3;
        Xq = t;
        break;
    }
    case CFH_GATE_X:   // X Z X = -Z
        Zq.e = (Zq.e + 2) & 3;
        break;
    case CFH_GATE_Z:   // Z X Z = -X
        Xq.e = (Xq.e + 2) & 3;
        break;
    case CFH_GATE_Y:   // Y Z Y = -Z, Y X Y = -X
        Zq.e = (Zq.e + 2) & 3;
        Xq.e = (Xq.e + 2) & 3;
        break;
    case CFH_GATE_CNOT: // Z_t -> Z_c Z_t, X_c -> X_c X_t
        f->zf[q1] = pauli_mul(f->zf[q0], f->zf[q1]);
        f->xf[q0] = pauli_mul(f->xf[q0], f->xf[q1]);
        break;
    case CFH_GATE_CZ: { // X_a -> X_a Z_b, X_b -> Z_a X_b
        Pauli xa = pauli_mul(f->xf[q0], f->zf[q1]);
        Pauli xb = pauli_mul(f->zf[q0], f->xf[q1]);
        f->xf[q0] = xa;
        f->xf[q1] = xb;
        break;
    }
    case CFH_GATE_SWAP:
        std::swap(f->zf[q0], f->zf[q1]);
        std::swap(f->xf[q0], f->xf[q1]);
        break;
    default:
        return set_error(CFH_E_INVAL, "cfh_frame_apply_clifford: unknown gate code");
    }
    return CFH_OK;
}

cfh_status cfh_frame_apply_gates(cfh_frame f, const int32_t *gates, size_t m)
{
    if (!f || (m && !gates)) return set_error(CFH_E_INVAL, "cfh_frame_apply_gates: null argument");
    for (size_t i = 0; i < m; ++i) {
        cfh_status s = cfh_frame_apply_clifford(f, gates[3 * i], gates[3 * i + 1], gates[3 * i + 2]);
        if (s) return s;
    }
    return CFH_OK;
}

cfh_status cfh_frame_row(cfh_frame f, int q, cfh_pauli *effZ, cfh_pauli *effX)
{
    if (!f || q < 0 || q >= f->n) return set_error(CFH_E_INVAL, "cfh_frame_row: bad frame or qubit");
    if (effZ) *effZ = cfh_pauli{f->zf[q].x, f->zf[q].z, f->zf[q].e, 0};
    if (effX) *effX = cfh_pauli{f->xf[q].x, f->xf[q].z, f->xf[q].e, 0};
    return CFH_OK;
}

// F(P) = i^e prod_{j in supp P} L_j with L_j = effX_j (X), effZ_j (Z) and
// U^dag Y_j U = U^dag (i X_j Z_j) U = i effX_j effZ_j (equal to -i effZ_j effX_j,
// the effY_j of Eq. framemat).  Factors of different qubits commute, so the
// order of the product does not matter.
cfh_status cfh_frame_conjugate(cfh_frame f, const cfh_pauli *p, cfh_pauli *out)
{
    if (!f || !p || !out) return set_error(CFH_E_INVAL, "cfh_frame_conjugate: null argument");
    cfh_status s = check_pauli(*p, f->n, false, "cfh_frame_conjugate");
    if (s) return s;
    Pauli r;
    r.e = p->e & 3;
    uint64_t supp = p->x | p->z;
    while (supp) {
        const int j = __builtin_ctzll(supp);
        supp &= supp - 1;
        const bool xb = (p->x >> j) & 1, zb = (p->z >> j) & 1;
        if (xb && zb) {
            Pauli y = pauli_mul(f->xf[j], f->zf[j]);
            y.e = (y.e + 1) & 3;
            r = pauli_mul(r, y);
        } else if (xb) {
            r = pauli_mul(r, f->xf[j]);
        } else {
            r = pauli_mul(r, f->zf[j]);
        }
    }
    *out = cfh_pauli{r.x, r.z, r.e, 0};
    return CFH_OK;
}

cfh_status cfh_frame_conjugate_many(cfh_frame f, const cfh_pauli *in, cfh_pauli *out, size_t m)
{
    if (!f || (m && (!in || !out))) return set_error(CFH_E_INVAL, "cfh_frame_conjugate_many: null argument");
    for (size_t i = 0; i < m; ++i) {
        cfh_pauli t;
        cfh_status s = cfh_frame_conjugate(f, &in[i], &t);
        if (s) return s;
        out[i] = t;
    }
    return CFH_OK;
}

cfh_status cfh_circuit_translate(cfh_frame f, const int32_t *gates, const double *angles, size_t m,
                                 cfh_pauli *rot, double *theta, size_t cap, size_t *nrot)
{
    if (!f || !nrot || (m && !gates)) return set_error(CFH_E_INVAL, "cfh_circuit_translate: null argument");
    std::vector<cfh_pauli> r;
    std::vector<double> th;
    size_t stop = 0;
    cfh_status s = circuit_translate(*f, gates, angles, 0, m, r, th, &stop);
    if (s) return s;
    if (stop < m)
        return set_error(CFH_E_UNSUPPORTED,
                         "cfh_circuit_translate: measurement and reset rows need the state (cfh_circuit_run)");
    *nrot = r.size();
    if (r.size() > cap) return set_error(CFH_E_RANGE, "cfh_circuit_translate: more rotations than cap");
    if (!r.empty() && (!rot || !theta)) return set_error(CFH_E_INVAL, "cfh_circuit_translate: null output");
    for (size_t i = 0; i < r.size(); ++i) {
        rot[i] = r[i];
        theta[i] = th[i];
    }
    return CFH_OK;
}

cfh_status cfh_frame_flush_rotations(cfh_frame f, cfh_pauli *rot, double *theta, size_t cap, size_t *m)
{
    if (!f || !m) return set_error(CFH_E_INVAL, "cfh_frame_flush_rotations: null argument");
    std::vector<Pauli> q;
    std::vector<double> th;
    cfh_status s = frame_flush_rotations(*f, q, th);
    if (s) return s;
    *m = q.size();
    if (q.size() > cap) return set_error(CFH_E_RANGE, "cfh_frame_flush_rotations: more rotations than cap");
    if (!q.empty() && (!rot || !theta)) return set_error(CFH_E_INVAL, "cfh_frame_flush_rotations: null output");
    for (size_t i = 0; i < q.size(); ++i) {
        rot[i] = cfh_pauli{q[i].x, q[i].z, q[i].e, 0};
        theta[i] = th[i];
    }
    return CFH_OK;
}

} // extern "C"
