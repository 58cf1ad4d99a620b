// Host side of libcfh: error reporting, Pauli encoding and the bit-packed
// Pauli frame tracker in the backward interpretation (Sec. 4.1).
#include <cstring>
#include <new>
#include <string>

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

} // extern "C"
