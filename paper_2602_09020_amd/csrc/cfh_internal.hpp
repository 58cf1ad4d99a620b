// Internal declarations shared by the host planner and the gfx950 kernels of
// libcfh.  Not installed; the public interface is include/cfh.h.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "cfh.h"

namespace cfh {

constexpr int kMaxStateQubits = 34;   // 2^34 c128 amplitudes = 256 GiB
constexpr int kMaxFrameQubits = 63;
constexpr int kMaxTileBits = 16;      // basis vectors carried per pass
constexpr int kMaxRun = 32;           // rotations per fused pass (kernel argument capacity)
constexpr int kMaxGroupsPerPass = 64; // x-groups per read-only Hamiltonian pass

// ------------------------------------------------------------- Pauli algebra
// P = i^e (x)_j sigma(x_j, z_j), sigma(1,1) = Y.  Writing sigma(x,z) = i^{xz} X^x Z^z
// and moving Z^{z1} past X^{x2} (one sign per shared qubit) gives the product
// rule below (the phase group of Sec. 2.1, Eq. pauli_group).
struct Pauli {
    uint64_t x = 0, z = 0;
    int e = 0;
};

inline int popc(uint64_t v) { return __builtin_popcountll(v); }

inline Pauli pauli_mul(const Pauli &a, const Pauli &b)
{
    Pauli r;
    r.x = a.x ^ b.x;
    r.z = a.z ^ b.z;
    r.e = (a.e + b.e + popc(a.x & a.z) + popc(b.x & b.z) + 2 * popc(a.z & b.x) - popc(r.x & r.z)) & 3;
    return r;
}

// Anticommutation flag lambda(P, Q) of Sec. 2.1: parity of the symplectic form.
inline bool anticommute(uint64_t x1, uint64_t z1, uint64_t x2, uint64_t z2)
{
    return (popc(x1 & z2) ^ popc(z1 & x2)) & 1;
}

// ---------------------------------------------------------- pass descriptors
// A fused pass works on the cosets y + V of a b-dimensional subspace V of
// GF(2)^n.  V is held in reduced echelon form: basis vector v[i] owns pivot
// bit p_i, which no other basis vector has set.  A coset is addressed by its
// base (any assignment of the non-pivot bits, `outer_mask`) and its elements
// by the local index a: y = base ^ (xor of v[i] over set bits i of a).
// A rotation with x in V maps every coset onto itself; in local coordinates
// its x is xl (bit i set iff x has pivot bit p_i) and the parity of y & z is
// parity(base & z) ^ parity(a & zl) with zl_i = parity(v[i] & z).
struct RotDesc {
    uint32_t xl;   // local x mask, 0 for a diagonal rotation
    uint32_t zl;   // local z parity mask
    uint64_t z;    // global z mask (sign of the coset base)
    int32_t hb;    // highest set bit of xl, -1 when xl == 0
    int32_t k;     // rotation index (angle, coefficient and gradient slot)
    int32_t w;     // omega exponent: (e - |x&z| + 3) mod 4
    int32_t dsign; // parity(x & z): sign difference between the two pair members
};

struct PassArgs {
    uint64_t outer_mask;
    uint64_t v[kMaxTileBits];
    int32_t b;
    int32_t nrot;
    int32_t inverse;     // 1: apply R^dag (negated angles) in reverse order
    int32_t tile_base;   // first coset handled by block 0 (for split launches)
    RotDesc rot[kMaxRun];
};

// One x-group of a read-only Hamiltonian pass (device memory).
struct HamGroupDev {
    uint32_t xl;
    int32_t hb;
    int32_t term_begin;
    int32_t term_count;
};
struct HamTermDev {
    uint64_t z;   // global z (coset sign)
    uint32_t zl;  // local z parity mask
    uint32_t pad;
    double wre;   // coeff * i^{(e - |x&z|) mod 4}, real part
    double wim;   // imaginary part
};
struct HamPassArgs {
    uint64_t outer_mask;
    uint64_t v[kMaxTileBits];
    int32_t b;
    int32_t group_begin;
    int32_t group_count;
    int32_t pad;
};

// ------------------------------------------------------------ host objects
struct PassPlan {
    int b = 0;
    uint64_t outer_mask = 0;
    std::vector<uint64_t> v;   // b basis vectors, local bit i <-> v[i]
    std::vector<int> rots;     // rotation indices in application order
};

struct TuningResolved {
    int tile_bits, low_bits, max_run, lookahead, unfused, block_threads;
};

TuningResolved resolve_tuning(const cfh_tuning *t, int n, int dtype, bool adjoint_tiles);

// Builds the passes of a rotation sequence (the fusion planner).
std::vector<PassPlan> plan_rotations(int n, const std::vector<Pauli> &rot, const TuningResolved &tu);

// Builds read-only passes covering the x-groups of a Hamiltonian.
struct HamGroup {
    uint64_t x;
    std::vector<int> terms;
};
struct HamPass {
    int b = 0;
    uint64_t outer_mask = 0;
    std::vector<uint64_t> v;
    std::vector<int> groups;
};
std::vector<HamPass> plan_hamiltonian(int n, const std::vector<HamGroup> &groups, const TuningResolved &tu);

// Fill a kernel descriptor for one rotation inside pass `pp`.
RotDesc make_rot_desc(const PassPlan &pp, const Pauli &p, int k);
uint32_t local_coords(const std::vector<uint64_t> &v, uint64_t x, bool *in_span);
uint32_t local_zmask(const std::vector<uint64_t> &v, uint64_t z);

// ------------------------------------------------------------------ errors
cfh_status set_error(cfh_status code, const std::string &msg);
void clear_error();
cfh_status check_pauli(const cfh_pauli &p, int n, bool need_hermitian, const char *what);

} // namespace cfh

// Opaque handle bodies.
struct cfh_frame_s {
    int n;
    std::vector<cfh::Pauli> zf, xf;  // effZ_q, effX_q
};
