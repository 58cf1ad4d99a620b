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
    int32_t pad;
    uint64_t tile_base;  // first coset handled by block 0 (for split launches)
    RotDesc rot[kMaxRun];
};

// Register-tiled form of a pass.  Inside the coset, a run is split into
// micro-groups: consecutive rotations whose local x masks span at most
// kRegDims dimensions U = span(u_0..u_3).  During a micro-group every thread
// holds the 16 amplitudes base_t ^ U[j] (j = 0..15) of one coset of U in
// registers, so each rotation pairs register j with register j ^ cx.  Between
// micro-groups the tile is transposed through LDS.  base_t deposits the
// thread index into the non-pivot local bits `npiv` of the micro-group.
constexpr int kRegDims = 4;
constexpr int kRegs = 1 << kRegDims;
constexpr int kMaxMG = 12;

struct RotDesc2 {
    uint32_t zl;     // local z parity mask
    uint16_t msign;  // bit j = parity(U[j] & zl)
    uint8_t cx;      // partner mask in register coordinates, 0 = diagonal
    uint8_t flags;   // bit 0: beta imaginary (w odd); bit 1: negate (w & 2); bit 2: i^{(e-|x&z|)} negative
    uint64_t z;      // global z (coset base sign)
    int32_t k;       // rotation index
    uint32_t zt;     // thread-index parity mask: parity(t & zt) = parity(bt & zl)
    uint32_t kase;   // cx | zr << 4 | imag << 8, zr_i = parity(u_i & zl); msign_j = parity(j & zr)
    int32_t pad;
};

struct MGDesc2 {
    uint32_t U[kRegs];   // local offset of register j
    uint32_t UC[kRegs];  // U[j] with the anchor bit removed (half-tile LDS index)
    uint32_t npiv;       // local bits that enumerate threads
    int32_t rot_begin;
    int32_t rot_count;
    int32_t pad;
};

struct PassArgs2 {
    uint64_t outer_mask;
    uint64_t v[kMaxTileBits];        // local -> global basis
    uint64_t LU_first[kRegs];        // global offset of register j, first micro-group layout
    uint64_t LU_last[kRegs];         // same for the last micro-group layout
    int32_t b;
    int32_t nmg;
    int32_t inverse;                 // negate angles (order already reversed on the host)
    int32_t qbit;                    // anchor pivot bit (register dim 0 of every micro-group), -1 = none
    int32_t xrot;                    // p > 0: the 2^p cosets sharing a 128-byte line go to one XCD; 0 = index order; -1 = bit-reversed
    int32_t pad;
    MGDesc2 mg[kMaxMG];
    RotDesc2 rot[kMaxRun];
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
    int tile_bits, low_bits, max_run, lookahead, unfused, block_threads, variant, tile_order;
};

enum { kTuneForward = 0, kTuneAdjoint = 1, kTuneHamiltonian = 2, kTuneMeasure = 3, kTuneAdjoint2 = 4 };
TuningResolved resolve_tuning(const cfh_tuning *t, int n, int dtype, int kind);

// Coset order of a register-tiled pass.  p > 0: the number of low coset-index
// bits that address amplitudes inside one 128-byte line (the outer bits below
// the line size), for the XCD-aware order.  -1 (bit-reversed coset index) when
// the tiles use whole lines or there are fewer than 8 * 2^p cosets, or when
// tile_order is 2.  0 (index order) when tile_order is 1.
int line_share_bits(uint64_t outer_mask, int n, int b, int amp_bytes, int tile_order);

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
std::vector<HamPass> plan_hamiltonian(int n, const std::vector<HamGroup> &groups, const TuningResolved &tu,
                                      int max_groups = kMaxGroupsPerPass, int max_terms = 1 << 30);
// Order the terms idx of one pass (all commute inside a sum) so that
// consecutive terms share register micro-groups: terms whose local x already
// lies in the current 4-dimensional span first, then the dimension that
// brings the most remaining terms in.
std::vector<int> order_for_microgroups(const std::vector<uint64_t> &basis, const std::vector<Pauli> &p,
                                      const std::vector<int> &idx, bool anchor);

// Fill a kernel descriptor for one rotation inside pass `pp`.
RotDesc make_rot_desc(const PassPlan &pp, const Pauli &p, int k);
// Register-tiled kernel arguments for one pass (forward or inverse order);
// false if the pass does not fit (more than kMaxMG micro-groups, b < kRegDims).
// anchor: seed every micro-group with the same vector (register dimension 0),
// so transposes can move the tile through LDS in two halves.
bool build_pass_args2(const PassPlan &pp, const std::vector<Pauli> &rot, bool inverse, bool anchor, PassArgs2 &a);
// Claim order of a persistent batched run: cache group by cache group,
// level by level (pass lv of every circuit of the group whose chain is that
// long), circuits with the most work left (amplitudes x passes left) first,
// each pass's work items in index order.  Every item comes after all items of
// the pass before it in its chain (prev[p], -1 for a chain's first pass), so
// a schedule that claims tickets in this order never waits on a later one.
void batch_ticket_order(const std::vector<std::vector<int>> &chains, const std::vector<int> &pass_items,
                        const std::vector<double> &circ_amps, const std::vector<std::pair<int, int>> &groups,
                        std::vector<std::pair<int, int>> &tickets, std::vector<int> &prev);
uint32_t local_coords(const std::vector<uint64_t> &v, uint64_t x, bool *in_span);
uint32_t local_zmask(const std::vector<uint64_t> &v, uint64_t z);

// ------------------------------------------------------------------ errors
cfh_status set_error(cfh_status code, const std::string &msg);
void clear_error();
cfh_status check_pauli(const cfh_pauli &p, int n, bool need_hermitian, const char *what);

// Observable planning (plan.cpp): the x-groups of the terms in first-appearance
// order; how <H> runs (measurement tuning, register tiles or LDS-staged,
// anchored half-tile transposes); the register-tiled term passes.
// How <H> runs: the measurement tuning, whether it runs on register tiles
// (tiles of 2^10..2^14 amplitudes, not tuning variant 1), and whether its
// micro-groups share an anchor vector for half-tile transposes (required at
// 2^14, the default at complex128, selectable by variant 5).
struct MeasureSettings {
    TuningResolved tm;
    bool reg, anchor;
};
std::vector<HamGroup> group_terms(const cfh_pauli *terms, size_t m);
MeasureSettings measure_settings(const cfh_tuning *tuning, int n, int dtype, size_t m);
cfh_status term_passes(int n, int dtype, const std::vector<HamGroup> &groups, const std::vector<Pauli> &tp,
                       const TuningResolved &tm, bool anchor, std::vector<PassArgs2> &out, const char *what);


} // namespace cfh

// Opaque handle bodies.
struct cfh_frame_s {
    int n;
    std::vector<cfh::Pauli> zf, xf;  // effZ_q, effX_q
};

namespace cfh {
// Rotations (angles pi/2 or pi) whose product applied to Phi, in order, gives
// U Phi up to a global phase; the frame is not changed.
cfh_status frame_flush_rotations(const cfh_frame_s &f, std::vector<Pauli> &rot, std::vector<double> &theta);
// Gate rows begin.. in circuit order: Clifford rows update the frame, RX/RY/RZ
// rows become rotations about the frame image of their one-qubit Pauli; stops
// at the first measurement or reset row (*stop = its index, else m).
cfh_status circuit_translate(cfh_frame_s &f, const int32_t *gates, const double *angles, size_t begin, size_t m,
                             std::vector<cfh_pauli> &rot, std::vector<double> &theta, size_t *stop);
// Rows back to the identity frame (effZ_q = Z_q, effX_q = X_q).
void frame_reset(cfh_frame_s &f);
} // namespace cfh
