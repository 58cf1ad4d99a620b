// Host-side planning for libcfh: tuning defaults, the fusion planner that
// packs rotations into LDS tile passes, and the grouping of Hamiltonian terms
// into read-only passes.
#include <algorithm>
#include <cstring>
#include <map>
#include <string>
#include <numeric>

#include "cfh_internal.hpp"

namespace cfh {

TuningResolved resolve_tuning(const cfh_tuning *t, int n, int dtype, int kind)
{
    TuningResolved r;
    const bool c64 = dtype == CFH_C64;
    // Defaults measured on MI355X at 28 qubits: the register-tiled kernel with
    // 128-byte contiguous chunks (8 complex128 / 16 complex64 amplitudes),
    // which leaves the most free dimensions per pass at full cache-line use;
    // complex128 on 2^14-amplitude tiles (half-tile transposes), complex64 on
    // 2^13.  Small states keep at least 128 tiles per pass: their passes are
    // short and latency-bound, so fewer, larger passes win until the grid gets
    // too small (measured at 18-24 qubits).  The adjoint holds two tiles in LDS and uses 2^11 (c128) / 2^12
    // (c64).  The LDS-staged Hamiltonian passes use 2^12 / 2^13 tiles with
    // 32-amplitude chunks.
    int b = c64 ? 13 : 14;
    if (kind == kTuneAdjoint) b = c64 ? 12 : 11;
    if (kind == kTuneHamiltonian) b = c64 ? 13 : 12;
    if (kind == kTuneAdjoint2) b = 13;
    // read-only <H> passes (and the H psi passes, whose tile follows): 2^11
    // tiles at complex128, 2^12 at complex64.  Smaller tiles hold fewer terms
    // per pass but need fewer micro-group transposes per term, and more
    // workgroups fit a CU, down to 2^11.  Measured on the 28-qubit,
    // 2,000-term observable, complex128: <H> 2^10 135 ms, 2^11 99.6 ms, 2^12
    // 103 ms, 2^13 110 ms, 2^14 132 ms; H psi 351 / 309 / 324 / 333 ms at
    // 2^10..2^13; complex64 <H> 83.0 / 82.2 / 85.5 ms at 2^11..2^13, H psi
    // 265 / 332 ms at 2^12 / 2^13.
    if (kind == kTuneMeasure) b = c64 ? 12 : 11;
    // the adjoint holds two vectors per workgroup (fewer workgroups per CU),
    // so it keeps at least 256 tiles
    b = std::max(std::min(b, n - (kind == kTuneAdjoint2 ? 8 : 7)), std::min(n, 10));
    r.tile_bits = (t && t->tile_bits > 0) ? t->tile_bits : b;
    const int c_def = kind == kTuneHamiltonian ? 5
                      : ((kind == kTuneForward || kind == kTuneMeasure || kind == kTuneAdjoint2) && !c64) ? 3
                                                                                                          : 4;
    r.low_bits = (t && t->low_bits > 0) ? t->low_bits : c_def;
    r.max_run = (t && t->max_run > 0) ? t->max_run : kMaxRun;
    r.lookahead = (t && t->lookahead != 0) ? t->lookahead : 512;
    r.unfused = (t && t->unfused) ? 1 : 0;
    r.block_threads = (t && t->block_threads > 0) ? t->block_threads : 256;
    r.variant = t ? t->variant : 0;
    r.tile_order = t ? t->tile_order : 0;
    r.max_run = std::min(r.max_run, kMaxRun);
    r.tile_bits = std::min(r.tile_bits, std::min(n, kMaxTileBits));
    r.low_bits = std::min(r.low_bits, r.tile_bits);
    // keep one free dimension so every pass can take at least one rotation/group
    if (r.tile_bits < n) r.low_bits = std::min(r.low_bits, r.tile_bits - 1);
    return r;
}

namespace {

// Subspace of GF(2)^64 in reduced echelon form (each vector owns a pivot bit
// that no other vector has set).
struct Span {
    std::vector<uint64_t> v;
    std::vector<int> piv;
    uint64_t pivmask = 0;

    uint64_t reduce(uint64_t x) const
    {
        for (size_t i = 0; i < v.size(); ++i)
            if ((x >> piv[i]) & 1) x ^= v[i];
        return x;
    }
    void add(uint64_t r)  // r must be reduced and nonzero
    {
        const int p = 63 - __builtin_clzll(r);
        for (auto &w : v)
            if ((w >> p) & 1) w ^= r;
        v.push_back(r);
        piv.push_back(p);
        pivmask |= 1ull << p;
    }
    int dim() const { return (int)v.size(); }
};

uint64_t full_mask(int n) { return n >= 64 ? ~0ull : ((1ull << n) - 1); }

// Complete to dimension b with unit vectors of the lowest free bits and order
// the basis so that unit vectors come first by bit position: then the low
// local index bits address contiguous amplitudes.
void finish_basis(Span &s, int n, int b, std::vector<uint64_t> &v_out, uint64_t &outer)
{
    for (int j = 0; j < n && s.dim() < b; ++j) {
        const uint64_t e = 1ull << j;
        const uint64_t r = s.reduce(e);
        if (r) s.add(r);
    }
    std::vector<int> idx(s.dim());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int c) {
        const bool ua = __builtin_popcountll(s.v[a]) == 1, uc = __builtin_popcountll(s.v[c]) == 1;
        if (ua != uc) return ua;
        return s.piv[a] < s.piv[c];
    });
    v_out.clear();
    for (int i : idx) v_out.push_back(s.v[i]);
    outer = full_mask(n) & ~s.pivmask;
}

} // namespace

uint32_t local_coords(const std::vector<uint64_t> &v, uint64_t x, bool *in_span)
{
    // In reduced echelon form bit i of the local coordinates is the pivot bit
    // of v[i] in x; the pivot of v[i] is its highest bit not shared with any
    // other basis vector.  Recompute pivots from the vectors themselves.
    uint32_t xl = 0;
    uint64_t acc = 0;
    uint64_t others_or = 0;
    (void)others_or;
    for (size_t i = 0; i < v.size(); ++i) {
        uint64_t own = v[i];
        for (size_t j = 0; j < v.size(); ++j)
            if (j != i) own &= ~v[j];
        const int p = 63 - __builtin_clzll(own);
        if ((x >> p) & 1) {
            xl |= 1u << i;
            acc ^= v[i];
        }
    }
    if (in_span) *in_span = (acc == x);
    return xl;
}

uint32_t local_zmask(const std::vector<uint64_t> &v, uint64_t z)
{
    uint32_t zl = 0;
    for (size_t i = 0; i < v.size(); ++i)
        if (popc(v[i] & z) & 1) zl |= 1u << i;
    return zl;
}

RotDesc make_rot_desc(const PassPlan &pp, const Pauli &p, int k)
{
    RotDesc d{};
    bool ok = true;
    d.xl = local_coords(pp.v, p.x, &ok);
    d.zl = local_zmask(pp.v, p.z);
    d.z = p.z;
    d.hb = d.xl ? 31 - __builtin_clz(d.xl) : -1;
    d.k = k;
    d.w = (p.e - popc(p.x & p.z) + 3) & 3;
    d.dsign = popc(p.x & p.z) & 1;
    return d;
}

int line_share_bits(uint64_t outer_mask, int n, int b, int amp_bytes, int tile_order)
{
    if (tile_order == 1) return 0;   // index order
    if (tile_order == 2) return -1;  // bit-reversed order
    const int line_amps = 128 / amp_bytes;
    const int p = popc(outer_mask & (uint64_t)(line_amps - 1));
    // the cosets of a line group and the 8 XCDs must tile the coset range;
    // otherwise bit-reversed (measured 1.3% faster per complex128 pass at
    // 28 qubits than index order, equal at complex64)
    if (p == 0 || n - b < 3 + p) return -1;
    return p;
}

std::vector<PassPlan> plan_rotations(int n, const std::vector<Pauli> &rot, const TuningResolved &tu)
{
    const int m = (int)rot.size();
    const int b = tu.tile_bits, c = tu.low_bits;
    std::vector<PassPlan> out;
    std::vector<char> taken(m, 0);
    std::vector<int> skipped;
    int first = 0;
    while (first < m) {
        Span s;
        for (int j = 0; j < c; ++j) s.add(1ull << j);
        PassPlan pp;
        skipped.clear();
        int scanned = 0;
        for (int j = first; j < m && (int)pp.rots.size() < tu.max_run; ++j) {
            if (taken[j]) continue;
            if (tu.lookahead >= 0 && scanned > tu.lookahead) break;
            ++scanned;
            const uint64_t r = s.reduce(rot[j].x);
            bool ok = (r == 0) || s.dim() < b;
            if (ok) {
                // may move ahead of the skipped rotations only if it commutes with all of them
                for (int q : skipped)
                    if (anticommute(rot[q].x, rot[q].z, rot[j].x, rot[j].z)) { ok = false; break; }
            }
            if (ok) {
                if (r) s.add(r);
                pp.rots.push_back(j);
                taken[j] = 1;
            } else {
                skipped.push_back(j);
                if (tu.lookahead < 0) break;
            }
        }
        finish_basis(s, n, b, pp.v, pp.outer_mask);
        pp.b = b;
        out.push_back(std::move(pp));
        while (first < m && taken[first]) ++first;
    }
    return out;
}

bool build_pass_args2(const PassPlan &pp, const std::vector<Pauli> &rot, bool inverse, bool anchor, PassArgs2 &a)
{
    std::memset(&a, 0, sizeof(a));
    const int b = pp.b;
    if (b < kRegDims || b > kMaxTileBits) return false;
    a.outer_mask = pp.outer_mask;
    for (int j = 0; j < b; ++j) a.v[j] = pp.v[j];
    a.b = b;
    a.inverse = inverse ? 1 : 0;
    std::vector<int> order = pp.rots;
    if (inverse) std::reverse(order.begin(), order.end());
    const int D = (int)order.size();
    std::vector<uint32_t> xl(D), zl(D);
    for (int i = 0; i < D; ++i) {
        bool ok = false;
        xl[i] = local_coords(pp.v, rot[order[i]].x, &ok);
        if (!ok) return false;
        zl[i] = local_zmask(pp.v, rot[order[i]].z);
    }
    // split into micro-groups of at most kRegDims local dimensions; with an
    // anchor every group starts from the same vector, which keeps its pivot
    // (the anchor bit) and stays register dimension 0 throughout the pass
    uint64_t anc = 0;
    if (anchor)
        for (int i = 0; i < D && !anc; ++i) anc = xl[i];
    std::vector<Span> spans;
    std::vector<std::vector<int>> members;
    auto open_group = [&]() {
        spans.emplace_back();
        members.emplace_back();
        if (anc) spans.back().add(anc);
    };
    for (int i = 0; i < D; ++i) {
        if (spans.empty()) open_group();
        uint64_t r = spans.back().reduce(xl[i]);
        if (r && spans.back().dim() == kRegDims) {
            open_group();
            r = spans.back().reduce(xl[i]);
        }
        if (r) spans.back().add(r);
        members.back().push_back(i);
    }
    if (spans.empty()) open_group();
    if ((int)spans.size() > kMaxMG) return false;
    a.qbit = anc ? 63 - __builtin_clzll(anc) : -1;
    auto compress = [&](uint32_t u) {
        if (a.qbit < 0) return u;
        const uint32_t lo = (1u << a.qbit) - 1;
        return (u & lo) | ((u >> (a.qbit + 1)) << a.qbit);
    };
    const uint32_t full = (uint32_t)((1ull << b) - 1);
    int ri = 0;
    for (size_t g = 0; g < spans.size(); ++g) {
        Span &s = spans[g];
        // pad with the highest free local unit vectors: pivots stay above the lane bits
        for (int bit = b - 1; bit >= 0 && s.dim() < kRegDims; --bit) {
            const uint64_t e = s.reduce(1ull << bit);
            if (e) s.add(e);
        }
        if (s.dim() != kRegDims) return false;
        MGDesc2 &m = a.mg[g];
        m.npiv = full & ~(uint32_t)s.pivmask;
        for (int j = 0; j < kRegs; ++j) {
            uint64_t u = 0;
            for (int i = 0; i < kRegDims; ++i)
                if ((j >> i) & 1) u ^= s.v[i];
            m.U[j] = (uint32_t)u;
            m.UC[j] = compress(m.U[j]);
        }
        m.rot_begin = ri;
        m.rot_count = (int)members[g].size();
        for (int i : members[g]) {
            const Pauli &p = rot[order[i]];
            RotDesc2 &d = a.rot[ri++];
            uint32_t cx = 0;
            uint64_t chk = 0;
            for (int q = 0; q < kRegDims; ++q)
                if ((xl[i] >> s.piv[q]) & 1) {
                    cx |= 1u << q;
                    chk ^= s.v[q];
                }
            if (chk != xl[i]) return false;
            d.cx = (uint8_t)cx;
            d.zl = zl[i];
            uint32_t ms = 0;
            for (int j = 0; j < kRegs; ++j)
                if (popc(m.U[j] & zl[i]) & 1) ms |= 1u << j;
            d.msign = (uint16_t)ms;
            const int w = (p.e - popc(p.x & p.z) + 3) & 3;
            // bit 2: sign of i^{(e-|x&z|)}, the phase of P psi (adjoint gradient)
            const int wp = (p.e - popc(p.x & p.z)) & 3;
            d.flags = (uint8_t)((w & 1) | ((w & 2) ? 2 : 0) | ((wp & 2) ? 4 : 0));
            // register signs are linear in j (U is spanned by the four u_q), so
            // they are fixed by a 4-bit mask; the thread part by a mask on t
            uint32_t zr = 0;
            for (int q = 0; q < kRegDims; ++q)
                if (popc(s.v[q] & zl[i]) & 1) zr |= 1u << q;
            d.kase = cx | (zr << 4) | ((uint32_t)(w & 1) << 8);
            // the compile-time bodies take the imaginary coefficient from
            // (cx, zr): for a Hermitian string it is set exactly when
            // parity(cx & zr) = |x & z| mod 2 is even
            if ((w & 1) != ((cx == 0 || !(popc(cx & zr) & 1)) ? 1 : 0)) return false;
            uint32_t zt = 0;
            int tb = 0;
            for (int bit = 0; bit < b; ++bit)
                if ((m.npiv >> bit) & 1) {
                    if ((zl[i] >> bit) & 1) zt |= 1u << tb;
                    ++tb;
                }
            d.zt = zt;
            d.z = p.z;
            d.k = order[i];
        }
    }
    a.nmg = (int)spans.size();
    auto Lmap = [&](uint32_t loc) {
        uint64_t y = 0;
        for (int i = 0; i < b; ++i)
            if ((loc >> i) & 1) y ^= pp.v[i];
        return y;
    };
    for (int j = 0; j < kRegs; ++j) {
        a.LU_first[j] = Lmap(a.mg[0].U[j]);
        a.LU_last[j] = Lmap(a.mg[a.nmg - 1].U[j]);
    }
    return true;
}

std::vector<HamPass> plan_hamiltonian(int n, const std::vector<HamGroup> &groups, const TuningResolved &tu,
                                      int max_groups, int max_terms)
{
    const int b = tu.tile_bits, c = tu.low_bits;
    const int G = (int)groups.size();
    std::vector<char> done(G, 0);
    // groups not yet placed, ascending: the scans below visit only these
    std::vector<int> rem(G);
    std::iota(rem.begin(), rem.end(), 0);
    // red[g]: groups[g].x reduced against the current span (zero at every
    // pivot; unique), kept up to date as vectors join the span
    std::vector<uint64_t> red(G);
    // open-addressing table: reduced mask -> number of candidate groups with
    // that mask; only the slots used in a step are cleared after it
    int lg = 4;
    while ((1ll << lg) < 2ll * G) ++lg;
    const size_t cap = (size_t)1 << lg;
    std::vector<uint64_t> hkey(cap, 0);
    std::vector<int32_t> hcnt(cap, 0);
    std::vector<size_t> hused;
    auto slot = [&](uint64_t r) {
        size_t i = (size_t)((r * 0x9E3779B97F4A7C15ull) >> (64 - lg));
        while (hkey[i] != 0 && hkey[i] != r) i = (i + 1) & (cap - 1);
        return i;
    };
    std::vector<HamPass> out;
    while (!rem.empty()) {
        int nterms = 0;
        // Grow a b-dimensional subspace greedily: each step adds one reduced
        // x mask as one new dimension, and every group whose x then lies in
        // the span joins for free.  (Covering a group by whole qubits, one unit
        // vector per new qubit, spends more dimensions per group; it packed
        // fewer groups per pass both for JW strings and for the dense masks
        // that a Clifford prefix leaves.)  Every group fits some pass, since a
        // single x adds at most one dimension.
        Span s;
        for (int j = 0; j < c; ++j) s.add(1ull << j);
        for (const int g : rem) red[g] = s.reduce(groups[g].x);
        // e: reduced and nonzero; the basis stays reduced, and so does every
        // red[g].  Groups whose red[g] becomes zero are collected in rem order.
        std::vector<int> newly;
        auto add = [&](uint64_t e) {
            const int p = 63 - __builtin_clzll(e);
            s.add(e);
            for (const int g : rem)
                if ((red[g] >> p) & 1) {
                    red[g] ^= e;
                    if (!red[g]) newly.push_back(g);
                }
        };
        std::vector<int> chosen;
        std::vector<char> in(G, 0);
        auto fits = [&](int g) { return nterms + (int)groups[g].terms.size() <= max_terms; };
        auto take = [&](int g) {
            if ((int)chosen.size() < max_groups && !in[g] && fits(g) && red[g] == 0) {
                in[g] = 1;
                chosen.push_back(g);
                nterms += (int)groups[g].terms.size();
            }
        };
        // the groups inside the span, ascending; later sweeps need only the
        // groups that entered it since, because a group that did not fit
        // never fits again (nterms only grows)
        for (const int g : rem) take(g);
        auto sweep = [&]() {
            std::sort(newly.begin(), newly.end());
            for (const int g : newly) take(g);
            newly.clear();
        };
        while ((int)chosen.size() < max_groups && nterms < max_terms && s.dim() < b) {
            // The reduced mask shared by the most candidate groups (those not
            // taken that still fit): adding it brings all of them into the
            // span at the cost of one dimension.  Ties go to the mask with the
            // fewest set bits, then to the first group in rem order.  (A
            // candidate that reduces to zero was taken by the sweep.)
            for (const int g : rem) {
                if (in[g] || !fits(g) || !red[g]) continue;
                const size_t i = slot(red[g]);
                if (!hkey[i]) {
                    hkey[i] = red[g];
                    hused.push_back(i);
                }
                ++hcnt[i];
            }
            int best = -1, best_n = 0, best_cost = 1 << 30;
            uint64_t best_r = 0;
            for (const int g : rem) {
                if (in[g] || !fits(g) || !red[g]) continue;
                const int nn = hcnt[slot(red[g])], cost = popc(red[g]);
                if (nn > best_n || (nn == best_n && cost < best_cost)) {
                    best_n = nn;
                    best_cost = cost;
                    best = g;
                    best_r = red[g];
                }
            }
            for (const size_t i : hused) {
                hkey[i] = 0;
                hcnt[i] = 0;
            }
            hused.clear();
            if (best < 0) break;
            add(best_r);
            sweep();
        }
        if (chosen.empty()) {
            // every remaining group is larger than max_terms on its own (the
            // caller splits such groups); take one so the loop always ends
            const int g = rem.front();
            if (red[g]) add(red[g]);
            chosen.push_back(g);
        }
        HamPass hp;
        hp.b = b;
        finish_basis(s, n, b, hp.v, hp.outer_mask);
        for (int g : chosen) done[g] = 1;
        rem.erase(std::remove_if(rem.begin(), rem.end(), [&](int g) { return done[g] != 0; }), rem.end());
        hp.groups = std::move(chosen);
        out.push_back(std::move(hp));
    }
    return out;
}

namespace {

// Term order inside one pass for a given anchor (0 = none): every term whose
// local x lies in the current micro-group span is taken at once; otherwise the
// span grows by the dimension that brings the most remaining terms into it;
// a full span (kRegDims dimensions) starts over from the anchor.  Returns
// positions into xl.
std::vector<int> microgroup_order(const std::vector<uint64_t> &xl, uint64_t anc)
{
    const int m = (int)xl.size();
    std::vector<char> used(m, 0);
    std::vector<uint64_t> red(m);
    std::vector<int> out;
    out.reserve(m);
    Span s;
    if (anc) s.add(anc);
    int left = m;
    while (left > 0) {
        for (int i = 0; i < m; ++i)
            if (!used[i] && (red[i] = s.reduce(xl[i])) == 0) {
                used[i] = 1;
                out.push_back(i);
                --left;
            }
        if (!left) break;
        if (s.dim() >= kRegDims) {
            s = Span();
            if (anc) s.add(anc);
            continue;
        }
        // adding an unused term's reduced x r brings into the span exactly the
        // unused terms whose reduced x is r (x is in span(s, r) iff its
        // reduction against s is 0 or r, and 0 was taken above)
        int best = -1, best_cov = -1;
        for (int i = 0; i < m; ++i) {
            if (used[i]) continue;
            int cov = 0;
            for (int j = 0; j < m; ++j) cov += !used[j] && red[j] == red[i];
            if (cov > best_cov) {
                best_cov = cov;
                best = i;
            }
        }
        s.add(red[best]);
    }
    return out;
}

// The micro-groups build_pass_args2 cuts from terms in this order: spans of
// at most kRegDims dimensions, each seeded with the anchor.
int count_microgroups(const std::vector<uint64_t> &xl, const std::vector<int> &order, uint64_t anc)
{
    int groups = 1;
    Span s;
    if (anc) s.add(anc);
    for (const int i : order) {
        uint64_t r = s.reduce(xl[i]);
        if (r && s.dim() == kRegDims) {
            ++groups;
            s = Span();
            if (anc) s.add(anc);
            r = s.reduce(xl[i]);
        }
        if (r) s.add(r);
    }
    return groups;
}

} // namespace

std::vector<int> order_for_microgroups(const std::vector<uint64_t> &basis, const std::vector<Pauli> &p,
                                      const std::vector<int> &idx, bool anchor)
{
    const int m = (int)idx.size();
    std::vector<uint64_t> xl(m);
    for (int i = 0; i < m; ++i) {
        bool ok = false;
        xl[i] = local_coords(basis, p[idx[i]].x, &ok);
    }
    std::vector<int> best;
    if (!anchor) {
        best = microgroup_order(xl, 0);
    } else {
        // The anchor is register dimension 0 of every micro-group, so it
        // decides how many micro-groups (and LDS transposes) the pass needs:
        // try each distinct local x as the anchor and keep the order with the
        // fewest micro-groups (the first candidate on ties).  The chosen
        // anchor's term comes first among the nonzero ones, as the
        // descriptor builder expects.
        int best_n = 1 << 30;
        std::vector<uint64_t> tried;
        for (int c = 0; c < m; ++c) {
            const uint64_t a = xl[c];
            if (!a || std::find(tried.begin(), tried.end(), a) != tried.end()) continue;
            tried.push_back(a);
            std::vector<int> o = microgroup_order(xl, a);
            const int n_mg = count_microgroups(xl, o, a);
            if (n_mg < best_n) {
                best_n = n_mg;
                best = std::move(o);
            }
        }
        if (best.empty()) best = microgroup_order(xl, 0);  // only diagonal terms
    }
    std::vector<int> out(best.size());
    for (size_t i = 0; i < best.size(); ++i) out[i] = idx[best[i]];
    return out;
}

void batch_ticket_order(const std::vector<std::vector<int>> &chains, const std::vector<int> &pass_items,
                        const std::vector<double> &circ_amps, const std::vector<std::pair<int, int>> &groups,
                        std::vector<std::pair<int, int>> &tickets, std::vector<int> &prev)
{
    tickets.clear();
    prev.assign(pass_items.size(), -1);
    for (const auto &cg : groups) {
        size_t maxlen = 0;
        for (int c = cg.first; c < cg.second; ++c) maxlen = std::max(maxlen, chains[c].size());
        std::vector<int> at;
        for (size_t lv = 0; lv < maxlen; ++lv) {
            at.clear();
            for (int c = cg.first; c < cg.second; ++c)
                if (lv < chains[c].size()) at.push_back(c);
            // the circuits with the most work left in their chains first
            std::stable_sort(at.begin(), at.end(), [&](int a, int b) {
                return circ_amps[a] * (double)(chains[a].size() - lv) > circ_amps[b] * (double)(chains[b].size() - lv);
            });
            for (int c : at) {
                const int p = chains[c][lv];
                prev[p] = lv ? chains[c][lv - 1] : -1;
                for (int i = 0; i < pass_items[p]; ++i) tickets.push_back({p, i});
            }
        }
    }
}

// The x-groups of an observable's terms, in first-appearance order.
std::vector<HamGroup> group_terms(const cfh_pauli *terms, size_t m)
{
    std::map<uint64_t, int> gid;
    std::vector<HamGroup> groups;
    for (size_t i = 0; i < m; ++i) {
        auto it = gid.find(terms[i].x);
        if (it == gid.end()) {
            gid[terms[i].x] = (int)groups.size();
            groups.push_back(HamGroup{terms[i].x, {(int)i}});
        } else {
            groups[it->second].terms.push_back((int)i);
        }
    }
    return groups;
}

MeasureSettings measure_settings(const cfh_tuning *tuning, int n, int dtype, size_t m)
{
    MeasureSettings ms;
    ms.tm = resolve_tuning(tuning, n, dtype, kTuneMeasure);
    ms.reg = ms.tm.variant != 1 && ms.tm.tile_bits >= 10 && ms.tm.tile_bits <= 14 && m > 0;
    ms.anchor = ms.tm.tile_bits == 14 || ms.tm.variant == 5 || (ms.tm.variant == 0 && dtype == CFH_C128);
    return ms;
}

// Register-tiled passes over the terms of an observable: the x-groups (split
// to at most kMaxRun terms) planned onto tiles, each pass's terms ordered so
// consecutive ones share register micro-groups (anchored for half-tile
// transposes), runs that need more micro-groups split in two.
cfh_status term_passes(int n, int dtype, const std::vector<HamGroup> &groups, const std::vector<Pauli> &tp,
                       const TuningResolved &tm, bool anchor, std::vector<PassArgs2> &out, const char *what)
{
    std::vector<HamGroup> mg;
    for (const HamGroup &g : groups)
        for (size_t i = 0; i < g.terms.size(); i += kMaxRun)
            mg.push_back(HamGroup{g.x, std::vector<int>(g.terms.begin() + (std::ptrdiff_t)i,
                                                        g.terms.begin() +
                                                            (std::ptrdiff_t)std::min(g.terms.size(), i + kMaxRun))});
    std::vector<PassPlan> todo;
    for (const HamPass &hp : plan_hamiltonian(n, mg, tm, kMaxGroupsPerPass, kMaxRun)) {
        std::vector<int> idx;
        for (int g : hp.groups) idx.insert(idx.end(), mg[g].terms.begin(), mg[g].terms.end());
        PassPlan pp;
        pp.b = hp.b;
        pp.outer_mask = hp.outer_mask;
        pp.v = hp.v;
        pp.rots = order_for_microgroups(hp.v, tp, idx, anchor);
        todo.push_back(std::move(pp));
    }
    std::reverse(todo.begin(), todo.end());
    PassArgs2 a2;
    while (!todo.empty()) {
        PassPlan pp = std::move(todo.back());
        todo.pop_back();
        if (build_pass_args2(pp, tp, false, anchor, a2)) {
            a2.xrot = line_share_bits(a2.outer_mask, n, a2.b, dtype == CFH_C64 ? 8 : 16, tm.tile_order);
            out.push_back(a2);
            continue;
        }
        if (pp.rots.size() < 2) return set_error(CFH_E_INVAL, std::string(what) + ": a term does not fit the tile");
        PassPlan hi = pp;
        const size_t half = pp.rots.size() / 2;
        hi.rots.assign(pp.rots.begin() + (std::ptrdiff_t)half, pp.rots.end());
        pp.rots.resize(half);
        todo.push_back(std::move(hi));
        todo.push_back(std::move(pp));
    }
    return CFH_OK;
}

} // namespace cfh

using namespace cfh;

extern "C" cfh_status cfh_batch_order(int count, const int32_t *chain_len, const int32_t *pass_items,
                                      const double *circ_amps, int32_t *ticket_pass, int32_t *ticket_item,
                                      int32_t *prev)
{
    if (count < 0 || (count && (!chain_len || !circ_amps)))
        return set_error(CFH_E_INVAL, "cfh_batch_order: null argument");
    std::vector<std::vector<int>> chains(count);
    int np = 0;
    for (int c = 0; c < count; ++c) {
        if (chain_len[c] < 0) return set_error(CFH_E_INVAL, "cfh_batch_order: negative chain length");
        for (int i = 0; i < chain_len[c]; ++i) chains[c].push_back(np++);
    }
    if (np && (!pass_items || !prev)) return set_error(CFH_E_INVAL, "cfh_batch_order: null argument");
    std::vector<int> items(pass_items, pass_items + np);
    int64_t nt = 0;
    for (int p = 0; p < np; ++p) {
        if (items[p] < 1) return set_error(CFH_E_INVAL, "cfh_batch_order: a pass without work items");
        nt += items[p];
    }
    if (nt && (!ticket_pass || !ticket_item)) return set_error(CFH_E_INVAL, "cfh_batch_order: null argument");
    std::vector<std::pair<int, int>> tickets;
    std::vector<int> pv;
    batch_ticket_order(chains, items, std::vector<double>(circ_amps, circ_amps + count), {{0, count}}, tickets, pv);
    for (size_t k = 0; k < tickets.size(); ++k) {
        ticket_pass[k] = tickets[k].first;
        ticket_item[k] = tickets[k].second;
    }
    for (int p = 0; p < np; ++p) prev[p] = pv[p];
    return CFH_OK;
}

extern "C" cfh_status cfh_plan_dry_run(int n, int dtype, const cfh_pauli *rot, size_t m, const cfh_tuning *tuning,
                                       int64_t *n_passes, int64_t *pass_start, int64_t *order)
{
    if (!n_passes || !pass_start || (m && (!rot || !order)))
        return set_error(CFH_E_INVAL, "cfh_plan_dry_run: null argument");
    if (n < 1 || n > kMaxStateQubits) return set_error(CFH_E_UNSUPPORTED, "cfh_plan_dry_run: n must be in 1..34");
    if (dtype != CFH_C64 && dtype != CFH_C128) return set_error(CFH_E_UNSUPPORTED, "cfh_plan_dry_run: dtype");
    std::vector<Pauli> r(m);
    for (size_t i = 0; i < m; ++i) {
        cfh_status st = check_pauli(rot[i], n, true, "cfh_plan_dry_run");
        if (st) return st;
        r[i] = Pauli{rot[i].x, rot[i].z, rot[i].e & 3};
    }
    const TuningResolved tu = resolve_tuning(tuning, n, dtype, kTuneForward);
    int64_t o = 0;
    if (tu.unfused) {
        for (size_t i = 0; i < m; ++i) {
            pass_start[i] = (int64_t)i;
            order[i] = (int64_t)i;
        }
        pass_start[m] = (int64_t)m;
        *n_passes = (int64_t)m;
        return CFH_OK;
    }
    const std::vector<PassPlan> passes = plan_rotations(n, r, tu);
    for (size_t i = 0; i < passes.size(); ++i) {
        pass_start[i] = o;
        for (int k : passes[i].rots) order[o++] = k;
    }
    pass_start[passes.size()] = o;
    *n_passes = (int64_t)passes.size();
    return CFH_OK;
}

extern "C" cfh_status cfh_ham_dry_run(int n, int dtype, const cfh_pauli *terms, size_t m, const cfh_tuning *tuning,
                           int64_t *n_passes, int64_t *pass_start, int64_t *order, int32_t *pass_bits,
                           uint64_t *basis)
{
    if (!n_passes || !pass_start || (m && (!terms || !order || !pass_bits || !basis)))
        return set_error(CFH_E_INVAL, "cfh_ham_dry_run: null argument");
    if (n < 1 || n > kMaxStateQubits) return set_error(CFH_E_UNSUPPORTED, "cfh_ham_dry_run: n must be in 1..34");
    if (dtype != CFH_C64 && dtype != CFH_C128) return set_error(CFH_E_UNSUPPORTED, "cfh_ham_dry_run: dtype");
    for (size_t i = 0; i < m; ++i) {
        cfh_status st = check_pauli(terms[i], n, true, "cfh_ham_dry_run");
        if (st) return st;
    }
    const MeasureSettings ms = measure_settings(tuning, n, dtype, m);
    if (m && !ms.reg)
        return set_error(CFH_E_UNSUPPORTED, "cfh_ham_dry_run: <H> does not run on register tiles under this tuning");
    std::vector<PassArgs2> margs;
    if (m) {
        std::vector<Pauli> tp(m);
        for (size_t i = 0; i < m; ++i) tp[i] = Pauli{terms[i].x, terms[i].z, terms[i].e & 3};
        cfh_status st = term_passes(n, dtype, group_terms(terms, m), tp, ms.tm, ms.anchor, margs, "cfh_ham_dry_run");
        if (st) return st;
    }
    // every pass holds at least one term and every term one place, so the
    // caller's m-entry arrays suffice; checked before each write
    int64_t o = 0;
    pass_start[0] = 0;
    for (size_t p = 0; p < margs.size(); ++p) {
        const PassArgs2 &a = margs[p];
        const int nt = a.nmg > 0 ? a.mg[a.nmg - 1].rot_begin + a.mg[a.nmg - 1].rot_count : 0;
        if (p >= m || o + nt > (int64_t)m)
            return set_error(CFH_E_INVAL, "cfh_ham_dry_run: the plan places more terms than given");
        for (int j = 0; j < nt; ++j) order[o++] = a.rot[j].k;
        pass_start[p + 1] = o;
        pass_bits[p] = a.b;
        for (int i = 0; i < kMaxTileBits; ++i) basis[p * kMaxTileBits + i] = i < a.b ? a.v[i] : 0;
    }
    *n_passes = (int64_t)margs.size();
    return CFH_OK;
}
