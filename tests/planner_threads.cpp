// Runs the host planners (rotation fusion planning, Hamiltonian pass
// planning, micro-group ordering, register-tile kernel descriptors) on
// several threads at once, as cfh_batch_create and cfh_ham_create do, and
// checks every thread's plans against a run on this thread.  Built with
// ThreadSanitizer by tests/test_planner_threads.py: a data race between the
// planners fails the run.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include "cfh_internal.hpp"

using namespace cfh;

namespace {

struct Input {
    int n;
    std::vector<Pauli> rot, terms;
    std::vector<HamGroup> groups;
};

Input make_input(int n, int m, int mh, unsigned seed)
{
    std::mt19937_64 g(seed);
    Input in;
    in.n = n;
    const uint64_t full = (1ull << n) - 1;
    auto letters = [&](int w) {
        uint64_t x = 0, z = 0;
        for (int k = 0; k < w; ++k) {
            const int q = (int)(g() % (uint64_t)n), l = 1 + (int)(g() % 3);  // X, Y, Z
            if (l == 1 || l == 2) x ^= 1ull << q;
            if (l == 2 || l == 3) z ^= 1ull << q;
        }
        return Pauli{x & full, z & full, 0};  // phase exponent 0: Hermitian
    };
    for (int i = 0; i < m; ++i) in.rot.push_back(letters(2 + (int)(g() % 4)));
    for (int i = 0; i < mh; ++i) in.terms.push_back(letters(1 + (int)(g() % 4)));
    for (int i = 0; i < mh; ++i) {
        bool found = false;
        for (auto &gr : in.groups)
            if (gr.x == in.terms[i].x) {
                gr.terms.push_back(i);
                found = true;
                break;
            }
        if (!found) in.groups.push_back(HamGroup{in.terms[i].x, {i}});
    }
    return in;
}

// A digest of every plan the batch and observable paths make for one input.
uint64_t plan_digest(const Input &in)
{
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t v) { h = (h ^ v) * 1099511628211ull; };
    cfh_tuning t{};
    t.tile_bits = 12;
    const TuningResolved tu = resolve_tuning(&t, in.n, CFH_C128, kTuneForward);
    PassArgs2 a2;
    for (const PassPlan &pp : plan_rotations(in.n, in.rot, tu)) {
        mix(pp.outer_mask);
        for (uint64_t v : pp.v) mix(v);
        for (int k : pp.rots) mix((uint64_t)k);
        if (build_pass_args2(pp, in.rot, false, true, a2)) {
            mix((uint64_t)a2.nmg);
            for (int j = 0; j < a2.nmg; ++j) mix(a2.mg[j].npiv);
        }
    }
    const TuningResolved tm = resolve_tuning(nullptr, in.n, CFH_C128, kTuneMeasure);
    for (const HamPass &hp : plan_hamiltonian(in.n, in.groups, tm, kMaxGroupsPerPass, kMaxRun)) {
        std::vector<int> idx;
        for (int g : hp.groups) idx.insert(idx.end(), in.groups[g].terms.begin(), in.groups[g].terms.end());
        for (int k : order_for_microgroups(hp.v, in.terms, idx, true)) mix((uint64_t)k);
        mix(hp.outer_mask);
    }
    return h;
}

} // namespace

int main()
{
    std::vector<Input> inputs;
    for (unsigned s = 0; s < 6; ++s) inputs.push_back(make_input(14 + (int)s, 300, 120, 1000 + s));
    std::vector<uint64_t> ref(inputs.size());
    for (size_t i = 0; i < inputs.size(); ++i) ref[i] = plan_digest(inputs[i]);
    const int T = 6;
    std::vector<std::vector<uint64_t>> got(T, std::vector<uint64_t>(inputs.size()));
    std::vector<std::thread> pool;
    for (int t = 0; t < T; ++t)
        pool.emplace_back([&, t] {
            // every thread plans every input, starting at a different one
            for (size_t k = 0; k < inputs.size(); ++k) {
                const size_t i = (k + (size_t)t) % inputs.size();
                got[t][i] = plan_digest(inputs[i]);
            }
        });
    for (auto &th : pool) th.join();
    int bad = 0;
    for (int t = 0; t < T; ++t)
        for (size_t i = 0; i < inputs.size(); ++i) bad += got[t][i] != ref[i];
    printf("planner digests: %d of %zu differ\n", bad, (size_t)T * inputs.size());
    return bad ? 1 : 0;
}
