// Batched hybrid simulation: many independent circuits (own qubit count,
// rotations, angles and observable) run together.
//
// Every circuit is a chain of passes: its fused rotation passes (the first
// one builds the initial basis state on the fly), then the read-only
// Hamiltonian passes that accumulate lam = H psi (the last one also reduces
// E = Re <psi|lam>, Eq. chfsexp), then, for gradients, its rotation passes
// walked backwards with the adjoint rule g_k = Im <lam|P_k|psi> while both
// vectors are rewound.  Passes are cut into work items of a few cosets.
//
// Execution is level-synchronous: level l holds pass l of every circuit whose
// chain is that long, one workgroup per work item, launched as one kernel;
// a second small kernel then reduces the per-item partial sums of the level's
// adjoint and energy passes in a fixed order (bitwise reproducible results).
// Kernel boundaries order the levels, so no workgroup ever waits for another.
// The whole sequence is enqueued by cfh_batch_run and captured once into a
// hipGraph by cfh_batch_graph_launch.
//
// Tuning variant 1 runs the same work items, in one persistent kernel per run
// instead of one launch per level and kind: resident workgroups claim items in
// a dependency-respecting order and wait, with bounded waits, only for the
// pass before an item in its own circuit (k_batch_persist).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "batch.hpp"
#include "cfh_internal.hpp"
#include "device_common.hpp"

using namespace cfh;
using namespace cfh::dev;

namespace {

// One work item: a range of cosets of one pass.
template <typename Amp, int BMAX>
__global__ void __launch_bounds__(kBThreads) k_batch_level(const BatchArgs A, const BItem *__restrict__ items)
{
    constexpr int T = kBThreads;
    constexpr int NMAX = 1 << BMAX;
    __shared__ Amp tp[NMAX];
    __shared__ Amp tl[NMAX];
    __shared__ double wacc[kMaxRun][kBWaves];
    __shared__ double ered[kBWaves];
    const int t = threadIdx.x;
    const BItem it = items[blockIdx.x];
    const BPass &P = A.passes[it.pass];
    const BCirc &C = A.circs[P.circ];
    Amp *psi = reinterpret_cast<Amp *>(A.psi) + C.psi_off;
    Amp *lam = reinterpret_cast<Amp *>(A.lam) + C.psi_off;
    const int b = P.b;
    const int N = 1 << b;
    const uint64_t ntiles = 1ull << (C.n - b);
    const uint64_t tile0 = (uint64_t)it.idx * P.tiles_per_item;
    const uint64_t tile1 = std::min<uint64_t>(ntiles, tile0 + P.tiles_per_item);
    if ((P.flags & kFlagStart) && it.idx == 0 && t == 0) A.t_start[P.circ] = wall_clock64();
    for (int i = t; i < kMaxRun * kBWaves; i += T) (&wacc[0][0])[i] = 0.0;
    double eacc = 0.0;
    __syncthreads();

    // local element a = t + k*T maps to base ^ Lt ^ Lk[k]: the thread part
    // (bits below log2 T) and the register part are disjoint, so their images
    // under the basis combine by XOR
    constexpr int LT = 8;
    static_assert(T == 1 << LT, "work items use 256 threads");
    constexpr int KMAX = NMAX > T ? NMAX / T : 1;
    uint64_t Lt = 0;
    for (int i = 0; i < LT && i < b; ++i)
        if ((t >> i) & 1) Lt ^= P.v[i];
    uint64_t Lk[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
        uint64_t y = 0;
        for (int i = LT; i < b; ++i)
            if ((k >> (i - LT)) & 1) y ^= P.v[i];
        Lk[k] = y;
    }
    for (uint64_t tile = tile0; tile < tile1; ++tile) {
        const uint64_t base = deposit(tile, P.outer_mask);
        // global index of this thread's k-th element a = t + k*T
        auto gk = [&](int k) { return base ^ Lt ^ Lk[k]; };
        if (P.type == kPassFwd) {
            #pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                const int a = t + k * T;
                if (a >= N) break;
                const uint64_t y = gk(k);
                if (P.flags & kFlagInit) st(tp[a], make_double2(y == C.init ? 1.0 : 0.0, 0.0));
                else tp[a] = psi[y];
            }
            __syncthreads();
            for (int ri = 0; ri < P.count; ++ri) {
                const RotDesc &d = A.rot[P.first + ri];
                const double2 cs = A.coef[C.theta_off + d.k];
                const double c = cs.x;
                const double sr = (d.w & 2) ? -cs.y : cs.y;
                const bool imag = d.w & 1;
                const int so = par64(base & d.z);
                if (d.xl == 0) {
                    for (int a = t; a < N; a += T) {
                        const double sj = (par32(a & d.zl) ^ so) ? -sr : sr;
                        st(tp[a], rot_diag(ld(tp[a]), c, sj, imag));
                    }
                } else {
                    const uint32_t lowm = (1u << d.hb) - 1;
                    for (uint32_t q = t; q < (uint32_t)(N >> 1); q += T) {
                        const uint32_t a0 = ((q & ~lowm) << 1) | (q & lowm);
                        const uint32_t a1 = a0 ^ d.xl;
                        const int sg0 = par32(a0 & d.zl) ^ so;
                        const double s0 = sg0 ? -sr : sr;
                        const double s1 = (sg0 ^ d.dsign) ? -sr : sr;
                        double2 u = ld(tp[a0]), v = ld(tp[a1]);
                        rot_pair(u, v, c, s0, s1, imag);
                        st(tp[a0], u);
                        st(tp[a1], v);
                    }
                }
                __syncthreads();
            }
            #pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                const int a = t + k * T;
                if (a >= N) break;
                psi[gk(k)] = tp[a];
            }
        } else if (P.type == kPassHam) {
            #pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                const int a = t + k * T;
                if (a >= N) break;
                tp[a] = psi[gk(k)];
            }
            __syncthreads();
            #pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                const int a = t + k * T;
                if (a >= N) break;
                double ar = 0.0, ai = 0.0;
                for (int g = P.first; g < P.first + P.count; ++g) {
                    const HamGroupDev G = A.groups[g];
                    const double2 v = ld(tp[a ^ G.xl]);
                    for (int j = G.term_begin; j < G.term_begin + G.term_count; ++j) {
                        const HamTermDev tm = A.terms[j];
                        const double sg = (par32(a & tm.zl) ^ par64(base & tm.z)) ? -1.0 : 1.0;
                        ar += sg * (tm.wre * v.x - tm.wim * v.y);
                        ai += sg * (tm.wre * v.y + tm.wim * v.x);
                    }
                }
                const uint64_t y = gk(k);
                double2 o = make_double2(ar, ai);
                if (P.flags & kFlagAccumulate) {
                    const double2 p = ld(lam[y]);
                    o.x += p.x;
                    o.y += p.y;
                }
                st(lam[y], o);
                if (P.flags & kFlagEnergy) {
                    const double2 u = ld(tp[a]);
                    const double2 oo = ld(lam[y]);   // the stored (rounded) value
                    eacc += u.x * oo.x + u.y * oo.y;
                }
            }
        } else {  // adjoint
            #pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                const int a = t + k * T;
                if (a >= N) break;
                const uint64_t y = gk(k);
                tp[a] = psi[y];
                tl[a] = lam[y];
            }
            __syncthreads();
            for (int ri = P.count - 1; ri >= 0; --ri) {
                const RotDesc &d = A.rot[P.first + ri];
                const double2 cs = A.coef[C.theta_off + d.k];
                const double c = cs.x;
                const double sr = (d.w & 2) ? cs.y : -cs.y;  // R^dag: negated angle
                const bool imag = d.w & 1;
                const int wp = (d.w + 1) & 3;
                const int so = par64(base & d.z);
                double g = 0.0;
                if (d.xl == 0) {
                    for (int a = t; a < N; a += T) {
                        const int sg = par32(a & d.zl) ^ so;
                        const double2 u = ld(tp[a]), l = ld(tl[a]);
                        const double zr = l.x * u.x + l.y * u.y, zi = l.x * u.y - l.y * u.x;
                        const double im = (wp & 1) ? zr : zi;
                        g += ((wp & 2) ? -im : im) * (sg ? -1.0 : 1.0);
                        const double sj = sg ? -sr : sr;
                        st(tp[a], rot_diag(u, c, sj, imag));
                        st(tl[a], rot_diag(l, c, sj, imag));
                    }
                } else {
                    const uint32_t lowm = (1u << d.hb) - 1;
                    for (uint32_t q = t; q < (uint32_t)(N >> 1); q += T) {
                        const uint32_t a0 = ((q & ~lowm) << 1) | (q & lowm);
                        const uint32_t a1 = a0 ^ d.xl;
                        const int sg0 = par32(a0 & d.zl) ^ so;
                        const int sg1 = sg0 ^ d.dsign;
                        double2 u0 = ld(tp[a0]), u1 = ld(tp[a1]);
                        double2 l0 = ld(tl[a0]), l1 = ld(tl[a1]);
                        const double z0r = l0.x * u1.x + l0.y * u1.y, z0i = l0.x * u1.y - l0.y * u1.x;
                        const double z1r = l1.x * u0.x + l1.y * u0.y, z1i = l1.x * u0.y - l1.y * u0.x;
                        const double zr = (sg0 ? -z0r : z0r) + (sg1 ? -z1r : z1r);
                        const double zi = (sg0 ? -z0i : z0i) + (sg1 ? -z1i : z1i);
                        const double im = (wp & 1) ? zr : zi;
                        g += (wp & 2) ? -im : im;
                        const double s0 = sg0 ? -sr : sr, s1 = sg1 ? -sr : sr;
                        rot_pair(u0, u1, c, s0, s1, imag);
                        rot_pair(l0, l1, c, s0, s1, imag);
                        st(tp[a0], u0);
                        st(tp[a1], u1);
                        st(tl[a0], l0);
                        st(tl[a1], l1);
                    }
                }
                g = wave_sum<64>(g);
                if ((t & 63) == 0) wacc[ri][t >> 6] += g;
                __syncthreads();
            }
            #pragma unroll
            for (int k = 0; k < KMAX; ++k) {
                const int a = t + k * T;
                if (a >= N) break;
                const uint64_t y = gk(k);
                psi[y] = tp[a];
                lam[y] = tl[a];
            }
        }
        __syncthreads();
    }

    // per-item partial sums
    if (P.type == kPassAdj) {
        if (t < P.count) {
            double s = 0.0;
            for (int w = 0; w < kBWaves; ++w) s += wacc[t][w];
            A.gpart[C.gpart_off + (int64_t)it.idx * kMaxRun + t] = s;
        }
    } else if (P.flags & kFlagEnergy) {
        eacc = wave_sum<64>(eacc);
        if ((t & 63) == 0) ered[t >> 6] = eacc;
        __syncthreads();
        if (t == 0) {
            double s = 0.0;
            for (int w = 0; w < kBWaves; ++w) s += ered[w];
            A.epart[C.epart_off + it.idx] = s;
        }
    }
}

// Fixed-order reduction of the per-item partial sums of one pass per workgroup.
__global__ void __launch_bounds__(kBThreads) k_batch_reduce(const BatchArgs A, const int *__restrict__ passes)
{
    __shared__ double sh[kBThreads];
    reduce_pass(A, passes[blockIdx.x], sh);
}

__global__ void k_batch_reset(uint64_t *t_start, uint64_t *t_end, int ncirc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ncirc) {
        t_start[i] = 0;
        t_end[i] = 0;
    }
}

// Before a persistent run: clear its pass counters, control words and
// timestamps, and turn the angles into (cos, sin) pairs.
__global__ void __launch_bounds__(256)
k_batch_persist_reset(uint32_t *done, uint32_t *ready, int npass, uint32_t *ctl, uint64_t *t_start, uint64_t *t_end,
                      int ncirc, const double *__restrict__ theta, double2 *__restrict__ coef, int64_t m)
{
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = i0; i < npass; i += step) {
        done[i] = 0;
        ready[i] = 0;
    }
    if (i0 < kCtlWords) ctl[i0] = 0;
    for (int64_t i = i0; i < ncirc; i += step) {
        t_start[i] = 0;
        t_end[i] = 0;
    }
    for (int64_t k = i0; k < m; k += step) {
        double sn, cs;
        sincos(0.5 * theta[k], &sn, &cs);
        coef[k] = make_double2(cs, sn);
    }
}

__global__ void k_batch_coef(const double *__restrict__ theta, double2 *__restrict__ coef, int64_t m)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) {
        double s, c;
        sincos(0.5 * theta[k], &s, &c);
        coef[k] = make_double2(c, s);
    }
}

inline bool hip_ok(hipError_t e, const char *what, cfh_status *st)
{
    if (e == hipSuccess) return true;
    *st = set_error(CFH_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return false;
}

} // namespace

struct cfh_batch_s {
    int count = 0, dtype = 0, bmax = 0;
    int64_t total_rot = 0, total_amp = 0;
    std::vector<int> n, m;
    std::vector<BPass> passes;
    // per level: [offset, count) into the item table and into the reduction list
    struct Level {
        int64_t red_off, red_cnt;
        int64_t off[kKernCount], cnt[kKernCount];  // items of each kernel (kKern*)
    };
    std::vector<Level> levels[2];   // [0] forward + energy, [1] with gradients
    int64_t n_items[2] = {0, 0};
    int n_groups = 0;               // cache groups of circuits
    int64_t n_passes = 0;           // passes of the gradient chains (forward, Hamiltonian, adjoint)
    double bytes[2] = {0.0, 0.0};   // algorithmic HBM bytes of one forward / gradient run
    void *arena = nullptr;
    BPass *d_passes = nullptr;
    BCirc *d_circs = nullptr;
    BItem *d_items[2][kKernCount] = {};
    PassArgs2 *d_pa = nullptr;
    double2 *d_mw = nullptr;
    int reg_fwd = 0;                // circuits with n >= reg_bits run on register tiles
    int reg_bits = kBatchRegTile;   // log2 amplitudes of a register tile
    int *d_reduce[2] = {nullptr, nullptr};
    RotDesc *d_rot = nullptr;
    HamGroupDev *d_groups = nullptr;
    HamTermDev *d_terms = nullptr;
    double *d_theta = nullptr, *d_grad = nullptr, *d_energy = nullptr, *d_gpart = nullptr, *d_epart = nullptr;
    double2 *d_coef = nullptr;
    void *d_psi = nullptr, *d_lam = nullptr;
    uint64_t *d_tstart = nullptr, *d_tend = nullptr;
    // persistent runs (tuning variant 1)
    bool persist = false;
    BItem *d_tickets[2] = {nullptr, nullptr};  // claim order of the forward / gradient run
    int32_t *d_prev[2] = {nullptr, nullptr};   // per pass: the pass before it in that run's chain
    int64_t n_tickets[2] = {0, 0};
    uint32_t *d_done = nullptr, *d_ready = nullptr, *d_ctl = nullptr;
    uint64_t max_wait_ticks = 0;  // a dependency wait gives up after this many wall-clock ticks
    double tick_hz = 1e8;
    uint32_t need = 1;            // 2: every wait gives up (the give-up path, for tests)
    int max_grid = 0;             // 0: every resident workgroup
    int grid_used = 0;
    std::vector<int64_t> psi_off;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    ~cfh_batch_s()
    {
        for (int i = 0; i < 2; ++i) {
            if (exec[i]) (void)hipGraphExecDestroy(exec[i]);
            if (graph[i]) (void)hipGraphDestroy(graph[i]);
        }
        if (arena) (void)hipFree(arena);
    }
};

namespace {

template <typename Amp>
cfh_status launch_level(int bmax, unsigned grid, hipStream_t s, const BatchArgs &A, const BItem *items)
{
    switch (bmax) {
    case 8: hipLaunchKernelGGL((k_batch_level<Amp, 8>), dim3(grid), dim3(kBThreads), 0, s, A, items); break;
    case 9: hipLaunchKernelGGL((k_batch_level<Amp, 9>), dim3(grid), dim3(kBThreads), 0, s, A, items); break;
    case 10: hipLaunchKernelGGL((k_batch_level<Amp, 10>), dim3(grid), dim3(kBThreads), 0, s, A, items); break;
    case 11: hipLaunchKernelGGL((k_batch_level<Amp, 11>), dim3(grid), dim3(kBThreads), 0, s, A, items); break;
    case 12:
        if constexpr (sizeof(Amp) == 8) {
            hipLaunchKernelGGL((k_batch_level<Amp, 12>), dim3(grid), dim3(kBThreads), 0, s, A, items);
            break;
        }
        [[fallthrough]];
    default:
        return set_error(CFH_E_UNSUPPORTED, "cfh_batch_run: tile_bits");
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(CFH_E_HIP, std::string("k_batch_level: ") + hipGetErrorString(e));
    return CFH_OK;
}

// The planning of one circuit of a batch: argument checks, its rotation
// passes (LDS-staged, or register-tiled with their forward and adjoint kernel
// descriptors, a run that needs more micro-groups than a pass carries split
// in two) and its observable's passes.  It depends on nothing but the circuit
// and the batch settings, so circuits are planned on worker threads; the
// batch tables are then assembled from these plans in circuit order.
struct CircPlan {
    cfh_status st = CFH_OK;
    std::string msg;
    std::vector<Pauli> r;                     // rotations
    TuningResolved tu;                        // LDS-staged tuning
    int b = 0, tpi = 1, nitems = 1, tpi2 = 1, nitems2 = 1;
    bool reg = false;                         // register-tiled passes
    std::vector<PassPlan> fw;                 // LDS-staged forward passes
    std::vector<std::pair<PassPlan, PassArgs2>> fwd2, adj2, meas2, ham2;  // register-tiled passes, in order
    std::vector<HamGroup> groups;             // the terms grouped by x mask (first-appearance order)
    std::vector<HamPass> hp;                  // LDS-staged Hamiltonian passes
};

struct BatchSettings {
    int dtype, bmax, reg_bits, max_items;
    bool reg_fwd, persist;
    const cfh_tuning *tuning;
};

void plan_circuit(const cfh_circuit_desc &d, const BatchSettings &S, CircPlan &out)
{
    auto fail = [&](cfh_status st) {
        out.st = st;
        out.msg = cfh_last_error();
    };
    const size_t ab = S.dtype == CFH_C64 ? 8 : 16;
    const cfh_tuning *tuning = S.tuning;
    if (d.n < 8 || d.n > 30) return fail(set_error(CFH_E_UNSUPPORTED, "cfh_batch_create: circuit n must be in 8..30"));
    if ((d.m && (!d.rot || !d.theta)) || (d.mh && (!d.terms || !d.coeff)) || d.m < 0 || d.mh < 0)
        return fail(set_error(CFH_E_INVAL, "cfh_batch_create: null rotation or term arrays"));
    if (d.init_index >> d.n) return fail(set_error(CFH_E_RANGE, "cfh_batch_create: init_index >= 2^n"));
    std::vector<Pauli> &r = out.r;
    r.resize(d.m);
    for (int64_t i = 0; i < d.m; ++i) {
        cfh_status st = check_pauli(d.rot[i], d.n, true, "cfh_batch_create");
        if (st) return fail(st);
        r[i] = Pauli{d.rot[i].x, d.rot[i].z, d.rot[i].e & 3};
    }
    for (int64_t i = 0; i < d.mh; ++i) {
        cfh_status st = check_pauli(d.terms[i], d.n, true, "cfh_batch_create");
        if (st) return fail(st);
    }
    cfh_tuning tc{};
    tc.tile_bits = std::min(S.bmax, d.n);
    tc.low_bits = tuning && tuning->low_bits > 0 ? tuning->low_bits : 4;
    tc.max_run = tuning && tuning->max_run > 0 ? tuning->max_run : kMaxRun;
    out.tu = resolve_tuning(&tc, d.n, S.dtype, kTuneForward);
    const TuningResolved &tu = out.tu;
    out.b = tu.tile_bits;
    const uint64_t ntiles = 1ull << (d.n - out.b);
    out.tpi = (int)std::clamp<uint64_t>((ntiles + S.max_items - 1) / S.max_items, 1, kBatchMaxTilesPerItem);
    out.nitems = (int)((ntiles + out.tpi - 1) / out.tpi);
    const bool reg = S.reg_fwd && d.n >= S.reg_bits && d.m > 0;
    out.reg = reg;
    if (S.persist && !reg)
        return fail(set_error(CFH_E_UNSUPPORTED, "cfh_batch_create: a persistent batch needs every circuit on "
                                                 "register tiles (n >= reg_tile_bits and at least one rotation)"));
    const uint64_t nt2 = reg ? 1ull << (d.n - S.reg_bits) : 1;
    out.tpi2 = (int)std::clamp<uint64_t>((nt2 + S.max_items - 1) / S.max_items, 1, kBatchMaxTilesPerItem);
    out.nitems2 = (int)((nt2 + out.tpi2 - 1) / out.tpi2);
    // LDS-staged plan of circuits below the register tile (or under tuning
    // variant 2): forward passes and, walked backwards, adjoint passes
    if (!reg) out.fw = plan_rotations(d.n, r, tu);
    if (reg) {
        // forward passes on register tiles of 2^reg_bits amplitudes (128-byte chunks);
        // a run needing more micro-groups than a pass carries is split in two
        cfh_tuning t2{};
        t2.tile_bits = S.reg_bits;
        t2.max_run = tc.max_run;
        const TuningResolved tu2 = resolve_tuning(&t2, d.n, S.dtype, kTuneForward);
        std::vector<PassPlan> todo;
        for (PassPlan &pp : plan_rotations(d.n, r, tu2)) todo.push_back(std::move(pp));
        std::reverse(todo.begin(), todo.end());
        PassArgs2 a2;
        while (!todo.empty()) {
            PassPlan pp = std::move(todo.back());
            todo.pop_back();
            if (!build_pass_args2(pp, r, false, batch_fwd_half((int)ab), a2)) {
                if (pp.rots.size() < 2)
                    return fail(set_error(CFH_E_INVAL, "cfh_batch_create: a rotation does not fit the register tile"));
                PassPlan hi = pp;
                const size_t half = pp.rots.size() / 2;
                hi.rots.assign(pp.rots.begin() + (std::ptrdiff_t)half, pp.rots.end());
                pp.rots.resize(half);
                todo.push_back(std::move(hi));
                todo.push_back(std::move(pp));
                continue;
            }
            if (a2.b != S.reg_bits) return fail(set_error(CFH_E_INVAL, "cfh_batch_create: register tile size"));
            out.fwd2.emplace_back(std::move(pp), a2);
        }
        // adjoint passes: the same runs walked backwards (anchored
        // micro-groups and half-tile transposes at complex128); a run that
        // needs more micro-groups so is split, its later half walked first
        std::vector<PassPlan> rtodo;
        for (const auto &f : out.fwd2) rtodo.push_back(f.first);
        while (!rtodo.empty()) {
            PassPlan pp = std::move(rtodo.back());
            rtodo.pop_back();
            if (!build_pass_args2(pp, r, true, batch_fwd_half((int)ab), a2)) {
                if (pp.rots.size() < 2)
                    return fail(set_error(CFH_E_INVAL, "cfh_batch_create: a rotation does not fit the register tile"));
                PassPlan hi = pp;
                const size_t half = pp.rots.size() / 2;
                hi.rots.assign(pp.rots.begin() + (std::ptrdiff_t)half, pp.rots.end());
                pp.rots.resize(half);
                rtodo.push_back(std::move(pp));
                rtodo.push_back(std::move(hi));
                continue;
            }
            out.adj2.emplace_back(std::move(pp), a2);
        }
    }
    // Hamiltonian passes (lam = H psi, energy on the last)
    std::map<uint64_t, int> gid;
    std::vector<HamGroup> &groups = out.groups;
    for (int64_t i = 0; i < d.mh; ++i) {
        auto itg = gid.find(d.terms[i].x);
        if (itg == gid.end()) {
            gid[d.terms[i].x] = (int)groups.size();
            groups.push_back(HamGroup{d.terms[i].x, {(int)i}});
        } else {
            groups[itg->second].terms.push_back((int)i);
        }
    }
    if (!reg) out.hp = plan_hamiltonian(d.n, groups, tu);
    if (reg) {
        // terms planned on register tiles: read-only measurement passes for
        // forward runs, H psi passes (psi and lam in registers; anchored,
        // half-tile transposes at complex128) for gradient runs
        cfh_tuning t3{};
        t3.tile_bits = S.reg_bits;
        const TuningResolved tm = resolve_tuning(&t3, d.n, S.dtype, kTuneMeasure);
        std::vector<HamGroup> mgr;
        for (const HamGroup &g : groups)
            for (size_t i = 0; i < g.terms.size(); i += kMaxRun)
                mgr.push_back(HamGroup{g.x, std::vector<int>(g.terms.begin() + (std::ptrdiff_t)i,
                                                             g.terms.begin() + (std::ptrdiff_t)std::min(
                                                                                   g.terms.size(), i + kMaxRun))});
        std::vector<Pauli> tp(d.mh);
        for (int64_t i = 0; i < d.mh; ++i) tp[i] = Pauli{d.terms[i].x, d.terms[i].z, d.terms[i].e & 3};
        const std::vector<HamPass> mps = plan_hamiltonian(d.n, mgr, tm, kMaxGroupsPerPass, kMaxRun);
        for (const bool ham : {false, true}) {
            // measurement and H psi items use half-tile transposes where the forward items do
            const bool anchored = batch_fwd_half((int)ab);
            std::vector<PassPlan> todo;
            for (const HamPass &mp : mps) {
                std::vector<int> idx;
                for (int g : mp.groups) idx.insert(idx.end(), mgr[g].terms.begin(), mgr[g].terms.end());
                PassPlan pp;
                pp.b = mp.b;
                pp.outer_mask = mp.outer_mask;
                pp.v = mp.v;
                pp.rots = order_for_microgroups(mp.v, tp, idx, anchored);
                todo.push_back(std::move(pp));
            }
            std::reverse(todo.begin(), todo.end());
            PassArgs2 a3;
            while (!todo.empty()) {
                PassPlan pp = std::move(todo.back());
                todo.pop_back();
                if (!build_pass_args2(pp, tp, false, anchored, a3)) {
                    if (pp.rots.size() < 2)
                        return fail(set_error(CFH_E_INVAL, "cfh_batch_create: a term does not fit the register tile"));
                    PassPlan hi = pp;
                    const size_t half = pp.rots.size() / 2;
                    hi.rots.assign(pp.rots.begin() + (std::ptrdiff_t)half, pp.rots.end());
                    pp.rots.resize(half);
                    todo.push_back(std::move(hi));
                    todo.push_back(std::move(pp));
                    continue;
                }
                if (a3.b != S.reg_bits) return fail(set_error(CFH_E_INVAL, "cfh_batch_create: register tile size"));
                (ham ? out.ham2 : out.meas2).emplace_back(std::move(pp), a3);
            }
        }
    }
}

// Plans every circuit, on up to 16 threads (this one included); a thread
// that cannot be started leaves its share to the others.
void plan_circuits(const cfh_circuit_desc *circ, int count, const BatchSettings &S, std::vector<CircPlan> &plans)
{
    std::atomic<int> next{0};
    auto work = [&] {
        for (int c; (c = next.fetch_add(1)) < count;) {
            try {
                plan_circuit(circ[c], S, plans[c]);
            } catch (...) {
                plans[c].st = CFH_E_NOMEM;
                plans[c].msg = "cfh_batch_create: host memory";
            }
        }
    };
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const unsigned nthreads = std::min<unsigned>({hw, 16u, (unsigned)count});
    std::vector<std::thread> pool;
    for (unsigned i = 1; i < nthreads; ++i) {
        try {
            pool.emplace_back(work);
        } catch (...) {
            break;
        }
    }
    work();
    for (auto &t : pool) t.join();
}

} // namespace

extern "C" {

cfh_status cfh_batch_create(const cfh_circuit_desc *circ, int count, int dtype, const cfh_tuning *tuning,
                            cfh_batch *out)
{
    if (!out || !circ || count < 1) return set_error(CFH_E_INVAL, "cfh_batch_create: bad arguments");
    if (dtype != CFH_C64 && dtype != CFH_C128) return set_error(CFH_E_UNSUPPORTED, "cfh_batch_create: dtype");
    if (tuning && (tuning->variant < 0 || tuning->variant > 2))
        return set_error(CFH_E_UNSUPPORTED,
                         "cfh_batch_create: variant 0 (level launches, register-tiled passes where n >= the "
                         "register tile), 1 (one persistent kernel per run, every circuit register-tiled) or 2 "
                         "(level launches, LDS-staged passes only)");
    std::unique_ptr<cfh_batch_s> B(new (std::nothrow) cfh_batch_s);
    if (!B) return set_error(CFH_E_NOMEM, "cfh_batch_create: host memory");
    B->count = count;
    B->dtype = dtype;
    B->reg_fwd = !(tuning && tuning->variant == 2);
    B->persist = tuning && tuning->variant == 1;
    B->reg_bits = (tuning && tuning->reg_tile_bits > 0) ? tuning->reg_tile_bits : kBatchRegTile;
    if (B->reg_bits < 11 || B->reg_bits > 13)
        return set_error(CFH_E_UNSUPPORTED, "cfh_batch_create: reg_tile_bits must be in 11..13");
    const int bcap = dtype == CFH_C128 ? 11 : 12;
    B->bmax = (tuning && tuning->tile_bits > 0) ? tuning->tile_bits : 10;
    if (B->bmax < 8 || B->bmax > bcap)
        return set_error(CFH_E_UNSUPPORTED, "cfh_batch_create: tile_bits must be in 8..11 (c128) / 8..12 (c64)");
    const int max_items = (tuning && tuning->batch_items > 0) ? tuning->batch_items : 32;
    const size_t ab = dtype == CFH_C64 ? 8 : 16;

    std::vector<BCirc> circs(count);
    std::vector<RotDesc> rots;
    std::vector<PassArgs2> pa;
    std::vector<double2> mw_all;
    std::vector<HamGroupDev> gdev;
    std::vector<HamTermDev> tdev;
    std::vector<double> theta_all;
    std::vector<std::vector<int>> chain_fwd(count), chain_grad(count);
    int64_t amp = 0, gpart = 0, epart = 0;
    std::vector<CircPlan> plans(count);
    plan_circuits(circ, count, BatchSettings{dtype, B->bmax, B->reg_bits, max_items, B->reg_fwd != 0, B->persist, tuning},
                  plans);
    {
        // the tables' final sizes (kernel descriptors are 3 KiB each): no regrowth copies
        size_t npa = 0, npass = 0, nrot = 0, nmw = 0;
        for (int c = 0; c < count; ++c) {
            const CircPlan &CP = plans[c];
            const size_t n2 = CP.fwd2.size() + CP.adj2.size() + CP.meas2.size() + CP.ham2.size();
            npa += n2;
            npass += n2 + 2 * CP.fw.size() + CP.hp.size();
            for (const auto &f : CP.fwd2) nrot += f.first.rots.size();
            for (const auto &f : CP.fw) nrot += f.rots.size();
            nmw += (size_t)std::max<int64_t>(0, circ[c].mh);
        }
        pa.reserve(npa);
        B->passes.reserve(npass);
        rots.reserve(nrot);
        mw_all.reserve(nmw);
    }
    for (int c = 0; c < count; ++c) {
        const cfh_circuit_desc &d = circ[c];
        CircPlan &CP = plans[c];
        if (CP.st) return set_error(CP.st, CP.msg);
        const std::vector<Pauli> &r = CP.r;
        const bool reg = CP.reg;
        const int b = CP.b, tpi = CP.tpi, nitems = CP.nitems, tpi2 = CP.tpi2, nitems2 = CP.nitems2;
        BCirc &C = circs[c];
        C.psi_off = amp;
        C.init = d.init_index;
        C.theta_off = (int64_t)theta_all.size();
        C.gpart_off = gpart;
        C.epart_off = epart;
        C.mw_off = (int64_t)mw_all.size();
        C.n = d.n;
        for (int64_t i = 0; i < d.mh; ++i) {
            const int wp = (d.terms[i].e - popc(d.terms[i].x & d.terms[i].z)) & 3;  // i^wp
            const double cf = d.coeff[i];
            mw_all.push_back(make_double2(wp == 0 ? cf : wp == 2 ? -cf : 0.0, wp == 1 ? cf : wp == 3 ? -cf : 0.0));
        }
        B->psi_off.push_back(amp);
        amp += (int64_t)1 << d.n;
        gpart += (int64_t)std::max(nitems, nitems2) * kMaxRun;
        epart += std::max(nitems, nitems2);
        theta_all.insert(theta_all.end(), d.theta, d.theta + d.m);
        B->n.push_back(d.n);
        B->m.push_back((int)d.m);

        auto new_pass = [&](int type, int bb, uint64_t outer, const std::vector<uint64_t> &v, int first, int cnt,
                            int flags) {
            BPass P;
            std::memset(&P, 0, sizeof(P));
            P.outer_mask = outer;
            for (size_t i = 0; i < v.size(); ++i) P.v[i] = v[i];
            P.type = type;
            P.circ = c;
            P.b = bb;
            P.flags = flags;
            P.nitems = nitems;
            P.tiles_per_item = tpi;
            P.first = first;
            P.count = cnt;
            P.p2 = -1;
            B->passes.push_back(P);
            return (int)B->passes.size() - 1;
        };
        const std::vector<PassPlan> &fw = CP.fw;
        std::vector<int> fw_lds;  // LDS-staged pass of fw[i]
        for (size_t i = 0; i < fw.size(); ++i) {
            const int first = (int)rots.size();
            for (int k : fw[i].rots) rots.push_back(make_rot_desc(fw[i], r[k], k));
            fw_lds.push_back(new_pass(kPassFwd, b, fw[i].outer_mask, fw[i].v, first, (int)fw[i].rots.size(),
                                      (i == 0 ? kFlagInit | kFlagStart : 0)));
        }
        std::vector<int> fwd_ids, adj_reg;
        if (reg) {
            bool first_pass = true;
            for (const auto &f : CP.fwd2) {
                const PassPlan &pp = f.first;
                const int id = new_pass(kPassFwd, B->reg_bits, pp.outer_mask, pp.v, 0, (int)pp.rots.size(),
                                        first_pass ? kFlagInit | kFlagStart : 0);
                B->passes[id].p2 = (int)pa.size();
                B->passes[id].nitems = nitems2;
                B->passes[id].tiles_per_item = tpi2;
                pa.push_back(f.second);
                fwd_ids.push_back(id);
                first_pass = false;
            }
            for (const auto &f : CP.adj2) {
                const PassPlan &pp = f.first;
                const PassArgs2 &a2 = f.second;
                // gradient slot t of the pass belongs to rotation a2.rot[t].k
                const int first = (int)rots.size();
                const int nr = a2.mg[a2.nmg - 1].rot_begin + a2.mg[a2.nmg - 1].rot_count;
                for (int t = 0; t < nr; ++t) {
                    RotDesc rd{};
                    rd.k = a2.rot[t].k;
                    rots.push_back(rd);
                }
                const int id = new_pass(kPassAdj, B->reg_bits, pp.outer_mask, pp.v, first, nr, 0);
                B->passes[id].p2 = (int)pa.size();
                B->passes[id].nitems = nitems2;
                B->passes[id].tiles_per_item = tpi2;
                pa.push_back(a2);
                adj_reg.push_back(id);
            }
        } else {
            fwd_ids = fw_lds;
        }
        // Hamiltonian passes (lam = H psi, energy on the last)
        const std::vector<HamGroup> &groups = CP.groups;
        std::vector<int> ham_ids;
        const std::vector<HamPass> &hp = CP.hp;
        for (size_t i = 0; i < hp.size(); ++i) {
            const int first = (int)gdev.size();
            for (int g : hp[i].groups) {
                bool ok = false;
                HamGroupDev gd;
                gd.xl = local_coords(hp[i].v, groups[g].x, &ok);
                if (!ok) return set_error(CFH_E_INVAL, "cfh_batch_create: group outside its tile");
                gd.hb = gd.xl ? 31 - __builtin_clz(gd.xl) : -1;
                gd.term_begin = (int32_t)tdev.size();
                gd.term_count = (int32_t)groups[g].terms.size();
                for (int ti : groups[g].terms) {
                    const cfh_pauli &tp = d.terms[ti];
                    HamTermDev td;
                    td.z = tp.z;
                    td.zl = local_zmask(hp[i].v, tp.z);
                    td.pad = 0;
                    const int wp = (tp.e - popc(tp.x & tp.z)) & 3;
                    const double cf = d.coeff[ti];
                    td.wre = (wp == 0) ? cf : (wp == 2) ? -cf : 0.0;
                    td.wim = (wp == 1) ? cf : (wp == 3) ? -cf : 0.0;
                    tdev.push_back(td);
                }
                gdev.push_back(gd);
            }
            int flags = (i > 0 ? kFlagAccumulate : 0) | (i + 1 == hp.size() ? kFlagEnergy | kFlagEnd : 0);
            if (fwd_ids.empty() && i == 0) flags |= kFlagStart;
            ham_ids.push_back(new_pass(kPassHam, hp[i].b, hp[i].outer_mask, hp[i].v, first,
                                       (int)hp[i].groups.size(), flags));
        }
        if (!reg && ham_ids.empty())
            return set_error(CFH_E_INVAL, "cfh_batch_create: every circuit needs an observable");
        // forward runs of register-tiled circuits need only E: read-only
        // measurement passes on register tiles instead of writing lam = H psi
        std::vector<int> meas_ids, ham2_ids;
        if (reg) {
            for (const bool ham : {false, true}) {
                std::vector<int> &ids = ham ? ham2_ids : meas_ids;
                for (const auto &f : ham ? CP.ham2 : CP.meas2) {
                    const PassPlan &pp = f.first;
                    const int id = new_pass(ham ? kPassHam : kPassMeas, B->reg_bits, pp.outer_mask, pp.v, 0,
                                            (int)pp.rots.size(), ids.empty() ? 0 : kFlagAccumulate);
                    B->passes[id].p2 = (int)pa.size();
                    B->passes[id].nitems = nitems2;
                    B->passes[id].tiles_per_item = tpi2;
                    pa.push_back(f.second);
                    ids.push_back(id);
                }
            }
            if (meas_ids.empty() || ham2_ids.empty())
                return set_error(CFH_E_INVAL, "cfh_batch_create: every circuit needs an observable");
            B->passes[ham2_ids.back()].flags |= kFlagEnergy | kFlagEnd;
            B->passes[meas_ids.back()].flags |= kFlagEnergy | kFlagEnd;
        }
        if (fwd_ids.empty()) return set_error(CFH_E_INVAL, "cfh_batch_create: every circuit needs rotations");
        // adjoint passes: the forward passes walked backwards
        std::vector<int> adj_ids = adj_reg;
        if (!reg)
            for (int i = (int)fw.size() - 1; i >= 0; --i) {
                const BPass &F = B->passes[fw_lds[i]];
                adj_ids.push_back(new_pass(kPassAdj, F.b, F.outer_mask, fw[i].v, F.first, F.count, 0));
            }
        B->passes[adj_ids.back()].end_flag_grad = 1;
        // dependency chains
        std::vector<int> chain = fwd_ids;
        chain.insert(chain.end(), meas_ids.begin(), meas_ids.end());
        if (meas_ids.empty()) chain.insert(chain.end(), ham_ids.begin(), ham_ids.end());
        chain_fwd[c] = chain;
        chain = fwd_ids;
        if (reg)
            chain.insert(chain.end(), ham2_ids.begin(), ham2_ids.end());
        else
            chain.insert(chain.end(), ham_ids.begin(), ham_ids.end());
        chain.insert(chain.end(), adj_ids.begin(), adj_ids.end());
        chain_grad[c] = chain;
        CP = CircPlan();  // its descriptors are in the batch tables now
    }
    B->total_rot = (int64_t)theta_all.size();
    for (const auto &ch : chain_grad) B->n_passes += (int64_t)ch.size();
    B->total_amp = amp;
    // level tables: items of pass `lv` of every circuit, then the passes of the
    // level whose partial sums are reduced (adjoint passes, the energy pass)
    // Circuits run in consecutive groups whose psi and lam vectors fit the
    // cache budget, so a group's vectors stay in the Infinity Cache across its
    // levels; all levels of one group precede the next group.
    const int gm = tuning ? tuning->group_mib : 0;
    const int64_t budget = gm <= 0 ? INT64_MAX : (int64_t)gm << 20;
    std::vector<std::pair<int, int>> cgroups;
    {
        int c0 = 0;
        int64_t acc = 0;
        for (int c = 0; c < count; ++c) {
            const int64_t bytes = 2 * ((int64_t)ab << circs[c].n);
            if (c > c0 && acc + bytes > budget) {
                cgroups.push_back({c0, c});
                c0 = c;
                acc = 0;
            }
            acc += bytes;
        }
        cgroups.push_back({c0, count});
    }
    std::vector<BItem> items[2][kKernCount];
    std::vector<int> red[2];
    for (int g = 0; g < 2; ++g) {
        const auto &chains = g ? chain_grad : chain_fwd;
        for (const auto &cg : cgroups) {
            size_t maxlen = 0;
            for (int c = cg.first; c < cg.second; ++c) maxlen = std::max(maxlen, chains[c].size());
            for (size_t lv = 0; lv < maxlen; ++lv) {
                cfh_batch_s::Level L{};
                L.red_off = (int64_t)red[g].size();
                for (int k = 0; k < kKernCount; ++k) L.off[k] = (int64_t)items[g][k].size();
                for (int c = cg.first; c < cg.second; ++c) {
                    if (lv >= chains[c].size()) continue;
                    const int p = chains[c][lv];
                    const int ty = B->passes[p].type;
                    const int kk = B->passes[p].p2 < 0 ? kKernLds
                                   : ty == kPassAdj    ? kKernAdj2
                                   : ty == kPassMeas   ? kKernMeas2
                                   : ty == kPassHam    ? kKernHam2
                                                       : kKernFwd2;
                    auto &dst = items[g][kk];
                    for (int i = 0; i < B->passes[p].nitems; ++i) dst.push_back(BItem{p, i});
                    const BPass &P = B->passes[p];
                    const bool ends = g ? P.end_flag_grad : (P.flags & kFlagEnd);
                    if (P.type == kPassAdj || (P.flags & kFlagEnergy) || ends) red[g].push_back(p);
                }
                for (int k = 0; k < kKernCount; ++k) L.cnt[k] = (int64_t)items[g][k].size() - L.off[k];
                L.red_cnt = (int64_t)red[g].size() - L.red_off;
                B->levels[g].push_back(L);
            }
        }
        B->n_items[g] = 0;
        for (int k = 0; k < kKernCount; ++k) B->n_items[g] += (int64_t)items[g][k].size();
    }
    B->n_groups = (int)cgroups.size();
    std::vector<std::pair<int, int>> tickets[2];
    std::vector<int> prev[2];
    if (B->persist) {
        std::vector<int> pitems(B->passes.size());
        for (size_t p = 0; p < B->passes.size(); ++p) pitems[p] = B->passes[p].nitems;
        std::vector<double> camps(count);
        for (int c = 0; c < count; ++c) camps[c] = std::ldexp(1.0, circs[c].n);
        for (int g = 0; g < 2; ++g) {
            batch_ticket_order(g ? chain_grad : chain_fwd, pitems, camps, cgroups, tickets[g], prev[g]);
            B->n_tickets[g] = (int64_t)tickets[g].size();
            if (B->n_tickets[g] >= (int64_t)INT32_MAX / 2)
                return set_error(CFH_E_UNSUPPORTED, "cfh_batch_create: too many work items for a persistent run");
        }
    }
    // algorithmic bytes: a rotation pass reads and writes psi (the first one
    // only writes), a Hamiltonian pass reads psi and writes lam (and reads it
    // when accumulating), an adjoint pass reads and writes psi and lam
    for (int g = 0; g < 2; ++g)
        for (int c = 0; c < count; ++c)
            for (int p : (g ? chain_grad : chain_fwd)[c]) {
                const BPass &P = B->passes[p];
                const double S = (double)((int64_t)ab << circs[c].n);
                B->bytes[g] += P.type == kPassFwd    ? ((P.flags & kFlagInit) ? 1.0 : 2.0) * S
                               : P.type == kPassHam  ? ((P.flags & kFlagAccumulate) ? 3.0 : 2.0) * S
                               : P.type == kPassMeas ? S
                                                     : 4.0 * S;
            }

    // one device arena
    const int npass = (int)B->passes.size();
    std::vector<std::pair<void **, size_t>> parts = {
        {(void **)&B->d_passes, npass * sizeof(BPass)},
        {(void **)&B->d_circs, count * sizeof(BCirc)},
        {(void **)&B->d_mw, std::max<size_t>(1, mw_all.size()) * sizeof(double2)},
        {(void **)&B->d_pa, std::max<size_t>(1, pa.size()) * sizeof(PassArgs2)},
        {(void **)&B->d_reduce[0], std::max<size_t>(1, red[0].size()) * sizeof(int)},
        {(void **)&B->d_reduce[1], std::max<size_t>(1, red[1].size()) * sizeof(int)},
        {(void **)&B->d_rot, std::max<size_t>(1, rots.size()) * sizeof(RotDesc)},
        {(void **)&B->d_groups, std::max<size_t>(1, gdev.size()) * sizeof(HamGroupDev)},
        {(void **)&B->d_terms, std::max<size_t>(1, tdev.size()) * sizeof(HamTermDev)},
        {(void **)&B->d_theta, B->total_rot * sizeof(double)},
        {(void **)&B->d_coef, B->total_rot * sizeof(double2)},
        {(void **)&B->d_grad, B->total_rot * sizeof(double)},
        {(void **)&B->d_energy, count * sizeof(double)},
        {(void **)&B->d_gpart, gpart * sizeof(double)},
        {(void **)&B->d_epart, epart * sizeof(double)},
        {(void **)&B->d_psi, amp * ab},
        {(void **)&B->d_lam, amp * ab},
        {(void **)&B->d_tstart, count * sizeof(uint64_t)},
        {(void **)&B->d_tend, count * sizeof(uint64_t)},
    };
    for (int g = 0; g < 2; ++g)
        for (int k = 0; k < kKernCount; ++k)
            parts.push_back({(void **)&B->d_items[g][k], std::max<size_t>(1, items[g][k].size()) * sizeof(BItem)});
    if (B->persist) {
        for (int g = 0; g < 2; ++g) {
            parts.push_back({(void **)&B->d_tickets[g], std::max<size_t>(1, tickets[g].size()) * sizeof(BItem)});
            parts.push_back({(void **)&B->d_prev[g], (size_t)npass * sizeof(int32_t)});
        }
        parts.push_back({(void **)&B->d_done, (size_t)npass * sizeof(uint32_t)});
        parts.push_back({(void **)&B->d_ready, (size_t)npass * sizeof(uint32_t)});
        parts.push_back({(void **)&B->d_ctl, kCtlWords * sizeof(uint32_t)});
    }
    size_t total = 0;
    for (auto &p : parts) total += (p.second + 255) & ~(size_t)255;
    cfh_status st = CFH_OK;
    if (!hip_ok(hipMalloc(&B->arena, total), "cfh_batch_create: hipMalloc", &st)) return st;
    size_t off = 0;
    for (auto &p : parts) {
        *p.first = (char *)B->arena + off;
        off += (p.second + 255) & ~(size_t)255;
    }
    auto up = [&](void *dst, const void *src, size_t bytes) {
        return bytes == 0 || hip_ok(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice), "cfh_batch_create: copy", &st);
    };
    if (!up(B->d_passes, B->passes.data(), npass * sizeof(BPass)) ||
        !up(B->d_circs, circs.data(), count * sizeof(BCirc)) ||
        !up(B->d_mw, mw_all.data(), mw_all.size() * sizeof(double2)) ||
        !up(B->d_pa, pa.data(), pa.size() * sizeof(PassArgs2)) ||
        !up(B->d_reduce[0], red[0].data(), red[0].size() * sizeof(int)) ||
        !up(B->d_reduce[1], red[1].data(), red[1].size() * sizeof(int)) ||
        !up(B->d_rot, rots.data(), rots.size() * sizeof(RotDesc)) ||
        !up(B->d_groups, gdev.data(), gdev.size() * sizeof(HamGroupDev)) ||
        !up(B->d_terms, tdev.data(), tdev.size() * sizeof(HamTermDev)) ||
        !up(B->d_theta, theta_all.data(), theta_all.size() * sizeof(double)))
        return st;
    for (int g = 0; g < 2; ++g)
        for (int k = 0; k < kKernCount; ++k)
            if (!up(B->d_items[g][k], items[g][k].data(), items[g][k].size() * sizeof(BItem))) return st;
    if (B->persist) {
        for (int g = 0; g < 2; ++g) {
            std::vector<BItem> tk(tickets[g].size());
            for (size_t k = 0; k < tk.size(); ++k) tk[k] = BItem{tickets[g][k].first, tickets[g][k].second};
            std::vector<int32_t> pv(prev[g].begin(), prev[g].end());
            if (!up(B->d_tickets[g], tk.data(), tk.size() * sizeof(BItem)) ||
                !up(B->d_prev[g], pv.data(), pv.size() * sizeof(int32_t)))
                return st;
        }
        int khz = 0, dev = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            B->tick_hz = khz * 1000.0;
        B->max_wait_ticks = (uint64_t)(kPersistWaitSeconds * B->tick_hz);
    }
    *out = B.release();
    return CFH_OK;
}

cfh_status cfh_batch_destroy(cfh_batch b)
{
    delete b;
    return CFH_OK;
}

cfh_status cfh_batch_info(cfh_batch b, int64_t *n_items_grad, int64_t *n_passes, int64_t *n_rot, double *state_bytes,
                          double *bytes_fwd, double *bytes_grad, int32_t *n_groups)
{
    if (!b) return set_error(CFH_E_INVAL, "cfh_batch_info: null batch");
    if (n_items_grad) *n_items_grad = b->n_items[1];
    if (n_passes) *n_passes = b->n_passes;
    if (n_rot) *n_rot = b->total_rot;
    if (state_bytes) *state_bytes = (double)b->total_amp * (b->dtype == CFH_C64 ? 8 : 16);
    if (bytes_fwd) *bytes_fwd = b->bytes[0];
    if (bytes_grad) *bytes_grad = b->bytes[1];
    if (n_groups) *n_groups = b->n_groups;
    return CFH_OK;
}

cfh_status cfh_batch_set_theta(cfh_batch b, const double *theta_host)
{
    if (!b || !theta_host) return set_error(CFH_E_INVAL, "cfh_batch_set_theta: null argument");
    cfh_status st = CFH_OK;
    hip_ok(hipMemcpy(b->d_theta, theta_host, b->total_rot * sizeof(double), hipMemcpyHostToDevice),
           "cfh_batch_set_theta", &st);
    return st;
}

} // extern "C"

namespace {

BatchArgs batch_args(const cfh_batch_s *b, int g)
{
    BatchArgs A;
    std::memset(&A, 0, sizeof(A));
    A.passes = b->d_passes;
    A.circs = b->d_circs;
    A.rot = b->d_rot;
    A.groups = b->d_groups;
    A.terms = b->d_terms;
    A.coef = b->d_coef;
    A.mw = b->d_mw;
    A.psi = b->d_psi;
    A.lam = b->d_lam;
    A.grad = b->d_grad;
    A.energy = b->d_energy;
    A.gpart = b->d_gpart;
    A.epart = b->d_epart;
    A.t_start = b->d_tstart;
    A.t_end = b->d_tend;
    A.with_grad = g;
    return A;
}

// One persistent run: a kernel that clears the pass counters, control words
// and timestamps and computes the (cos, sin) table, then the persistent
// kernel over every ticket of the run.
cfh_status run_persistent(cfh_batch_s *b, int g, hipStream_t s)
{
    const int npass = (int)b->passes.size();
    const int64_t span = std::max<int64_t>({(int64_t)npass, (int64_t)b->count, b->total_rot, (int64_t)kCtlWords});
    const unsigned rgrid = (unsigned)std::min<int64_t>(1024, (span + 255) / 256);
    hipLaunchKernelGGL(k_batch_persist_reset, dim3(rgrid), dim3(256), 0, s, b->d_done, b->d_ready, npass, b->d_ctl,
                       b->d_tstart, b->d_tend, b->count, b->d_theta, b->d_coef, b->total_rot);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return set_error(CFH_E_HIP, std::string("k_batch_persist_reset: ") + hipGetErrorString(e));
    PersistArgs Q;
    Q.tickets = b->d_tickets[g];
    Q.prev = b->d_prev[g];
    Q.done = b->d_done;
    Q.ready = b->d_ready;
    Q.ctl = b->d_ctl;
    Q.max_wait = b->max_wait_ticks;
    Q.nt = (int32_t)b->n_tickets[g];
    Q.need = b->need;
    const BatchArgs A = batch_args(b, g);
    return b->dtype == CFH_C128
               ? launch_batch_persist<double2>(b->reg_bits, g != 0, b->max_grid, s, A, b->d_pa, Q, &b->grid_used)
               : launch_batch_persist<float2>(b->reg_bits, g != 0, b->max_grid, s, A, b->d_pa, Q, &b->grid_used);
}

} // namespace

extern "C" {

cfh_status cfh_batch_run(cfh_batch b, int with_grad, void *stream)
{
    if (!b) return set_error(CFH_E_INVAL, "cfh_batch_run: null batch");
    hipStream_t s = (hipStream_t)stream;
    const int g = with_grad ? 1 : 0;
    if (b->persist) return run_persistent(b, g, s);
    hipLaunchKernelGGL(k_batch_reset, dim3((b->count + 255) / 256), dim3(256), 0, s, b->d_tstart, b->d_tend,
                       b->count);
    if (b->total_rot)
        hipLaunchKernelGGL(k_batch_coef, dim3((unsigned)((b->total_rot + 255) / 256)), dim3(256), 0, s, b->d_theta,
                           b->d_coef, b->total_rot);
    const BatchArgs A = batch_args(b, g);
    const bool c128 = b->dtype == CFH_C128;
    for (const auto &L : b->levels[g]) {
        for (int k = 0; k < kKernCount; ++k) {
            if (!L.cnt[k]) continue;
            const unsigned n = (unsigned)L.cnt[k];
            const BItem *it = b->d_items[g][k] + L.off[k];
            cfh_status st = CFH_OK;
            switch (k) {
            case kKernLds:
                st = c128 ? launch_level<double2>(b->bmax, n, s, A, it) : launch_level<float2>(b->bmax, n, s, A, it);
                break;
            case kKernFwd2:
                st = c128 ? launch_batch_fwd2<double2>(b->reg_bits, n, s, A, b->d_pa, it)
                          : launch_batch_fwd2<float2>(b->reg_bits, n, s, A, b->d_pa, it);
                break;
            case kKernAdj2:
                st = c128 ? launch_batch_adj2<double2>(b->reg_bits, n, s, A, b->d_pa, it)
                          : launch_batch_adj2<float2>(b->reg_bits, n, s, A, b->d_pa, it);
                break;
            case kKernMeas2:
                st = c128 ? launch_batch_meas2<double2>(b->reg_bits, n, s, A, b->d_pa, it)
                          : launch_batch_meas2<float2>(b->reg_bits, n, s, A, b->d_pa, it);
                break;
            default:
                st = c128 ? launch_batch_ham2<double2>(b->reg_bits, n, s, A, b->d_pa, it)
                          : launch_batch_ham2<float2>(b->reg_bits, n, s, A, b->d_pa, it);
                break;
            }
            if (st) return st;
        }
        if (L.red_cnt) {
            hipLaunchKernelGGL(k_batch_reduce, dim3((unsigned)L.red_cnt), dim3(kBThreads), 0, s, A,
                               b->d_reduce[g] + L.red_off);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return set_error(CFH_E_HIP, std::string("k_batch_reduce: ") + hipGetErrorString(e));
        }
    }
    return CFH_OK;
}

cfh_status cfh_batch_graph_launch(cfh_batch b, int with_grad, void *stream)
{
    if (!b) return set_error(CFH_E_INVAL, "cfh_batch_graph_launch: null batch");
    if (!stream) return set_error(CFH_E_INVAL, "cfh_batch_graph_launch: graph capture needs a non-default stream");
    hipStream_t s = (hipStream_t)stream;
    const int g = with_grad ? 1 : 0;
    cfh_status st = CFH_OK;
    if (!b->exec[g]) {
        if (!hip_ok(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture", &st))
            return st;
        const cfh_status rs = cfh_batch_run(b, with_grad, stream);
        const hipError_t e = hipStreamEndCapture(s, &b->graph[g]);
        if (rs) return rs;
        if (!hip_ok(e, "hipStreamEndCapture", &st)) return st;
        if (!hip_ok(hipGraphInstantiate(&b->exec[g], b->graph[g], nullptr, nullptr, 0), "hipGraphInstantiate", &st))
            return st;
    }
    hip_ok(hipGraphLaunch(b->exec[g], s), "hipGraphLaunch", &st);
    return st;
}

cfh_status cfh_batch_results(cfh_batch b, double *energies, double *grads, uint64_t *t_start, uint64_t *t_end,
                             double *tick_hz, void *stream)
{
    if (!b) return set_error(CFH_E_INVAL, "cfh_batch_results: null batch");
    cfh_status st = CFH_OK;
    if (!hip_ok(hipStreamSynchronize((hipStream_t)stream), "cfh_batch_results: sync", &st)) return st;
    if (energies && !hip_ok(hipMemcpy(energies, b->d_energy, b->count * sizeof(double), hipMemcpyDeviceToHost),
                            "copy", &st))
        return st;
    if (grads && b->total_rot &&
        !hip_ok(hipMemcpy(grads, b->d_grad, b->total_rot * sizeof(double), hipMemcpyDeviceToHost), "copy", &st))
        return st;
    if (t_start && !hip_ok(hipMemcpy(t_start, b->d_tstart, b->count * sizeof(uint64_t), hipMemcpyDeviceToHost),
                           "copy", &st))
        return st;
    if (t_end && !hip_ok(hipMemcpy(t_end, b->d_tend, b->count * sizeof(uint64_t), hipMemcpyDeviceToHost), "copy", &st))
        return st;
    if (tick_hz) {
        int khz = 0, dev = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
        *tick_hz = khz * 1000.0;
    }
    if (b->persist) {
        uint32_t status = 0;
        if (!hip_ok(hipMemcpy(&status, b->d_ctl + kCtlStatus, sizeof(status), hipMemcpyDeviceToHost), "copy", &st))
            return st;
        if (status)
            return set_error(CFH_E_TIMEOUT, "cfh_batch_results: the persistent run gave up waiting for a pass; "
                                            "its results are incomplete");
    }
    return CFH_OK;
}

cfh_status cfh_batch_persist_config(cfh_batch b, double max_wait_s, int hold, int max_grid)
{
    if (!b) return set_error(CFH_E_INVAL, "cfh_batch_persist_config: null batch");
    if (!b->persist) return set_error(CFH_E_UNSUPPORTED, "cfh_batch_persist_config: not a persistent batch");
    if (!(max_wait_s > 0.0) || max_wait_s > 600.0 || (hold != 0 && hold != 1) || max_grid < 0)
        return set_error(CFH_E_INVAL, "cfh_batch_persist_config: max_wait_s in (0, 600], hold 0 or 1, max_grid >= 0");
    b->max_wait_ticks = std::max<uint64_t>(1, (uint64_t)(max_wait_s * b->tick_hz));
    b->need = hold ? 2u : 1u;
    b->max_grid = max_grid;
    // captured graphs hold the old kernel arguments
    cfh_status st = CFH_OK;
    for (int i = 0; i < 2; ++i) {
        if (b->exec[i] && !hip_ok(hipGraphExecDestroy(b->exec[i]), "hipGraphExecDestroy", &st)) return st;
        if (b->graph[i] && !hip_ok(hipGraphDestroy(b->graph[i]), "hipGraphDestroy", &st)) return st;
        b->exec[i] = nullptr;
        b->graph[i] = nullptr;
    }
    return CFH_OK;
}

cfh_status cfh_batch_persist_info(cfh_batch b, int32_t *grid, int64_t *tickets_fwd, int64_t *tickets_grad)
{
    if (!b) return set_error(CFH_E_INVAL, "cfh_batch_persist_info: null batch");
    if (!b->persist) return set_error(CFH_E_UNSUPPORTED, "cfh_batch_persist_info: not a persistent batch");
    if (grid) *grid = b->grid_used;
    if (tickets_fwd) *tickets_fwd = b->n_tickets[0];
    if (tickets_grad) *tickets_grad = b->n_tickets[1];
    return CFH_OK;
}

cfh_status cfh_batch_state(cfh_batch b, int i, void *dst_dev, void *stream)
{
    if (!b || !dst_dev || i < 0 || i >= b->count) return set_error(CFH_E_INVAL, "cfh_batch_state: bad arguments");
    const size_t ab = b->dtype == CFH_C64 ? 8 : 16;
    cfh_status st = CFH_OK;
    hip_ok(hipMemcpyAsync(dst_dev, (char *)b->d_psi + b->psi_off[i] * ab, ((size_t)1 << b->n[i]) * ab,
                          hipMemcpyDeviceToDevice, (hipStream_t)stream),
           "cfh_batch_state", &st);
    return st;
}

} // extern "C"
