// C ABI of the directional diffusion splitting solver: context set-up,
// device tables, sweep drivers (eq. (10)), stationary iteration, parabolic
// march, eq. (11) initial guess, residual, geometry export, kernel timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "adr_internal.h"
#include "adr_kernels.h"

using adr::Error;

namespace {

thread_local std::string g_setup_error;

constexpr int kSlotStep = 0, kSlotLin = 1, kSlotTime = 2, kSlotGuess = 3, kSlotHalf = 4, kSlots = 5;
constexpr int kBlock = 256;
constexpr int kTile = 16;
constexpr size_t kLdsLimit = 160 * 1024;
// the longest curve: 12 nodes per thread of a 256-thread workgroup
constexpr int kMaxNodes = 3072;

#define HIPCHK(x)                                                                              \
    do {                                                                                       \
        hipError_t e_ = (x);                                                                   \
        if (e_ != hipSuccess) throw Error{ADR_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)}; \
    } while (0)

template <typename T>
T *dalloc(size_t n, std::vector<void *> &owned) {
    if (n == 0) n = 1;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) throw Error{ADR_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)};
    owned.push_back(p);
    return static_cast<T *>(p);
}

template <typename T>
T *upload(const std::vector<T> &h, std::vector<void *> &owned, hipStream_t st) {
    T *d = dalloc<T>(h.size(), owned);
    (void)st;  // synchronous: the host vector may be a temporary
    if (!h.empty()) HIPCHK(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return d;
}

template <typename T>
std::vector<T> to_type(const std::vector<double> &v) {
    return std::vector<T>(v.begin(), v.end());
}

// One node's direct-transfer record in the FP32 sweeps' 10-byte form
// (LineArgs::dk0, dkd, dwp); koff shifts the source nodes into the packed
// numbering of the other family.  The weights become the left bracket's weight
// wL = w0 + w1 (10 bits) and the positions t = w1 / wL, w3 / wR on the two
// source segments (11 bits each); the right weight is 1 - wL, so every row
// keeps the sum 1 of its brackets.
void pack_direct(const adr::DirRec &r, int64_t koff, int32_t &k0, int16_t &kd, uint32_t &wp) {
    const int64_t kl = r.k[0] < 0 ? -1 : koff + r.k[0], kr = r.k[1] < 0 ? -1 : koff + r.k[1];
    if (kl < 0 && kr >= 0) {
        k0 = static_cast<int32_t>(kr);
        kd = adr::kDirNoLeft;
    } else {
        k0 = static_cast<int32_t>(kl);
        kd = kr < 0 ? adr::kDirNoRight
                    : (std::llabs(kr - kl) <= adr::kDirMaxDelta ? static_cast<int16_t>(kr - kl) : adr::kDirEscape);
    }
    const double wl = r.w[0] + r.w[1], wr = r.w[2] + r.w[3];
    const double tl = wl > 0.0 ? r.w[1] / wl : 0.0, tr = wr > 0.0 ? r.w[3] / wr : 0.0;
    auto q = [](double x, double scale, uint32_t top) {
        const double v = std::nearbyint(std::min(std::max(x, 0.0), 1.0) * scale);
        return std::min(static_cast<uint32_t>(v), top);
    };
    wp = q(wl, 1023.0, 1023u) | (q(tl, 2047.0, 2047u) << 10) | (q(tr, 2047.0, 2047u) << 21);
}

struct DevFam {
    int n_lines = 0;
    int nmax = 0;  // nodes of the longest curve (sizes the launch's LDS)
    int64_t n_nodes = 0, n_unknowns = 0;
    adr::LineArgs<double> a64{};
    adr::LineArgs<double> a64d{};  // the same with the direct-transfer records (options.transfer = 1)
    adr::LineArgs<float> a32{};
    adr::LineArgs<float> a32d{};
    adr::ScatterArgs<double> s64{};
    adr::ScatterArgs<float> s32{};
    double *v64 = nullptr;
    float *v32 = nullptr;
    // launch-list compaction (batched stationary solves): lines of unfinished instances
    std::vector<int> inst_lines, inst_nmax;  // per instance: curves, longest curve
    std::vector<int64_t> inst_unk;           // per instance: line unknowns
    int *lidx = nullptr;                      // compacted line list (device)
    int act = -1, act_nmax = 0;               // its length and longest curve; -1: full list
    int64_t act_unk = 0;                      // line unknowns of the compacted list
    // length buckets: the list is ordered longest first, so bucket b is the
    // range bstart[b] .. bstart[b+1]-1 of the full list (abstart: of the
    // compacted list); bnmax: its longest curve
    int bstart[adr::kLineBuckets + 1] = {}, bnmax[adr::kLineBuckets] = {};
    int bshape[adr::kLineBuckets] = {};  // workgroup shape of each bucket's launch (adr_autotune)
    // the single launch's dispatch (full list): list positions in XCD order
    // (sidx), each XCD's share (xs, 9 entries, device), the grid (xgrid)
    const int *sidx = nullptr;
    const int *xs = nullptr;
    int xgrid = 0;
    int abstart[adr::kLineBuckets + 1] = {}, abnmax[adr::kLineBuckets] = {};
    std::vector<std::array<int, adr::kLineBuckets>> inst_bl, inst_bnmax;  // per instance and bucket
};

}  // namespace

struct adr_ctx {
    int n_inst = 0;
    std::vector<int64_t> goff;
    int64_t n_grid = 0, n_unknowns = 0;
    int64_t n_blocked = 0;  // size of the blocked (8 x 4) FP32 increment fields
    adr_options opt{};
    hipStream_t st = nullptr;
    std::vector<void *> owned;
    DevFam fam[2];
    int *blk_start = nullptr, *inst_bstride = nullptr;
    int *slot_rm = nullptr, *slot_b = nullptr;  // interior node of each scatter slot: row-major / blocked
    const int *blk_inst_d = nullptr;            // instance of each scatter block (device)
    int npad = 0;
    double *Ub = nullptr;  // the state in the blocked layout during a call
    int n_blocks = 0;
    std::vector<int> inst_blocks;                      // per instance: 256-slot scatter blocks
    std::vector<int64_t> inst_grid;                    // per instance: interior grid nodes
    int64_t act_grid = 0;                              // interior grid nodes of the compacted blocks
    int *blist = nullptr, *cscan = nullptr, *ccount = nullptr;  // compacted block list, scan scratch, count
    int act_blocks = -1;                               // length of blist; -1: full list
    std::vector<int> act_set;                          // the flags blist was compacted from
    // interpolation-free transfer (options.transfer = 1): per gamma-curve update
    // sums grouped by instance, their ranges, and |Phi(0)| of the direct sweep
    double *lpart = nullptr, *cnorm_d = nullptr;
    int *inst_lstart = nullptr;
    bool cnorm_d_valid = false;
    // direct increments on the grid route (options.increments = 1): the FP32
    // sum of a block's gamma-curve increments
    float *hsum = nullptr;
    double *par = nullptr;  // [slot][fam][inst][8]
    std::vector<double> par_h;
    double *Uh64 = nullptr, *Z64 = nullptr, *partial = nullptr, *cnorm = nullptr, *rel = nullptr;
    double *rel_fb = nullptr;  // residual of a fallback start (adr_split_iterate_judged)
    float *d32 = nullptr, *D32 = nullptr;
    int *done = nullptr, *never = nullptr, *conv_it = nullptr;
    int *sing = nullptr;  // per instance: a line solve met a bad pivot (ADR_ESINGULAR)
    // fitted beta-lines (options.stabilize): per beta node the element's |beta|_e h_e
    // (mu-free part of its Peclet number) and phi(Pe) in FP64 and FP32
    std::vector<double> fit_wlh;
    double *phi64 = nullptr;
    float *phi32 = nullptr;
    // phi per beta node from fit_wlh and the instances' mu (0 at line starts)
    void fill_phi(const std::vector<double> &mu_i) {
        std::vector<double> ph(fit_wlh.size(), 0.0);
        for (int i = 0; i < n_inst; ++i)
            for (int64_t k = noffB[i]; k < noffB[i + 1]; ++k) {
                const double wlh = fit_wlh[static_cast<size_t>(k)];
                if (wlh > 0.0) {
                    const double pe = wlh / (2.0 * mu_i[i]);
                    ph[static_cast<size_t>(k)] = pe / std::tanh(pe);
                }
            }
        std::vector<float> p32(ph.begin(), ph.end());
        HIPCHK(hipMemcpy(phi64, ph.data(), sizeof(double) * ph.size(), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(phi32, p32.data(), sizeof(float) * p32.size(), hipMemcpyHostToDevice));
    }
    // GMRES acceleration (options.krylov = m > 0), allocated on first use
    std::vector<int64_t> boff_h;  // blocked offset of each instance (n_inst + 1)
    adr::KChunks kch{};
    int kmax = 0;                 // basis vectors allocated (m + 1)
    double *kV = nullptr;         // the basis, kmax fields of n_blocked
    double *kWh = nullptr;        // half step of the linear sweeps (zero outside the interior)
    double *kpart = nullptr, *kout = nullptr, *kcoef = nullptr;
    int *kskip = nullptr;         // done, or finished inside the current Arnoldi cycle
    double last_theta = -1, last_dt = -1;
    std::vector<double> mu, sg;
    std::string err;
    std::vector<adr::Family> geo[2];  // per instance, for export
    std::vector<adr::InstanceGeo> host_geo;  // host-only contexts: the whole set-up, for export
    std::vector<adr::Grid> grids;     // per instance
    std::vector<adr_problem> shape;   // per instance: grid and domain (pointers cleared)
    std::vector<int64_t> noffB;       // first beta-line node of each instance
    double *L64 = nullptr;            // packed loads (mutable views of the line tables)
    double *L64base = nullptr;        // the problem's own loads (the converged time steps shift L64)
    float *L32 = nullptr;
    // timing
    struct Tick {
        int prec, cls;
        int64_t units;  // line unknowns (line solves) or interior grid nodes (scatters) of the launch
        hipEvent_t a, b;
    };
    std::vector<Tick> ticks;
    std::vector<hipEvent_t> ev_pool;
    double ms[2][5] = {};
    int64_t cnt[2][5] = {}, units[2][5] = {};

    const double *par_ptr(int slot, int f) const { return par + (static_cast<size_t>(slot) * 2 + f) * n_inst * 8; }

    template <typename F>
    void timed(int prec, int cls, int64_t work, F &&fn) {
        if (!opt.timing) {
            HIPCHK(fn());
            return;
        }
        // events come from a pool (created once, reused after each collection)
        while (ev_pool.size() < 2 * (ticks.size() + 1)) {
            hipEvent_t e = nullptr;
            HIPCHK(hipEventCreate(&e));
            ev_pool.push_back(e);
        }
        Tick t{prec, cls, work, ev_pool[2 * ticks.size()], ev_pool[2 * ticks.size() + 1]};
        HIPCHK(hipEventRecord(t.a, st));
        HIPCHK(fn());
        HIPCHK(hipEventRecord(t.b, st));
        ticks.push_back(t);
        // bound the outstanding records: fold them in every 4096 launches
        if (ticks.size() >= 4096) collect_ticks();
    }

    void collect_ticks() {
        if (ticks.empty()) return;
        HIPCHK(hipStreamSynchronize(st));
        for (auto &t : ticks) {
            float e = 0.f;
            HIPCHK(hipEventElapsedTime(&e, t.a, t.b));
            ms[t.prec][t.cls] += e;
            cnt[t.prec][t.cls] += 1;
            units[t.prec][t.cls] += t.units;
        }
        ticks.clear();
    }

    // line and scatter arguments with the compacted lists when they are active
    template <typename T>
    adr::LineArgs<T> largs(const DevFam &F, const adr::LineArgs<T> &a) const {
        adr::LineArgs<T> r = a;
        if (F.act >= 0) r.lidx = F.lidx;
        return r;
    }
    template <typename T>
    adr::ScatterArgs<T> sargs(const adr::ScatterArgs<T> &a) const {
        adr::ScatterArgs<T> r = a;
        if (act_blocks >= 0) {
            r.blist = blist;
            r.nblist = act_blocks;
        }
        return r;
    }
    // the line solves of family f: one launch, or one per non-empty length bucket
    template <typename T>
    hipError_t lines(int f, const adr::LineArgs<T> &base, const T *fin, T *vout, const double *par, const int *dn) {
        const DevFam &F = fam[f];
        adr::LineArgs<T> a = largs(F, base);
        a.lbase = 0;
        if (!opt.split_lines) {
            const int nl = F.act >= 0 ? F.act : F.n_lines, nm = F.act >= 0 ? F.act_nmax : F.nmax;
            if (F.act < 0 && F.xs) {
                // the full list: chunks of neighbouring curves dealt to the XCDs
                a.lidx = F.sidx;
                a.xs = F.xs;
                return adr::launch_line<T>(f, -1, 0, a, F.xgrid, fin, vout, par, dn, nm, st);
            }
            return adr::launch_line<T>(f, -1, 0, a, nl, fin, vout, par, dn, nm, st);
        }
        const int *bs = F.act >= 0 ? F.abstart : F.bstart;
        const int *bn = F.act >= 0 ? F.abnmax : F.bnmax;
        // concurrent: the longest bucket on st, the next on side[0], the short ones
        // in turn on side[1] (not inside a graph capture, which runs on cap; st may
        // be the null stream, so the test is on cap being in use)
        const bool conc = opt.split_lines == 2 && !(cap != nullptr && st == cap);
        hipError_t e = hipSuccess;
        if (conc) {
            if (!side[0]) {
                for (int k = 0; k < 2; ++k) {
                    if ((e = hipStreamCreateWithFlags(&side[k], hipStreamNonBlocking)) != hipSuccess) return e;
                    if ((e = hipEventCreateWithFlags(&join_ev[k], hipEventDisableTiming)) != hipSuccess) return e;
                }
                if ((e = hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming)) != hipSuccess) return e;
            }
            if ((e = hipEventRecord(fork_ev, st)) != hipSuccess) return e;
            for (int k = 0; k < 2; ++k)
                if ((e = hipStreamWaitEvent(side[k], fork_ev, 0)) != hipSuccess) return e;
        }
        for (int b = 0; b < adr::kLineBuckets; ++b) {
            if (bs[b + 1] == bs[b]) continue;
            a.lbase = bs[b];
            hipStream_t sb = !conc || b == 0 ? st : side[b == 1 ? 0 : 1];
            if ((e = adr::launch_line<T>(f, b, F.bshape[b], a, bs[b + 1] - bs[b], fin, vout, par, dn, bn[b], sb)) !=
                hipSuccess)
                return e;
        }
        if (conc)
            for (int k = 0; k < 2; ++k) {
                if ((e = hipEventRecord(join_ev[k], side[k])) != hipSuccess) return e;
                if ((e = hipStreamWaitEvent(st, join_ev[k], 0)) != hipSuccess) return e;
            }
        return hipSuccess;
    }
    // milliseconds of `reps` FP32 line solves of bucket b (both families, full
    // lists) with workgroup shape `shape`, after one untimed run (the direct
    // transfer's line solves in a direct context)
    double time_bucket(int b, int shape, int reps) {
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        const bool dir = opt.transfer == 1;
        auto run = [&]() {
            for (int f = 0; f < 2; ++f) {
                const DevFam &F = fam[f];
                adr::LineArgs<float> a = dir ? F.a32d : F.a32;
                a.lidx = nullptr;
                a.lbase = F.bstart[b];
                HIPCHK(adr::launch_line<float>(f, b, shape, a, F.bstart[b + 1] - F.bstart[b],
                                               dir ? fam[1 - f].v32 : d32, F.v32, par_ptr(kSlotLin, f), never,
                                               F.bnmax[b], st));
            }
        };
        run();
        HIPCHK(hipEventRecord(e0, st));
        for (int r = 0; r < reps; ++r) run();
        HIPCHK(hipEventRecord(e1, st));
        HIPCHK(hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return ms;
    }
    // work of a launch over the current (possibly compacted) lists
    int64_t line_work(int f) const { return fam[f].act >= 0 ? fam[f].act_unk : fam[f].n_unknowns; }
    int64_t grid_work() const { return act_blocks >= 0 ? act_grid : n_unknowns; }
    void line64(int f, int slot, const double *fin, const int *dn) {
        timed(0, f, line_work(f), [&] { return lines<double>(f, fam[f].a64, fin, fam[f].v64, par_ptr(slot, f), dn); });
    }
    void line32(int f, int slot, const float *fin, const int *dn) {
        timed(1, f, line_work(f), [&] { return lines<float>(f, fam[f].a32, fin, fam[f].v32, par_ptr(slot, f), dn); });
    }

    // One FP64 sweep of eq. (10) from U.  mode of the final scatter: 0 write U,
    // 1 write U + d32 + partial, 3 partial only (U unchanged).
    void sweep64(int slot, const double *U_in, double *U_out, int mode, const int *dn) {
        line64(0, slot, U_in, dn);
        timed(0, 2, grid_work(), [&] { return adr::launch_scatter<double, double>(0, sargs(fam[0].s64), fam[0].v64, Uh64, d32, partial, dn, st); });
        line64(1, slot, Uh64, dn);
        timed(0, 3, grid_work(), [&] { return adr::launch_scatter<double, double>(mode, sargs(fam[1].s64), fam[1].v64, U_out, d32, partial, dn, st); });
    }
    // One symmetric step of the march: beta substep over dt/2 (slot kSlotHalf),
    // gamma substep over dt (kSlotTime), beta substep over dt/2, each writing
    // the state in place (a line solve has gathered its input before its
    // scatter runs).
    void strang_step(double *U) {
        for (int half = 0; half < 2; ++half) {
            if (half == 1) {
                line64(1, kSlotTime, U, never);
                timed(0, 3, grid_work(), [&] { return adr::launch_scatter<double, double>(0, sargs(fam[1].s64), fam[1].v64, U, d32, partial, never, st); });
            }
            line64(0, kSlotHalf, U, never);
            timed(0, 2, grid_work(), [&] { return adr::launch_scatter<double, double>(0, sargs(fam[0].s64), fam[0].v64, U, d32, partial, never, st); });
        }
    }
    // out = T in (T the linear part of the FP64 sweep: no load, zero Dirichlet
    // data) on the interior nodes; in and out have zero outside the interior.
    void linear_sweep(const double *in, double *out, const int *dn) {
        line64(0, kSlotLin, in, dn);
        adr::ScatterArgs<double> s0 = sargs(fam[0].s64), s1 = sargs(fam[1].s64);
        s0.gb = nullptr;
        s1.gb = nullptr;
        timed(0, 2, grid_work(), [&] { return adr::launch_scatter<double, double>(0, s0, fam[0].v64, kWh, d32, partial, dn, st); });
        line64(1, kSlotLin, kWh, dn);
        timed(0, 3, grid_work(), [&] { return adr::launch_scatter<double, double>(0, s1, fam[1].v64, out, d32, partial, dn, st); });
    }
    // the GMRES work arrays for m basis steps (allocated once, grown on demand)
    void krylov_alloc(int m) {
        if (!kch.n) {
            const int64_t C = adr::krylov_chunk();
            std::vector<int> ci, ic(n_inst + 1, 0);
            std::vector<int64_t> cb, ce;
            for (int i = 0; i < n_inst; ++i) {
                ic[i] = static_cast<int>(ci.size());
                for (int64_t b = boff_h[i]; b < boff_h[i + 1]; b += C) {
                    ci.push_back(i);
                    cb.push_back(b);
                    ce.push_back(std::min(b + C, boff_h[i + 1]));
                }
            }
            ic[n_inst] = static_cast<int>(ci.size());
            kch = adr::KChunks{upload(ci, owned, st), upload(cb, owned, st), upload(ce, owned, st),
                               upload(ic, owned, st), static_cast<int>(ci.size()), n_inst};
            kWh = dalloc<double>(n_blocked, owned);
            HIPCHK(hipMemsetAsync(kWh, 0, sizeof(double) * n_blocked, st));
            kskip = dalloc<int>(n_inst, owned);
        }
        if (m + 1 > kmax) {
            // a larger basis replaces the smaller one
            HIPCHK(hipStreamSynchronize(st));
            for (void *q : {static_cast<void *>(kV), static_cast<void *>(kpart), static_cast<void *>(kout),
                            static_cast<void *>(kcoef)}) {
                if (!q) continue;
                owned.erase(std::remove(owned.begin(), owned.end(), q), owned.end());
                (void)hipFree(q);
            }
            kmax = m + 1;
            kV = dalloc<double>(static_cast<size_t>(kmax) * n_blocked, owned);
            HIPCHK(hipMemsetAsync(kV, 0, sizeof(double) * kmax * n_blocked, st));
            kpart = dalloc<double>(static_cast<size_t>(kch.n) * kmax, owned);
            kout = dalloc<double>(static_cast<size_t>(n_inst) * kmax, owned);
            kcoef = dalloc<double>(static_cast<size_t>(n_inst) * kmax, owned);
        }
    }
    // One FP32 increment sweep: d32 <- T d32, U += d32.
    void sweep32(double *U, const int *dn) {
        line32(0, kSlotLin, d32, dn);
        timed(1, 2, grid_work(), [&] { return adr::launch_scatter<float, float>(0, sargs(fam[0].s32), fam[0].v32, D32, nullptr, partial, dn, st); });
        line32(1, kSlotLin, D32, dn);
        timed(1, 3, grid_work(), [&] { return adr::launch_scatter<float, double>(2, sargs(fam[1].s32), fam[1].v32, U, d32, partial, dn, st); });
    }

    // Restricts the line and scatter launches to the instances not done (dn,
    // the host copy of the device flags `flags`, default the done flags): the
    // lists are compacted on the device from the flags, their lengths counted
    // here.  The kernels still test their flags, so instances that finish later
    // are skipped as before.  A launch's workgroups then all carry work.
    void compact(const std::vector<int> &dn, const int *flags = nullptr) {
        if (!flags) flags = done;
        if (act_blocks >= 0 ? dn == act_set : std::none_of(dn.begin(), dn.end(), [](int v) { return v != 0; }))
            return;  // unchanged set
        int nb = 0;
        int64_t ng = 0;
        for (int i = 0; i < n_inst; ++i)
            if (!dn[i]) {
                nb += inst_blocks[i];
                ng += inst_grid[i];
            }
        HIPCHK(adr::launch_compact(blk_inst_d, n_blocks, flags, cscan, blist, ccount, st));
        act_set = dn;
        act_blocks = nb;
        act_grid = ng;
        for (int f = 0; f < 2; ++f) {
            DevFam &F = fam[f];
            int nl = 0, nm = 0;
            int64_t nu = 0;
            int bl[adr::kLineBuckets] = {};
            for (int b = 0; b < adr::kLineBuckets; ++b) F.abnmax[b] = 0;
            for (int i = 0; i < n_inst; ++i)
                if (!dn[i]) {
                    nl += F.inst_lines[i];
                    nu += F.inst_unk[i];
                    nm = std::max(nm, F.inst_nmax[i]);
                    for (int b = 0; b < adr::kLineBuckets; ++b) {
                        bl[b] += F.inst_bl[i][b];
                        F.abnmax[b] = std::max(F.abnmax[b], F.inst_bnmax[i][b]);
                    }
                }
            HIPCHK(adr::launch_compact(F.a64.linst, F.n_lines, flags, cscan, F.lidx, ccount, st));
            F.act = nl;
            F.act_nmax = nm;
            F.act_unk = nu;
            // the compaction keeps the list order, so the buckets stay contiguous ranges
            F.abstart[0] = 0;
            for (int b = 0; b < adr::kLineBuckets; ++b) F.abstart[b + 1] = F.abstart[b] + bl[b];
        }
    }
    void uncompact() {
        act_blocks = -1;
        fam[0].act = fam[1].act = -1;
    }
    // ADR_ESINGULAR with the flagged instances named, or ADR_OK (synchronises)
    adr_status singular_status() {
        std::vector<int> sg_h(n_inst, 0);
        HIPCHK(hipMemcpyAsync(sg_h.data(), sing, sizeof(int) * n_inst, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        std::string which;
        int cnt = 0;
        for (int i = 0; i < n_inst; ++i)
            if (sg_h[i]) {
                if (cnt < 8) which += (cnt ? ", " : "") + std::to_string(i);
                ++cnt;
            }
        if (!cnt) return ADR_OK;
        err = "a line solve met a pivot below the threshold or not finite in " + std::to_string(cnt) +
              " instance(s): " + which + (cnt > 8 ? ", ..." : "");
        return ADR_ESINGULAR;
    }
    void norm(int count, double tol, int mode) {
        timed(0, 4, 0, [&] {
            return adr::launch_norm(n_inst, partial, blk_start, cnorm, rel, done, conv_it, count, tol, mode, st);
        });
    }

    // One sweep of eq. (10) with the direct transfer: the beta-lines take their
    // input from the gamma-curve values, the gamma-lines from the beta-curve
    // values (in place into fam[1].v64, with the per-line update sums; with
    // keep_d the update also goes to fam[1].v32 as the first FP32 increment).
    void direct_sweep(const int *dn, bool keep_d) {
        timed(0, 0, line_work(0), [&] {
            return lines<double>(0, fam[0].a64d, fam[1].v64, fam[0].v64, par_ptr(kSlotStep, 0), dn);
        });
        adr::LineArgs<double> g = fam[1].a64d;
        if (keep_d) g.dout = fam[1].v32;
        timed(0, 1, line_work(1), [&] {
            return lines<double>(1, g, fam[0].v64, fam[1].v64, par_ptr(kSlotStep, 1), dn);
        });
    }
    // One FP32 increment sweep with the direct transfer: d <- T d on the curve
    // values (fam[f].v32), the gamma increments added to the FP64 state (or,
    // with sum32, to the FP32 sum of the grid route's direct increments).
    void direct_sweep32(const int *dn, float *sum32 = nullptr) {
        timed(1, 0, line_work(0), [&] {
            return lines<float>(0, fam[0].a32d, fam[1].v32, fam[0].v32, par_ptr(kSlotLin, 0), dn);
        });
        adr::LineArgs<float> g = fam[1].a32d;
        if (sum32) g.vacc32 = sum32;
        else g.vacc = fam[1].v64;
        timed(1, 1, line_work(1), [&] {
            return lines<float>(1, g, fam[0].v32, fam[1].v32, par_ptr(kSlotLin, 1), dn);
        });
    }
    void direct_norm(int count, double tol, int mode) {
        timed(0, 4, 0, [&] {
            return adr::launch_norm(n_inst, lpart, inst_lstart, cnorm_d, rel, done, conv_it,
                                    count, tol, mode, st);
        });
    }

    // the caller's row-major state in and out of the blocked state Ub (interior nodes)
    void to_blocked(const double *u) { HIPCHK(adr::launch_layout(slot_rm, slot_b, npad, u, Ub, true, st)); }
    void from_blocked(double *u) { HIPCHK(adr::launch_layout(slot_rm, slot_b, npad, Ub, u, false, st)); }

    // one block of the stationary iteration: FP32 increment sweeps, then an FP64
    // sweep with the update norm (the first block has no FP32 sweeps)
    void block(double *u, int fp32_sweeps, double tol) {
        if (hsum && opt.increments == 1 && fp32_sweeps > 0) {
            hybrid_increments(u, fp32_sweeps);
        } else {
            for (int k = 0; k < fp32_sweeps; ++k) sweep32(u, done);
        }
        sweep64(kSlotStep, u, u, 1, done);
        norm(fp32_sweeps + 1, tol, 0);
    }
    // The block's m FP32 increments with the direct transfer (options.increments
    // = 1): the last FP64 update d (d32) gathered onto the gamma-curves, m direct
    // increment sweeps v <- T v summed into S (FP32, zero at the curve ends),
    // then one scatter U += P_G S (the FP32 increment scatter).  The increments
    // only steer the iterate: the FP64 grid-route sweeps fix the limit and
    // measure the residual.  Timed as FP32 classes 2 (the gather) and 3 (the
    // scatter).
    void hybrid_increments(double *u, int m) {
        DevFam &G = fam[1];
        adr::LineArgs<float> a = largs(G, G.a32);
        a.gend = nullptr;
        const int nl = G.act >= 0 ? G.act : G.n_lines;
        timed(1, 2, line_work(1), [&] { return adr::launch_line_values32(a, nl, d32, G.v32, hsum, st); });
        for (int q = 0; q < m; ++q) direct_sweep32(done, hsum);
        timed(1, 3, grid_work(), [&] {
            return adr::launch_scatter<float, double>(2, sargs(G.s32), hsum, u, d32, partial, done, st);
        });
    }

    // Adaptive schedule: after each FP64 sweep the per-instance rel is
    // read with the done flags; an unfinished instance whose rel fell from r0
    // (sweep k0) to r (sweep k) is expected to reach tol after
    // ceil(log(tol / r) / log(rho)) more sweeps, rho = (r / r0)^(1 / (k - k0)).
    // The next block ends on the earliest such sweep (at most fp32_sweeps FP32
    // sweeps; at least half of that while several instances run, so that one
    // instance about to finish does not cut every block short).
    template <typename AllDone, typename Run>
    void adaptive_blocks(double *ub, int max_iters, double tol, std::vector<int> &dn, AllDone &&all_done, Run &&run,
                         bool may_compact) {
        const int mmax = opt.fp32_sweeps;
        std::vector<double> rel_h(n_inst, 0.0), r0(n_inst, -1.0);
        std::vector<int> k0(n_inst, 0);
        auto read_rel = [&]() {
            HIPCHK(hipMemcpyAsync(rel_h.data(), rel, sizeof(double) * n_inst, hipMemcpyDeviceToHost, st));
        };
        int k = 1;  // the first FP64 sweep has run
        read_rel();
        if (all_done()) return;  // synchronises (rel_h is valid too)
        for (int i = 0; i < n_inst; ++i) { r0[i] = rel_h[i]; k0[i] = k; }
        int m = std::min(mmax, max_iters - k - 1);
        while (m >= 0 && k + m + 1 <= max_iters) {
            run(m);
            k += m + 1;
            read_rel();
            if (all_done()) return;
            if (may_compact && n_inst > 1) compact(dn);
            int target = k + mmax + 1, active = 0;
            for (int i = 0; i < n_inst; ++i) {
                if (dn[i]) continue;
                ++active;
                const double r = rel_h[i];
                if (tol > 0.0 && r > 0.0 && r0[i] > r && std::isfinite(r)) {
                    const double rho = std::pow(r / r0[i], 1.0 / (k - k0[i]));
                    const double more = std::ceil(std::log(tol / r) / std::log(rho));
                    if (rho > 0.0 && rho < 1.0 && more >= 0.0 && more < 1e6)
                        target = std::min(target, k + static_cast<int>(more));
                }
                r0[i] = r;
                k0[i] = k;
            }
            const int lo = active > 1 ? mmax / 2 : 0;
            m = std::min(std::max(lo, std::min(mmax, target - k - 1)), max_iters - k - 1);
        }
    }

    // captured graphs of whole blocks (m FP32 sweeps, an FP64 sweep, the norm),
    // one per block length m, captured on first use and replayed; all are
    // dropped when the state pointer, tol or the line launches change
    struct GBlock {
        hipGraph_t g = nullptr;
        hipGraphExec_t x = nullptr;
    };
    std::map<int, GBlock> gblocks;
    const double *g_u = nullptr;
    double g_tol = -1.0;
    int g_split = -1;  // the line launches (options.split_lines) of the captured graphs
    int g_inc = -1;    // and their increment sweeps (options.increments)
    hipStream_t cap = nullptr;
    // concurrent bucket launches (options.split_lines == 2): two more streams of
    // the default priority, forked from and joined back into st by events
    hipStream_t side[2] = {nullptr, nullptr};
    hipEvent_t fork_ev = nullptr, join_ev[2] = {nullptr, nullptr};
    void drop_graph() {
        for (auto &kv : gblocks) {
            if (kv.second.x) (void)hipGraphExecDestroy(kv.second.x);
            if (kv.second.g) (void)hipGraphDestroy(kv.second.g);
        }
        gblocks.clear();
    }
    // one block replayed from its graph (captured now if new) on st, the
    // capture stream; the launch lists must be the full ones (not compacted)
    void graph_block(double *ub, int m, double tol) {
        if (g_u != ub || g_tol != tol || g_split != opt.split_lines || g_inc != opt.increments) {
            drop_graph();
            g_u = ub;
            g_tol = tol;
            g_split = opt.split_lines;
            g_inc = opt.increments;
        }
        auto it = gblocks.find(m);
        if (it == gblocks.end()) {
            GBlock b;
            HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            try {
                block(ub, m, tol);
            } catch (...) {
                // leave no capture open on the stream
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(st, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            HIPCHK(hipStreamEndCapture(st, &b.g));
            const hipError_t e = hipGraphInstantiate(&b.x, b.g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(b.g);
                HIPCHK(e);
            }
            it = gblocks.emplace(m, b).first;
        }
        HIPCHK(hipGraphLaunch(it->second.x, st));
    }

};

namespace {

void fill_params(std::vector<double> &ph, int n_inst, int slot, const std::vector<double> &mu,
                 const std::vector<double> &sg, double theta, double dt) {
    for (int f = 0; f < 2; ++f)
        for (int i = 0; i < n_inst; ++i) {
            double *p = ph.data() + ((static_cast<size_t>(slot) * 2 + f) * n_inst + i) * 8;
            std::fill(p, p + 8, 0.0);
            if (slot == kSlotGuess) {
                if (f == 0) { p[0] = sg[i]; p[1] = mu[i]; p[2] = 1.0; p[6] = 1.0; p[7] = 1.0; }
                continue;
            }
            // p[7]: the sweep carries the state, so the curve ends take the
            // Dirichlet data (the increment sweeps carry zero there)
            p[7] = slot == kSlotLin ? 0.0 : 1.0;
            const double td = theta * dt, ed = (1.0 - theta) * dt;
            if (f == 0) {
                p[0] = 1.0 + td * sg[i]; p[1] = td * mu[i]; p[2] = td;
                p[3] = 1.0 - ed * sg[i]; p[4] = -ed * mu[i]; p[5] = -ed;
                p[6] = slot == kSlotLin ? 0.0 : dt;
            } else {
                p[0] = 1.0; p[1] = td * mu[i]; p[2] = 0.0;
                p[3] = 1.0; p[4] = -ed * mu[i]; p[5] = 0.0; p[6] = 0.0;
            }
        }
}

adr_status fail_ctx(adr_ctx *c, const Error &e) {
    if (c) c->err = e.msg;
    return e.code;
}

}  // namespace

extern "C" {

adr_status adr_setup(const adr_problem *probs, int32_t n_probs, const adr_options *opt, adr_ctx **out) {
    if (!out) return ADR_EINVAL;
    *out = nullptr;
    std::unique_ptr<adr_ctx> C(new adr_ctx);
    try {
        if (!probs || n_probs <= 0 || !opt) throw Error{ADR_EINVAL, "probs, n_probs > 0 and opt are required"};
        if (!(opt->theta > 0.0 && opt->theta <= 1.0)) throw Error{ADR_EINVAL, "theta must be in (0, 1]"};
        if (!(opt->dt > 0.0) || !std::isfinite(opt->dt)) throw Error{ADR_EINVAL, "dt must be > 0"};
        if (opt->precision != ADR_PREC_FP64 && opt->precision != ADR_PREC_FP32_LINES)
            throw Error{ADR_EINVAL, "unknown precision"};
        if (opt->splitting != 0 && opt->splitting != 1) throw Error{ADR_EINVAL, "splitting must be 0 or 1"};
        if (opt->stabilize != 0 && opt->stabilize != 1) throw Error{ADR_EINVAL, "stabilize must be 0 or 1"};
        if (opt->krylov < 0 || opt->krylov > 200) throw Error{ADR_EINVAL, "krylov must be in 0..200"};
        if (opt->transfer != 0 && opt->transfer != 1) throw Error{ADR_EINVAL, "transfer must be 0 or 1"};
        if (opt->transfer == 1 && opt->krylov != 0)
            throw Error{ADR_EINVAL, "krylov applies to the grid transfer (transfer = 0)"};
        if (opt->increments != 0 && opt->increments != 1) throw Error{ADR_EINVAL, "increments must be 0 or 1"};
        if (opt->fp32_sweeps < 0) throw Error{ADR_EINVAL, "fp32_sweeps must be >= 0"};
        C->opt = *opt;
        C->n_inst = n_probs;
        C->st = static_cast<hipStream_t>(opt->stream);
        const int n = n_probs;

        // host geometry, instances in parallel.  Instances that share the grid,
        // the domain and the beta arrays (same pointers) share their curves:
        // they are traced once and only the load vector is rebuilt.
        std::vector<adr::InstanceGeo> G(n);
        std::vector<Error> errs(n, Error{ADR_OK, ""});
        std::vector<int> rep(n);
        {
            std::map<std::vector<double>, int> first;
            for (int i = 0; i < n; ++i) {
                const adr_problem &p = probs[i];
                std::vector<double> key = {double(p.nx), double(p.ny), p.a, p.b, p.c, p.d, double(p.domain),
                                           double(reinterpret_cast<uintptr_t>(p.beta1)),
                                           double(reinterpret_cast<uintptr_t>(p.beta2)),
                                           double(reinterpret_cast<uintptr_t>(p.beta1 ? nullptr : p.psi)),
                                           double(reinterpret_cast<uintptr_t>(p.g))};
                for (int k = 0; k < p.n_dom_params && p.dom_params; ++k) key.push_back(p.dom_params[k]);
                auto it = first.find(key);
                if (it == first.end()) { first.emplace(key, i); rep[i] = i; }
                else rep[i] = it->second;
            }
        }
        auto run_pool = [&](auto &&work) {
            unsigned nt = std::max(1u, std::min<unsigned>(std::thread::hardware_concurrency(), 16u));
            nt = std::min<unsigned>(nt, static_cast<unsigned>(n));
            std::atomic<int> next{0};
            std::vector<std::thread> pool;
            for (unsigned t = 0; t < nt; ++t)
                pool.emplace_back([&] {
                    for (int i = next++; i < n; i = next++) {
                        try {
                            work(i);
                        } catch (const Error &e) {
                            errs[i] = e;
                        } catch (const std::bad_alloc &) {
                            errs[i] = Error{ADR_ENOMEM, "host allocation failed"};
                        }
                    }
                });
            for (auto &th : pool) th.join();
        };
        run_pool([&](int i) { if (rep[i] == i) adr::build_instance(probs[i], G[i]); });
        for (int i = 0; i < n; ++i)
            if (errs[rep[i]].code != ADR_OK && rep[i] != i) errs[i] = errs[rep[i]];
        run_pool([&](int i) {
            if (rep[i] != i && errs[rep[i]].code == ADR_OK) adr::rebuild_for_source(G[rep[i]], probs[i], G[i]);
        });
        for (int i = 0; i < n; ++i)
            if (errs[i].code != ADR_OK)
                throw Error{errs[i].code, "instance " + std::to_string(i) + ": " + errs[i].msg};
        const bool direct_recs = opt->transfer == 1 || opt->increments == 1;
        if (direct_recs) {
            run_pool([&](int i) {
                adr::build_direct(G[i].g, G[i].fam[0], G[i].hk[0], G[i].fam[1], G[i].drec[0]);
                adr::build_direct(G[i].g, G[i].fam[1], G[i].hk[1], G[i].fam[0], G[i].drec[1]);
            });
            for (int i = 0; i < n; ++i)
                if (errs[i].code != ADR_OK)
                    throw Error{errs[i].code, "instance " + std::to_string(i) + ": " + errs[i].msg};
        }

        if (opt->host_only) {
            C->goff.assign(n + 1, 0);
            for (int i = 0; i < n; ++i) {
                C->goff[i + 1] = C->goff[i] + static_cast<int64_t>(G[i].g.nx) * G[i].g.ny;
                C->n_unknowns += static_cast<int64_t>(G[i].inner_list.size());
                for (int f = 0; f < 2; ++f) {
                    const adr::Family &fa = G[i].fam[f];
                    C->fam[f].n_lines += static_cast<int>(fa.off.size()) - 1;
                    C->fam[f].n_nodes += static_cast<int64_t>(fa.x.size());
                    C->fam[f].n_unknowns += static_cast<int64_t>(fa.x.size()) - 2 * (static_cast<int64_t>(fa.off.size()) - 1);
                    C->geo[f].push_back(fa);
                }
            }
            C->host_geo = std::move(G);
            *out = C.release();
            return ADR_OK;
        }

        // packing
        C->goff.assign(n + 1, 0);
        std::vector<double> mu(n), sg(n);
        for (int i = 0; i < n; ++i) {
            C->goff[i + 1] = C->goff[i] + static_cast<int64_t>(G[i].g.nx) * G[i].g.ny;
            mu[i] = G[i].mu;
            sg[i] = G[i].sigma;
        }
        C->n_grid = C->goff[n];
        if (C->n_grid > (int64_t(1) << 31) - 1) throw Error{ADR_EINVAL, "packed grid exceeds 2^31 nodes"};
        // blocked layout of the sweep fields: 8 x 4-node blocks per instance
        std::vector<int64_t> boff(n + 1, 0);
        std::vector<int> inst_bstride(n);
        for (int i = 0; i < n; ++i) {
            const int nx8 = (G[i].g.nx + 7) / 8, ny4 = (G[i].g.ny + 3) / 4;
            boff[i + 1] = boff[i] + int64_t(32) * nx8 * ny4;
            inst_bstride[i] = 32 * nx8;
        }
        C->n_blocked = boff[n];
        C->boff_h = boff;
        if (C->n_blocked > (int64_t(1) << 31) - 1) throw Error{ADR_EINVAL, "packed grid exceeds 2^31 nodes"};
        hipStream_t st = C->st;
        auto &own = C->owned;
        C->inst_bstride = upload(inst_bstride, own, st);
        bool any_g = false;
        for (int i = 0; i < n; ++i) any_g = any_g || probs[i].g != nullptr;
        C->sing = dalloc<int>(n, own);
        HIPCHK(hipMemsetAsync(C->sing, 0, sizeof(int) * n, st));

        // scatter slots, padded per instance to whole blocks
        std::vector<int> blk_start(n + 1, 0);
        for (int i = 0; i < n; ++i)
            blk_start[i + 1] = blk_start[i] + static_cast<int>((G[i].inner_list.size() + kBlock - 1) / kBlock);
        const int nblk = blk_start[n];
        const int npad = nblk * kBlock;
        C->n_blocks = nblk;
        // slot order: 16 x 16 tiles of the grid (row-major inside a tile), so that
        // a wavefront's nodes are a compact patch whose crossing records come
        // from few curves (cache-line reuse of the line values)
        std::vector<std::vector<int>> order(n);
        for (int i = 0; i < n; ++i) {
            const int nxi = G[i].g.nx;
            std::vector<int> &o = order[i];
            o.resize(G[i].inner_list.size());
            for (size_t s = 0; s < o.size(); ++s) o[s] = static_cast<int>(s);
            auto key = [&](int s) {
                const int g = G[i].inner_list[s], gi = g % nxi, gj = g / nxi;
                return std::make_tuple(gj / kTile, gi / kTile, gj % kTile, gi % kTile);
            };
            std::stable_sort(o.begin(), o.end(), [&](int a, int b) { return key(a) < key(b); });
        }
        std::vector<int> gidx(npad, -1), gidx_b(npad, -1), blk_inst(nblk);
        for (int i = 0; i < n; ++i) {
            const int nxi = G[i].g.nx;
            for (int b = blk_start[i]; b < blk_start[i + 1]; ++b) blk_inst[b] = i;
            for (size_t s = 0; s < order[i].size(); ++s) {
                const int g = G[i].inner_list[order[i][s]];
                gidx[blk_start[i] * kBlock + s] = static_cast<int>(C->goff[i] + g);
                gidx_b[blk_start[i] * kBlock + s] =
                    adr::blocked_index(g % nxi, g / nxi, static_cast<int>(boff[i]), inst_bstride[i]);
            }
            C->n_unknowns += static_cast<int64_t>(G[i].inner_list.size());
        }
        C->inst_grid.resize(n);
        for (int i = 0; i < n; ++i) C->inst_grid[i] = static_cast<int64_t>(G[i].inner_list.size());
        C->slot_rm = upload(gidx, own, st);
        int *d_gidx = upload(gidx_b, own, st);
        C->slot_b = d_gidx;
        C->npad = npad;
        int *d_blk_inst = upload(blk_inst, own, st);
        C->blk_start = upload(blk_start, own, st);
        C->blk_inst_d = d_blk_inst;
        C->inst_blocks.resize(n);
        for (int i = 0; i < n; ++i) C->inst_blocks[i] = blk_start[i + 1] - blk_start[i];
        C->blist = dalloc<int>(std::max(nblk, 1), own);
        HIPCHK(hipMemsetAsync(C->blist, 0, sizeof(int) * std::max(nblk, 1), st));  // valid indices from the start

        // node offsets of each family's instances (the direct records of one
        // family index the other's nodes)
        std::vector<int64_t> noffs[2];
        for (int f = 0; f < 2; ++f) {
            noffs[f].assign(n + 1, 0);
            for (int i = 0; i < n; ++i) noffs[f][i + 1] = noffs[f][i] + static_cast<int64_t>(G[i].fam[f].x.size());
        }
        for (int f = 0; f < 2; ++f) {
            DevFam &F = C->fam[f];
            std::vector<int64_t> noff(n + 1, 0);
            std::vector<std::pair<int, int>> lines;  // (instance, local line)
            for (int i = 0; i < n; ++i) {
                const adr::Family &fa = G[i].fam[f];
                noff[i + 1] = noff[i] + static_cast<int64_t>(fa.x.size());
                for (size_t l = 0; l + 1 < fa.off.size(); ++l) lines.emplace_back(i, static_cast<int>(l));
            }
            F.n_nodes = noff[n];
            if (F.n_nodes > (int64_t(1) << 31) - 2) throw Error{ADR_EINVAL, "too many line nodes"};
            F.n_lines = static_cast<int>(lines.size());
            for (auto &li : lines) {
                const adr::Family &fa = G[li.first].fam[f];
                const int64_t cnt = fa.off[li.second + 1] - fa.off[li.second];
                if (cnt > kMaxNodes)
                    throw Error{ADR_EINVAL, "a curve has " + std::to_string(cnt) + " nodes; the line solver holds " +
                                                std::to_string(kMaxNodes)};
            }
            // list order: length bucket (longest first), then instance, then curve
            // length (longest first): the order of the bucketed launches and of
            // lists compacted to the unfinished instances.  In a batch each bucket
            // holds the instances one after another, so that a chunk of
            // neighbouring positions (one XCD's, see k_line_b) holds one
            // instance's curves
            std::stable_sort(lines.begin(), lines.end(), [&](const std::pair<int, int> &x, const std::pair<int, int> &y) {
                const adr::Family &fx = G[x.first].fam[f], &fy = G[y.first].fam[f];
                const int nx = static_cast<int>(fx.off[x.second + 1] - fx.off[x.second]);
                const int ny = static_cast<int>(fy.off[y.second + 1] - fy.off[y.second]);
                const int bx = adr::line_bucket(nx), by = adr::line_bucket(ny);
                if (bx != by) return bx < by;
                if (x.first != y.first) return x.first < y.first;
                return nx > ny;
            });
            std::vector<int> loff, lcnt, linst;
            std::vector<double> gend;  // per list position: the Dirichlet data at the two ends
            loff.reserve(lines.size());
            F.inst_lines.assign(n, 0);
            F.inst_nmax.assign(n, 0);
            F.inst_unk.assign(n, 0);
            F.inst_bl.assign(n, {});
            F.inst_bnmax.assign(n, {});
            int bcount[adr::kLineBuckets] = {};
            F.lidx = dalloc<int>(std::max(F.n_lines, 1), own);
            HIPCHK(hipMemsetAsync(F.lidx, 0, sizeof(int) * std::max(F.n_lines, 1), st));
            for (auto &li : lines) {
                const adr::Family &fa = G[li.first].fam[f];
                const int cnt = static_cast<int>(fa.off[li.second + 1] - fa.off[li.second]);
                loff.push_back(static_cast<int>(noff[li.first] + fa.off[li.second]));
                lcnt.push_back(cnt);
                linst.push_back(li.first);
                gend.push_back(G[li.first].gend[f][2 * li.second]);
                gend.push_back(G[li.first].gend[f][2 * li.second + 1]);
                F.nmax = std::max(F.nmax, cnt);
                F.inst_lines[li.first] += 1;
                F.inst_unk[li.first] += cnt - 2;
                F.inst_nmax[li.first] = std::max(F.inst_nmax[li.first], cnt);
                F.n_unknowns += cnt - 2;
                const int b = adr::line_bucket(cnt);
                bcount[b] += 1;
                F.bnmax[b] = std::max(F.bnmax[b], cnt);
                F.inst_bl[li.first][b] += 1;
                F.inst_bnmax[li.first][b] = std::max(F.inst_bnmax[li.first][b], cnt);
            }
            F.bstart[0] = 0;
            for (int b = 0; b < adr::kLineBuckets; ++b) F.bstart[b + 1] = F.bstart[b] + bcount[b];
            {
                // dispatch of the single launch: the curves in their own order
                // (instance, then seeds along the inflow boundary, so
                // neighbours), cut into chunks of adr::kXcdChunk, chunk c to XCD c mod 8
                std::vector<int> nat(lines.size());
                for (size_t p = 0; p < nat.size(); ++p) nat[p] = static_cast<int>(p);
                std::sort(nat.begin(), nat.end(), [&](int x, int y) { return lines[x] < lines[y]; });
                const int nl = static_cast<int>(nat.size());
                const int nch = (nl + adr::kXcdChunk - 1) / adr::kXcdChunk;
                std::vector<int> sp, xs(9, 0);
                sp.reserve(nat.size());
                for (int x = 0; x < 8; ++x) {
                    xs[x] = static_cast<int>(sp.size());
                    for (int c = x; c < nch; c += 8)
                        for (int q = c * adr::kXcdChunk; q < std::min(nl, (c + 1) * adr::kXcdChunk); ++q) sp.push_back(nat[q]);
                }
                xs[8] = static_cast<int>(sp.size());
                int most = 0;
                for (int x = 0; x < 8; ++x) most = std::max(most, xs[x + 1] - xs[x]);
                F.sidx = upload(sp, own, st);
                F.xs = upload(xs, own, st);
                F.xgrid = 8 * most;
            }
            if (F.nmax > kMaxNodes || adr::line_lds_bytes<double>(f, F.nmax) > kLdsLimit)
                throw Error{ADR_EINVAL, "a curve has " + std::to_string(F.nmax) +
                                            " nodes: longer than the LDS-resident line solver holds"};
            // per node data (cellb: the cell's corner in the blocked fields)
            std::vector<int> cellb(F.n_nodes, -1);
            std::vector<double> lx(F.n_nodes), ly(F.n_nodes), h(F.n_nodes), w, L;
            if (f == 0) { w.resize(F.n_nodes); L.resize(F.n_nodes); }
            for (int i = 0; i < n; ++i) {
                const adr::Family &fa = G[i].fam[f];
                for (size_t k = 0; k < fa.x.size(); ++k) {
                    const int64_t gk = noff[i] + static_cast<int64_t>(k);
                    const int c = G[i].cellk[f][k];
                    if (c >= 0) {
                        const int nx = G[i].g.nx;
                        cellb[gk] = adr::blocked_index(c % nx, c / nx, static_cast<int>(boff[i]), inst_bstride[i]);
                    }
                    lx[gk] = G[i].lxk[f][k];
                    ly[gk] = G[i].lyk[f][k];
                    h[gk] = G[i].hk[f][k];
                    if (f == 0) { w[gk] = G[i].wk[k]; L[gk] = G[i].Lk[k]; }
                }
            }
            if (f == 0) C->noffB = noff;
            const int *d_loff = upload(loff, own, st), *d_lcnt = upload(lcnt, own, st);
            const int *d_linst = upload(linst, own, st), *d_cellb = upload(cellb, own, st);
            double *dL64 = f == 0 ? upload(L, own, st) : nullptr;
            float *dL32 = f == 0 ? upload(to_type<float>(L), own, st) : nullptr;
            if (f == 0) { C->L64 = dL64; C->L32 = dL32; C->L64base = upload(L, own, st); }
            F.a64 = adr::LineArgs<double>{d_loff, d_lcnt, d_linst, C->inst_bstride, d_cellb,
                                          upload(lx, own, st), upload(ly, own, st), upload(h, own, st),
                                          f == 0 ? upload(w, own, st) : nullptr, dL64};
            F.a32 = adr::LineArgs<float>{d_loff, d_lcnt, d_linst, C->inst_bstride, d_cellb,
                                         upload(to_type<float>(lx), own, st), upload(to_type<float>(ly), own, st),
                                         upload(to_type<float>(h), own, st),
                                         f == 0 ? upload(to_type<float>(w), own, st) : nullptr, dL32};
            // Dirichlet data (FP64 state sweeps only; the FP32 sweeps carry increments)
            F.a64.gend = any_g ? upload(gend, own, st) : nullptr;
            F.a64.sing = C->sing;
            F.a32.sing = C->sing;
            F.a64.ptol = opt->pivot_tol > 0.0 ? opt->pivot_tol : 64.0 * 2.220446049250313e-16;
            if (f == 0 && opt->stabilize) {
                // per node: |beta|_e h_e of the element ending there, |beta|_e the mean of its ends
                C->fit_wlh.assign(static_cast<size_t>(F.n_nodes), 0.0);
                for (int i = 0; i < n; ++i) {
                    const adr::Family &fa = G[i].fam[0];
                    for (size_t l = 0; l + 1 < fa.off.size(); ++l)
                        for (int64_t k = fa.off[l] + 1; k < fa.off[l + 1]; ++k) {
                            const double wl = 0.5 * (G[i].wk[static_cast<size_t>(k)] + G[i].wk[static_cast<size_t>(k - 1)]);
                            C->fit_wlh[static_cast<size_t>(noff[i] + k)] = wl * G[i].hk[0][static_cast<size_t>(k)];
                        }
                }
                C->phi64 = dalloc<double>(static_cast<size_t>(F.n_nodes), own);
                C->phi32 = dalloc<float>(static_cast<size_t>(F.n_nodes), own);
                C->fill_phi(mu);
                F.a64.phi = C->phi64;
                F.a32.phi = C->phi32;
            }
            F.a32.ptol = opt->pivot_tol > 0.0 ? opt->pivot_tol : 64.0 * 1.1920928955078125e-07;
            if (direct_recs) {
                // direct-transfer records: source nodes in the other family's packed numbering
                std::vector<int> dk(2 * static_cast<size_t>(F.n_nodes), -1);
                std::vector<double> dw(4 * static_cast<size_t>(F.n_nodes), 0.0);
                for (int i = 0; i < n; ++i) {
                    const std::vector<adr::DirRec> &D = G[i].drec[f];
                    for (size_t k = 0; k < D.size(); ++k) {
                        const size_t gk = static_cast<size_t>(noff[i]) + k;
                        for (int e = 0; e < 2; ++e)
                            dk[2 * gk + e] = D[k].k[e] < 0 ? -1 : static_cast<int>(noffs[1 - f][i] + D[k].k[e]);
                        for (int e = 0; e < 4; ++e) dw[4 * gk + e] = D[k].w[e];
                    }
                }
                F.a64d = F.a64;
                F.a64d.dk = reinterpret_cast<const int2 *>(upload(dk, own, st));
                F.a64d.dw = upload(dw, own, st);
                // FP32 increment sweeps: the records packed into 10 bytes per node
                std::vector<int32_t> dk0(static_cast<size_t>(F.n_nodes), -1);
                std::vector<int16_t> dkd(static_cast<size_t>(F.n_nodes), adr::kDirNoRight);
                std::vector<uint32_t> dwp(static_cast<size_t>(F.n_nodes), 0u);
                for (int i = 0; i < n; ++i) {
                    const std::vector<adr::DirRec> &D = G[i].drec[f];
                    for (size_t k = 0; k < D.size(); ++k) {
                        const size_t gk = static_cast<size_t>(noff[i]) + k;
                        pack_direct(D[k], noffs[1 - f][i], dk0[gk], dkd[gk], dwp[gk]);
                    }
                }
                F.a32d = F.a32;
                F.a32d.dk = F.a64d.dk;  // the escapes' full records (and the direct mode's flag)
                F.a32d.dk0 = upload(dk0, own, st);
                F.a32d.dkd = reinterpret_cast<const short *>(upload(dkd, own, st));
                F.a32d.dwp = upload(dwp, own, st);
                if (f == 1) {
                    // update sums of the gamma-curves, grouped by instance in list order
                    std::vector<int> start(n + 1, 0), slot(F.n_lines);
                    for (int i = 0; i < n; ++i) start[i + 1] = start[i] + F.inst_lines[i];
                    std::vector<int> next(start.begin(), start.end() - 1);
                    for (int l = 0; l < F.n_lines; ++l) slot[l] = next[linst[l]]++;
                    C->inst_lstart = upload(start, own, st);
                    C->lpart = dalloc<double>(std::max(F.n_lines, 1), own);
                    F.a64d.lpart = C->lpart;
                    F.a64d.lslot = upload(slot, own, st);
                }
            }
            // scatter records
            std::vector<int> rk(4 * static_cast<size_t>(npad), -1);
            std::vector<double> rf(6 * static_cast<size_t>(npad), 0.0);  // FP64 factors
            std::vector<double> gb(any_g ? npad : 0, 0.0);
            // FP32 tables: the stencil's factors, quantised (weights to ~3e-5)
            std::vector<unsigned> sw(npad, 0u), rt(2 * static_cast<size_t>(npad), 0u);
            auto q16 = [](double v) { return static_cast<unsigned>(std::lround(std::min(std::max(v, 0.0), 1.0) * 65535.0)); };
            auto q15 = [](double v) { return static_cast<unsigned>(std::lround(std::min(std::max(v, 0.0), 1.0) * 32767.0)); };
            for (int i = 0; i < n; ++i)
                for (size_t s = 0; s < order[i].size(); ++s) {
                    const size_t slot = static_cast<size_t>(blk_start[i]) * kBlock + s;
                    const adr::Rec4 &R = G[i].rec[f][order[i][s]];
                    if (any_g) gb[slot] = R.gb;
                    const unsigned wcode = R.wh == 0.0 ? 0u : (R.wh == 0.5 ? 1u : 2u);
                    sw[slot] = wcode | (q15(R.lam[0]) << 2) | (q15(R.lam[1]) << 17);
                    rt[slot] = q16(R.t[0]) | (q16(R.t[1]) << 16);
                    rt[static_cast<size_t>(npad) + slot] = q16(R.t[2]) | (q16(R.t[3]) << 16);
                    rf[slot] = R.lam[0];
                    rf[static_cast<size_t>(npad) + slot] = R.lam[1];
                    for (int r = 0; r < 4; ++r) {
                        rk[r * static_cast<size_t>(npad) + slot] = R.k[r] < 0 ? -1 : static_cast<int>(noff[i] + R.k[r]);
                        rf[(2 + r) * static_cast<size_t>(npad) + slot] = R.t[r];
                    }
                }
            const int *d_rk = upload(rk, own, st);
            // compact form: the first record's node and 16-bit offsets of the others
            std::vector<int> rk0(npad, -1);
            std::vector<short> rd(3 * static_cast<size_t>(npad), adr::kRecMissing);
            for (size_t slot = 0; slot < static_cast<size_t>(npad); ++slot) {
                const int k0 = rk[slot];
                rk0[slot] = k0;
                for (int r = 1; r < 4; ++r) {
                    const int kr = rk[r * static_cast<size_t>(npad) + slot];
                    short &d = rd[(r - 1) * static_cast<size_t>(npad) + slot];
                    if (kr < 0) d = adr::kRecMissing;
                    else if (k0 >= 0 && std::abs(static_cast<int64_t>(kr) - k0) <= adr::kRecMaxDelta)
                        d = static_cast<short>(kr - k0);
                    else d = adr::kRecEscape;
                }
            }
            const int *d_rk0 = upload(rk0, own, st);
            const short *d_rd = upload(rd, own, st);
            const unsigned *d_sw = upload(sw, own, st);
            F.s64 = adr::ScatterArgs<double>{d_gidx, d_blk_inst, d_rk, d_rk0, d_rd, d_sw, nullptr,
                                             upload(rf, own, st), npad};
            F.s64.gb = any_g ? upload(gb, own, st) : nullptr;
            F.s32 = adr::ScatterArgs<float>{d_gidx, d_blk_inst, d_rk, d_rk0, d_rd, d_sw, upload(rt, own, st),
                                            nullptr, npad};
            F.v64 = dalloc<double>(F.n_nodes, own);
            F.v32 = dalloc<float>(F.n_nodes, own);
            if (f == 1 && opt->increments == 1 && opt->transfer == 0) C->hsum = dalloc<float>(F.n_nodes, own);
            for (int i = 0; i < n; ++i) C->geo[f].push_back(G[i].fam[f]);
        }

        for (int i = 0; i < n; ++i) {
            C->grids.push_back(G[i].g);
            adr_problem sh = probs[i];
            sh.beta1 = sh.beta2 = sh.f = sh.g = sh.psi = nullptr;
            sh.dom_params = nullptr;
            C->shape.push_back(sh);
        }
        // state scratch: non-interior nodes of the state fields hold the
        // Dirichlet data (never written later), of the increment fields zero
        C->Ub = dalloc<double>(C->n_blocked, own);
        C->Uh64 = dalloc<double>(C->n_blocked, own);
        C->Z64 = dalloc<double>(C->n_blocked, own);
        C->d32 = dalloc<float>(C->n_blocked, own);
        C->D32 = dalloc<float>(C->n_blocked, own);
        if (any_g) {
            std::vector<double> bf(C->n_blocked, 0.0);
            for (int i = 0; i < n; ++i) {
                if (!probs[i].g) continue;
                const int nxi = G[i].g.nx, nyi = G[i].g.ny;
                for (int j = 0; j < nyi; ++j)
                    for (int x = 0; x < nxi; ++x)
                        if (!G[i].inner[static_cast<size_t>(j) * nxi + x])
                            bf[adr::blocked_index(x, j, static_cast<int>(boff[i]), inst_bstride[i])] =
                                probs[i].g[static_cast<size_t>(j) * nxi + x];
            }
            for (double *fld : {C->Ub, C->Uh64, C->Z64})
                HIPCHK(hipMemcpyAsync(fld, bf.data(), sizeof(double) * C->n_blocked, hipMemcpyHostToDevice, st));
            HIPCHK(hipStreamSynchronize(st));  // bf leaves scope
        } else {
            HIPCHK(hipMemsetAsync(C->Ub, 0, sizeof(double) * C->n_blocked, st));
            HIPCHK(hipMemsetAsync(C->Uh64, 0, sizeof(double) * C->n_blocked, st));
            HIPCHK(hipMemsetAsync(C->Z64, 0, sizeof(double) * C->n_blocked, st));
        }
        HIPCHK(hipMemsetAsync(C->d32, 0, sizeof(float) * C->n_blocked, st));
        HIPCHK(hipMemsetAsync(C->D32, 0, sizeof(float) * C->n_blocked, st));
        C->partial = dalloc<double>(std::max(nblk, 1), own);
        {
            const int most = std::max({nblk, C->fam[0].n_lines, C->fam[1].n_lines});
            C->cscan = dalloc<int>((most + 255) / 256 + 1, own);
            C->ccount = dalloc<int>(1, own);
        }
        C->cnorm = dalloc<double>(n, own);
        C->cnorm_d = dalloc<double>(n, own);
        C->rel = dalloc<double>(n, own);
        C->rel_fb = dalloc<double>(n, own);
        C->done = dalloc<int>(n, own);
        C->never = dalloc<int>(n, own);
        C->conv_it = dalloc<int>(n, own);
        HIPCHK(hipMemsetAsync(C->never, 0, sizeof(int) * n, st));
        HIPCHK(hipMemsetAsync(C->done, 0, sizeof(int) * n, st));

        C->par_h.assign(static_cast<size_t>(kSlots) * 2 * n * 8, 0.0);
        fill_params(C->par_h, n, kSlotStep, mu, sg, opt->theta, opt->dt);
        fill_params(C->par_h, n, kSlotLin, mu, sg, opt->theta, opt->dt);
        fill_params(C->par_h, n, kSlotGuess, mu, sg, 1.0, 1.0);
        C->par = upload(C->par_h, own, st);
        C->mu = mu;
        C->sg = sg;

        // |Phi(0)| per instance: one FP64 sweep from zero
        C->sweep64(kSlotStep, C->Z64, C->Z64, 3, C->never);
        C->norm(0, 0.0, 1);
        HIPCHK(hipStreamSynchronize(st));
        C->collect_ticks();
        for (auto &r : C->ms) for (auto &v : r) v = 0.0;
        for (auto &r : C->cnt) for (auto &v : r) v = 0;
    } catch (const Error &e) {
        g_setup_error = e.msg;
        for (void *p : C->owned) (void)hipFree(p);
        C->owned.clear();
        return e.code;
    } catch (const std::bad_alloc &) {
        g_setup_error = "host allocation failed";
        for (void *p : C->owned) (void)hipFree(p);
        C->owned.clear();
        return ADR_ENOMEM;
    }
    *out = C.release();
    return ADR_OK;
}

adr_status adr_layout(const adr_ctx *ctx, int64_t *offsets) {
    if (!ctx || !offsets) return ADR_EINVAL;
    for (int i = 0; i <= ctx->n_inst; ++i) offsets[i] = ctx->goff[i];
    return ADR_OK;
}

adr_status adr_counts(const adr_ctx *ctx, int64_t *grid_unknowns, int64_t *lines_b, int64_t *lines_g,
                      int64_t *line_unknowns_b, int64_t *line_unknowns_g) {
    if (!ctx) return ADR_EINVAL;
    if (grid_unknowns) *grid_unknowns = ctx->n_unknowns;
    if (lines_b) *lines_b = ctx->fam[0].n_lines;
    if (lines_g) *lines_g = ctx->fam[1].n_lines;
    if (line_unknowns_b) *line_unknowns_b = ctx->fam[0].n_unknowns;
    if (line_unknowns_g) *line_unknowns_g = ctx->fam[1].n_unknowns;
    return ADR_OK;
}

adr_status adr_update(adr_ctx *ctx, const adr_problem *probs, int32_t n_probs) {
    if (!ctx || !probs) return ADR_EINVAL;
    if (ctx->opt.host_only || n_probs != ctx->n_inst) {
        ctx->err = "adr_update needs the set-up's instance count on a device context";
        return ADR_EINVAL;
    }
    ctx->cnorm_d_valid = false;
    try {
        const int n = ctx->n_inst;
        for (int i = 0; i < n; ++i) {
            const adr_problem &p = probs[i], &q = ctx->shape[i];
            if (p.nx != q.nx || p.ny != q.ny || p.a != q.a || p.b != q.b || p.c != q.c || p.d != q.d ||
                p.domain != q.domain)
                throw Error{ADR_EINVAL, "instance " + std::to_string(i) + ": grid or domain differs from the set-up"};
            if (!(p.mu > 0.0) || !(p.sigma >= 0.0) || !p.f)
                throw Error{ADR_EINVAL, "instance " + std::to_string(i) + ": mu > 0, sigma >= 0 and f are required"};
            const size_t nn = static_cast<size_t>(p.nx) * p.ny;
            for (size_t k = 0; k < nn; ++k)
                if (!std::isfinite(p.f[k])) throw Error{ADR_ENONFINITE, "non-finite f"};
        }
        const int64_t nB = ctx->fam[0].n_nodes;
        std::vector<double> L(nB, 0.0);
        {
            std::atomic<int> next{0};
            unsigned nt = std::max(1u, std::min<unsigned>(std::thread::hardware_concurrency(), 16u));
            nt = std::min<unsigned>(nt, static_cast<unsigned>(n));
            std::vector<std::thread> pool;
            for (unsigned t = 0; t < nt; ++t)
                pool.emplace_back([&] {
                    std::vector<double> Li;
                    for (int i = next++; i < n; i = next++) {
                        adr::load_from_positions(ctx->grids[i], ctx->geo[0][i], probs[i].f, Li);
                        std::copy(Li.begin(), Li.end(), L.begin() + ctx->noffB[i]);
                    }
                });
            for (auto &th : pool) th.join();
        }
        HIPCHK(hipStreamSynchronize(ctx->st));
        HIPCHK(hipMemcpy(ctx->L64, L.data(), sizeof(double) * nB, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(ctx->L64base, L.data(), sizeof(double) * nB, hipMemcpyHostToDevice));
        std::vector<float> L32(L.begin(), L.end());
        HIPCHK(hipMemcpy(ctx->L32, L32.data(), sizeof(float) * nB, hipMemcpyHostToDevice));
        for (int i = 0; i < n; ++i) {
            ctx->mu[i] = probs[i].mu;
            ctx->sg[i] = probs[i].sigma;
        }
        if (ctx->phi64) ctx->fill_phi(ctx->mu);
        fill_params(ctx->par_h, n, kSlotStep, ctx->mu, ctx->sg, ctx->opt.theta, ctx->opt.dt);
        fill_params(ctx->par_h, n, kSlotLin, ctx->mu, ctx->sg, ctx->opt.theta, ctx->opt.dt);
        fill_params(ctx->par_h, n, kSlotGuess, ctx->mu, ctx->sg, 1.0, 1.0);
        HIPCHK(hipMemcpy(ctx->par, ctx->par_h.data(), sizeof(double) * ctx->par_h.size(), hipMemcpyHostToDevice));
        ctx->last_theta = -1.0;  // the time-step slot is refilled on its next use
        ctx->sweep64(kSlotStep, ctx->Z64, ctx->Z64, 3, ctx->never);
        ctx->norm(0, 0.0, 1);
        HIPCHK(hipStreamSynchronize(ctx->st));
        return ADR_OK;
    } catch (const Error &e) {
        return fail_ctx(ctx, e);
    }
}

// GMRES(m) on (I - T) U = c, c = Phi(0): the stationary fixed point by a Krylov
// route (options.krylov = m).  FP64 throughout: every application of I - T is a
// linear FP64 sweep; each cycle starts from the exact residual r = Phi(U) - U
// (one FP64 sweep), whose relative norm is the iteration's stopping measure.
// Per instance its own Krylov space; the Hessenberg columns and Givens
// rotations are kept on the host (two small reads per basis step).
static adr_status krylov_iterate(adr_ctx *ctx, double *u, int32_t max_iters, double tol, int32_t *iters,
                                 double *rel_res) {
    const int n = ctx->n_inst, m = ctx->opt.krylov;
    hipStream_t st = ctx->st;
    ctx->krylov_alloc(m);
    const int K = ctx->kmax;
    const int64_t stride = ctx->n_blocked;
    double *V = ctx->kV;
    auto Vp = [&](int j) { return V + static_cast<int64_t>(j) * stride; };
    std::vector<double> cn(n), out(static_cast<size_t>(n) * K), coef(static_cast<size_t>(n) * K, 0.0);
    HIPCHK(hipMemcpyAsync(cn.data(), ctx->cnorm, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    HIPCHK(adr::launch_fill_int(ctx->done, 0, n, st));
    HIPCHK(adr::launch_fill_int(ctx->sing, 0, n, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<int> dn(n, 0), skip(n, 0), sweeps(n, 0), steps(n, 0);
    std::vector<double> rel(n, NAN);
    auto read_out = [&]() {
        HIPCHK(hipMemcpyAsync(out.data(), ctx->kout, sizeof(double) * n * K, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
    };
    auto put = [&](int *dflag, const std::vector<int> &h) {
        HIPCHK(hipMemcpyAsync(dflag, h.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
    };
    auto put_coef = [&]() {
        HIPCHK(hipMemcpyAsync(ctx->kcoef, coef.data(), sizeof(double) * n * K, hipMemcpyHostToDevice, st));
    };
    // per instance: H (K x m, column-major), rotations, right-hand side g
    std::vector<double> H(static_cast<size_t>(n) * K * m), cs(static_cast<size_t>(n) * m), sn(cs.size()),
        g(static_cast<size_t>(n) * K);
    ctx->to_blocked(u);
    while (true) {
        // exact residual r = Phi(U) - U into V_0; rel = |r| / |Phi(0)|
        if (n > 1) ctx->compact(dn);
        ctx->sweep64(kSlotStep, ctx->Ub, Vp(0), 0, ctx->done);
        HIPCHK(adr::launch_kresidual(ctx->slot_b, ctx->npad, Vp(0), ctx->Ub, Vp(0), st));
        HIPCHK(adr::launch_kdot(Vp(0), Vp(0), stride, 1, K, ctx->kch, ctx->done, ctx->kpart, ctx->kout, st));
        read_out();
        bool all = true;
        for (int i = 0; i < n; ++i) {
            if (dn[i]) continue;
            ++sweeps[i];
            const double r = std::sqrt(out[static_cast<size_t>(i) * K]);
            rel[i] = r / (cn[i] > 0.0 ? cn[i] : 1.0);
            if (rel[i] <= tol || !std::isfinite(rel[i]) || sweeps[i] >= max_iters) dn[i] = 1;
            else {
                all = false;
                coef[static_cast<size_t>(i) * K] = 1.0 / r;  // scale of V_0
                g[static_cast<size_t>(i) * K] = r;
            }
            skip[i] = dn[i];
            steps[i] = 0;
        }
        put(ctx->done, dn);
        put(ctx->kskip, skip);
        if (all) break;
        put_coef();
        HIPCHK(adr::launch_kscale(Vp(0), ctx->kcoef, K, ctx->kch, ctx->kskip, st));
        for (int j = 0; j < m; ++j) {
            // z = T V_j into V_{j+1}; h_ij = delta_ij - (T V_j, V_i)
            if (n > 1) ctx->compact(skip, ctx->kskip);
            ctx->linear_sweep(Vp(j), Vp(j + 1), ctx->kskip);
            HIPCHK(adr::launch_kdot(Vp(j + 1), V, stride, j + 1, K, ctx->kch, ctx->kskip, ctx->kpart, ctx->kout, st));
            read_out();
            for (int i = 0; i < n; ++i) {
                if (skip[i]) continue;
                ++sweeps[i];
                double *h = &H[(static_cast<size_t>(i) * m + j) * K];
                for (int q = 0; q <= j; ++q) {
                    h[q] = (q == j ? 1.0 : 0.0) - out[static_cast<size_t>(i) * K + q];
                    coef[static_cast<size_t>(i) * K + q] = h[q];
                }
            }
            put_coef();
            // w = V_j - T V_j - sum h_ij V_i (in V_{j+1}); |w| = h_{j+1,j}
            HIPCHK(adr::launch_kupdate(Vp(j + 1), V, stride, j, j + 1, K, ctx->kcoef, ctx->kch, ctx->kskip,
                                       ctx->kpart, ctx->kout, st));
            read_out();
            bool any = false;
            for (int i = 0; i < n; ++i) {
                if (skip[i]) continue;
                double *h = &H[(static_cast<size_t>(i) * m + j) * K];
                double *c_ = &cs[static_cast<size_t>(i) * m], *s_ = &sn[static_cast<size_t>(i) * m];
                double *gi = &g[static_cast<size_t>(i) * K];
                const double hn = std::sqrt(out[static_cast<size_t>(i) * K]);
                h[j + 1] = hn;
                coef[static_cast<size_t>(i) * K] = hn > 0.0 ? 1.0 / hn : 0.0;
                for (int q = 0; q < j; ++q) {  // earlier rotations on the new column
                    const double t = c_[q] * h[q] + s_[q] * h[q + 1];
                    h[q + 1] = -s_[q] * h[q] + c_[q] * h[q + 1];
                    h[q] = t;
                }
                const double den = std::hypot(h[j], h[j + 1]);
                c_[j] = den > 0.0 ? h[j] / den : 1.0;
                s_[j] = den > 0.0 ? h[j + 1] / den : 0.0;
                h[j] = den;
                h[j + 1] = 0.0;
                gi[j + 1] = -s_[j] * gi[j];
                gi[j] = c_[j] * gi[j];
                steps[i] = j + 1;
                const double est = std::fabs(gi[j + 1]) / (cn[i] > 0.0 ? cn[i] : 1.0);
                // this instance's cycle ends once its estimate reaches tol (or its sweeps run out)
                if (est <= tol || hn == 0.0 || sweeps[i] + 1 >= max_iters) skip[i] = 1;
                else any = true;
            }
            put_coef();
            HIPCHK(adr::launch_kscale(Vp(j + 1), ctx->kcoef, K, ctx->kch, ctx->kskip, st));
            put(ctx->kskip, skip);
            if (!any) break;
        }
        // U += sum_q y_q V_q, y from the triangular H y = g of each instance's cycle
        std::fill(coef.begin(), coef.end(), 0.0);
        for (int i = 0; i < n; ++i) {
            if (dn[i]) continue;
            const int k = steps[i];
            double *y = &coef[static_cast<size_t>(i) * K];
            for (int q = k - 1; q >= 0; --q) {
                double acc = g[static_cast<size_t>(i) * K + q];
                for (int t = q + 1; t < k; ++t) acc -= H[(static_cast<size_t>(i) * m + t) * K + q] * y[t];
                const double d = H[(static_cast<size_t>(i) * m + q) * K + q];
                y[q] = d != 0.0 ? acc / d : 0.0;
            }
        }
        put_coef();
        HIPCHK(adr::launch_kcombine(ctx->Ub, V, stride, m, K, ctx->kcoef, ctx->kch, ctx->done, st));
    }
    ctx->uncompact();
    ctx->from_blocked(u);
    const adr_status sst = ctx->singular_status();
    adr_status status = ADR_OK;
    for (int i = 0; i < n; ++i) {
        if (iters) iters[i] = sweeps[i];
        if (rel_res) rel_res[i] = rel[i];
        if (!std::isfinite(rel[i])) status = ADR_ENONFINITE;
        else if (!(rel[i] <= tol) && status == ADR_OK) status = ADR_ENOTCONV;
    }
    if (sst != ADR_OK) return sst;
    if (status == ADR_ENONFINITE) ctx->err = "non-finite residual";
    return status;
}

// The stationary iteration with the interpolation-free transfer: the state is
// the gamma-curve values (fam[1].v64).  The start is the bilinear gather of u
// onto the gamma-curves; an instance stops at the first FP64 sweep whose
// update |v' - v| over its interior gamma nodes is <= tol |Phi(0)| (Phi(0):
// the sweep from zero interior values).  FP64 precision: every sweep FP64, the
// done flags read every kDirectCheck sweeps.  FP32_LINES: the FP64 sweep also
// keeps its update as an FP32 increment d, and fp32_sweeps FP32 sweeps
// d <- T d (each adding d to the state) precede every further FP64 sweep
// (the block lengths chosen as in the grid route's adaptive schedule when
// options.adaptive).  The launch lists follow the unfinished instances.  u
// receives the scatter of the last gamma values (Sec. 6).
constexpr int kDirectCheck = 4;
static adr_status direct_iterate(adr_ctx *ctx, double *u, int32_t max_iters, double tol, int32_t *iters,
                                 double *rel_res) {
    const int n = ctx->n_inst;
    hipStream_t st = ctx->st;
    DevFam &FG = ctx->fam[1];
    HIPCHK(adr::launch_fill_int(ctx->done, 0, n, st));
    HIPCHK(adr::launch_fill_int(ctx->conv_it, 0, n, st));
    HIPCHK(adr::launch_fill_int(ctx->sing, 0, n, st));
    if (!ctx->cnorm_d_valid) {
        HIPCHK(adr::launch_line_values(FG.a64d, FG.n_lines, nullptr, FG.v64, st));
        ctx->direct_sweep(ctx->never, false);
        ctx->direct_norm(0, 0.0, 1);
        ctx->cnorm_d_valid = true;
    }
    ctx->to_blocked(u);
    HIPCHK(adr::launch_line_values(FG.a64d, FG.n_lines, ctx->Ub, FG.v64, st));
    std::vector<int> dn(n, 0);
    auto all_done = [&]() {
        HIPCHK(hipMemcpyAsync(dn.data(), ctx->done, sizeof(int) * n, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return std::all_of(dn.begin(), dn.end(), [](int v) { return v != 0; });
    };
    const bool fp32 = ctx->opt.precision == ADR_PREC_FP32_LINES;
    if (!fp32) {
        int k = 0;
        while (k < max_iters) {
            const int m = std::min(kDirectCheck, max_iters - k);
            for (int q = 0; q < m; ++q) {
                ctx->direct_sweep(ctx->done, false);
                ctx->direct_norm(1, tol, 0);
            }
            k += m;
            if (all_done()) break;
            if (n > 1) ctx->compact(dn);
        }
    } else if (max_iters > 0) {
        // a block: m FP32 increment sweeps, then the FP64 sweep and its norm
        auto run = [&](int m) {
            for (int q = 0; q < m; ++q) ctx->direct_sweep32(ctx->done);
            ctx->direct_sweep(ctx->done, true);
            ctx->direct_norm(m + 1, tol, 0);
        };
        run(0);
        if (ctx->opt.adaptive) {
            ctx->adaptive_blocks(ctx->Ub, max_iters, tol, dn, all_done, run, true);
        } else {
            const int m = ctx->opt.fp32_sweeps, period = m + 1;
            const int blocks = (max_iters - 1) / period;
            const int check = std::max(1, 8 / period);
            for (int b = 0; b < blocks; ++b) {
                run(m);
                if ((b + 1) % check == 0) {
                    if (all_done()) break;
                    if (n > 1) ctx->compact(dn);
                }
            }
        }
        all_done();
    }
    ctx->uncompact();
    HIPCHK((adr::launch_scatter<double, double>(0, FG.s64, FG.v64, ctx->Ub, ctx->d32, ctx->partial, ctx->never, st)));
    ctx->from_blocked(u);
    std::vector<int> ci(n, 0);
    std::vector<double> rr(n, 0.0);
    HIPCHK(hipMemcpyAsync(ci.data(), ctx->conv_it, sizeof(int) * n, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(rr.data(), ctx->rel, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const adr_status sst = ctx->singular_status();
    adr_status status = ADR_OK;
    for (int i = 0; i < n; ++i) {
        if (iters) iters[i] = ci[i];
        if (rel_res) rel_res[i] = max_iters > 0 ? rr[i] : NAN;
        if (max_iters > 0 && !std::isfinite(rr[i])) status = ADR_ENONFINITE;
        else if (!dn[i] && status == ADR_OK) status = ADR_ENOTCONV;
    }
    if (sst != ADR_OK) return sst;
    if (status == ADR_ENONFINITE) ctx->err = "non-finite residual";
    return status;
}

// The stationary iteration; with a fallback start, the start u is judged by
// the first sweep (see adr_split_iterate_judged).
static adr_status split_iterate(adr_ctx *ctx, double *u, const double *fallback, int32_t max_iters, double tol,
                                int32_t *iters, double *rel_res, int32_t *used_fallback) {
    if (ctx->opt.transfer == 1) {
        if (fallback)
            return fail_ctx(ctx, Error{ADR_EINVAL, "the judged solve runs on the grid transfer (transfer = 0)"});
        try {
            return direct_iterate(ctx, u, max_iters, tol, iters, rel_res);
        } catch (const Error &e) {
            ctx->uncompact();
            return fail_ctx(ctx, e);
        }
    }
    if (ctx->opt.krylov > 0 && !fallback && max_iters > 0) {
        try {
            return krylov_iterate(ctx, u, max_iters, tol, iters, rel_res);
        } catch (const Error &e) {
            return fail_ctx(ctx, e);
        }
    }
    try {
        const int n = ctx->n_inst;
        hipStream_t user = ctx->st;
        const bool use_graph = ctx->opt.graph != 0 && !ctx->opt.timing;
        if (use_graph) {
            // run on the context's own stream (capturable), ordered after the caller's work
            if (!ctx->cap) HIPCHK(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
            hipEvent_t ev;
            HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
            HIPCHK(hipEventRecord(ev, user));
            HIPCHK(hipStreamWaitEvent(ctx->cap, ev, 0));
            HIPCHK(hipEventDestroy(ev));
            ctx->st = ctx->cap;
        }
        hipStream_t st = ctx->st;
        const bool fp32 = ctx->opt.precision == ADR_PREC_FP32_LINES;
        const int m = fp32 ? ctx->opt.fp32_sweeps : 0;
        const int period = m + 1;
        HIPCHK(adr::launch_fill_int(ctx->done, 0, n, st));
        HIPCHK(adr::launch_fill_int(ctx->conv_it, 0, n, st));
        HIPCHK(adr::launch_fill_int(ctx->sing, 0, n, st));
        std::vector<int> dn(n, 0);
        auto all_done = [&]() {
            HIPCHK(hipMemcpyAsync(dn.data(), ctx->done, sizeof(int) * n, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            return std::all_of(dn.begin(), dn.end(), [](int v) { return v != 0; });
        };
        double *const ub = ctx->Ub;
        if (fallback) {
            // the fallback's residual, kept aside: an FP64 sweep that leaves the state alone
            ctx->to_blocked(fallback);
            ctx->sweep64(kSlotStep, ub, ub, 3, ctx->never);
            ctx->norm(0, 0.0, 2);
            HIPCHK(hipMemcpyAsync(ctx->rel_fb, ctx->rel, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        }
        ctx->to_blocked(u);
        if (max_iters > 0) {
            ctx->block(ub, 0, tol);  // first FP64 sweep
            if (fallback) {
                // its update is the start's residual: an instance whose residual is
                // not below the fallback's (or not finite) restarts from the fallback
                std::vector<double> rn(n), rf(n);
                HIPCHK(hipMemcpyAsync(rn.data(), ctx->rel, sizeof(double) * n, hipMemcpyDeviceToHost, st));
                HIPCHK(hipMemcpyAsync(rf.data(), ctx->rel_fb, sizeof(double) * n, hipMemcpyDeviceToHost, st));
                HIPCHK(hipMemcpyAsync(dn.data(), ctx->done, sizeof(int) * n, hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
                bool any = false;
                for (int i = 0; i < n; ++i) {
                    const bool back = !(rn[i] < rf[i]);
                    if (used_fallback) used_fallback[i] = back ? 1 : 0;
                    if (back) {
                        any = true;
                        dn[i] = 0;
                    }
                }
                if (any) {
                    ctx->from_blocked(u);  // u = Phi(start) on every instance
                    for (int i = 0; i < n; ++i)
                        if (used_fallback ? used_fallback[i] : !(rn[i] < rf[i]))
                            HIPCHK(hipMemcpyAsync(u + ctx->goff[i], fallback + ctx->goff[i],
                                                  sizeof(double) * (ctx->goff[i + 1] - ctx->goff[i]),
                                                  hipMemcpyDeviceToDevice, st));
                    ctx->to_blocked(u);
                    HIPCHK(hipMemcpyAsync(ctx->done, dn.data(), sizeof(int) * n, hipMemcpyHostToDevice, st));
                    // one more first sweep: from the fallback where restarted, a second
                    // sweep for the other unfinished instances
                    ctx->block(ub, 0, tol);
                }
            }
            const int blocks = (max_iters - 1) / period;
            const int check = std::max(1, 8 / period);
            // a block: replayed from its captured graph (full launch lists), or
            // eager launches that follow the compacted lists of the active instances
            auto run = [&](int mb) {
                if (use_graph) ctx->graph_block(ub, mb, tol);
                else ctx->block(ub, mb, tol);
            };
            if (fp32 && ctx->opt.adaptive) {
                ctx->adaptive_blocks(ub, max_iters, tol, dn, all_done, run, !use_graph);
            } else {
                for (int b = 0; b < blocks; ++b) {
                    run(m);
                    if ((b + 1) % check == 0) {
                        if (all_done()) break;
                        // the graph's launches are fixed; eager launches follow the active set
                        if (!use_graph && n > 1) ctx->compact(dn);
                    }
                }
            }
        }
        ctx->uncompact();
        ctx->from_blocked(u);
        std::vector<int> ci(n, 0);
        std::vector<double> rr(n, 0.0);
        HIPCHK(hipMemcpyAsync(dn.data(), ctx->done, sizeof(int) * n, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(ci.data(), ctx->conv_it, sizeof(int) * n, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(rr.data(), ctx->rel, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        const adr_status sst = ctx->singular_status();
        if (use_graph) ctx->st = user;
        adr_status status = ADR_OK;
        for (int i = 0; i < n; ++i) {
            if (iters) iters[i] = ci[i];
            if (rel_res) rel_res[i] = max_iters > 0 ? rr[i] : NAN;
            if (max_iters > 0 && !std::isfinite(rr[i])) status = ADR_ENONFINITE;
            else if (!dn[i] && status == ADR_OK) status = ADR_ENOTCONV;
        }
        if (sst != ADR_OK) return sst;
        if (status == ADR_ENONFINITE) ctx->err = "non-finite residual";
        return status;
    } catch (const Error &e) {
        ctx->uncompact();
        if (ctx->opt.graph) ctx->st = static_cast<hipStream_t>(ctx->opt.stream);
        return fail_ctx(ctx, e);
    }
}

adr_status adr_split_iterate(adr_ctx *ctx, double *u, int32_t max_iters, double tol, int32_t *iters,
                             double *rel_res) {
    if (!ctx) return ADR_EINVAL;
    if (!u || max_iters < 0 || !(tol >= 0.0)) {
        ctx->err = "u, max_iters >= 0 and tol >= 0 are required";
        return ADR_EINVAL;
    }
    return split_iterate(ctx, u, nullptr, max_iters, tol, iters, rel_res, nullptr);
}

adr_status adr_split_iterate_judged(adr_ctx *ctx, double *u, const double *fallback, int32_t max_iters, double tol,
                                    int32_t *iters, double *rel_res, int32_t *used_fallback) {
    if (!ctx) return ADR_EINVAL;
    if (!u || !fallback || max_iters < 1 || !(tol >= 0.0) || ctx->opt.host_only) {
        ctx->err = "u, fallback, max_iters >= 1, tol >= 0 and a device context are required";
        return ADR_EINVAL;
    }
    return split_iterate(ctx, u, fallback, max_iters, tol, iters, rel_res, used_fallback);
}

adr_status adr_autotune(adr_ctx *ctx, double *work, int32_t max_iters, double tol, int32_t *best_fp32_sweeps,
                        int32_t *best_adaptive, double *best_ms, int32_t *best_split, int32_t *best_shapes,
                        int32_t *best_krylov, int32_t *best_increments) {
    if (!ctx) return ADR_EINVAL;
    if (!work || max_iters < 1 || !(tol >= 0.0) || ctx->opt.precision != ADR_PREC_FP32_LINES) {
        ctx->err = "adr_autotune needs work, max_iters >= 1, tol >= 0 and FP32_LINES precision";
        return ADR_EINVAL;
    }
    // (FP32 sweeps per FP64 sweep or their maximum, adaptive)
    static const int kCand[][2] = {{2, 0}, {3, 0}, {4, 0}, {6, 0}, {6, 1}, {8, 1}, {12, 1}, {16, 1}, {24, 1}};
    const int32_t saved = ctx->opt.fp32_sweeps, saved_ad = ctx->opt.adaptive, saved_split = ctx->opt.split_lines;
    const int32_t saved_kr = ctx->opt.krylov, saved_inc = ctx->opt.increments;
    ctx->opt.krylov = 0;
    // the increment kinds to try: the grid route's, and the direct transfer's
    // when the context holds its records (set up with increments = 1)
    const int n_inc = ctx->hsum ? 2 : 1;
    const size_t nbytes = sizeof(double) * static_cast<size_t>(ctx->goff.back());
    auto restore = [&]() {
        ctx->opt.fp32_sweeps = saved;
        ctx->opt.adaptive = saved_ad;
        ctx->opt.split_lines = saved_split;
        ctx->opt.krylov = saved_kr;
        ctx->opt.increments = saved_inc;
        ctx->drop_graph();
    };
    // one timed solve from zero (the second of two runs: the first also
    // captures the graph in graph mode); ms < 0 on a device error
    auto time_solve = [&](double &ms) -> adr_status {
        ms = INFINITY;
        for (int rep = 0; rep < 2; ++rep) {
            if (hipMemsetAsync(work, 0, nbytes, ctx->st) != hipSuccess || hipStreamSynchronize(ctx->st) != hipSuccess) {
                ctx->err = "adr_autotune: device error";
                return ADR_EDEVICE;
            }
            const auto t0 = std::chrono::steady_clock::now();
            const adr_status st = adr_split_iterate(ctx, work, max_iters, tol, nullptr, nullptr);
            ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
            if (st != ADR_OK && st != ADR_ENOTCONV) return st;
        }
        return ADR_OK;
    };
    // 1. the line launches (one, or one per length bucket) under the current schedule
    int split = saved_split;
    {
        double best_t = INFINITY;
        for (int sp = 0; sp < 3; ++sp) {
            ctx->opt.split_lines = sp;
            double t;
            const adr_status st = time_solve(t);
            if (st != ADR_OK) {
                restore();
                return st;
            }
            if (t < best_t) {
                best_t = t;
                split = sp;
            }
        }
        ctx->opt.split_lines = split;
    }
    // 1b. with bucketed launches: each bucket's workgroup shape, from its FP32
    //     line solves timed alone (both families, the bucket's curves of every instance)
    if (split) {
        try {
            for (int b = 0; b < adr::kLineBuckets; ++b) {
                const int ns = adr::line_shapes(b);
                if (ns < 2 || (ctx->fam[0].bstart[b + 1] == ctx->fam[0].bstart[b] &&
                               ctx->fam[1].bstart[b + 1] == ctx->fam[1].bstart[b]))
                    continue;
                int bs = 0;
                double bt = INFINITY;
                for (int sh = 0; sh < ns; ++sh) {
                    const double t = ctx->time_bucket(b, sh, 3);
                    if (t < bt) {
                        bt = t;
                        bs = sh;
                    }
                }
                ctx->fam[0].bshape[b] = ctx->fam[1].bshape[b] = bs;
            }
        } catch (const Error &e) {
            restore();
            return fail_ctx(ctx, e);
        }
        ctx->drop_graph();  // a graph captured in step 1 holds the launches of the old shapes
    }
    // 2. the FP32/FP64 sweep schedule and the kind of increments with those launches
    int best = saved, best_ad = saved_ad, best_inc = 0;
    double best_t = INFINITY;
    for (int inc = 0; inc < n_inc; ++inc)
        for (const auto &cand : kCand) {
            const int c = cand[0];
            ctx->opt.fp32_sweeps = c;
            ctx->opt.adaptive = cand[1];
            ctx->opt.increments = inc;
            double t;
            const adr_status st = time_solve(t);
            if (st != ADR_OK) {
                restore();
                return st;
            }
            if (t < best_t) {
                best_t = t;
                best = c;
                best_ad = cand[1];
                best_inc = inc;
            }
        }
    ctx->opt.fp32_sweeps = best;
    ctx->opt.adaptive = best_ad;
    ctx->opt.increments = best_inc;
    // 3. GMRES(m) on (I - T) U = c (FP64 sweeps) with those launches, against the best
    //    schedule (the grid transfer only)
    int best_kr = 0;
    for (int m : {10, 20, 30}) {
        if (ctx->opt.transfer != 0) break;
        ctx->opt.krylov = m;
        double t;
        const adr_status st = time_solve(t);
        if (st != ADR_OK) {
            restore();
            return st;
        }
        if (t < best_t) {
            best_t = t;
            best_kr = m;
        }
    }
    ctx->opt.krylov = best_kr;
    if (ctx->opt.timing)
        for (int prec = 0; prec < 2; ++prec) (void)adr_kernel_times(ctx, prec, nullptr, nullptr, nullptr, 1);
    if (best_fp32_sweeps) *best_fp32_sweeps = best;
    if (best_adaptive) *best_adaptive = best_ad;
    if (best_ms) *best_ms = best_t;
    if (best_split) *best_split = split;
    if (best_shapes)
        for (int b = 0; b < adr::kLineBuckets; ++b) best_shapes[b] = ctx->fam[0].bshape[b];
    if (best_krylov) *best_krylov = best_kr;
    if (best_increments) *best_increments = best_inc;
    return ADR_OK;
}

adr_status adr_set_graph(adr_ctx *ctx, int32_t on) {
    if (!ctx || ctx->opt.host_only) return ADR_EINVAL;
    ctx->opt.graph = on ? 1 : 0;
    ctx->drop_graph();
    return ADR_OK;
}

adr_status adr_set_line_shapes(adr_ctx *ctx, const int32_t *shapes) {
    if (!ctx) return ADR_EINVAL;
    if (!shapes || ctx->opt.host_only) {
        ctx->err = "shapes and a device context are required";
        return ADR_EINVAL;
    }
    for (int b = 0; b < adr::kLineBuckets; ++b)
        if (shapes[b] < 0 || shapes[b] >= adr::line_shapes(b)) {
            ctx->err = "bucket " + std::to_string(b) + " has " + std::to_string(adr::line_shapes(b)) + " shapes";
            return ADR_EINVAL;
        }
    for (int b = 0; b < adr::kLineBuckets; ++b) ctx->fam[0].bshape[b] = ctx->fam[1].bshape[b] = shapes[b];
    ctx->drop_graph();  // a captured block holds the old launches
    return ADR_OK;
}

// Converged implicit Euler steps: each step (u - u_n)/dt + A u = f is the
// stationary problem with sigma + 1/dt and the beta-curves' load L + M G u_n/dt,
// solved by the stationary iteration (the context's pseudo step, schedule and
// launches) from u_n.  The stationary coefficients, loads and |Phi(0)| are
// restored afterwards.
static adr_status converged_steps(adr_ctx *ctx, double *u, double dt, int32_t nsteps, int32_t inner_max,
                                  double inner_tol, int32_t *inner_iters) {
    const int n = ctx->n_inst;
    const size_t nB = static_cast<size_t>(ctx->fam[0].n_nodes);
    auto set_sigma = [&](const std::vector<double> &sg) {
        fill_params(ctx->par_h, n, kSlotStep, ctx->mu, sg, ctx->opt.theta, ctx->opt.dt);
        fill_params(ctx->par_h, n, kSlotLin, ctx->mu, sg, ctx->opt.theta, ctx->opt.dt);
        HIPCHK(hipMemcpyAsync(ctx->par, ctx->par_h.data(), sizeof(double) * 2 * 2 * n * 8, hipMemcpyHostToDevice,
                              ctx->st));
        HIPCHK(hipStreamSynchronize(ctx->st));  // par_h is host memory the copy reads
    };
    auto restore = [&]() {
        set_sigma(ctx->sg);
        HIPCHK(hipMemcpyAsync(ctx->L64, ctx->L64base, sizeof(double) * nB, hipMemcpyDeviceToDevice, ctx->st));
        ctx->sweep64(kSlotStep, ctx->Z64, ctx->Z64, 3, ctx->never);
        ctx->norm(0, 0.0, 1);
        HIPCHK(hipStreamSynchronize(ctx->st));
    };
    std::vector<double> sg2(n);
    for (int i = 0; i < n; ++i) sg2[i] = ctx->sg[i] + 1.0 / dt;
    adr_status status = ADR_OK;
    try {
        set_sigma(sg2);
        std::vector<int32_t> it(n, 0);
        for (int s = 0; s < nsteps; ++s) {
            ctx->to_blocked(u);  // u_n
            HIPCHK(adr::launch_shift_load(ctx->fam[0].a64, ctx->fam[0].n_lines, ctx->fam[0].nmax, ctx->L64base,
                                          ctx->Ub, ctx->L64, 1.0 / dt, ctx->st));
            ctx->sweep64(kSlotStep, ctx->Z64, ctx->Z64, 3, ctx->never);  // |Phi(0)| of the step's problem
            ctx->norm(0, 0.0, 1);
            const adr_status st = split_iterate(ctx, u, nullptr, inner_max, inner_tol, it.data(), nullptr, nullptr);
            if (inner_iters)
                for (int i = 0; i < n; ++i) inner_iters[static_cast<size_t>(s) * n + i] = it[i];
            if (st < 0) {
                status = st;
                break;
            }
            if (st == ADR_ENOTCONV) status = ADR_ENOTCONV;
        }
        const std::string msg = ctx->err;
        restore();
        ctx->err = msg;
        return status;
    } catch (const Error &e) {
        try {
            restore();
        } catch (const Error &) {
        }
        return fail_ctx(ctx, e);
    }
}

adr_status adr_time_step(adr_ctx *ctx, double *u, double theta, double dt, int32_t nsteps, int32_t inner_max,
                         double inner_tol, int32_t *inner_iters) {
    if (!ctx) return ADR_EINVAL;
    if (!u || nsteps < 0 || !(theta > 0.0 && theta <= 1.0) || !(dt > 0.0) || inner_max < 0) {
        ctx->err = "u, nsteps >= 0, theta in (0,1], dt > 0 and inner_max >= 0 are required";
        return ADR_EINVAL;
    }
    if (inner_max > 0 && theta != 1.0) {
        ctx->err = "the converged mode (inner_max > 0) is implicit Euler: theta = 1";
        return ADR_EINVAL;
    }
    if (inner_max > 0) return converged_steps(ctx, u, dt, nsteps, inner_max, inner_tol, inner_iters);
    try {
        if (theta != ctx->last_theta || dt != ctx->last_dt) {
            fill_params(ctx->par_h, ctx->n_inst, kSlotTime, ctx->mu, ctx->sg, theta, dt);
            fill_params(ctx->par_h, ctx->n_inst, kSlotHalf, ctx->mu, ctx->sg, theta, 0.5 * dt);
            for (int slot : {kSlotTime, kSlotHalf})
                HIPCHK(hipMemcpy(ctx->par + static_cast<size_t>(slot) * 2 * ctx->n_inst * 8,
                                 ctx->par_h.data() + static_cast<size_t>(slot) * 2 * ctx->n_inst * 8,
                                 sizeof(double) * 2 * ctx->n_inst * 8, hipMemcpyHostToDevice));
            ctx->last_theta = theta;
            ctx->last_dt = dt;
        }
        ctx->to_blocked(u);
        if (ctx->opt.splitting == 1) {
            for (int s = 0; s < nsteps; ++s) ctx->strang_step(ctx->Ub);
        } else {
            for (int s = 0; s < nsteps; ++s) ctx->sweep64(kSlotTime, ctx->Ub, ctx->Ub, 0, ctx->never);
        }
        ctx->from_blocked(u);
        return ADR_OK;
    } catch (const Error &e) {
        return fail_ctx(ctx, e);
    }
}

adr_status adr_residual(adr_ctx *ctx, const double *u, double *rel_res) {
    if (!ctx) return ADR_EINVAL;
    if (!u || !rel_res) {
        ctx->err = "u and rel_res are required";
        return ADR_EINVAL;
    }
    try {
        HIPCHK(adr::launch_fill_int(ctx->sing, 0, ctx->n_inst, ctx->st));
        ctx->to_blocked(u);
        ctx->sweep64(kSlotStep, ctx->Ub, ctx->Ub, 3, ctx->never);
        ctx->norm(0, 0.0, 2);
        HIPCHK(hipMemcpyAsync(rel_res, ctx->rel, sizeof(double) * ctx->n_inst, hipMemcpyDeviceToHost, ctx->st));
        HIPCHK(hipStreamSynchronize(ctx->st));
        const adr_status sst = ctx->singular_status();
        if (sst != ADR_OK) return sst;
        for (int i = 0; i < ctx->n_inst; ++i)
            if (!std::isfinite(rel_res[i])) {
                ctx->err = "non-finite residual";
                return ADR_ENONFINITE;
            }
        return ADR_OK;
    } catch (const Error &e) {
        return fail_ctx(ctx, e);
    }
}

adr_status adr_initial_guess(adr_ctx *ctx, double *u) {
    if (!ctx) return ADR_EINVAL;
    if (!u) {
        ctx->err = "u is required";
        return ADR_EINVAL;
    }
    try {
        ctx->line64(0, kSlotGuess, ctx->Z64, ctx->never);
        ctx->timed(0, 2, ctx->n_unknowns, [&] {
            return adr::launch_scatter<double, double>(0, ctx->fam[0].s64, ctx->fam[0].v64, ctx->Ub, ctx->d32,
                                                       ctx->partial, ctx->never, ctx->st);
        });
        ctx->from_blocked(u);
        return ADR_OK;
    } catch (const Error &e) {
        return fail_ctx(ctx, e);
    }
}

adr_status adr_export_lines(const adr_ctx *ctx, int32_t inst, int32_t family, int64_t *n_lines, int64_t *n_nodes,
                            int64_t *offsets, double *x, double *y) {
    if (!ctx || inst < 0 || inst >= ctx->n_inst || family < 0 || family > 1) return ADR_EINVAL;
    const adr::Family &F = ctx->geo[family][inst];
    if (n_lines) *n_lines = static_cast<int64_t>(F.off.size()) - 1;
    if (n_nodes) *n_nodes = static_cast<int64_t>(F.x.size());
    if (offsets) std::copy(F.off.begin(), F.off.end(), offsets);
    if (x) std::copy(F.x.begin(), F.x.end(), x);
    if (y) std::copy(F.y.begin(), F.y.end(), y);
    return ADR_OK;
}

adr_status adr_export_scatter(const adr_ctx *ctx, int32_t inst, int32_t family, int64_t *n_rows,
                              int32_t *node, int32_t *k, double *ca, double *cb, double *gb) {
    if (!ctx || !ctx->opt.host_only || inst < 0 || inst >= ctx->n_inst || family < 0 || family > 1)
        return ADR_EINVAL;
    const adr::InstanceGeo &G = ctx->host_geo[inst];
    const std::vector<adr::Rec4> &R = G.rec[family];
    if (n_rows) *n_rows = static_cast<int64_t>(R.size());
    for (size_t r = 0; r < R.size(); ++r) {
        if (node) node[r] = G.inner_list[r];
        if (gb) gb[r] = R[r].gb;
        for (int q = 0; q < 4; ++q) {
            if (k) k[4 * r + q] = R[r].k[q];
            if (ca) ca[4 * r + q] = R[r].ca[q];
            if (cb) cb[4 * r + q] = R[r].cb[q];
        }
    }
    return ADR_OK;
}

adr_status adr_export_scatter_factors(const adr_ctx *ctx, int32_t inst, int32_t family, int64_t *n_rows,
                                      double *wh, double *lam, double *t) {
    if (!ctx || !ctx->opt.host_only || inst < 0 || inst >= ctx->n_inst || family < 0 || family > 1)
        return ADR_EINVAL;
    const std::vector<adr::Rec4> &R = ctx->host_geo[inst].rec[family];
    if (n_rows) *n_rows = static_cast<int64_t>(R.size());
    for (size_t r = 0; r < R.size(); ++r) {
        if (wh) wh[r] = R[r].wh;
        for (int q = 0; q < 2; ++q)
            if (lam) lam[2 * r + q] = R[r].lam[q];
        for (int q = 0; q < 4; ++q)
            if (t) t[4 * r + q] = R[r].t[q];
    }
    return ADR_OK;
}

adr_status adr_export_direct(const adr_ctx *ctx, int32_t inst, int32_t family, int64_t *n_nodes, int32_t *k,
                             double *w) {
    if (!ctx || !ctx->opt.host_only || (ctx->opt.transfer != 1 && ctx->opt.increments != 1) || inst < 0 || inst >= ctx->n_inst || family < 0 ||
        family > 1)
        return ADR_EINVAL;
    const std::vector<adr::DirRec> &D = ctx->host_geo[inst].drec[family];
    if (n_nodes) *n_nodes = static_cast<int64_t>(D.size());
    for (size_t q = 0; q < D.size(); ++q) {
        for (int e = 0; e < 2; ++e)
            if (k) k[2 * q + e] = D[q].k[e];
        for (int e = 0; e < 4; ++e)
            if (w) w[4 * q + e] = D[q].w[e];
    }
    return ADR_OK;
}

adr_status adr_export_direct_packed(const adr_ctx *ctx, int32_t inst, int32_t family, int64_t *n_nodes,
                                    int32_t *k0, int16_t *kd, uint32_t *wp) {
    if (!ctx || !ctx->opt.host_only || (ctx->opt.transfer != 1 && ctx->opt.increments != 1) || inst < 0 ||
        inst >= ctx->n_inst || family < 0 || family > 1)
        return ADR_EINVAL;
    const std::vector<adr::DirRec> &D = ctx->host_geo[inst].drec[family];
    if (n_nodes) *n_nodes = static_cast<int64_t>(D.size());
    if (k0 && kd && wp)
        for (size_t q = 0; q < D.size(); ++q) pack_direct(D[q], 0, k0[q], kd[q], wp[q]);
    return ADR_OK;
}

adr_status adr_set_timing(adr_ctx *ctx, int32_t on) {
    if (!ctx || ctx->opt.host_only) return ADR_EINVAL;
    try {
        ctx->collect_ticks();
        ctx->opt.timing = on ? 1 : 0;
        return ADR_OK;
    } catch (const Error &e) {
        return fail_ctx(ctx, e);
    }
}

adr_status adr_kernel_times(adr_ctx *ctx, int32_t precision, double *ms_out, int64_t *count_out,
                            int64_t *work_out, int32_t reset) {
    if (!ctx || precision < 0 || precision > 1) return ADR_EINVAL;
    try {
        ctx->collect_ticks();
        for (int k = 0; k < 5; ++k) {
            if (ms_out) ms_out[k] = ctx->ms[precision][k];
            if (count_out) count_out[k] = ctx->cnt[precision][k];
            if (work_out) work_out[k] = ctx->units[precision][k];
        }
        if (reset)
            for (int k = 0; k < 5; ++k) {
                ctx->ms[precision][k] = 0.0;
                ctx->cnt[precision][k] = 0;
                ctx->units[precision][k] = 0;
            }
        return ADR_OK;
    } catch (const Error &e) {
        return fail_ctx(ctx, e);
    }
}

adr_status adr_destroy(adr_ctx *ctx) {
    if (!ctx) return ADR_OK;
    if (ctx->opt.host_only) {
        delete ctx;
        return ADR_OK;
    }
    (void)hipStreamSynchronize(ctx->st);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    ctx->drop_graph();
    if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    for (int k = 0; k < 2; ++k) {
        if (ctx->side[k]) (void)hipStreamSynchronize(ctx->side[k]);
        if (ctx->side[k]) (void)hipStreamDestroy(ctx->side[k]);
        if (ctx->join_ev[k]) (void)hipEventDestroy(ctx->join_ev[k]);
    }
    if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
    for (void *p : ctx->owned) (void)hipFree(p);
    delete ctx;
    return ADR_OK;
}

const char *adr_last_error(const adr_ctx *ctx) {
    if (!ctx) return g_setup_error.c_str();
    return ctx->err.c_str();
}

}  // extern "C"

namespace adr {
void set_thread_error(const std::string &msg) { g_setup_error = msg; }
}  // namespace adr
