// batch.cpp -- many independent solves of different sizes advanced together.
//
// Every problem runs the mixed-precision refinement of the single-problem
// MIXED form (FP32 V(2,2) cycle for the correction, FP64 update and FP64
// residual fused into the last finest-level launch).  A step of the whole
// batch is a fixed sequence of launches:
//   for each level size s, largest first: one persistent row-march launch over
//     the (problem, tile) list of every problem that has a level of size s
//     (relaxation + residual + restriction);
//   one launch with one workgroup per problem for the levels of <= 32 cells;
//   for each size s, smallest first: the prolongating launches (coarse levels,
//     and the finest levels with the FP64 update);
//   one launch that turns each problem's partial sums into its relative
//   residual, history entry and "done" flag.
// Converged problems keep their flag set and every launch skips their tiles.
// The sequence is captured once into a hipGraph per step parity (the FP64
// iterate and the FP32 residual alternate between two buffers) and replayed;
// kernels read all pointers from descriptor arrays in the workspace, so a new
// set of caller arrays only needs a descriptor upload.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "batch.h"

using namespace ccmg;

namespace {

constexpr int kMaxLevelsB = 16;
constexpr int kStatBlocksB = 64;
constexpr int kMinTyB = 8;
constexpr int kMinOutwB = 112;
constexpr int kMaxWaves = 4096;

size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
long pitch_of(int n) { return (long)((n + 2 + 31) & ~31); }
int tiles_max(int n) { return ((n + kMinOutwB - 1) / kMinOutwB) * ((n + kMinTyB - 1) / kMinTyB); }
int log2i(int n) { return 31 - __builtin_clz((unsigned)n); }

// Per-problem workspace (FP32 levels, FP64 second iterate, partial sums).
struct ProbLay {
    int n = 0, L = 0, lt = 0;
    double h = 0;
    size_t lev_a[kMaxLevelsB], lev_b[kMaxLevelsB], lev_f[kMaxLevelsB], fpart[kMaxLevelsB];
    long pitch[kMaxLevelsB];
    size_t r2 = 0, qb = 0, normpart = 0, part3[2] = {0, 0};
    size_t total = 0;
};

ProbLay prob_layout(const ccmg_problem &p) {
    ProbLay pl;
    pl.n = p.n;
    while ((p.n >> pl.L) >= 2) ++pl.L;
    pl.lt = pl.L - 1;
    for (int l = 0; l < pl.L; ++l)
        if ((p.n >> l) <= kCoarseMax) {
            pl.lt = l;
            break;
        }
    pl.h = (p.xmax - p.xmin) / p.n;
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off = al256(off + b);
        return o;
    };
    for (int l = 0; l <= pl.lt; ++l) {
        const int n = p.n >> l;
        pl.pitch[l] = pitch_of(n);
        const size_t bytes = sizeof(float) * (size_t)(n + 2) * (size_t)pl.pitch[l];
        pl.lev_a[l] = take(bytes);
        pl.lev_b[l] = take(bytes);
        pl.lev_f[l] = take(bytes);
        pl.fpart[l] = l > 0 ? take(sizeof(double) * tiles_max(2 * n)) : 0;
    }
    pl.r2 = take(sizeof(float) * (size_t)(p.n + 2) * (size_t)pl.pitch[0]);
    pl.qb = take(sizeof(double) * (size_t)(p.n + 2) * (size_t)pl.pitch[0]);
    pl.normpart = take(sizeof(double) * 2 * tiles_max(p.n));
    pl.part3[0] = take(sizeof(double) * tiles_max(p.n));
    pl.part3[1] = take(sizeof(double) * tiles_max(p.n));
    pl.total = off;
    return pl;
}

// Per-problem device words (ints) in the batch arena.
enum { I_DONE = 0, I_CYC = 1, I_R32CNT = 2, I_FPCNT = 4, kInts = I_FPCNT + kMaxLevelsB };

// Kinds of launches in a step.
enum Kind { K_PRE = 0, K_POSTC = 1, K_POSTF = 2, K_TAILF = 3, K_START = 4, K_START_GUESS = 5 };

struct Launch {
    int kind = 0;
    int size = 0;          // level size class (cells per side)
    size_t desc_off = 0;   // device byte offsets in the arena
    size_t item_off = 0;
    int ndesc = 0;
    int nitems = 0;
};

struct HostLaunch {
    Launch L;
    std::vector<MarchArgs<float>> d32;
    std::vector<MarchArgs<double>> d64;
    std::vector<WorkItem> items;
};

}  // namespace

struct ccmg_batch {
    int m = 0;
    std::vector<ccmg_problem> prob;
    std::vector<ProbLay> pl;
    std::vector<size_t> base;       // byte offset of each problem's workspace
    char *ws = nullptr;
    size_t ws_bytes = 0;
    size_t arena = 0, arena_bytes = 0;
    size_t off_probs[2] = {0, 0}, off_fin = 0, off_ints = 0, off_hist = 0, off_stat = 0, off_scal = 0;
    size_t off_coarse[2] = {0, 0};
    size_t desc_cap = 0, item_cap = 0, off_desc = 0, off_items = 0;
    hipStream_t user = nullptr, stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_sync[2] = {nullptr, nullptr};
    hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;
    double *hrec = nullptr, *drec = nullptr;   // host-mapped per-problem records
    std::map<int, int> ty;                     // rows per band for each level size class
    std::vector<int> sizes;                    // march level sizes present (descending)
    int waves = kMaxWaves;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    bool graph_ok = false;
    // descriptors of the last upload
    std::vector<Launch> step[2];
    Launch start;
    // caller arrays of the last upload
    std::vector<const double *> cf;
    std::vector<double *> cphi;
    std::vector<long> cpitch;
    int c_guess = -1;
    bool opt_eager = false;                    // CCMG_BATCH_OPT_EAGER

    template <typename T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
    template <typename T>
    T *pat(int i, size_t off) const { return reinterpret_cast<T *>(ws + base[i] + off); }
    int *ints(int i) const { return at<int>(off_ints) + kInts * i; }
};

namespace {

bool batch_problem_ok(const ccmg_problem &p) {
    return ccmg_problem_check(&p) == CCMG_OK && p.nu1 == 2 && p.nu2 == 2;
}

template <typename T>
void consts_for(const ccmg_problem &p, const ProbLay &pl, int l, MarchArgs<T> &a) {
    const double h = pl.h * (double)(1 << l);
    const double c = p.beta / (h * h);
    a.cc = (T)c;
    a.invd = (T)(1.0 / (p.alpha + 4.0 * c));
    a.alpha = (T)p.alpha;
    a.beta = (T)p.beta;
    a.ih2 = (T)(1.0 / (h * h));
    a.n = p.n >> l;
    for (int s = 0; s < 4; ++s) a.bc[s] = p.bc[s];
}

// Tile geometry of one (level, variant) as the single-launch path computes it.
template <typename T>
void set_tiles(MarchArgs<T> &a, int outw, int ty) {
    a.outw = outw;
    a.ty = ty < a.n ? ty : a.n;
    a.strips = (a.n + a.outw - 1) / a.outw;
    a.chunks = (a.n + a.ty - 1) / a.ty;
    a.ntiles = a.strips * a.chunks;
    a.ety = a.ty;
    a.echunks = 0;  // work lists keep one band height for every strip
    a.groups_per_xcd = 0;
}

int outw_of(int nu, bool prolong, bool post) {
    const int hxc = 2 * nu + (post ? 1 : 0) + (prolong ? 2 : 0);
    return 128 - 2 * ((hxc + 1) & ~1);
}

bool singular_of(const ccmg_problem &p) {
    if (p.alpha != 0.0) return false;
    for (int s = 0; s < 4; ++s)
        if (p.bc[s] == CCMG_BC_DIRICHLET) return false;
    return true;
}

// Build every launch of a step of parity `par` (and the start pass) on the host.
void build_step(const ccmg_batch *B, int par, std::vector<HostLaunch> &out) {
    out.clear();
    const int rin = 1 - par, rout = par;  // step k reads buffers of parity (k-1)&1
    auto r_ptr = [&](int i, int which) -> float * {
        return which == 0 ? B->pat<float>(i, B->pl[i].lev_f[0]) : B->pat<float>(i, B->pl[i].r2);
    };
    auto q_ptr = [&](int i, int which) -> double * { return which == 0 ? B->cphi[i] : B->pat<double>(i, B->pl[i].qb); };
    auto q_pitch = [&](int i, int which) -> long { return which == 0 ? B->cpitch[i] : B->pl[i].pitch[0]; };
    auto add_items = [&](HostLaunch &H, int desc, int ntiles) {
        for (int t = 0; t < ntiles; ++t) H.items.push_back(WorkItem{desc, t});
    };
    auto ir_fill = [&](int i, MarchArgs<float> &a) {
        const ccmg_problem &p = B->prob[i];
        const ProbLay &pl = B->pl[i];
        a.q_in = q_ptr(i, rin);
        a.pq_in = q_pitch(i, rin);
        a.q_out = q_ptr(i, rout);
        a.pq_out = q_pitch(i, rout);
        a.g = B->cf[i];
        a.pg = B->cpitch[i];
        a.r_out = r_ptr(i, rout);
        a.pr = pl.pitch[0];
        a.partial = B->pat<double>(i, pl.normpart);
        a.partial3 = B->pat<double>(i, pl.part3[rout]);
        a.count_out = B->ints(i) + I_R32CNT + rout;
        a.alpha64 = p.alpha;
        a.beta64 = p.beta;
        a.ih2_64 = 1.0 / (pl.h * pl.h);
        a.phi_shift = singular_of(p) ? B->at<double>(B->off_scal) + (size_t)kScal * i + S_PHIMEAN : nullptr;
        a.skip = B->ints(i) + I_DONE;
    };
    auto fmean_fill = [&](int i, int l, MarchArgs<float> &a) {
        if (!singular_of(B->prob[i])) return;
        if (l == 0) {
            a.fmean_part = B->pat<double>(i, B->pl[i].part3[rin]);
            a.fmean_count_ptr = B->ints(i) + I_R32CNT + rin;
        } else {
            a.fmean_part = B->pat<double>(i, B->pl[i].fpart[l]);
            a.fmean_count_ptr = B->ints(i) + I_FPCNT + l;
        }
    };
    // down: relaxation + restriction per size class
    for (int s : B->sizes) {
        HostLaunch H;
        H.L.kind = K_PRE;
        H.L.size = s;
        for (int i = 0; i < B->m; ++i) {
            const ccmg_problem &p = B->prob[i];
            const ProbLay &pl = B->pl[i];
            if (p.n < s) continue;
            const int l = log2i(p.n / s);
            if (l >= pl.lt) continue;
            MarchArgs<float> a{};
            consts_for(p, pl, l, a);
            set_tiles(a, outw_of(2, false, true), B->ty.at(s));
            a.f = l == 0 ? r_ptr(i, rin) : B->pat<float>(i, pl.lev_f[l]);
            a.pf = pl.pitch[l];
            fmean_fill(i, l, a);
            a.phi_in = B->pat<float>(i, pl.lev_a[l]);
            a.pin = pl.pitch[l];
            a.phi_out = B->pat<float>(i, pl.lev_b[l]);
            a.pout = pl.pitch[l];
            a.aux = B->pat<float>(i, pl.lev_f[l + 1]);
            a.paux = pl.pitch[l + 1];
            a.partial = B->pat<double>(i, pl.fpart[l + 1]);
            a.count_out = B->ints(i) + I_FPCNT + l + 1;
            a.skip = B->ints(i) + I_DONE;
            add_items(H, (int)H.d32.size(), a.ntiles);
            H.d32.push_back(a);
        }
        if (!H.d32.empty()) out.push_back(std::move(H));
    }
    // (the one-workgroup tail is launched between the two halves; see record_step)
    // up: prolongation + relaxation, coarse levels and finest levels apart
    std::vector<int> asc(B->sizes.rbegin(), B->sizes.rend());
    for (int s : asc) {
        HostLaunch HC, HF;
        HC.L.kind = K_POSTC;
        HF.L.kind = K_POSTF;
        HC.L.size = HF.L.size = s;
        for (int i = 0; i < B->m; ++i) {
            const ccmg_problem &p = B->prob[i];
            const ProbLay &pl = B->pl[i];
            if (p.n < s) continue;
            const int l = log2i(p.n / s);
            if (l >= pl.lt) continue;
            MarchArgs<float> a{};
            consts_for(p, pl, l, a);
            set_tiles(a, outw_of(2, true, l == 0), B->ty.at(s));
            a.f = l == 0 ? r_ptr(i, rin) : B->pat<float>(i, pl.lev_f[l]);
            a.pf = pl.pitch[l];
            fmean_fill(i, l, a);
            a.phi_in = B->pat<float>(i, pl.lev_b[l]);
            a.pin = pl.pitch[l];
            a.phi_out = B->pat<float>(i, pl.lev_a[l]);
            a.pout = pl.pitch[l];
            a.ec = B->pat<float>(i, pl.lev_a[l + 1]);
            a.pc = pl.pitch[l + 1];
            a.skip = B->ints(i) + I_DONE;
            if (l == 0) {
                ir_fill(i, a);
                add_items(HF, (int)HF.d32.size(), a.ntiles);
                HF.d32.push_back(a);
            } else {
                add_items(HC, (int)HC.d32.size(), a.ntiles);
                HC.d32.push_back(a);
            }
        }
        if (!HC.d32.empty()) out.push_back(std::move(HC));
        if (!HF.d32.empty()) out.push_back(std::move(HF));
    }
    // problems that fit the tail entirely: the FP64 update as its own pass
    {
        HostLaunch H;
        H.L.kind = K_TAILF;
        for (int i = 0; i < B->m; ++i) {
            const ccmg_problem &p = B->prob[i];
            const ProbLay &pl = B->pl[i];
            if (pl.lt != 0) continue;
            MarchArgs<float> a{};
            consts_for(p, pl, 0, a);
            set_tiles(a, outw_of(0, false, true), p.n);
            a.f = r_ptr(i, rin);
            a.pf = pl.pitch[0];
            fmean_fill(i, 0, a);
            a.phi_in = B->pat<float>(i, pl.lev_a[0]);
            a.pin = pl.pitch[0];
            ir_fill(i, a);
            add_items(H, (int)H.d32.size(), a.ntiles);
            H.d32.push_back(a);
        }
        if (!H.d32.empty()) out.push_back(std::move(H));
    }
}

// The starting pass: r32 = f - A phi (FP64), its norm, and (no guess) phi = 0.
void build_start(const ccmg_batch *B, bool guess, HostLaunch &H) {
    H = HostLaunch();
    H.L.kind = guess ? K_START_GUESS : K_START;
    for (int i = 0; i < B->m; ++i) {
        const ccmg_problem &p = B->prob[i];
        const ProbLay &pl = B->pl[i];
        MarchArgs<double> a{};
        consts_for(p, pl, 0, a);
        set_tiles(a, outw_of(0, false, true), B->ty.count(p.n) ? B->ty.at(p.n) : 16);
        a.f = B->cf[i];
        a.pf = B->cpitch[i];
        a.phi_in = B->cphi[i];
        a.pin = B->cpitch[i];
        a.phi_out = guess ? nullptr : B->cphi[i];  // writes the zero starting iterate
        a.pout = B->cpitch[i];
        a.r_out = B->pat<float>(i, pl.lev_f[0]);
        a.pr = pl.pitch[0];
        a.partial = B->pat<double>(i, pl.normpart);
        a.partial3 = B->pat<double>(i, pl.part3[0]);
        a.count_out = B->ints(i) + I_R32CNT + 0;
        for (int t = 0; t < a.ntiles; ++t) H.items.push_back(WorkItem{(int)H.d64.size(), t});
        H.d64.push_back(a);
    }
}

std::vector<CoarseArgs<float>> build_coarse(const ccmg_batch *B, int par) {
    std::vector<CoarseArgs<float>> v(B->m);
    const int rin = 1 - par;
    for (int i = 0; i < B->m; ++i) {
        const ccmg_problem &p = B->prob[i];
        const ProbLay &pl = B->pl[i];
        CoarseArgs<float> &c = v[i];
        std::memset(&c, 0, sizeof(c));
        const int l = pl.lt;
        c.f = l == 0 ? (rin == 0 ? B->pat<float>(i, pl.lev_f[0]) : B->pat<float>(i, pl.r2))
                     : B->pat<float>(i, pl.lev_f[l]);
        c.pf = pl.pitch[l];
        c.phi_in = B->pat<float>(i, pl.lev_a[l]);
        c.pin = pl.pitch[l];
        c.phi_out = B->pat<float>(i, pl.lev_a[l]);
        c.pout = pl.pitch[l];
        c.skip = B->ints(i) + I_DONE;
        c.n_top = p.n >> l;
        for (int q = 0; q < 4; ++q) c.bc[q] = p.bc[q];
        c.alpha = p.alpha;
        c.beta = p.beta;
        c.h_top = pl.h * (double)(1 << l);
        c.nu1 = p.nu1;
        c.nu2 = p.nu2;
        c.nu_bottom = p.nu_bottom;
        c.load_phi = 0;
        c.sub_top_mean = singular_of(p) ? 1 : 0;
        c.singular = singular_of(p) ? 1 : 0;
        coarse_fill_consts(c);
    }
    return v;
}

std::vector<BatchProb> build_probs(const ccmg_batch *B, int par) {
    std::vector<BatchProb> v(B->m);
    for (int i = 0; i < B->m; ++i) {
        const ccmg_problem &p = B->prob[i];
        BatchProb &b = v[i];
        std::memset(&b, 0, sizeof(b));
        b.f = B->cf[i];
        b.pf = B->cpitch[i];
        b.n = p.n;
        b.singular = singular_of(p) ? 1 : 0;
        b.rtol = p.rtol;
        b.max_cycles = p.max_cycles;
        b.scal = B->at<double>(B->off_scal) + (size_t)kScal * i;
        b.hist = B->at<double>(B->off_hist) + (size_t)CCMG_HISTORY * i;
        b.done = B->ints(i) + I_DONE;
        b.cycles = B->ints(i) + I_CYC;
        b.normpart = B->pat<double>(i, B->pl[i].normpart);
        b.norm_count = B->ints(i) + I_R32CNT + par;  // written by the launch that wrote normpart
        b.stat_part = B->at<double>(B->off_stat) + (size_t)4 * kStatBlocksB * i;
        b.host = B->drec + 8 * i;
    }
    return v;
}

// Upload host launches into the descriptor arena; fills L.desc_off / item_off.
hipError_t upload(ccmg_batch *B, std::vector<HostLaunch> &H, size_t &dcur, size_t &icur) {
    for (auto &h : H) {
        const size_t dbytes = h.d32.size() * sizeof(MarchArgs<float>) + h.d64.size() * sizeof(MarchArgs<double>);
        const size_t ibytes = h.items.size() * sizeof(WorkItem);
        if (dcur + dbytes > B->desc_cap || icur + ibytes > B->item_cap) return hipErrorOutOfMemory;
        h.L.desc_off = B->off_desc + dcur;
        h.L.item_off = B->off_items + icur;
        h.L.ndesc = (int)(h.d32.size() + h.d64.size());
        h.L.nitems = (int)h.items.size();
        hipError_t e = hipSuccess;
        if (!h.d32.empty())
            e = hipMemcpyAsync(B->ws + h.L.desc_off, h.d32.data(), h.d32.size() * sizeof(MarchArgs<float>),
                               hipMemcpyHostToDevice, B->stream);
        if (e == hipSuccess && !h.d64.empty())
            e = hipMemcpyAsync(B->ws + h.L.desc_off, h.d64.data(), h.d64.size() * sizeof(MarchArgs<double>),
                               hipMemcpyHostToDevice, B->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(B->ws + h.L.item_off, h.items.data(), ibytes, hipMemcpyHostToDevice, B->stream);
        if (e != hipSuccess) return e;
        dcur = al256(dcur + dbytes);
        icur = al256(icur + ibytes);
    }
    return hipSuccess;
}

hipError_t launch_one(ccmg_batch *B, const Launch &L) {
    const int waves = std::min(B->waves, std::max(L.nitems, 1));
    const WorkItem *it = B->at<WorkItem>(L.item_off);
    switch (L.kind) {
        case K_PRE:
            return launch_list_variant<float, 2, false, false, POST_RESTRICT>(B->at<MarchArgs<float>>(L.desc_off), it,
                                                                            L.nitems, waves, B->stream);
        case K_POSTC:
            return launch_list_variant<float, 2, true, true, POST_NONE>(B->at<MarchArgs<float>>(L.desc_off), it,
                                                                      L.nitems, waves, B->stream);
        case K_POSTF:
            return launch_list_variant<float, 2, true, true, POST_IR>(B->at<MarchArgs<float>>(L.desc_off), it,
                                                                    L.nitems, waves, B->stream);
        case K_TAILF:
            return launch_list_variant<float, 0, true, false, POST_IR>(B->at<MarchArgs<float>>(L.desc_off), it,
                                                                     L.nitems, waves, B->stream);
        case K_START:
            return launch_list_variant<double, 0, false, false, POST_R32>(B->at<MarchArgs<double>>(L.desc_off), it,
                                                                        L.nitems, waves, B->stream);
        case K_START_GUESS:
            return launch_list_variant<double, 0, true, false, POST_R32>(B->at<MarchArgs<double>>(L.desc_off), it,
                                                                       L.nitems, waves, B->stream);
    }
    return hipErrorInvalidValue;
}

// The launches of one step of parity `par`, in order.
hipError_t record_step(ccmg_batch *B, int par) {
    hipError_t e = hipSuccess;
    bool tail_done = false;
    for (const Launch &L : B->step[par]) {
        if (!tail_done && L.kind != K_PRE) {
            e = launch_coarse_list<float>(B->at<CoarseArgs<float>>(B->off_coarse[par]), B->m, B->stream);
            tail_done = true;
            if (e != hipSuccess) return e;
        }
        e = launch_one(B, L);
        if (e != hipSuccess) return e;
    }
    if (!tail_done) e = launch_coarse_list<float>(B->at<CoarseArgs<float>>(B->off_coarse[par]), B->m, B->stream);
    if (e == hipSuccess) e = launch_batch_cycle_end(B->at<BatchProb>(B->off_probs[par]), B->m, 0, B->stream);
    return e;
}

void drop_graphs(ccmg_batch *B) {
    for (int k = 0; k < 2; ++k)
        if (B->graph[k]) {
            hipGraphExecDestroy(B->graph[k]);
            B->graph[k] = nullptr;
        }
    B->graph_ok = false;
}

hipError_t capture_graphs(ccmg_batch *B) {
    drop_graphs(B);
    for (int par = 0; par < 2; ++par) {
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return e;
        hipError_t e2 = record_step(B, par);
        e = hipStreamEndCapture(B->stream, &g);
        if (e2 != hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&B->graph[par], g, nullptr, nullptr, 0);
        if (g) hipGraphDestroy(g);
        if (e != hipSuccess) return e;
    }
    B->graph_ok = true;
    return hipSuccess;
}

// Build and upload every descriptor for the given caller arrays; recapture the
// graphs only when the launch structure changed (it does not depend on the arrays).
hipError_t prepare(ccmg_batch *B, const double *const *f, double *const *phi, const ptrdiff_t *pitch, bool guess,
                   bool restructure) {
    bool same = B->c_guess == (int)guess && (int)B->cf.size() == B->m;
    for (int i = 0; same && i < B->m; ++i)
        same = B->cf[i] == f[i] && B->cphi[i] == phi[i] && B->cpitch[i] == pitch[i];
    if (same && !restructure) return hipSuccess;
    B->cf.assign(f, f + B->m);
    B->cphi.assign(phi, phi + B->m);
    B->cpitch.assign(pitch, pitch + B->m);
    B->c_guess = guess ? 1 : 0;
    size_t dcur = 0, icur = 0;
    hipError_t e = hipSuccess;
    for (int par = 0; par < 2 && e == hipSuccess; ++par) {
        std::vector<HostLaunch> H;
        build_step(B, par, H);
        e = upload(B, H, dcur, icur);
        B->step[par].clear();
        for (auto &h : H) B->step[par].push_back(h.L);
        std::vector<CoarseArgs<float>> c = build_coarse(B, par);
        if (e == hipSuccess)
            e = hipMemcpyAsync(B->ws + B->off_coarse[par], c.data(), c.size() * sizeof(CoarseArgs<float>),
                               hipMemcpyHostToDevice, B->stream);
        std::vector<BatchProb> pr = build_probs(B, par);
        if (e == hipSuccess)
            e = hipMemcpyAsync(B->ws + B->off_probs[par], pr.data(), pr.size() * sizeof(BatchProb),
                               hipMemcpyHostToDevice, B->stream);
        // host vectors must outlive the asynchronous copies
        if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
    }
    if (e == hipSuccess) {
        std::vector<HostLaunch> H(1);
        build_start(B, guess, H[0]);
        e = upload(B, H, dcur, icur);
        B->start = H[0].L;
        if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
    }
    // the graphs hold launch geometry only (descriptor contents are read at run time)
    if (e == hipSuccess && (restructure || !B->graph_ok)) e = capture_graphs(B);
    return e;
}

}  // namespace

extern "C" {

size_t ccmg_batch_workspace_bytes(int m, const ccmg_problem *probs) {
    if (m <= 0 || !probs) return 0;
    size_t tot = 0, items = 0, descs = 0;
    for (int i = 0; i < m; ++i) {
        if (!batch_problem_ok(probs[i])) return 0;
        const ProbLay pl = prob_layout(probs[i]);
        tot = al256(tot + pl.total);
        for (int l = 0; l < pl.L; ++l) items += (size_t)tiles_max(probs[i].n >> l);
        descs += (size_t)pl.L + 2;
    }
    // arena: 2 parities x (pre + post launches) + the start pass
    const size_t per = al256(sizeof(BatchProb) * m) * 2 + al256(sizeof(BatchFinish) * m) +
                       al256(sizeof(int) * kInts * m) + al256(sizeof(double) * CCMG_HISTORY * m) +
                       al256(sizeof(double) * 4 * kStatBlocksB * m) + al256(sizeof(double) * kScal * m) +
                       al256(sizeof(CoarseArgs<float>) * m) * 2;
    const size_t dcap = al256((descs * 2 * 2 + 2 * m) * sizeof(MarchArgs<double>) + 64 * 256);
    const size_t icap = al256((items * 2 * 2 + items) * sizeof(WorkItem) + 64 * 256);
    return tot + per + dcap + icap;
}

int ccmg_batch_create(int m, const ccmg_problem *probs, void *d_ws, size_t ws_bytes, void *stream,
                      ccmg_batch **out) {
    if (!out) return CCMG_EINVAL;
    *out = nullptr;
    if (m <= 0 || !probs) return CCMG_EINVAL;
    for (int i = 0; i < m; ++i) {
        const int st = ccmg_problem_check(&probs[i]);
        if (st != CCMG_OK) return st;
        if (probs[i].nu1 != 2 || probs[i].nu2 != 2) return CCMG_EINVAL;
    }
    const size_t need = ccmg_batch_workspace_bytes(m, probs);
    if (!d_ws || ws_bytes < need || (reinterpret_cast<uintptr_t>(d_ws) & 255)) return CCMG_EWORKSPACE;
    ccmg_batch *B = new (std::nothrow) ccmg_batch();
    if (!B) return CCMG_EINVAL;
    B->m = m;
    B->prob.assign(probs, probs + m);
    B->ws = static_cast<char *>(d_ws);
    B->ws_bytes = ws_bytes;
    size_t off = 0;
    size_t items = 0, descs = 0;
    for (int i = 0; i < m; ++i) {
        B->pl.push_back(prob_layout(probs[i]));
        B->base.push_back(off);
        off = al256(off + B->pl.back().total);
        for (int l = 0; l < B->pl.back().L; ++l) items += (size_t)tiles_max(probs[i].n >> l);
        descs += (size_t)B->pl.back().L + 2;
    }
    auto take = [&](size_t b) {
        size_t o = off;
        off = al256(off + b);
        return o;
    };
    B->off_probs[0] = take(sizeof(BatchProb) * m);
    B->off_probs[1] = take(sizeof(BatchProb) * m);
    B->off_fin = take(sizeof(BatchFinish) * m);
    B->off_ints = take(sizeof(int) * kInts * m);
    B->off_hist = take(sizeof(double) * CCMG_HISTORY * m);
    B->off_stat = take(sizeof(double) * 4 * kStatBlocksB * m);
    B->off_scal = take(sizeof(double) * kScal * m);
    B->off_coarse[0] = take(sizeof(CoarseArgs<float>) * m);
    B->off_coarse[1] = take(sizeof(CoarseArgs<float>) * m);
    B->desc_cap = al256((descs * 2 * 2 + 2 * m) * sizeof(MarchArgs<double>) + 64 * 256);
    B->item_cap = al256((items * 2 * 2 + items) * sizeof(WorkItem) + 64 * 256);
    B->off_desc = take(B->desc_cap);
    B->off_items = take(B->item_cap);
    // level size classes handled by row-march launches
    for (int i = 0; i < m; ++i)
        for (int l = 0; l < B->pl[i].lt; ++l) B->ty[probs[i].n >> l] = 0;
    for (auto &kv : B->ty) {
        const int s = kv.first;
        kv.second = s >= 512 ? 16 : 8;
        B->sizes.push_back(s);
    }
    std::sort(B->sizes.rbegin(), B->sizes.rend());
    B->user = static_cast<hipStream_t>(stream);
    hipError_t e = hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&B->ev_sync[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&B->ev_sync[1], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreate(&B->ev_t0);
    if (e == hipSuccess) e = hipEventCreate(&B->ev_t1);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&B->hrec), sizeof(double) * 8 * m,
                          hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void **>(&B->drec), B->hrec, 0);
    if (e != hipSuccess) {
        ccmg_batch_destroy(B);
        return CCMG_EHIP;
    }
    *out = B;
    return CCMG_OK;
}

int ccmg_batch_set_option(ccmg_batch *B, int option, double value) {
    if (!B) return CCMG_EINVAL;
    if (option == CCMG_BATCH_OPT_EAGER && (value == 0.0 || value == 1.0)) {
        B->opt_eager = value != 0.0;
        return CCMG_OK;
    }
    return CCMG_EINVAL;
}

int ccmg_batch_destroy(ccmg_batch *B) {
    if (!B) return CCMG_EINVAL;
    if (B->stream) hipStreamSynchronize(B->stream);
    drop_graphs(B);
    if (B->hrec) hipHostFree(B->hrec);
    for (hipEvent_t ev : {B->ev_in, B->ev_out, B->ev_sync[0], B->ev_sync[1], B->ev_t0, B->ev_t1})
        if (ev) hipEventDestroy(ev);
    if (B->stream) hipStreamDestroy(B->stream);
    delete B;
    return CCMG_OK;
}

// Every problem's arrays: present, pitch >= n + 2, fewer than 2^31 elements
// (the kernels form row offsets in 32 bits).
static bool arrays_ok(const ccmg_batch *B, const double *const *d_f, double *const *d_phi, const ptrdiff_t *pitch) {
    if (!d_f || !d_phi || !pitch) return false;
    for (int i = 0; i < B->m; ++i) {
        const long rows = B->prob[i].n + 2;
        if (!d_f[i] || !d_phi[i] || pitch[i] < rows || (double)pitch[i] * (double)rows >= 2147483648.0)
            return false;
    }
    return true;
}

int ccmg_batch_solve(ccmg_batch *B, const double *const *d_f, double *const *d_phi, const ptrdiff_t *pitch,
                     int use_guess, ccmg_result *out, ccmg_batch_info *info) {
    if (!B || !arrays_ok(B, d_f, d_phi, pitch)) return CCMG_EINVAL;
    const int m = B->m;
    hipError_t e = hipEventRecord(B->ev_in, B->user);  // order after the caller's prior work
    if (e == hipSuccess) e = hipStreamWaitEvent(B->stream, B->ev_in, 0);
    if (e == hipSuccess) e = prepare(B, d_f, d_phi, pitch, use_guess != 0, false);
    if (e != hipSuccess) return CCMG_EHIP;
    e = hipEventRecord(B->ev_t0, B->stream);
    // statistics, flags, the starting FP64 residual and its norm
    if (e == hipSuccess) e = launch_batch_fstats(B->at<BatchProb>(B->off_probs[0]), m, kStatBlocksB, B->stream);
    if (e == hipSuccess) e = launch_one(B, B->start);
    if (e == hipSuccess) e = launch_batch_cycle_end(B->at<BatchProb>(B->off_probs[0]), m, 1, B->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
    if (e != hipSuccess) return CCMG_EHIP;
    int max_steps = 0;
    for (int i = 0; i < m; ++i) max_steps = std::max(max_steps, B->prob[i].max_cycles);
    auto all_done = [&]() {
        for (int i = 0; i < m; ++i)
            if (B->hrec[8 * i + 2] == 0.0) return false;
        return true;
    };
    int steps = 0;
    // CCMG_BATCH_OPT_EAGER issues each step's launches directly instead of
    // replaying the captured graphs (same launches; used to check the replays)
    const bool eager = B->opt_eager;
    auto run_step = [&](int k) -> hipError_t {
        return eager ? record_step(B, k & 1) : hipGraphLaunch(B->graph[k & 1], B->stream);
    };
    if (!all_done() && max_steps > 0) {
        // step k replays graph (k & 1); step k+1 is queued before step k is checked
        e = run_step(1);
        if (e == hipSuccess) e = hipEventRecord(B->ev_sync[1], B->stream);
        for (int k = 1; e == hipSuccess; ++k) {
            if (k < max_steps) {
                e = run_step(k + 1);
                if (e == hipSuccess) e = hipEventRecord(B->ev_sync[(k + 1) & 1], B->stream);
                if (e != hipSuccess) break;
            }
            e = hipEventSynchronize(B->ev_sync[k & 1]);
            if (e != hipSuccess) break;
            steps = k;
            if (all_done() || k >= max_steps) break;
        }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
    if (e != hipSuccess) return CCMG_EHIP;
    // read the per-problem scalars and histories
    std::vector<double> scal((size_t)kScal * m), hist((size_t)CCMG_HISTORY * m);
    std::vector<int> ints((size_t)kInts * m);
    e = hipMemcpy(scal.data(), B->ws + B->off_scal, scal.size() * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess)
        e = hipMemcpy(hist.data(), B->ws + B->off_hist, hist.size() * sizeof(double), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(ints.data(), B->ws + B->off_ints, ints.size() * sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return CCMG_EHIP;
    // returned fields: the iterate after step c sits in the caller's array if c is even
    std::vector<BatchFinish> fin(m);
    int nmax = 0;
    for (int i = 0; i < m; ++i) {
        const int c = ints[(size_t)kInts * i + I_CYC];
        BatchFinish &q = fin[i];
        std::memset(&q, 0, sizeof(q));
        q.src = (c & 1) ? B->pat<double>(i, B->pl[i].qb) : d_phi[i];
        q.psrc = (c & 1) ? B->pl[i].pitch[0] : pitch[i];
        q.dst = d_phi[i];
        q.pdst = pitch[i];
        q.n = B->prob[i].n;
        for (int s = 0; s < 4; ++s) q.bc[s] = B->prob[i].bc[s];
        q.shift = singular_of(B->prob[i]) ? B->at<double>(B->off_scal) + (size_t)kScal * i + S_PHIMEAN : nullptr;
        q.zero = scal[(size_t)kScal * i + S_F2] == 0.0 ? 1 : 0;
        nmax = std::max(nmax, q.n);
    }
    e = hipMemcpyAsync(B->ws + B->off_fin, fin.data(), sizeof(BatchFinish) * m, hipMemcpyHostToDevice, B->stream);
    if (e == hipSuccess) e = launch_batch_finish(B->at<BatchFinish>(B->off_fin), m, nmax, B->stream);
    if (e == hipSuccess) e = hipEventRecord(B->ev_t1, B->stream);
    if (e == hipSuccess) e = hipEventSynchronize(B->ev_t1);
    if (e == hipSuccess) e = hipEventRecord(B->ev_out, B->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(B->user, B->ev_out, 0);
    if (e != hipSuccess) return CCMG_EHIP;
    float ms = 0.f;
    hipEventElapsedTime(&ms, B->ev_t0, B->ev_t1);
    int worst = CCMG_OK, converged = 0;
    for (int i = 0; i < m; ++i) {
        const double *sc = &scal[(size_t)kScal * i];
        const int c = ints[(size_t)kInts * i + I_CYC];
        const double rho = B->hrec[8 * i + 0];
        int st = rho <= B->prob[i].rtol ? CCMG_OK : CCMG_NOT_CONVERGED;
        if (sc[S_FBAD] > 0 || !std::isfinite(rho)) st = CCMG_ENONFINITE;
        if (sc[S_F2] == 0.0) st = CCMG_OK;
        if (singular_of(B->prob[i]) && std::fabs(sc[S_FSUM]) > 1e-12 * sc[S_FABS]) st = CCMG_EINCOMPAT;
        if (st == CCMG_OK) ++converged;
        if (st < 0 && worst >= 0) worst = st;
        else if (st == CCMG_NOT_CONVERGED && worst == CCMG_OK) worst = st;
        if (out) {
            ccmg_result &R = out[i];
            std::memset(&R, 0, sizeof(R));
            R.status = st;
            R.cycles = c;
            R.inner_cycles = c;
            for (int k = 0; k <= c && k < CCMG_HISTORY; ++k) R.history[k] = hist[(size_t)CCMG_HISTORY * i + k];
            R.rel_resid0 = R.history[0];
            R.rel_resid = rho;
            R.ms = ms;
            if (sc[S_F2] == 0.0) {  // phi = 0 solves it exactly, as ccmg_solve reports
                R.cycles = R.inner_cycles = 0;
                R.rel_resid0 = R.rel_resid = 0.0;
                for (int k = 0; k < CCMG_HISTORY; ++k) R.history[k] = 0.0;
            }
        }
    }
    if (info) {
        info->steps = steps;
        info->converged = converged;
        info->ms = ms;
    }
    return worst;
}

// Time the candidate rows-per-band of every level size class on the given
// arrays (whole steps replayed) and keep the fastest; recaptures the graphs.
int ccmg_batch_autotune(ccmg_batch *B, const double *const *d_f, double *const *d_phi, const ptrdiff_t *pitch) {
    if (!B || !arrays_ok(B, d_f, d_phi, pitch)) return CCMG_EINVAL;
    hipError_t e = prepare(B, d_f, d_phi, pitch, false, true);
    if (e != hipSuccess) return CCMG_EHIP;
    // reset the flags so that every launch does its work while being timed
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return CCMG_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return CCMG_EHIP;
    }
    const int cands[] = {8, 16, 32, 64};
    const int wave_cands[] = {1024, 2048, 4096};
    auto time_steps = [&](float &ms) -> hipError_t {
        hipError_t x = launch_batch_fstats(B->at<BatchProb>(B->off_probs[0]), B->m, kStatBlocksB, B->stream);
        if (x == hipSuccess) x = launch_one(B, B->start);
        if (x == hipSuccess) x = launch_batch_cycle_end(B->at<BatchProb>(B->off_probs[0]), B->m, 1, B->stream);
        if (x == hipSuccess) x = hipEventRecord(e0, B->stream);
        for (int k = 1; k <= 2 && x == hipSuccess; ++k) x = hipGraphLaunch(B->graph[k & 1], B->stream);
        if (x == hipSuccess) x = hipEventRecord(e1, B->stream);
        if (x == hipSuccess) x = hipEventSynchronize(e1);
        if (x == hipSuccess) x = hipEventElapsedTime(&ms, e0, e1);
        return x;
    };
    for (int s : B->sizes) {
        int best_ty = B->ty[s];
        float best = 1e30f;
        for (int ty : cands) {
            if (ty > s) continue;
            B->ty[s] = ty;
            e = prepare(B, d_f, d_phi, pitch, false, true);
            float ms = 0.f;
            if (e == hipSuccess) e = time_steps(ms);
            if (e != hipSuccess) break;
            if (ms < best) {
                best = ms;
                best_ty = ty;
            }
        }
        if (e != hipSuccess) break;
        B->ty[s] = best_ty;
    }
    if (e == hipSuccess) {
        int best_w = B->waves;
        float best = 1e30f;
        for (int w : wave_cands) {
            B->waves = w;
            e = prepare(B, d_f, d_phi, pitch, false, true);
            float ms = 0.f;
            if (e == hipSuccess) e = time_steps(ms);
            if (e != hipSuccess) break;
            if (ms < best) {
                best = ms;
                best_w = w;
            }
        }
        B->waves = best_w;
    }
    if (e == hipSuccess) e = prepare(B, d_f, d_phi, pitch, false, true);
    if (e == hipSuccess) e = hipStreamSynchronize(B->stream);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return e == hipSuccess ? CCMG_OK : CCMG_EHIP;
}

int ccmg_batch_shapes(ccmg_batch *B, int *sizes, int *ty, int max, int *count, int *waves) {
    if (!B || !count) return CCMG_EINVAL;
    *count = (int)B->sizes.size();
    for (int k = 0; k < *count && k < max; ++k) {
        if (sizes) sizes[k] = B->sizes[k];
        if (ty) ty[k] = B->ty[B->sizes[k]];
    }
    if (waves) *waves = B->waves;
    return CCMG_OK;
}

}  // extern "C"
