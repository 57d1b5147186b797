// plan.cpp -- host side of the ccmg C ABI: validation, workspace layout, the
// V-cycle schedule (which kernel runs on which level) and the solve loop.
//
// Schedule of one V(nu1, nu2) cycle (pyro paper, Sec. 3.3):
//   for each level l from the finest while it has more than kCoarseMax cells per side:
//     row-march: nu1 red-black iterations, residual, four-cell restriction into
//     the rhs of level l+1 (plus that rhs's partial sums, for singular problems)
//   one workgroup: the whole rest of the cycle (coarse.hip), down to 2x2 and back
//   for each of those levels back up:
//     row-march: prolongation of the level-(l+1) correction, nu2 iterations,
//     and on the finest level the residual norm and the sum of phi
//   one workgroup: residual norm -> relative residual, mean of phi, done flag
// The stop test reads the relative residual back after each cycle while the
// next cycle is already queued; the device "done" flag turns that queued cycle
// into no-ops once the tolerance is met, so the GPU never waits on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "internal.h"

using namespace ccmg;

namespace {

constexpr int kMinTy = 8;       // smallest rows-per-tile the shape picker uses
constexpr int kMinOutw = 100;   // narrowest output width of any march variant (the first fused one)
constexpr int kStatBlocks = 2048;  // f statistics: workgroups (8 waves per SIMD)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
long pitch_for(int n) { return (long)((n + 2 + 31) & ~31); }
bool pow2(int n) { return n >= 2 && (n & (n - 1)) == 0; }


int max_tiles(int n) {
    const int strips = (n + kMinOutw - 1) / kMinOutw;
    const int chunks = (n + kMinTy - 1) / kMinTy;
    // plus the edge strips' halved bands (at least kEdgeSplitMinTy / 2 rows)
    const int ety = kEdgeSplitMinTy / 2;
    return strips * chunks + 2 * ((n + ety - 1) / ety);
}

// Tiles of a row-march launch of an n^2 level in bands of ty rows (as the
// launcher cuts it: x-edge strips in halved bands when `xwalls`).
int march_tiles(int n, int outw, int ty, bool xwalls) {
    const int strips = (n + outw - 1) / outw;
    const int chunks = (n + ty - 1) / ty;
    if (!xwalls || strips < 3 || ty < kEdgeSplitMinTy) return strips * chunks;
    const int ety = edge_band_rows(ty);
    return (strips - 2) * chunks + 2 * ((n + ety - 1) / ety);
}

struct LevelLay {
    int n = 0;
    double h = 0;
    long pitch = 0;        // pitch of the workspace arrays of this level
    size_t a = 0, b = 0, f = 0;  // byte offsets of phi (two buffers) and f in the level's precision
    size_t c = 0;          // FP64 level 0 (below the tail): the post-smoothed iterate of a fused launch
    size_t f2 = 0;         // MIXED level 0: second FP32 residual buffer
    size_t fpart = 0;      // partial sums of this level's rhs
    int fpart_cap = 0;
};

constexpr int kMaxLevels = 16;  // n <= 16384: at most 14 levels

struct Layout {
    int L = 0;             // levels n, n/2, ..., 2
    int lt = 0;            // first level handled by the one-workgroup tail
    size_t elem = 8;       // bytes per value of the relaxed levels (8 FP64, 4 MIXED)
    LevelLay lev[kMaxLevels];
    size_t qb = 0;         // MIXED: second FP64 iterate buffer (finest level)
    size_t normpart = 0;
    int normpart_cap = 0;
    size_t part3 = 0;      // MIXED: per-tile sums of the FP32 residual (two buffers: one read,
    size_t part3b = 0;     // one written by the same launch)
    size_t fstats = 0;
    size_t scal = 0, hist = 0, flags = 0;
    size_t ainv = 0;       // inverse operator of an exact-bottom level (FP64)
    size_t total = 0;
};

bool build_layout(const ccmg_problem &p, Layout &lay) {
    const int n = p.n;
    const bool mixed = p.prec == CCMG_MIXED;
    lay.elem = mixed ? sizeof(float) : sizeof(double);
    lay.L = 0;
    while ((n >> lay.L) >= 2) ++lay.L;
    for (int l = 0; l < kMaxLevels; ++l) lay.lev[l] = LevelLay();
    const double h0 = (p.xmax - p.xmin) / n;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    lay.lt = lay.L - 1;
    for (int l = 0; l < lay.L; ++l) {
        if ((n >> l) <= kCoarseMax) {
            lay.lt = l;
            break;
        }
    }
    for (int l = 0; l < lay.L; ++l) {
        LevelLay &v = lay.lev[l];
        v.n = n >> l;
        v.h = h0 * (double)(1 << l);
        v.pitch = pitch_for(v.n);
        const size_t bytes = lay.elem * (size_t)(v.n + 2) * (size_t)v.pitch;
        if (l == 0 && !mixed) {
            v.b = take(bytes);  // the caller's phi is buffer a, its f the rhs
            if (lay.lt > 0) v.c = take(bytes);
        } else if (l == 0) {
            v.a = take(bytes);  // FP32 correction e (two buffers)
            v.b = take(bytes);
            v.f = take(bytes);  // FP32 residual r32 (two buffers)
            v.f2 = take(bytes);
            lay.qb = take(sizeof(double) * (size_t)(v.n + 2) * (size_t)v.pitch);
        } else if (l <= lay.lt) {
            v.a = take(bytes);
            v.b = take(bytes);
            v.f = take(bytes);
            // partial sums from the launch on the level above: row-march tiles
            // or 32 x 32 blocks of the 2-D tile kernel ((2n / 32)^2)
            v.fpart_cap = std::max(max_tiles(v.n * 2), (v.n / 16) * (v.n / 16));
            v.fpart = take(sizeof(double) * v.fpart_cap);
        }
    }
    lay.normpart_cap = max_tiles(n);
    lay.normpart = take(sizeof(double) * 2 * lay.normpart_cap);
    lay.part3 = take(sizeof(double) * lay.normpart_cap);
    lay.part3b = take(sizeof(double) * lay.normpart_cap);
    // f statistics: per workgroup of the statistics pass, or per tile of the
    // first restricting launch of a solve (which takes them from its own loads)
    lay.fstats = take(sizeof(double) * 4 * std::max(kStatBlocks, max_tiles(n)));
    lay.scal = take(sizeof(double) * kScal);
    lay.hist = take(sizeof(double) * CCMG_HISTORY);
    lay.flags = take(sizeof(int) * 16);
    lay.ainv = take(sizeof(double) * kDirectMax * kDirectMax * kDirectMax * kDirectMax);  // keep last
    lay.total = off;
    return true;
}

// Default rows per tile (before / without autotuning): long bands on the big
// levels keep the redundant halo rows (2 x 6 per band) small; small levels
// need short bands so that enough wavefronts run and each finishes quickly.
MarchShape shape_for(int n) {
    MarchShape s;
    s.wpb = 1;
    int ty;
    if (n >= 4096) ty = 64;
    else if (n >= 2048) ty = 32;
    else if (n >= 512) ty = 16;
    else ty = 8;
    s.ty = ty < n ? ty : n;
    if (s.ty < 2) s.ty = 2;
    return s;
}

// Default shape of a visit launch: its bands carry 8 halo rows on either
// side, so they are taller.
MarchShape visit_shape_for(int n) {
    MarchShape s;
    s.wpb = 1;
    const int ty = n >= 4096 ? 128 : (n >= 512 ? 64 : 32);
    s.ty = ty < n ? ty : n;
    return s;
}

}  // namespace

// Events bracketing finest-level launches while profiling is on.
struct KernelTimer {
    static constexpr int kKinds = 10;
    static constexpr int kPairs = 1024;
    bool on = false;
    std::vector<hipEvent_t> ev;          // 2 * kPairs
    int used = 0;
    int kind[kPairs];
    int cyc[kPairs];  // cycle (refinement step) of a solve the launch belongs to, 0 outside solves
    double bytes[kPairs];
    int launches[kKinds] = {};
    double ms[kKinds] = {}, tbytes[kKinds] = {};
};

struct ccmg_plan {
    ccmg_problem p;
    KernelTimer timer;
    MarchShape shp_pre[kMaxLevels], shp_post[kMaxLevels];  // launch shape per level (autotuned)
    // a level run as a visit: its restricting launch without the stored
    // iterate, and the visit launch (recomputed pre-smoothing, prolongation,
    // post-smoothing); visit[l]: the autotuner found the pair faster
    MarchShape shp_pre_v[kMaxLevels], shp_visit[kMaxLevels];
    bool visit[kMaxLevels] = {};
    MarchShape shp_fused{64, 1};  // the fused finest launch (autotuned)
    // the first fused launch of a solve from zero recomputing the first
    // pre-smoothing (fused0: the autotuner found that pair faster than a
    // stored pre-smoothing and the ordinary fused launch)
    MarchShape shp_fused0{64, 1};
    bool fused0 = false;
    MarchShape shp_fused32{64, 1};  // ... its FP32 form (inner cycles of a mixed step)
    // options (ccmg_plan_set_option)
    bool opt_fused = true;       // fused finest launch of FP64 V(2,2) solves
    double opt_fused_keep = 1.0;    // keep a cycle's own iterate while the extrapolated residual is
                                    // within this factor of the tolerance
    int opt_mixed_inner = 3;     // most FP32 cycles per refinement step
    int opt_fmg = 0;             // FMG start of FP64 solves without a guess: V-cycles per level (0: off)
    int opt_visit = 1;           // coarse levels as visits: 0 never, 1 where autotuned, 2 wherever they apply
    int n_bottom = 2;  // 4 or 8: exact solve on that level (ccmg_plan_set_bottom)
    int tcycle = 0;    // cycle being enqueued by the solve loop (tags timed launches)
    double *hrho = nullptr;   // host-mapped: relative residual of each cycle
    double *drho = nullptr;   // ... its device address
    Layout lay;
    char *ws = nullptr;
    hipStream_t stream = nullptr;
    int simds = 1024;         // SIMDs of the device (compute units x 4)
    bool singular = false;
    double *hpin = nullptr;  // pinned host: relative residual per cycle
    hipEvent_t ev_sync[2] = {nullptr, nullptr};
    // Events after cycles 2, 3, ... of a solve: the host then reads only the
    // cycle's residual from hrho, which is fine-grained (coherent) host memory
    // that the kernel writes directly, so these skip the system-scope fence
    // (a cache write-back the device otherwise idles for after every cycle);
    // the statistics copied to hpin are read after cycle 1's fenced event
    hipEvent_t ev_cyc[2] = {nullptr, nullptr};
    hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;

    template <typename T>
    T *at(size_t off) const { return reinterpret_cast<T *>(ws + off); }
    double *scal() const { return at<double>(lay.scal); }

    // Record the start event of a timed launch (returns the pair index or -1).
    int tstart(int kind, double bytes) {
        if (!timer.on || timer.used >= KernelTimer::kPairs) return -1;
        const int i = timer.used++;
        timer.kind[i] = kind;
        timer.cyc[i] = tcycle;
        timer.bytes[i] = bytes;
        hipEventRecord(timer.ev[2 * i], stream);
        return i;
    }
    void tstop(int i) {
        if (i >= 0) hipEventRecord(timer.ev[2 * i + 1], stream);
    }
    // Fold finished pairs into the per-kind totals.  Launches of cycles after
    // `last_cycle` were queued ahead of a convergence the device then flagged:
    // they exited at once and are not counted.
    void tcollect(int last_cycle = INT_MAX) {
        for (int i = 0; i < timer.used; ++i) {
            float ms = 0.f;
            if (timer.cyc[i] > last_cycle) continue;
            if (hipEventElapsedTime(&ms, timer.ev[2 * i], timer.ev[2 * i + 1]) == hipSuccess) {
                timer.launches[timer.kind[i]] += 1;
                timer.ms[timer.kind[i]] += ms;
                timer.tbytes[timer.kind[i]] += timer.bytes[i];
            }
        }
        timer.used = 0;
    }
    double *hist() const { return at<double>(lay.hist); }
    int *done() const { return at<int>(lay.flags); }
};

// Host side of ccmg_vcycle_noalloc: one plan object per device (guarded by
// a mutex each), built at library load, re-initialised by every call.
namespace {
constexpr int kNoallocDevices = 16;
ccmg_plan g_noalloc_plan[kNoallocDevices];
std::mutex g_noalloc_mu[kNoallocDevices];
}  // namespace

hipStream_t ccmg::plan_stream(const ccmg_plan *P) { return P->stream; }
int ccmg::plan_n(const ccmg_plan *P) { return P->lay.lev[0].n; }
const ccmg_problem *ccmg::plan_problem(const ccmg_plan *P) { return &P->p; }

namespace {
// The fused finest launch applies to FP64 plans with V(2,2) and levels below
// the finest (option CCMG_OPT_FUSED turns it off).
bool fused_eligible(const ccmg_plan *P) {
    return P->opt_fused && P->p.prec == CCMG_FP64 && P->lay.lt >= 1 && P->p.nu1 == 2 && P->p.nu2 == 2;
}
// Mixed-precision steps with several FP32 V-cycles per FP64 refinement: the
// most inner cycles per step (CCMG_OPT_MIXED_INNER, default 3; 1 = one cycle
// per step; one more is allowed when it is expected to end the solve).  More
// cycles per step do not pay on ill-conditioned problems: the FP32 residual
// of a smooth correction loses about log10(kappa) of its 7 digits, so a step
// cannot reduce the FP64 residual by much more than about 1e-4 there (seen on
// 4096^2 Poisson).  Needs the same cycle shape as the fused FP64 launch.
int mixed_inner_max(const ccmg_plan *P) {
    if (P->p.prec != CCMG_MIXED || P->lay.lt < 1 || P->p.nu1 != 2 || P->p.nu2 != 2) return 1;
    return P->opt_mixed_inner;
}
// Level l (below the finest, above the one-workgroup tail) may run as a visit
// in V(2,2) cycles: where its correction starts from zero, the restricting
// launch of the way down stores no iterate and one launch on the way up
// recomputes the two pre-smoothing iterations, adds the prolongated
// correction and runs the two post-smoothing iterations (the same arithmetic
// per cell: iterates are bitwise those of the two-launch form, and each cell
// of the level is written and read once less).
bool visit_level(const ccmg_plan *P, int l) {
    if (l < 1 || l >= P->lay.lt || l >= kMaxLevels || P->p.nu1 != 2 || P->p.nu2 != 2 || P->opt_visit == 0)
        return false;
    return P->opt_visit == 2 || P->visit[l];
}

}  // namespace

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? CCMG_OK : CCMG_EHIP; }

// Constants of the level-l operator: relaxation phi = (f + cc*sum) * invd and
// residual r = f - (alpha phi - beta ih2 lap).
template <typename T>
void level_consts(const ccmg_plan *P, int l, MarchArgs<T> &a) {
    const double h = P->lay.lev[l].h;
    const double c = P->p.beta / (h * h);
    a.cc = (T)c;
    a.invd = (T)(1.0 / (P->p.alpha + 4.0 * c));
    a.alpha = (T)P->p.alpha;
    a.beta = (T)P->p.beta;
    a.ih2 = (T)(1.0 / (h * h));
    a.n = P->lay.lev[l].n;
    for (int s = 0; s < 4; ++s) a.bc[s] = P->p.bc[s];
}

// Split nu (0..8) relaxations into launches of at most two iterations.
struct NuChain {
    int k[5];
    int count;
    size_t size() const { return (size_t)count; }
    int operator[](size_t i) const { return k[i]; }
    int front() const { return k[0]; }
    int back() const { return k[count - 1]; }
};
NuChain split_nu(int nu) {
    NuChain v{};
    if (nu == 0) {
        v.k[v.count++] = 0;
        return v;
    }
    if (nu & 1) v.k[v.count++] = 1;
    for (int i = 0; i < nu / 2; ++i) v.k[v.count++] = 2;
    return v;
}

template <typename T>
struct Buf {
    T *p;
    long pitch;
};

// What one V-cycle works on at the finest level (level 0).
template <typename T>
struct CycleIO {
    const T *f0 = nullptr;         // level-0 rhs
    long pf0 = 0;
    T *phi0 = nullptr;             // level-0 iterate; the result ends here (unless post0 == POST_IR)
    long pp0 = 0;
    T *phi0b = nullptr;            // second level-0 buffer
    long pp0b = 0;
    bool zero = false;             // the level-0 iterate starts at zero (not read)
    const double *phi_shift = nullptr;    // subtracted from the level-0 iterate as it is read
    const double *f0mean_part = nullptr;  // sums whose mean is removed from f0 (singular, MIXED)
    int f0mean_count = 0;
    int post0 = POST_NONE;         // what the last level-0 launch does after relaxing
    const int *skip = nullptr;
    // POST_IR: the FP64 side of a refinement step
    const double *q_in = nullptr;
    long pq_in = 0;
    double *q_out = nullptr;
    long pq_out = 0;
    const double *g = nullptr;
    long pg = 0;
    float *r_out = nullptr;
    long pr = 0;
    bool q_zero = false;           // the FP64 iterate is zero (first step without a guess)
    const double *q_shift = nullptr;  // subtracted from the FP64 iterate as it is read
    double *partial3_out = nullptr;   // per-tile sums of the new FP32 residual
    // levels >= 1 only (the fused FP64 driver runs the level-0 launches itself)
    bool coarse_only = false;
    int f1_count = 0;                 // partial sums of the level-1 rhs already restricted
    Buf<T> *l1_out = nullptr;         // receives the buffer holding level 1's final iterate
    // a cycle rooted at level top >= 1 (full multigrid): its rhs is that
    // level's f buffer, its iterate top_in (one of the level's two buffers;
    // ignored when `zero`), the buffer holding the result goes to *top_out
    int top = 0;
    Buf<T> top_in{nullptr, 0};
    Buf<T> *top_out = nullptr;
};

template <typename T>
void coarse_consts(const ccmg_plan *P, int l, CoarseArgs<T> &c) {
    for (int q = 0; q < 4; ++q) c.bc[q] = P->p.bc[q];
    c.alpha = P->p.alpha;
    c.beta = P->p.beta;
    c.h_top = P->lay.lev[l].h;
    c.nu1 = P->p.nu1;
    c.nu2 = P->p.nu2;
    c.nu_bottom = P->p.nu_bottom;
    c.n_top = P->lay.lev[l].n;
    c.n_bottom = P->n_bottom >= 4 ? P->n_bottom : 0;
    c.ainv = P->n_bottom >= 4 ? P->at<double>(P->lay.ainv) : nullptr;
}

// Enqueue one V-cycle in precision T.  Returns in *norm_tiles the tile count of
// the launch that wrote per-tile norm partials (POST_NORM / POST_IR), else 0.
template <typename T>
hipError_t enqueue_cycle(ccmg_plan *P, const CycleIO<T> &io, int *norm_tiles) {
    const Layout &lay = P->lay;
    hipStream_t s = P->stream;
    hipError_t e;
    Buf<T> cur[kMaxLevels] = {}, other[kMaxLevels] = {};
    int fpart_count[kMaxLevels] = {};
    bool visited[kMaxLevels] = {};
    const bool f64 = sizeof(T) == sizeof(double);
    // visits (tuned for the precision the plan relaxes its coarse levels in)
    const bool visits_ok = f64 == (P->p.prec == CCMG_FP64);
    *norm_tiles = 0;

    auto fptr = [&](int l) -> Buf<T> {
        if (l == 0) return Buf<T>{const_cast<T *>(io.f0), io.pf0};
        return Buf<T>{P->at<T>(lay.lev[l].f), lay.lev[l].pitch};
    };
    const int top = io.coarse_only ? 1 : io.top;
    auto setup_bufs = [&](int l) {
        if (l == 0) {
            cur[0] = Buf<T>{io.phi0, io.pp0};
            other[0] = Buf<T>{io.phi0b, io.pp0b};
        } else {
            cur[l] = Buf<T>{P->at<T>(lay.lev[l].a), lay.lev[l].pitch};
            other[l] = Buf<T>{P->at<T>(lay.lev[l].b), lay.lev[l].pitch};
            if (l == top && !io.coarse_only && io.top_in.p && io.top_in.p != cur[l].p) std::swap(cur[l], other[l]);
        }
    };
    auto fmean = [&](int l, MarchArgs<T> &a) {
        a.fmean_part = nullptr;
        a.fmean_count = 0;
        if (!P->singular) return;
        if (l > 0) {
            a.fmean_part = P->at<double>(lay.lev[l].fpart);
            a.fmean_count = fpart_count[l];
        } else if (io.f0mean_part) {
            a.fmean_part = io.f0mean_part;
            a.fmean_count = io.f0mean_count;
        }
    };
    auto ir_args = [&](MarchArgs<T> &a) {
        a.q_in = io.q_in;
        a.pq_in = io.pq_in;
        a.q_out = io.q_out;
        a.pq_out = io.pq_out;
        a.g = io.g;
        a.pg = io.pg;
        a.r_out = io.r_out;
        a.pr = io.pr;
        a.q_zero = io.q_zero ? 1 : 0;
        a.phi_shift = io.q_shift;
        a.partial = P->at<double>(lay.normpart);
        a.partial3 = io.partial3_out;
        const double h = lay.lev[0].h;
        a.alpha64 = P->p.alpha;
        a.beta64 = P->p.beta;
        a.ih2_64 = 1.0 / (h * h);
    };

    // down
    if (io.coarse_only) fpart_count[1] = io.f1_count;
    for (int l = top; l < lay.lt; ++l) {
        setup_bufs(l);
        const NuChain chain = split_nu(P->p.nu1);
        bool zero = io.coarse_only || l > top || io.zero;
        const bool vis = visits_ok && zero && visit_level(P, l);
        visited[l] = vis;
        const MarchShape sh = vis ? P->shp_pre_v[l] : P->shp_pre[l];
        for (size_t i = 0; i < chain.size(); ++i) {
            const bool last = i + 1 == chain.size();
            MarchArgs<T> a{};
            level_consts(P, l, a);
            const Buf<T> fb = fptr(l);
            a.f = fb.p;
            a.pf = fb.pitch;
            fmean(l, a);
            a.phi_in = cur[l].p;
            a.pin = cur[l].pitch;
            a.phi_out = vis ? nullptr : other[l].p;  // a visit recomputes this iterate
            a.pout = other[l].pitch;
            a.phi_shift = (l == 0 && i == 0 && !zero) ? io.phi_shift : nullptr;
            a.skip = io.skip;
            int post = POST_NONE;
            if (last) {
                post = POST_RESTRICT;
                a.aux = P->at<T>(lay.lev[l + 1].f);
                a.paux = lay.lev[l + 1].pitch;
                a.partial = P->at<double>(lay.lev[l + 1].fpart);
            }
            int nt = 0;
            const double nn = (double)lay.lev[l].n * lay.lev[l].n;
            const int ti = l == 0 ? P->tstart(f64 ? 0 : 2, sizeof(T) * nn * ((zero ? 2.0 : 3.0) + (last ? 0.25 : 0.0)))
                                  : -1;
            e = launch_march<T>(a, chain[i], !zero, false, post, sh, s, &nt);
            P->tstop(ti);
            if (e != hipSuccess) return e;
            if (last) fpart_count[l + 1] = nt;
            if (!vis) std::swap(cur[l], other[l]);
            zero = false;
        }
    }
    // bottom part in one workgroup
    {
        const int l = lay.lt;
        setup_bufs(l);
        CoarseArgs<T> c{};
        coarse_consts(P, l, c);
        const Buf<T> fb = fptr(l);
        c.f = fb.p;
        c.pf = fb.pitch;
        c.load_phi = (l == top && !io.coarse_only && !io.zero) ? 1 : 0;
        c.phi_in = cur[l].p;
        c.pin = cur[l].pitch;
        c.phi_out = cur[l].p;  // the tail reads everything into LDS first
        c.pout = cur[l].pitch;
        c.phi_shift = (l == 0) ? io.phi_shift : nullptr;
        c.skip = io.skip;
        // the top rhs is a restricted residual (or, MIXED, the FP32 residual): remove its mean
        c.sub_top_mean = (P->singular && (l > 0 || !f64)) ? 1 : 0;
        c.singular = P->singular ? 1 : 0;
        e = launch_coarse<T>(c, s);
        if (e != hipSuccess) return e;
    }
    // up
    for (int l = lay.lt - 1; l >= top; --l) {
        if (visited[l]) {
            MarchArgs<T> a{};
            level_consts(P, l, a);
            const Buf<T> fb = fptr(l);
            a.f = fb.p;
            a.pf = fb.pitch;
            fmean(l, a);
            a.phi_out = other[l].p;
            a.pout = other[l].pitch;
            a.skip = io.skip;
            a.ec = cur[l + 1].p;
            a.pc = cur[l + 1].pitch;
            int nt = 0;
            e = launch_march<T>(a, 4, false, true, POST_VISIT, P->shp_visit[l], s, &nt);
            if (e != hipSuccess) return e;
            std::swap(cur[l], other[l]);
            continue;
        }
        const MarchShape sh = P->shp_post[l];
        const NuChain chain = split_nu(P->p.nu2);
        for (size_t i = 0; i < chain.size(); ++i) {
            const bool last = i + 1 == chain.size();
            MarchArgs<T> a{};
            level_consts(P, l, a);
            const Buf<T> fb = fptr(l);
            a.f = fb.p;
            a.pf = fb.pitch;
            fmean(l, a);
            a.phi_in = cur[l].p;
            a.pin = cur[l].pitch;
            a.phi_out = other[l].p;
            a.pout = other[l].pitch;
            a.skip = io.skip;
            const bool prolong = i == 0;
            if (prolong) {
                a.ec = cur[l + 1].p;
                a.pc = cur[l + 1].pitch;
            }
            int post = POST_NONE;
            if (last && l == 0 && io.post0 != POST_NONE) {
                post = io.post0;
                if (post == POST_IR) ir_args(a);
                else a.partial = P->at<double>(lay.normpart);
            }
            int nt = 0;
            const double nn = (double)lay.lev[l].n * lay.lev[l].n;
            // POST_IR also reads the FP64 iterate and rhs, writes the iterate and the FP32 residual
            const double tb = sizeof(T) * nn * (3.0 + (prolong ? 0.25 : 0.0)) +
                              (post == POST_IR ? nn * (3.0 * sizeof(double) + sizeof(float)) : 0.0);
            const int ti = l == 0 ? P->tstart(f64 ? 1 : 3, tb) : -1;
            e = launch_march<T>(a, chain[i], true, prolong, post, sh, s, &nt);
            P->tstop(ti);
            if (e != hipSuccess) return e;
            if (post != POST_NONE) *norm_tiles = nt;
            std::swap(cur[l], other[l]);
        }
    }
    if (io.coarse_only) {
        if (io.l1_out) *io.l1_out = cur[1];
        return hipSuccess;
    }
    if (top > 0) {
        if (io.top_out) *io.top_out = cur[top];
        return hipSuccess;
    }
    // the result must end in phi0
    if (lay.lt > 0 && io.post0 != POST_IR && cur[0].p != io.phi0) {
        e = hipMemcpy2DAsync(io.phi0 + io.pp0 + 1, sizeof(T) * io.pp0, cur[0].p + cur[0].pitch + 1,
                             sizeof(T) * cur[0].pitch, sizeof(T) * lay.lev[0].n, lay.lev[0].n,
                             hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return e;
    }
    if (lay.lt == 0 && io.post0 != POST_NONE) {
        // the whole cycle ran in the tail: one more pass over level 0 for the norm
        // (and, MIXED, the FP64 update)
        MarchArgs<T> a{};
        level_consts(P, 0, a);
        a.f = io.f0;
        a.pf = io.pf0;
        a.phi_in = io.phi0;
        a.pin = io.pp0;
        a.skip = io.skip;
        if (io.post0 == POST_IR) ir_args(a);
        else a.partial = P->at<double>(lay.normpart);
        e = launch_march<T>(a, 0, true, false, io.post0, shape_for(lay.lev[0].n), s, norm_tiles);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// One FP64 V-cycle on the caller's arrays (the plain form).
hipError_t enqueue_vcycle64(ccmg_plan *P, const double *f0, long pf0, double *phi0, long pp0, bool first_zero,
                            const double *phi_shift, bool with_norm, int slot) {
    CycleIO<double> io;
    io.f0 = f0;
    io.pf0 = pf0;
    io.phi0 = phi0;
    io.pp0 = pp0;
    io.phi0b = P->at<double>(P->lay.lev[0].b);
    io.pp0b = P->lay.lev[0].pitch;
    io.zero = first_zero;
    io.phi_shift = phi_shift;
    io.post0 = with_norm ? POST_NORM : POST_NONE;
    io.skip = with_norm ? P->done() : nullptr;
    int nt = 0;
    hipError_t e = enqueue_cycle<double>(P, io, &nt);
    if (e == hipSuccess && with_norm)
        e = launch_cycle_end(P->at<double>(P->lay.normpart), nt, P->lay.lev[0].n, P->singular ? 1 : 0,
                             P->scal() + S_F2, P->p.rtol, P->hist() + slot, P->scal() + S_PHIMEAN, P->done(),
                             P->drho + slot, P->stream);
    return e;
}

// Full multigrid start (FP64).  f is restricted (four-cell means) level by
// level down to the coarse tail's top level c; there phi starts at zero and
// gets ncyc_top V-cycles of the tail; on each finer level phi is the
// prolongation of the coarser phi into a zero field, followed by ncyc
// V-cycles rooted at that level (its coarser levels' buffers serve as the
// cycle's corrections, the coarser phi being no longer needed).  Level 0's
// phi goes to phi0.  With norm_slot >= 0 the level-0 prolongation also takes
// the residual norm of its result and the cycle-end kernel files it in that
// history slot (the solve's starting residual), and no V-cycle runs on level
// 0; otherwise ncyc plain V-cycles follow there.  ncyc_top >= 1.
hipError_t enqueue_fmg(ccmg_plan *P, const double *f0, long pf0, double *phi0, long pp0, int ncyc_top, int ncyc,
                       int norm_slot, Buf<double> *l1_out = nullptr, bool f1_ready = false) {
    const Layout &lay = P->lay;
    hipStream_t s = P->stream;
    const int c = lay.lt;
    hipError_t e = hipSuccess;
    int nt = 0;
    if (c > 0) {
        // 1. the right-hand side on every level down to c
        for (int l = f1_ready ? 2 : 1; l <= c && e == hipSuccess; ++l) {
            const double *src = l == 1 ? f0 : P->at<double>(lay.lev[l - 1].f);
            const long ps = l == 1 ? pf0 : lay.lev[l - 1].pitch;
            e = launch_restrict(src, ps, P->at<double>(lay.lev[l].f), lay.lev[l].pitch, lay.lev[l].n, s);
        }
        // 2. level c: V-cycles of the tail from zero
        Buf<double> cur{P->at<double>(lay.lev[c].a), lay.lev[c].pitch};
        for (int k = 0; k < ncyc_top && e == hipSuccess; ++k) {
            CycleIO<double> io;
            io.top = c;
            io.zero = k == 0;
            io.top_in = cur;
            io.top_out = &cur;
            e = enqueue_cycle<double>(P, io, &nt);
        }
        // 3. levels c - 1 .. 1: prolongate, then V-cycles rooted there
        for (int l = c - 1; l >= 1 && e == hipSuccess; --l) {
            MarchArgs<double> a{};
            level_consts(P, l, a);
            a.f = P->at<double>(lay.lev[l].f);
            a.pf = lay.lev[l].pitch;
            a.phi_out = P->at<double>(lay.lev[l].a);
            a.pout = lay.lev[l].pitch;
            a.ec = cur.p;
            a.pc = cur.pitch;
            e = launch_march<double>(a, 0, false, true, POST_NONE, shape_for(lay.lev[l].n), s, &nt);
            cur = Buf<double>{P->at<double>(lay.lev[l].a), lay.lev[l].pitch};
            for (int k = 0; k < ncyc && e == hipSuccess; ++k) {
                CycleIO<double> io;
                io.top = l;
                io.top_in = cur;
                io.top_out = &cur;
                e = enqueue_cycle<double>(P, io, &nt);
            }
        }
        // 4. level 0 (or, with l1_out, left to the caller: the fused solve
        // prolongates inside its first pre-smoothing launch)
        if (l1_out) {
            *l1_out = cur;
            return e;
        }
        if (e == hipSuccess) {
            MarchArgs<double> a{};
            level_consts(P, 0, a);
            a.f = f0;
            a.pf = pf0;
            a.phi_out = phi0;
            a.pout = pp0;
            a.ec = cur.p;
            a.pc = cur.pitch;
            a.partial = P->at<double>(lay.normpart);
            e = launch_march<double>(a, 0, false, true, norm_slot >= 0 ? POST_NORM : POST_NONE,
                                     shape_for(lay.lev[0].n), s, &nt);
        }
        if (e == hipSuccess && norm_slot >= 0)
            return launch_cycle_end(P->at<double>(lay.normpart), nt, lay.lev[0].n, P->singular ? 1 : 0,
                                    P->scal() + S_F2, P->p.rtol, P->hist() + norm_slot, P->scal() + S_PHIMEAN,
                                    P->done(), P->drho + norm_slot, s);
        for (int k = 0; k < ncyc && e == hipSuccess; ++k)
            e = enqueue_vcycle64(P, f0, pf0, phi0, pp0, false, nullptr, false, 0);
        return e;
    }
    // the finest level is the tail's top: V-cycles from zero there
    for (int k = 0; k < ncyc_top && e == hipSuccess; ++k)
        e = enqueue_vcycle64(P, f0, pf0, phi0, pp0, k == 0, nullptr, false, 0);
    if (e == hipSuccess && norm_slot >= 0) {
        MarchArgs<double> a{};
        level_consts(P, 0, a);
        a.f = f0;
        a.pf = pf0;
        a.phi_in = phi0;
        a.pin = pp0;
        a.partial = P->at<double>(lay.normpart);
        e = launch_march<double>(a, 0, true, false, POST_NORM, shape_for(lay.lev[0].n), s, &nt);
        if (e == hipSuccess)
            e = launch_cycle_end(P->at<double>(lay.normpart), nt, lay.lev[0].n, P->singular ? 1 : 0,
                                 P->scal() + S_F2, P->p.rtol, P->hist() + norm_slot, P->scal() + S_PHIMEAN,
                                 P->done(), P->drho + norm_slot, s);
    }
    return e;
}

// State of the mixed-precision refinement between steps: which of the two FP64
// iterate buffers and which of the two FP32 residual buffers are current.
struct MixedState {
    double *q;     // current FP64 iterate
    long pq;
    double *qo;    // the other FP64 buffer
    long pqo;
    float *r;      // current FP32 residual (rhs of the next correction)
    float *ro;
    long pr;
    double *s3;    // per-tile sums of the current FP32 residual
    double *s3o;
    int r_tiles;   // tiles of the launch that wrote the current residual's partial sums
    bool q_zero;   // the FP64 iterate is still zero
};

// r32 = f - A phi64 in FP64 (and its norm -> hist[slot]); phi64 is not changed.
hipError_t enqueue_mixed_start(ccmg_plan *P, const double *d_f, long pf, MixedState &st, bool use_guess, int slot,
                               double *stats_host = nullptr) {
    MarchArgs<double> a{};
    level_consts(P, 0, a);
    a.f = d_f;
    a.pf = pf;
    a.phi_in = st.q;
    a.pin = st.pq;
    a.r_out = st.r;
    a.pr = st.pr;
    a.partial = P->at<double>(P->lay.normpart);
    a.partial3 = st.s3;
    // stats_host: f's statistics from this launch's loads too (summed before
    // the norm needs ||f||, then copied to the host)
    if (stats_host) a.fstat_part = P->at<double>(P->lay.fstats);
    int nt = 0;
    hipError_t e = launch_march<double>(a, 0, use_guess, false, POST_R32, P->shp_pre[0], P->stream, &nt);
    st.r_tiles = nt;
    if (e == hipSuccess && stats_host) e = launch_reduce4(P->at<double>(P->lay.fstats), nt, P->scal() + S_FSUM, P->stream);
    if (e == hipSuccess)
        e = launch_cycle_end(P->at<double>(P->lay.normpart), nt, P->lay.lev[0].n, P->singular ? 1 : 0,
                             P->scal() + S_F2, P->p.rtol, P->hist() + slot, P->scal() + S_PHIMEAN, P->done(),
                             P->drho + slot, P->stream);
    if (e == hipSuccess && stats_host)
        e = hipMemcpyAsync(stats_host, P->scal(), sizeof(double) * kScal, hipMemcpyDeviceToHost, P->stream);
    return e;
}

// One refinement step: an FP32 V-cycle for A e = r32 from e = 0, then (fused
// into its last launch) phi64 += e and the new FP64 residual -> r32.
hipError_t enqueue_mixed_step(ccmg_plan *P, const double *d_f, long pf, MixedState &st, const int *skip,
                              int slot) {
    const Layout &lay = P->lay;
    CycleIO<float> io;
    io.f0 = st.r;
    io.pf0 = st.pr;
    io.phi0 = P->at<float>(lay.lev[0].a);
    io.pp0 = lay.lev[0].pitch;
    io.phi0b = P->at<float>(lay.lev[0].b);
    io.pp0b = lay.lev[0].pitch;
    io.zero = true;
    io.f0mean_part = st.s3;
    io.f0mean_count = st.r_tiles;
    io.partial3_out = st.s3o;
    io.post0 = POST_IR;
    io.skip = skip;
    io.q_in = st.q;
    io.pq_in = st.pq;
    io.q_out = st.qo;
    io.pq_out = st.pqo;
    io.g = d_f;
    io.pg = pf;
    io.r_out = st.ro;
    io.pr = st.pr;
    io.q_zero = st.q_zero;
    // the mean of phi64 from the last norm pass is removed as it is read
    io.q_shift = P->singular ? P->scal() + S_PHIMEAN : nullptr;
    int nt = 0;
    hipError_t e = enqueue_cycle<float>(P, io, &nt);
    if (e != hipSuccess) return e;
    std::swap(st.q, st.qo);
    std::swap(st.pq, st.pqo);
    std::swap(st.r, st.ro);
    std::swap(st.s3, st.s3o);
    st.r_tiles = nt;
    st.q_zero = false;
    return launch_cycle_end(P->at<double>(lay.normpart), nt, lay.lev[0].n, P->singular ? 1 : 0, P->scal() + S_F2,
                            P->p.rtol, P->hist() + slot, P->scal() + S_PHIMEAN, skip ? P->done() : nullptr,
                            skip ? P->drho + slot : nullptr, P->stream);
}

// A refinement step with m >= 2 FP32 V-cycles for A e = r32 (e from zero):
// level-0 pre-smoothing of the first cycle, then m - 1 fused level-0
// launches (post-smoothing of one inner cycle, pre-smoothing and restriction
// of the next; no norm, nothing kept), levels >= 1 after each, and the last
// cycle's post-smoothing with the FP64 update and residual (POST_IR).
hipError_t enqueue_mixed_step_inner(ccmg_plan *P, const double *d_f, long pf, MixedState &st, const int *skip,
                                   int slot, int m) {
    const Layout &lay = P->lay;
    hipStream_t s = P->stream;
    const double nn = (double)lay.lev[0].n * lay.lev[0].n;
    Buf<float> cur{P->at<float>(lay.lev[0].a), lay.lev[0].pitch};
    Buf<float> oth{P->at<float>(lay.lev[0].b), lay.lev[0].pitch};
    auto l0_args = [&](MarchArgs<float> &a) {
        level_consts(P, 0, a);
        a.f = st.r;
        a.pf = st.pr;
        if (P->singular) {  // the FP32 residual's mean (its per-tile sums) is removed as it is read
            a.fmean_part = st.s3;
            a.fmean_count = st.r_tiles;
        }
        a.skip = skip;
    };
    auto coarse = [&](int f1_count, Buf<float> &l1) -> hipError_t {
        CycleIO<float> io;
        io.f0 = st.r;
        io.pf0 = st.pr;
        io.phi0 = cur.p;
        io.pp0 = cur.pitch;
        io.phi0b = oth.p;
        io.pp0b = oth.pitch;
        io.skip = skip;
        io.coarse_only = true;
        io.f1_count = f1_count;
        io.l1_out = &l1;
        int dummy = 0;
        return enqueue_cycle<float>(P, io, &dummy);
    };
    int nt = 0;
    MarchArgs<float> a{};
    l0_args(a);
    a.phi_in = cur.p;
    a.pin = cur.pitch;
    a.phi_out = cur.p;  // from zero: nothing is read
    a.pout = cur.pitch;
    a.aux = P->at<float>(lay.lev[1].f);
    a.paux = lay.lev[1].pitch;
    a.partial = P->at<double>(lay.lev[1].fpart);
    int ti = P->tstart(2, sizeof(float) * nn * 2.25);
    hipError_t e = launch_march<float>(a, 2, false, false, POST_RESTRICT, P->shp_pre[0], s, &nt);
    P->tstop(ti);
    Buf<float> l1{nullptr, 0};
    if (e == hipSuccess) e = coarse(nt, l1);
    for (int i = 2; i <= m && e == hipSuccess; ++i) {
        MarchArgs<float> b{};
        l0_args(b);
        b.phi_in = cur.p;
        b.pin = cur.pitch;
        b.phi_out = oth.p;
        b.pout = oth.pitch;
        b.ec = l1.p;
        b.pc = l1.pitch;
        b.aux = P->at<float>(lay.lev[1].f);
        b.paux = lay.lev[1].pitch;
        b.partial = P->at<double>(lay.lev[1].fpart);
        ti = P->tstart(5, sizeof(float) * nn * 3.5);
        e = launch_march<float>(b, 4, true, true, POST_FUSED, P->shp_fused32, s, &nt);
        P->tstop(ti);
        std::swap(cur, oth);
        if (e == hipSuccess) e = coarse(nt, l1);
    }
    if (e != hipSuccess) return e;
    // the last inner cycle's post-smoothing, the FP64 update and the FP64 residual
    MarchArgs<float> c{};
    l0_args(c);
    c.phi_in = cur.p;
    c.pin = cur.pitch;
    c.phi_out = oth.p;  // not written: POST_IR stores the FP64 iterate
    c.pout = oth.pitch;
    c.ec = l1.p;
    c.pc = l1.pitch;
    c.q_in = st.q;
    c.pq_in = st.pq;
    c.q_out = st.qo;
    c.pq_out = st.pqo;
    c.g = d_f;
    c.pg = pf;
    c.r_out = st.ro;
    c.pr = st.pr;
    c.q_zero = st.q_zero ? 1 : 0;
    c.phi_shift = P->singular ? P->scal() + S_PHIMEAN : nullptr;
    c.partial = P->at<double>(lay.normpart);
    c.partial3 = st.s3o;
    const double h = lay.lev[0].h;
    c.alpha64 = P->p.alpha;
    c.beta64 = P->p.beta;
    c.ih2_64 = 1.0 / (h * h);
    ti = P->tstart(3, sizeof(float) * nn * 3.25 + nn * (3.0 * sizeof(double) + sizeof(float)));
    e = launch_march<float>(c, 2, true, true, POST_IR, P->shp_post[0], s, &nt);
    P->tstop(ti);
    if (e != hipSuccess) return e;
    std::swap(st.q, st.qo);
    std::swap(st.pq, st.pqo);
    std::swap(st.r, st.ro);
    std::swap(st.s3, st.s3o);
    st.r_tiles = nt;
    st.q_zero = false;
    return launch_cycle_end(P->at<double>(lay.normpart), nt, lay.lev[0].n, P->singular ? 1 : 0, P->scal() + S_F2,
                            P->p.rtol, P->hist() + slot, P->scal() + S_PHIMEAN, skip ? P->done() : nullptr,
                            skip ? P->drho + slot : nullptr, s);
}

// Host-side state of a plan for problem p (validated): layout, side type
// flags, default launch shapes and options.  No device or host allocation.
void plan_init_host(ccmg_plan *P, const ccmg_problem &p) {
    P->p = p;
    build_layout(p, P->lay);
    P->singular = p.alpha == 0.0 && p.bc[0] != CCMG_BC_DIRICHLET && p.bc[1] != CCMG_BC_DIRICHLET &&
                  p.bc[2] != CCMG_BC_DIRICHLET && p.bc[3] != CCMG_BC_DIRICHLET;
    for (int l = 0; l < P->lay.L && l < kMaxLevels; ++l) {
        P->shp_pre[l] = P->shp_post[l] = P->shp_pre_v[l] = shape_for(P->lay.lev[l].n);
        P->shp_visit[l] = visit_shape_for(P->lay.lev[l].n);
        P->visit[l] = false;
    }
    P->shp_fused = shape_for(P->lay.lev[0].n);
    P->shp_fused0 = shape_for(P->lay.lev[0].n);
    P->fused0 = false;
    P->shp_fused32 = shape_for(P->lay.lev[0].n);
    P->n_bottom = 2;
    P->tcycle = 0;
    P->timer.on = false;
    P->timer.used = 0;
    P->opt_fused = true;
    P->opt_fused_keep = 1.0;
    P->opt_mixed_inner = 3;
    P->opt_visit = 1;
}

// pitch >= n + 2, and the array holds fewer than 2^31 elements (the kernels
// form row offsets in 32 bits)
int check_pitch(const ccmg_plan *P, int level, ptrdiff_t pitch) {
    if (level < 0 || level >= P->lay.L) return CCMG_EINVAL;
    const ptrdiff_t rows = P->lay.lev[level].n + 2;
    if (pitch < rows || (double)pitch * (double)rows >= 2147483648.0) return CCMG_EINVAL;
    return CCMG_OK;
}

}  // namespace

// ============================================================================
extern "C" {

const char *ccmg_status_str(int s) {
    switch (s) {
        case CCMG_OK: return "ok";
        case CCMG_NOT_CONVERGED: return "not converged within max_cycles";
        case CCMG_EINVAL: return "invalid argument";
        case CCMG_ESIZE: return "n must be a power of two in [2, 16384]";
        case CCMG_EBC: return "bad boundary condition (unknown type or unpaired periodic side)";
        case CCMG_EINCOMPAT: return "singular problem with a right-hand side of nonzero mean";
        case CCMG_ENONFINITE: return "non-finite value in f or in a residual norm";
        case CCMG_EHIP: return "HIP runtime error";
        case CCMG_EWORKSPACE: return "workspace missing, too small or not 256-byte aligned";
    }
    return "unknown status";
}

int ccmg_problem_init(ccmg_problem *p, int n) {
    if (!p) return CCMG_EINVAL;
    std::memset(p, 0, sizeof(*p));
    p->n = n;
    p->ng = 1;
    p->xmin = 0.0;
    p->xmax = 1.0;
    p->ymin = 0.0;
    p->ymax = 1.0;
    for (int s = 0; s < 4; ++s) p->bc[s] = CCMG_BC_DIRICHLET;
    p->alpha = 0.0;
    p->beta = -1.0;
    p->nu1 = 2;
    p->nu2 = 2;
    p->nu_bottom = 50;
    p->max_cycles = 100;
    p->rtol = 1e-10;
    p->prec = CCMG_FP64;
    return ccmg_problem_check(p);
}

int ccmg_problem_check(const ccmg_problem *p) {
    if (!p) return CCMG_EINVAL;
    if (!pow2(p->n) || p->n > 16384) return CCMG_ESIZE;
    if (p->ng != 1) return CCMG_EINVAL;
    for (int s = 0; s < 4; ++s)
        if (p->bc[s] < CCMG_BC_DIRICHLET || p->bc[s] > CCMG_BC_PERIODIC) return CCMG_EBC;
    if ((p->bc[0] == CCMG_BC_PERIODIC) != (p->bc[1] == CCMG_BC_PERIODIC)) return CCMG_EBC;
    if ((p->bc[2] == CCMG_BC_PERIODIC) != (p->bc[3] == CCMG_BC_PERIODIC)) return CCMG_EBC;
    const double lx = p->xmax - p->xmin, ly = p->ymax - p->ymin;
    if (!(lx > 0) || !(ly > 0) || !std::isfinite(lx) || !std::isfinite(ly)) return CCMG_EINVAL;
    if (std::fabs(lx - ly) > 1e-12 * lx) return CCMG_EINVAL;
    if (!std::isfinite(p->alpha) || !std::isfinite(p->beta)) return CCMG_EINVAL;
    if (p->nu1 < 0 || p->nu1 > 8 || p->nu2 < 0 || p->nu2 > 8) return CCMG_EINVAL;
    if (p->nu_bottom < 0 || p->nu_bottom > 100000) return CCMG_EINVAL;
    if (p->max_cycles < 0 || p->max_cycles >= CCMG_HISTORY) return CCMG_EINVAL;
    if (!(p->rtol >= 0) || !std::isfinite(p->rtol)) return CCMG_EINVAL;
    if (p->prec != CCMG_FP64 && p->prec != CCMG_MIXED) return CCMG_EINVAL;
    // every level's relaxation divides by alpha + 4 beta / h^2
    const double h0 = lx / p->n;
    for (int l = 0; (p->n >> l) >= 2; ++l) {
        const double h = h0 * (double)(1 << l);
        const double d = p->alpha + 4.0 * p->beta / (h * h);
        if (d == 0.0 || !std::isfinite(d)) return CCMG_EINVAL;
    }
    return CCMG_OK;
}

size_t ccmg_workspace_bytes(const ccmg_problem *p) {
    if (ccmg_problem_check(p) != CCMG_OK) return 0;
    Layout lay;
    build_layout(*p, lay);
    return lay.total;
}

int ccmg_plan_create(const ccmg_problem *p, void *d_ws, size_t ws_bytes, void *stream, ccmg_plan **out) {
    if (!out) return CCMG_EINVAL;
    *out = nullptr;
    int st = ccmg_problem_check(p);
    if (st != CCMG_OK) return st;
    ccmg_plan *P = new (std::nothrow) ccmg_plan();
    if (!P) return CCMG_EINVAL;
    plan_init_host(P, *p);
    if (!d_ws || ws_bytes < P->lay.total || (reinterpret_cast<uintptr_t>(d_ws) & 255)) {
        delete P;
        return CCMG_EWORKSPACE;
    }
    P->ws = static_cast<char *>(d_ws);
    P->stream = static_cast<hipStream_t>(stream);
    {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
            P->simds = 4 * ncu;
    }
    hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&P->hpin), sizeof(double) * (CCMG_HISTORY + kScal),
                                 hipHostMallocDefault);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&P->hrho), sizeof(double) * CCMG_HISTORY,
                          hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void **>(&P->drho), P->hrho, 0);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&P->ev_sync[0], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&P->ev_sync[1], hipEventDisableTiming);
    for (int i = 0; i < 2 && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&P->ev_cyc[i], hipEventDisableTiming | hipEventDisableSystemFence);
    if (e == hipSuccess) e = hipEventCreate(&P->ev_t0);
    if (e == hipSuccess) e = hipEventCreate(&P->ev_t1);
    if (e != hipSuccess) {
        ccmg_plan_destroy(P);
        return CCMG_EHIP;
    }
    *out = P;
    return CCMG_OK;
}

}  // extern "C"

namespace {
// Rows per band that make a launch's wave count just fit k waves per SIMD
// (k = 1 .. kmax), one wave per workgroup.  The dispatcher spreads such
// workgroups evenly, so a wave count slightly above a multiple of the SIMD
// count leaves some SIMDs a whole band more to march than the rest (at
// 4096^2 the fused launch takes 136 us with 1280 waves on 1024 SIMDs and
// 116 us with 1000).
std::vector<int> balanced_tys(int n, int outw, int simds, int kmax, bool xwalls) {
    std::vector<int> out;
    const int strips = (n + outw - 1) / outw;
    for (int k = 1; k <= kmax; ++k) {
        // the most bands whose waves (edge strips' halved bands included) fit
        for (int chunks = k * simds / strips; chunks >= 1; --chunks) {
            int ty = (n + chunks - 1) / chunks;
            ty += ty & 1;
            if (ty >= n) break;
            if (ty < kMinTy || march_tiles(n, outw, ty, xwalls) > k * simds) continue;
            if (std::find(out.begin(), out.end(), ty) == out.end()) out.push_back(ty);
            break;
        }
    }
    return out;
}

// Time every candidate launch shape of each row-march level (the nu1 half and
// the nu2 half of the cycle separately) and keep the fastest.  T is the
// precision of the relaxed levels (double for FP64 plans, float for MIXED).
template <typename T>
hipError_t autotune_levels(ccmg_plan *P, const double *d_f, double *d_phi, ptrdiff_t pitch) {
    const Layout &lay = P->lay;
    hipStream_t s = P->stream;
    const bool f64 = sizeof(T) == sizeof(double);
    const bool xwalls = P->p.bc[CCMG_XLO] != CCMG_BC_PERIODIC;  // edge strips run halved bands
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return hipErrorOutOfMemory;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return hipErrorOutOfMemory;
    }
    // the workspace is scratch between calls: start from zeros (values do not
    // change the timing, but keep them finite)
    // (all but the exact bottom's inverse, the last region, which is kept)
    hipError_t err = hipMemsetAsync(P->ws, 0, lay.ainv, s);
    const int tys[] = {0, 8, 16, 32, 64, 128, 256};
    const int wpbs[] = {1, 2, 4};
    const int reps = 4;
    for (int l = 0; l < lay.lt && err == hipSuccess; ++l) {
        const int n = lay.lev[l].n;
        // kinds 0 / 1: the level's restricting and prolongating launches;
        // 2 / 3: the same level as a visit (restricting launch without the
        // stored iterate, visit launch), on levels where a visit applies
        const bool visit_ok = l >= 1 && P->p.nu1 == 2 && P->p.nu2 == 2;
        float kbest[4] = {0.f, 0.f, 0.f, 0.f};
        for (int kind = 0; kind < (visit_ok ? 4 : 2) && err == hipSuccess; ++kind) {
            MarchArgs<T> a{};
            level_consts(P, l, a);
            if (l == 0 && f64) {
                a.f = reinterpret_cast<const T *>(d_f);
                a.pf = pitch;
            } else {
                a.f = P->at<T>(lay.lev[l].f);
                a.pf = lay.lev[l].pitch;
            }
            const bool caller_phi = l == 0 && f64;
            T *pa = caller_phi ? reinterpret_cast<T *>(d_phi) : P->at<T>(lay.lev[l].a);
            const long ppa = caller_phi ? pitch : lay.lev[l].pitch;
            int nu, post;
            bool load_phi, prolong;
            a.phi_in = pa;
            a.pin = ppa;
            a.phi_out = P->at<T>(lay.lev[l].b);
            a.pout = lay.lev[l].pitch;
            if (kind == 0 || kind == 2) {  // the restricting launch of the nu1 half
                if (kind == 2) a.phi_out = nullptr;
                nu = split_nu(P->p.nu1).back();
                load_phi = l == 0 && f64;
                prolong = false;
                post = POST_RESTRICT;
                a.aux = P->at<T>(lay.lev[l + 1].f);
                a.paux = lay.lev[l + 1].pitch;
                a.partial = P->at<double>(lay.lev[l + 1].fpart);
            } else if (kind == 3) {  // the visit launch
                nu = 4;
                load_phi = false;
                prolong = true;
                post = POST_VISIT;
                a.phi_in = nullptr;
                a.ec = P->at<T>(lay.lev[l + 1].a);
                a.pc = lay.lev[l + 1].pitch;
            } else {  // the prolongating launch of the nu2 half
                nu = split_nu(P->p.nu2).front();
                load_phi = true;
                prolong = true;
                const bool single = split_nu(P->p.nu2).size() == 1;
                post = POST_NONE;
                if (l == 0 && single) post = f64 ? POST_NORM : POST_IR;
                a.ec = P->at<T>(lay.lev[l + 1].a);
                a.pc = lay.lev[l + 1].pitch;
                a.partial = P->at<double>(lay.normpart);
                if (post == POST_IR) {
                    a.q_in = d_phi;  // read only
                    a.pq_in = pitch;
                    a.q_out = P->at<double>(lay.qb);
                    a.pq_out = lay.lev[0].pitch;
                    a.g = d_f;
                    a.pg = pitch;
                    a.r_out = P->at<float>(lay.lev[0].f2);
                    a.pr = lay.lev[0].pitch;
                    a.partial3 = P->at<double>(lay.part3);
                    a.alpha64 = P->p.alpha;
                    a.beta64 = P->p.beta;
                    a.ih2_64 = 1.0 / (lay.lev[0].h * lay.lev[0].h);
                }
            }
            float best = 1e30f;
            MarchShape *const slot[4] = {&P->shp_pre[l], &P->shp_post[l], &P->shp_pre_v[l], &P->shp_visit[l]};
            MarchShape bs = *slot[kind];
            // candidates: row-march shapes (powers of two, and bands that
            // balance the waves over the SIMDs), and (levels below the finest)
            // the 2-D LDS tile kernel, written as ty = 0 (not for the visit
            // launch, whose bands need 8 halo rows a side: none below 16 rows)
            const bool tile_ok = l > 0 && n >= kTileMinN && kind != 3;
            std::vector<MarchShape> cands;
            for (int ty : tys) {
                if (ty == 0) {
                    if (tile_ok) cands.push_back(MarchShape{0, 1});
                    continue;
                }
                if (ty > n || (kind == 3 && ty < 16 && ty < n)) continue;
                for (int wpb : wpbs) cands.push_back(MarchShape{ty < n ? ty : n, wpb});
            }
            const bool res = post != POST_NONE && post != POST_VISIT;
            for (int ty : balanced_tys(n, march_outw(nu, prolong, res), P->simds, 4, xwalls))
                if (kind != 3 || ty >= 16) cands.push_back(MarchShape{ty, 1});
            for (const MarchShape &sh : cands) {
                {
                    int nt;
                    err = launch_march<T>(a, nu, load_phi, prolong, post, sh, s, &nt);  // warm-up
                    if (err == hipSuccess) err = hipEventRecord(e0, s);
                    for (int r = 0; r < reps && err == hipSuccess; ++r)
                        err = launch_march<T>(a, nu, load_phi, prolong, post, sh, s, &nt);
                    if (err == hipSuccess) err = hipEventRecord(e1, s);
                    if (err == hipSuccess) err = hipEventSynchronize(e1);
                    float ms = 0.f;
                    if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
                    if (err != hipSuccess) break;
                    if (ms < best) {
                        best = ms;
                        bs = sh;
                    }
                }
                if (err != hipSuccess) break;
            }
            *slot[kind] = bs;
            kbest[kind] = best;
        }
        // the visit pair replaces the two launches where it is faster
        if (err == hipSuccess && l < kMaxLevels) P->visit[l] = visit_ok && kbest[2] + kbest[3] < kbest[0] + kbest[1];
    }
    // Visits, level by level from the top: decided on the coarse part of whole
    // cycles (levels 1 down, as the fused driver runs them), each form timed
    // three times, the faster kept.  A launch timed alone misses how it
    // shares the caches with its neighbours in the cycle, and the small
    // levels' launches differ by a few microseconds.
    if (err == hipSuccess && P->p.nu1 == 2 && P->p.nu2 == 2 && lay.lt >= 2) {
        const int saved = P->opt_visit;
        P->opt_visit = 1;
        auto time_cycles = [&](float *best) -> hipError_t {
            CycleIO<T> io;
            io.coarse_only = true;
            io.f1_count = 1;
            Buf<T> l1{nullptr, 0};
            io.l1_out = &l1;
            int nt = 0;
            hipError_t x = enqueue_cycle<T>(P, io, &nt);  // warm-up
            if (x == hipSuccess) x = hipEventRecord(e0, s);
            for (int r = 0; r < 4 && x == hipSuccess; ++r) x = enqueue_cycle<T>(P, io, &nt);
            if (x == hipSuccess) x = hipEventRecord(e1, s);
            if (x == hipSuccess) x = hipEventSynchronize(e1);
            float ms = 0.f;
            if (x == hipSuccess) x = hipEventElapsedTime(&ms, e0, e1);
            if (x == hipSuccess && ms < *best) *best = ms;
            return x;
        };
        for (int l = 1; l < lay.lt && l < kMaxLevels && err == hipSuccess; ++l) {
            float on = 1e30f, off = 1e30f;
            for (int round = 0; round < 3 && err == hipSuccess; ++round) {
                P->visit[l] = false;
                err = time_cycles(&off);
                P->visit[l] = true;
                if (err == hipSuccess) err = time_cycles(&on);
            }
            P->visit[l] = on < off;
        }
        P->opt_visit = saved;
    }
    // the fused finest launch (FP64 plans that use it; MIXED plans with
    // several inner cycles per step, in FP32 without norm or kept iterate)
    const bool tune_fused = f64 ? fused_eligible(P) : mixed_inner_max(P) > 1;
    if (err == hipSuccess && tune_fused) {
        MarchArgs<T> a{};
        level_consts(P, 0, a);
        if (f64) {
            a.f = reinterpret_cast<const T *>(d_f);
            a.pf = pitch;
            a.phi_in = reinterpret_cast<T *>(d_phi);  // read only
            a.pin = pitch;
            a.phi_mid = P->at<T>(lay.lev[0].c);
            a.pmid = lay.lev[0].pitch;
            a.partial_norm = P->at<double>(lay.normpart);
        } else {
            a.f = P->at<T>(lay.lev[0].f);
            a.pf = lay.lev[0].pitch;
            a.phi_in = P->at<T>(lay.lev[0].a);
            a.pin = lay.lev[0].pitch;
        }
        a.phi_out = P->at<T>(lay.lev[0].b);
        a.pout = lay.lev[0].pitch;
        a.ec = P->at<T>(lay.lev[1].a);
        a.pc = lay.lev[1].pitch;
        a.aux = P->at<T>(lay.lev[1].f);
        a.paux = lay.lev[1].pitch;
        a.partial = P->at<double>(lay.lev[1].fpart);
        const int n = lay.lev[0].n;
        float best = 1e30f;
        MarchShape bs = f64 ? P->shp_fused : P->shp_fused32;
        std::vector<MarchShape> cands;
        for (int ty : {16, 32, 64, 128, 256}) {
            if (ty > n && ty != 16) continue;
            for (int wpb : {1, 2}) cands.push_back(MarchShape{ty < n ? ty : n, wpb});
        }
        for (int ty : balanced_tys(n, march_outw(4, true, true), P->simds, 4, xwalls)) cands.push_back(MarchShape{ty, 1});
        for (const MarchShape &sh : cands) {
            {
                int nt;
                err = launch_march<T>(a, 4, true, true, POST_FUSED, sh, s, &nt);  // warm-up
                if (err == hipSuccess) err = hipEventRecord(e0, s);
                for (int r = 0; r < reps && err == hipSuccess; ++r)
                    err = launch_march<T>(a, 4, true, true, POST_FUSED, sh, s, &nt);
                if (err == hipSuccess) err = hipEventRecord(e1, s);
                if (err == hipSuccess) err = hipEventSynchronize(e1);
                float ms = 0.f;
                if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
                if (err != hipSuccess) break;
                if (ms < best) {
                    best = ms;
                    bs = sh;
                }
            }
            if (err != hipSuccess) break;
        }
        if (f64) P->shp_fused = bs;
        else P->shp_fused32 = bs;
        // FP64: the first cycle's end of a solve from zero, with the first
        // pre-smoothing stored and the ordinary fused launch, against the
        // pre-smoothing unstored and the fused launch that recomputes it
        // (its bands carry 14 halo rows a side instead of 10)
        if (f64 && err == hipSuccess) {
            MarchArgs<T> pre{};
            level_consts(P, 0, pre);
            pre.f = a.f;
            pre.pf = a.pf;
            pre.phi_out = a.phi_out;
            pre.pout = a.pout;
            pre.aux = a.aux;
            pre.paux = a.paux;
            pre.partial = a.partial;
            MarchArgs<T> af = a;  // (no kept iterate: the first cycle's end keeps none)
            af.phi_mid = nullptr;
            MarchArgs<T> z = af;
            z.phi_in = nullptr;
            auto pair = [&](bool recompute, MarchShape sh, float *ms) -> hipError_t {
                MarchArgs<T> p0 = pre;
                if (recompute) p0.phi_out = nullptr;
                int nt;
                hipError_t x = hipSuccess;
                for (int r = 0; r <= reps && x == hipSuccess; ++r) {  // the first pair warms up
                    if (r == 1) x = hipEventRecord(e0, s);
                    if (x == hipSuccess) x = launch_march<T>(p0, 2, false, false, POST_RESTRICT, P->shp_pre[0], s, &nt);
                    if (x == hipSuccess)
                        x = recompute ? launch_march<T>(z, 6, false, true, POST_FUSED0, sh, s, &nt)
                                      : launch_march<T>(af, 4, true, true, POST_FUSED, sh, s, &nt);
                }
                if (x == hipSuccess) x = hipEventRecord(e1, s);
                if (x == hipSuccess) x = hipEventSynchronize(e1);
                if (x == hipSuccess) x = hipEventElapsedTime(ms, e0, e1);
                return x;
            };
            float stored = 1e30f, best0 = 1e30f;
            MarchShape bs0 = P->shp_fused0;
            err = pair(false, P->shp_fused, &stored);
            for (const MarchShape &sh : cands) {
                if (err != hipSuccess) break;
                if (sh.ty < 16 && sh.ty < n) continue;  // 14 halo rows a side
                float ms = 1e30f;
                err = pair(true, sh, &ms);
                if (err == hipSuccess && ms < best0) {
                    best0 = ms;
                    bs0 = sh;
                }
            }
            if (err == hipSuccess) {
                P->shp_fused0 = bs0;
                P->fused0 = best0 < stored;
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    return err;
}
}  // namespace

extern "C" {

// Autotune the launch shapes of every row-march level on the caller's data.
// Inputs are only read; outputs go to workspace buffers.
int ccmg_plan_autotune(ccmg_plan *P, const double *d_f, double *d_phi, ptrdiff_t pitch) {
    if (!P || !d_f || !d_phi) return CCMG_EINVAL;
    if (check_pitch(P, 0, pitch) != CCMG_OK) return CCMG_EINVAL;
    if (P->p.prec == CCMG_MIXED) return hip_status(autotune_levels<float>(P, d_f, d_phi, pitch));
    return hip_status(autotune_levels<double>(P, d_f, d_phi, pitch));
}

int ccmg_plan_set_shape(ccmg_plan *P, int level, int kind, int ty, int wpb) {
    if (!P || level < 0 || level >= P->lay.L || level >= kMaxLevels || kind < 0 || kind > 6) return CCMG_EINVAL;
    if (kind == 6) {  // the first fused launch recomputing the first pre-smoothing; ty = 0: not used
        const int n = P->lay.lev[0].n;
        if (level != 0) return CCMG_EINVAL;
        if (ty == 0) {
            P->fused0 = false;
            return CCMG_OK;
        }
        if (ty < 2 || (ty & 1) || (ty < 16 && ty < n) || wpb < 1 || wpb > 4) return CCMG_EINVAL;
        P->shp_fused0 = MarchShape{ty < n ? ty : n, wpb};
        P->fused0 = true;
        return CCMG_OK;
    }
    if (kind == 5) {  // the visit launch; ty = 0: the level runs its two launches instead
        if (level == 0 || level >= P->lay.lt) return CCMG_EINVAL;
        const int n = P->lay.lev[level].n;
        if (ty == 0) {
            P->visit[level] = false;
            return CCMG_OK;
        }
        if (ty < 2 || (ty & 1) || (ty < 16 && ty < n) || wpb < 1 || wpb > 4) return CCMG_EINVAL;
        P->shp_visit[level] = MarchShape{ty < n ? ty : n, wpb};
        P->visit[level] = true;
        return CCMG_OK;
    }
    if (kind == 4 && (level == 0 || level >= P->lay.lt)) return CCMG_EINVAL;
    if (kind == 2 || kind == 3) {  // the fused finest launch (FP64 / FP32)
        const int n = P->lay.lev[0].n;
        if (level != 0 || ty < 2 || (ty & 1) || (ty < kMinTy && ty < n) || wpb < 1 || wpb > 4) return CCMG_EINVAL;
        const MarchShape sh{ty < n ? ty : n, wpb};
        if (kind == 2) P->shp_fused = sh;
        else P->shp_fused32 = sh;
        return CCMG_OK;
    }
    if (ty == 0) {  // the 2-D LDS tile kernel: levels below the finest that are not in the tail
        if (level == 0 || level >= P->lay.lt || P->lay.lev[level].n < kTileMinN) return CCMG_EINVAL;
        (kind == 0 ? P->shp_pre : kind == 1 ? P->shp_post : P->shp_pre_v)[level] = MarchShape{0, 1};
        return CCMG_OK;
    }
    if (ty < 2 || (ty & 1) || wpb < 1 || wpb > 4) return CCMG_EINVAL;
    // the partial-sum buffers are sized for bands of at least kMinTy rows
    const int n = P->lay.lev[level].n;
    if (ty < kMinTy && ty < n) return CCMG_EINVAL;
    MarchShape sh{ty < n ? ty : n, wpb};
    (kind == 0 ? P->shp_pre : kind == 1 ? P->shp_post : P->shp_pre_v)[level] = sh;
    return CCMG_OK;
}

int ccmg_plan_shape(ccmg_plan *P, int level, int kind, int *ty, int *wpb) {
    if (!P || !ty || !wpb || level < 0 || level >= P->lay.L || level >= kMaxLevels || kind < 0 || kind > 6)
        return CCMG_EINVAL;
    if ((kind == 2 || kind == 3 || kind == 6) && level != 0) return CCMG_EINVAL;
    if (kind == 6) {
        *ty = P->fused0 ? P->shp_fused0.ty : 0;
        *wpb = P->fused0 ? P->shp_fused0.wpb : 1;
        return CCMG_OK;
    }
    if ((kind == 4 || kind == 5) && (level == 0 || level >= P->lay.lt)) return CCMG_EINVAL;
    const MarchShape sh = kind == 0   ? P->shp_pre[level]
                          : kind == 1 ? P->shp_post[level]
                          : kind == 2 ? P->shp_fused
                          : kind == 3 ? P->shp_fused32
                          : kind == 4 ? P->shp_pre_v[level]
                                      : P->shp_visit[level];
    const bool none = kind == 5 && !P->visit[level];  // (0, 1): the level runs its two launches
    *ty = none ? 0 : sh.ty;
    *wpb = none ? 1 : sh.wpb;
    return CCMG_OK;
}

int ccmg_plan_set_option(ccmg_plan *P, int option, double value) {
    if (!P || !std::isfinite(value)) return CCMG_EINVAL;
    switch (option) {
        case CCMG_OPT_FUSED:
            if (value != 0.0 && value != 1.0) return CCMG_EINVAL;
            P->opt_fused = value != 0.0;
            return CCMG_OK;
        case CCMG_OPT_FUSED_KEEP:
            if (value < 0.0) return CCMG_EINVAL;
            P->opt_fused_keep = value;
            return CCMG_OK;
        case CCMG_OPT_MIXED_INNER:
            if (value != std::floor(value) || value < 1.0 || value > 8.0) return CCMG_EINVAL;
            P->opt_mixed_inner = (int)value;
            return CCMG_OK;
        case CCMG_OPT_FMG:
            if (value != std::floor(value) || value < 0.0 || value > 4.0) return CCMG_EINVAL;
            P->opt_fmg = (int)value;
            return CCMG_OK;
        case CCMG_OPT_VISIT:
            if (value != 0.0 && value != 1.0 && value != 2.0) return CCMG_EINVAL;
            P->opt_visit = (int)value;
            return CCMG_OK;
        default: return CCMG_EINVAL;
    }
}

int ccmg_plan_get_option(ccmg_plan *P, int option, double *value) {
    if (!P || !value) return CCMG_EINVAL;
    switch (option) {
        case CCMG_OPT_FUSED: *value = P->opt_fused ? 1.0 : 0.0; return CCMG_OK;
        case CCMG_OPT_FUSED_KEEP: *value = P->opt_fused_keep; return CCMG_OK;
        case CCMG_OPT_MIXED_INNER: *value = (double)P->opt_mixed_inner; return CCMG_OK;
        case CCMG_OPT_FMG: *value = (double)P->opt_fmg; return CCMG_OK;
        case CCMG_OPT_VISIT: *value = (double)P->opt_visit; return CCMG_OK;
        default: return CCMG_EINVAL;
    }
}

int ccmg_plan_set_bottom(ccmg_plan *P, int n_bottom) {
    if (!P) return CCMG_EINVAL;
    if (n_bottom == 2) {
        P->n_bottom = 2;
        return CCMG_OK;
    }
    const ccmg_problem &p = P->p;
    // a level the tail holds, and a definite operator (no pivoting in the inverse)
    if ((n_bottom != 4 && n_bottom != kDirectMax) || n_bottom > P->lay.lev[P->lay.lt].n) return CCMG_EINVAL;
    if (p.beta == 0.0 || p.alpha * p.beta < 0.0) return CCMG_EINVAL;
    int lb = 0;
    while (P->lay.lev[lb].n != n_bottom) ++lb;
    hipError_t e = launch_bottom_inverse(n_bottom, p.bc, p.alpha, p.beta, P->lay.lev[lb].h, P->singular ? 1 : 0,
                                         P->at<double>(P->lay.ainv), P->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
    if (e != hipSuccess) return CCMG_EHIP;
    P->n_bottom = n_bottom;
    return CCMG_OK;
}

// side data of a plan: NULL for a homogeneous side; a periodic side takes none
static int bc_data(const ccmg_plan *P, const double *const d_b[4], BcData &d) {
    for (int s = 0; s < 4; ++s) {
        d.type[s] = P->p.bc[s];
        d.b[s] = d_b ? d_b[s] : nullptr;
        if (d.b[s] && P->p.bc[s] == CCMG_BC_PERIODIC) return CCMG_EINVAL;
    }
    return CCMG_OK;
}

int ccmg_bc_rhs(ccmg_plan *P, const double *d_f, double *d_f_out, ptrdiff_t pitch, const double *const d_b[4]) {
    if (!P || !d_f || !d_f_out || d_f == d_f_out) return CCMG_EINVAL;
    if (check_pitch(P, 0, pitch) != CCMG_OK) return CCMG_EINVAL;
    BcData d;
    if (bc_data(P, d_b, d) != CCMG_OK) return CCMG_EINVAL;
    return hip_status(launch_bc_rhs(d_f, d_f_out, pitch, P->lay.lev[0].n, d, P->p.beta, P->lay.lev[0].h, P->stream));
}

int ccmg_fill_ghosts_bc(ccmg_plan *P, double *d_phi, ptrdiff_t pitch, const double *const d_b[4]) {
    if (!P || !d_phi) return CCMG_EINVAL;
    if (check_pitch(P, 0, pitch) != CCMG_OK) return CCMG_EINVAL;
    BcData d;
    if (bc_data(P, d_b, d) != CCMG_OK) return CCMG_EINVAL;
    const int n = P->lay.lev[0].n;
    hipError_t e = launch_fill_ghosts_f64(d_phi, pitch, n, P->p.bc, nullptr, P->stream);
    if (e == hipSuccess) e = launch_add_ghost_data(d_phi, pitch, n, d, P->lay.lev[0].h, P->stream);
    return hip_status(e);
}

int ccmg_solve_bc(ccmg_plan *P, const double *d_f, double *d_phi, ptrdiff_t pitch, int use_guess,
                  const double *const d_b[4], double *d_work, ccmg_result *out) {
    ccmg_result local;
    ccmg_result *R = out ? out : &local;
    std::memset(R, 0, sizeof(*R));
    if (!P || !d_f || !d_phi || !d_work || d_work == d_f || d_work == d_phi) return R->status = CCMG_EINVAL;
    int st = ccmg_bc_rhs(P, d_f, d_work, pitch, d_b);
    if (st != CCMG_OK) return R->status = st;
    st = ccmg_solve(P, d_work, d_phi, pitch, use_guess, R);
    if (st != CCMG_OK && st != CCMG_NOT_CONVERGED) return st;
    const int g = ccmg_fill_ghosts_bc(P, d_phi, pitch, d_b);
    if (g != CCMG_OK) return R->status = g;
    hipError_t e = hipStreamSynchronize(P->stream);
    if (e != hipSuccess) return R->status = CCMG_EHIP;
    return st;
}

int ccmg_project(ccmg_plan *P, double *d_u, double *d_v, ptrdiff_t pitch, double *d_phi, double *d_work,
                 ccmg_result *out) {
    ccmg_result local;
    ccmg_result *R = out ? out : &local;
    std::memset(R, 0, sizeof(*R));
    if (!P || !d_u || !d_v || !d_phi || !d_work) return R->status = CCMG_EINVAL;
    const double *arrs[4] = {d_u, d_v, d_phi, d_work};
    for (int a = 0; a < 4; ++a)
        for (int b = a + 1; b < 4; ++b)
            if (arrs[a] == arrs[b]) return R->status = CCMG_EINVAL;
    if (P->p.alpha != 0.0 || P->p.beta != -1.0) return R->status = CCMG_EINVAL;
    for (int s = 0; s < 4; ++s)
        if (P->p.bc[s] != CCMG_BC_PERIODIC) return R->status = CCMG_EINVAL;
    if (check_pitch(P, 0, pitch) != CCMG_OK) return R->status = CCMG_EINVAL;
    const int n = P->lay.lev[0].n;
    const double h = P->lay.lev[0].h;
    const double nn = (double)n * n;
    int ti = P->tstart(7, 3.0 * sizeof(double) * nn);
    hipError_t e = launch_divergence(d_u, d_v, d_work, pitch, n, h, P->stream);
    P->tstop(ti);
    if (e != hipSuccess) return R->status = CCMG_EHIP;
    const int st = ccmg_solve(P, d_work, d_phi, pitch, 0, R);
    if (st != CCMG_OK && st != CCMG_NOT_CONVERGED) return st;
    ti = P->tstart(8, 5.0 * sizeof(double) * nn);
    e = launch_subtract_gradient(d_phi, d_u, d_v, pitch, n, h, P->stream);
    P->tstop(ti);
    if (e == hipSuccess) e = hipStreamSynchronize(P->stream);
    if (e != hipSuccess) return R->status = CCMG_EHIP;
    return st;
}

int ccmg_cn_rhs(ccmg_plan *P, const double *d_phi, double *d_f, ptrdiff_t pitch) {
    if (!P || !d_phi || !d_f || d_phi == d_f) return CCMG_EINVAL;
    if (check_pitch(P, 0, pitch) != CCMG_OK) return CCMG_EINVAL;
    const int n = P->lay.lev[0].n;
    const int ti = P->tstart(6, 2.0 * sizeof(double) * (double)n * n);
    hipError_t e = launch_cn_rhs(d_phi, pitch, d_f, pitch, n, P->p.bc, P->p.beta, P->lay.lev[0].h, P->stream);
    P->tstop(ti);
    return hip_status(e);
}

int ccmg_cn_step(ccmg_plan *P, double *d_phi, double *d_work, ptrdiff_t pitch, ccmg_result *out) {
    ccmg_result local;
    ccmg_result *R = out ? out : &local;
    std::memset(R, 0, sizeof(*R));
    if (!P || !d_phi || !d_work || d_phi == d_work || P->p.alpha != 1.0) return R->status = CCMG_EINVAL;
    // FP64 solves with the fused launch form the right-hand side in their
    // first pre-smoothing launch (which loads the old level anyway)
    if (P->p.prec == CCMG_FP64 && fused_eligible(P) && P->p.max_cycles > 0 && !P->singular)
        return solve_impl(P, d_work, d_phi, pitch, 1, R, INFINITY, d_work);
    const int st = ccmg_cn_rhs(P, d_phi, d_work, pitch);
    if (st != CCMG_OK) return R->status = st;
    return ccmg_solve(P, d_work, d_phi, pitch, 1, R);
}

int ccmg_plan_fused_shape(ccmg_plan *P, int kind, int *ty, int *wpb) {
    if (!P || !ty || !wpb || (kind != 2 && kind != 3)) return CCMG_EINVAL;
    const MarchShape &sh = kind == 2 ? P->shp_fused : P->shp_fused32;
    *ty = sh.ty;
    *wpb = sh.wpb;
    return CCMG_OK;
}

int ccmg_plan_shapes(ccmg_plan *P, int *ty_pre, int *wpb_pre, int *ty_post, int *wpb_post, int max_levels) {
    if (!P || !ty_pre || !wpb_pre || !ty_post || !wpb_post) return CCMG_EINVAL;
    for (int l = 0; l < max_levels && l < P->lay.L && l < kMaxLevels; ++l) {
        ty_pre[l] = P->shp_pre[l].ty;
        wpb_pre[l] = P->shp_pre[l].wpb;
        ty_post[l] = P->shp_post[l].ty;
        wpb_post[l] = P->shp_post[l].wpb;
    }
    return CCMG_OK;
}

int ccmg_plan_profile(ccmg_plan *P, int enable) {
    if (!P) return CCMG_EINVAL;
    if (enable && P->timer.ev.empty()) {
        P->timer.ev.assign(2 * KernelTimer::kPairs, nullptr);
        for (auto &e : P->timer.ev)
            if (hipEventCreate(&e) != hipSuccess) return CCMG_EHIP;
    }
    if (hipStreamSynchronize(P->stream) != hipSuccess) return CCMG_EHIP;
    P->timer.used = 0;
    for (int k = 0; k < KernelTimer::kKinds; ++k) {
        P->timer.launches[k] = 0;
        P->timer.ms[k] = P->timer.tbytes[k] = 0.0;
    }
    P->timer.on = enable != 0;
    return CCMG_OK;
}

int ccmg_plan_kernel_stats(ccmg_plan *P, ccmg_kernel_stat *out, int max, int *count) {
    if (!P || !count || (max > 0 && !out)) return CCMG_EINVAL;
    if (hipStreamSynchronize(P->stream) != hipSuccess) return CCMG_EHIP;
    P->tcollect();
    static const char *names[KernelTimer::kKinds] = {"finest_pre", "finest_post", "mixed_finest_pre",
                                                      "mixed_finest_post_ir", "finest_fused",
                                                      "mixed_finest_fused", "cn_rhs", "divergence",
                                                      "subtract_gradient", "finest_fused_first"};
    *count = KernelTimer::kKinds;
    for (int k = 0; k < KernelTimer::kKinds && k < max; ++k) {
        std::memset(&out[k], 0, sizeof(out[k]));
        std::strncpy(out[k].name, names[k], sizeof(out[k].name) - 1);
        out[k].launches = P->timer.launches[k];
        out[k].ms = P->timer.ms[k];
        out[k].bytes = P->timer.tbytes[k];
    }
    return CCMG_OK;
}

}  // extern "C"

namespace ccmg {
// c = a + b over `count` doubles (even count, 16-byte aligned): the streaming
// probe with `blocks` workgroups of 256 threads, nontemporal accesses if nt
// (util.hip).
hipError_t launch_probe_stream(const double *a, const double *b, double *c, long count, int blocks, bool nt,
                               hipStream_t s);
}  // namespace ccmg

extern "C" {

int ccmg_probe_stream(const double *d_a, const double *d_b, double *d_c, size_t count, int reps, void *stream,
                      float *ms, int *config) {
    if (!d_a || !d_b || !d_c || !ms || reps < 1 || count == 0 || (count & 1) ||
        ((reinterpret_cast<uintptr_t>(d_a) | reinterpret_cast<uintptr_t>(d_b) | reinterpret_cast<uintptr_t>(d_c)) & 15))
        return CCMG_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return CCMG_EHIP;
    // workgroups per compute unit x {ordinary, nontemporal}: keep the fastest
    static const int kPerCu[] = {2, 4, 8, 32, 128};
    float best = 0.f;
    int best_cfg = 0;
    hipError_t e = hipSuccess;
    for (int nt = 0; nt < 2 && e == hipSuccess; ++nt)
        for (int w : kPerCu) {
            const int blocks = w * cus;
            e = launch_probe_stream(d_a, d_b, d_c, (long)count, blocks, nt != 0, s);  // warm-up
            if (e == hipSuccess) e = hipEventRecord(e0, s);
            for (int r = 0; r < reps && e == hipSuccess; ++r)
                e = launch_probe_stream(d_a, d_b, d_c, (long)count, blocks, nt != 0, s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (e != hipSuccess) break;
            t /= (float)reps;
            if (best == 0.f || t < best) {
                best = t;
                best_cfg = 1000 * nt + w;
            }
        }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (e != hipSuccess) return CCMG_EHIP;
    *ms = best;
    if (config) *config = best_cfg;
    return CCMG_OK;
}

int ccmg_plan_destroy(ccmg_plan *P) {
    if (!P) return CCMG_EINVAL;
    for (auto &e : P->timer.ev)
        if (e) hipEventDestroy(e);
    if (P->hpin) hipHostFree(P->hpin);
    if (P->hrho) hipHostFree(P->hrho);
    for (int i = 0; i < 2; ++i) {
        if (P->ev_sync[i]) hipEventDestroy(P->ev_sync[i]);
        if (P->ev_cyc[i]) hipEventDestroy(P->ev_cyc[i]);
    }
    if (P->ev_t0) hipEventDestroy(P->ev_t0);
    if (P->ev_t1) hipEventDestroy(P->ev_t1);
    delete P;
    return CCMG_OK;
}

}  // extern "C"

namespace {
MixedState mixed_state(ccmg_plan *P, double *d_phi, ptrdiff_t pitch, bool q_zero) {
    const Layout &lay = P->lay;
    MixedState st;
    st.q = d_phi;
    st.pq = pitch;
    st.qo = P->at<double>(lay.qb);
    st.pqo = lay.lev[0].pitch;
    st.r = P->at<float>(lay.lev[0].f);
    st.ro = P->at<float>(lay.lev[0].f2);
    st.pr = lay.lev[0].pitch;
    st.s3 = P->at<double>(lay.part3);
    st.s3o = P->at<double>(lay.part3b);
    st.r_tiles = 0;
    st.q_zero = q_zero;
    return st;
}

// Copy the valid cells of an FP64 level-0 array (the iterate ended in the workspace).
hipError_t copy_valid(double *dst, long pd, const double *src, long ps, int n, hipStream_t s) {
    if (dst == src) return hipSuccess;
    return hipMemcpy2DAsync(dst + pd + 1, sizeof(double) * pd, src + ps + 1, sizeof(double) * ps,
                            sizeof(double) * n, n, hipMemcpyDeviceToDevice, s);
}

// ---- FP64 solves with fused finest-level launches ----------------------------
// The post-smoothing of cycle k and the pre-smoothing (and restriction) of
// cycle k+1 touch the same finest-level data back to back, so one launch does
// both (POST_FUSED): per cycle the finest level is read once instead of twice.
// The norm of cycle k is taken inside that launch, after the post-smoothing;
// its post-smoothed iterate is kept (phi_mid) whenever cycle k may be the last.
// The arithmetic of every cell is that of the unfused cycle.

struct FusedCtx {
    Buf<double> cur;     // level-0 buffer the next level-0 launch reads
    bool pre_done;       // the next cycle's pre-smoothing and level-1 rhs are done
    bool first_zero;     // the first pre-smoothing starts from zero
    int f1_count;        // partial sums of the level-1 rhs
    Buf<double> res;     // where the last enqueued cycle's post-smoothed iterate is (p = null: not kept)
    Buf<double> next;    // the pre-smoothed iterate of the following cycle (fused end)
    Buf<double> first_ec{nullptr, 0};  // full multigrid start: the level-1 phi that the first
                                       // pre-smoothing prolongates into a zero field
    // the first pre-smoothing also takes f's statistics (into the scalars,
    // then copied to `stats_host`), the solve's separate pass being skipped
    bool first_stats = false;
    double *stats_host = nullptr;
    // the first pre-smoothing (from a guess) also takes the guess's residual
    // norm, filed as the history's entry 0 (the solve's separate pass skipped)
    bool first_norm = false;
    // Crank-Nicolson step: the first pre-smoothing (from the old level) forms
    // the right-hand side phi + beta Lap phi itself and writes it here
    double *cn_f = nullptr;
    // a first pre-smoothing from zero may leave its iterate unstored, the
    // first fused launch recomputing it (the solve allows at least 2 cycles);
    // `recompute`: the next fused launch must
    bool allow_recompute = false;
    bool recompute = false;
};

// One V-cycle of the fused driver: [level-0 pre] + levels >= 1 + level-0 end
// (fused or plain post) + stop test -> hist[slot].
hipError_t enqueue_fused_cycle(ccmg_plan *P, FusedCtx &cx, const double *d_f, long pf, Buf<double> A, int slot,
                               bool end_fused, bool with_mid) {
    const Layout &lay = P->lay;
    hipStream_t s = P->stream;
    const Buf<double> B{P->at<double>(lay.lev[0].b), lay.lev[0].pitch};
    const Buf<double> C{P->at<double>(lay.lev[0].c), lay.lev[0].pitch};
    // A (the caller's array) is written only by launches that produce a
    // cycle's final iterate (the kept post-smoothed iterate, or a plain post),
    // so a converged solve ends in A without a copy; intermediate iterates
    // alternate between B and C
    auto other = [&](const Buf<double> &x) { return x.p == B.p ? C : B; };
    const double nn = (double)lay.lev[0].n * lay.lev[0].n;
    hipError_t e = hipSuccess;
    int nt = 0;
    if (!cx.pre_done) {
        const Buf<double> out = other(cx.cur);
        MarchArgs<double> a{};
        level_consts(P, 0, a);
        a.f = d_f;
        a.pf = pf;
        a.phi_in = cx.cur.p;
        a.pin = cx.cur.pitch;
        a.phi_out = out.p;
        a.pout = out.pitch;
        a.phi_shift = (!cx.first_zero && P->singular) ? P->scal() + S_PHIMEAN : nullptr;
        a.skip = P->done();
        a.aux = P->at<double>(lay.lev[1].f);
        a.paux = lay.lev[1].pitch;
        a.partial = P->at<double>(lay.lev[1].fpart);
        if (cx.first_ec.p) {
            // phi = P (level-1 phi of the full multigrid pass), then the pre-smoothing
            a.ec = cx.first_ec.p;
            a.pc = cx.first_ec.pitch;
            a.phi_shift = nullptr;
            const int ti = P->tstart(0, sizeof(double) * nn * 2.5);
            e = launch_march<double>(a, 2, false, true, POST_RESTRICT, P->shp_pre[0], s, &nt);
            P->tstop(ti);
            cx.first_ec = Buf<double>{nullptr, 0};
        } else {
            if (cx.first_stats) a.fstat_part = P->at<double>(lay.fstats);
            const bool first_norm = cx.first_norm && !cx.first_zero;
            if (first_norm) a.in_norm_part = P->at<double>(lay.normpart);
            cx.recompute = cx.first_zero && cx.allow_recompute && end_fused;
            if (cx.recompute) a.phi_out = nullptr;
            int post = POST_RESTRICT;
            if (cx.cn_f && !cx.first_zero) {  // f is formed here, not read
                a.cn_f = cx.cn_f;
                a.pcnf = pf;
                a.cn_beta = P->p.beta;
                post = POST_CNPRE;
                cx.cn_f = nullptr;
            }
            const int ti = P->tstart(0, sizeof(double) * nn * ((cx.first_zero ? (cx.recompute ? 1.0 : 2.0) : 3.0) +
                                                               0.25));
            e = launch_march<double>(a, 2, !cx.first_zero, false, post, P->shp_pre[0], s, &nt);
            P->tstop(ti);
            if (e == hipSuccess && cx.first_stats) {
                e = launch_reduce4(P->at<double>(lay.fstats), nt, P->scal() + S_FSUM, s);
                // the guess's residual norm -> history entry 0 (a guess within
                // the tolerance sets the done flag: the rest of the cycle does nothing)
                if (e == hipSuccess && first_norm)
                    e = launch_cycle_end(P->at<double>(lay.normpart), nt, lay.lev[0].n, 0, P->scal() + S_F2,
                                         P->p.rtol, P->hist(), P->scal() + S_PHIMEAN, P->done(), P->drho, s);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(cx.stats_host, P->scal(), sizeof(double) * kScal, hipMemcpyDeviceToHost, s);
                cx.first_stats = false;
                cx.first_norm = false;
            }
        }
        if (e != hipSuccess) return e;
        cx.f1_count = nt;
        cx.cur = out;
        cx.first_zero = false;
    }
    CycleIO<double> io;
    io.f0 = d_f;
    io.pf0 = pf;
    io.phi0 = A.p;
    io.pp0 = A.pitch;
    io.phi0b = B.p;
    io.pp0b = B.pitch;
    io.skip = P->done();
    io.coarse_only = true;
    io.f1_count = cx.f1_count;
    Buf<double> l1{nullptr, 0};
    io.l1_out = &l1;
    int dummy = 0;
    e = enqueue_cycle<double>(P, io, &dummy);
    if (e != hipSuccess) return e;

    const Buf<double> out = other(cx.cur);
    MarchArgs<double> a{};
    level_consts(P, 0, a);
    a.f = d_f;
    a.pf = pf;
    a.phi_in = cx.cur.p;
    a.pin = cx.cur.pitch;
    a.phi_out = out.p;
    a.pout = out.pitch;
    a.ec = l1.p;
    a.pc = l1.pitch;
    a.skip = P->done();
    if (end_fused) {
        a.phi_mid = with_mid ? A.p : nullptr;  // the input is B or C here
        a.pmid = A.pitch;
        a.aux = P->at<double>(lay.lev[1].f);
        a.paux = lay.lev[1].pitch;
        a.partial = P->at<double>(lay.lev[1].fpart);
        a.partial_norm = P->at<double>(lay.normpart);
        if (cx.recompute) {  // the first cycle's pre-smoothing was not stored: recompute it from f
            a.phi_in = nullptr;
            const int ti = P->tstart(9, sizeof(double) * nn * (2.0 + 0.5 + (with_mid ? 1.0 : 0.0)));
            e = launch_march<double>(a, 6, false, true, POST_FUSED0, P->shp_fused0, s, &nt);
            P->tstop(ti);
            cx.recompute = false;
        } else {
            const int ti = P->tstart(4, sizeof(double) * nn * (3.0 + 0.5 + (with_mid ? 1.0 : 0.0)));
            e = launch_march<double>(a, 4, true, true, POST_FUSED, P->shp_fused, s, &nt);
            P->tstop(ti);
        }
        if (e != hipSuccess) return e;
        cx.f1_count = nt;
        cx.pre_done = true;
        cx.res = with_mid ? A : Buf<double>{nullptr, 0};
        cx.next = out;
        cx.cur = out;
    } else {
        if (cx.recompute) return hipErrorInvalidValue;  // (not reached: recompute only before a fused end)
        a.phi_out = A.p;
        a.pout = A.pitch;
        a.partial = P->at<double>(lay.normpart);
        const int ti = P->tstart(1, sizeof(double) * nn * 3.25);
        e = launch_march<double>(a, 2, true, true, POST_NORM, P->shp_post[0], s, &nt);
        P->tstop(ti);
        if (e != hipSuccess) return e;
        cx.pre_done = false;
        cx.res = A;
        cx.next = Buf<double>{nullptr, 0};
        cx.cur = A;
    }
    return launch_cycle_end(P->at<double>(lay.normpart), nt, lay.lev[0].n, P->singular ? 1 : 0, P->scal() + S_F2,
                            P->p.rtol, P->hist() + slot, P->scal() + S_PHIMEAN, P->done(), P->drho + slot, s);
}
}  // namespace

extern "C" {

int ccmg_vcycle(ccmg_plan *P, const double *d_f, double *d_phi, ptrdiff_t pitch) {
    if (!P || !d_f || !d_phi) return CCMG_EINVAL;
    if (check_pitch(P, 0, pitch) != CCMG_OK) return CCMG_EINVAL;
    if (P->p.prec == CCMG_FP64)
        return hip_status(enqueue_vcycle64(P, d_f, pitch, d_phi, pitch, false, nullptr, false, 0));
    // MIXED: one refinement step in place
    MixedState st = mixed_state(P, d_phi, pitch, false);
    hipError_t e = launch_set_int(P->done(), 1, 0, P->stream);
    if (e == hipSuccess) e = launch_set(P->scal(), kScal, 0.0, P->stream);
    if (e == hipSuccess) e = launch_fstats(d_f, pitch, P->lay.lev[0].n, P->at<double>(P->lay.fstats), kStatBlocks,
                                           P->scal() + S_FSUM, P->stream);
    if (e == hipSuccess) e = enqueue_mixed_start(P, d_f, pitch, st, true, 0);
    // the start pass may have set the done flag; the hook always runs the step
    if (e == hipSuccess) e = launch_set_int(P->done(), 1, 0, P->stream);
    if (e == hipSuccess) e = launch_set(P->scal() + S_PHIMEAN, 1, 0.0, P->stream);
    if (e == hipSuccess) e = enqueue_mixed_step(P, d_f, pitch, st, nullptr, 1);
    if (e == hipSuccess) e = copy_valid(d_phi, pitch, st.q, st.pq, P->lay.lev[0].n, P->stream);
    return hip_status(e);
}

// One V-cycle without a plan or workspace: the levels below the finest live in
// the library's static device scratch (one copy per device, see
// noalloc.hip).  The host side of the plan is a per-device static object, so
// nothing is allocated, on the device or the host.
int ccmg_vcycle_noalloc(const ccmg_problem *p, const double *d_f, double *d_phi, ptrdiff_t pitch, void *stream) {
    const int st = ccmg_problem_check(p);
    if (st != CCMG_OK) return st;
    if (!d_f || !d_phi || p->prec != CCMG_FP64) return CCMG_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return CCMG_EHIP;
    if (dev < 0 || dev >= kNoallocDevices) return CCMG_EINVAL;
    void *scratch = nullptr;
    size_t cap = 0;
    if (static_scratch(dev, &scratch, &cap) != hipSuccess) return CCMG_EHIP;
    std::lock_guard<std::mutex> lock(g_noalloc_mu[dev]);
    ccmg_plan *P = &g_noalloc_plan[dev];
    plan_init_host(P, *p);
    if (P->lay.total > cap) return CCMG_EWORKSPACE;
    P->ws = static_cast<char *>(scratch);
    P->stream = static_cast<hipStream_t>(stream);
    if (check_pitch(P, 0, pitch) != CCMG_OK) return CCMG_EINVAL;
    return hip_status(enqueue_vcycle64(P, d_f, pitch, d_phi, pitch, false, nullptr, false, 0));
}

size_t ccmg_noalloc_scratch_bytes(void) { return kStaticScratchBytes; }

}  // extern "C"

// ccmg_solve, and the learned solve's first attempt: with use_guess and a
// finite guess_reject, a guess whose relative residual is not finite or above
// guess_reject returns kGuessRejected before any cycle runs.
int ccmg::solve_impl(ccmg_plan *P, const double *d_f, double *d_phi, ptrdiff_t pitch, int use_guess,
                     ccmg_result *out, double guess_reject, double *cn_f) {
    ccmg_result local;
    ccmg_result *R = out ? out : &local;
    std::memset(R, 0, sizeof(*R));
    if (!P || !d_f || !d_phi) return R->status = CCMG_EINVAL;
    if (check_pitch(P, 0, pitch) != CCMG_OK) return R->status = CCMG_EINVAL;
    hipStream_t s = P->stream;
    const Layout &lay = P->lay;
    const int n = lay.lev[0].n;
    const bool mixed = P->p.prec == CCMG_MIXED;
    double *scal = P->scal();
    P->tcycle = 0;
    hipError_t e = hipEventRecord(P->ev_t0, s);

    // statistics of f, reset of the flags, and the starting residual
    if (e == hipSuccess) e = launch_set_int(P->done(), 1, 0, s);
    if (e == hipSuccess) e = launch_set(scal, kScal, 0.0, s);
    // full multigrid start: f's statistics and its restriction to level 1 from one read
    const bool fmg_f1 = P->opt_fmg > 0 && !use_guess && !mixed && lay.lt >= 1;
    // FP64 solves from zero with the fused finest launch take f's statistics
    // in the first pre-smoothing launch, from its own loads of f, and are
    // checked once the first cycle has run: no separate pass, and the device
    // does not wait for the host before the first cycle (on a bad f that
    // cycle's results are dropped)
    const bool stats_late = !use_guess && !mixed && P->opt_fmg == 0 && fused_eligible(P) && P->p.max_cycles > 0;
    // ... and from a guess (non-singular problems, no rejection bound): the
    // first launch also takes the guess's residual norm, read with the first
    // cycle's (the first cycle's end then waits for it on the host)
    const bool guess_late = use_guess && !mixed && fused_eligible(P) && P->p.max_cycles > 0 && !P->singular &&
                            !std::isfinite(guess_reject);
    // ... and MIXED solves: the start pass (the FP64 residual rounded to FP32)
    // takes f's statistics too, read with the first step's residual
    const bool mixed_late = mixed && P->p.max_cycles > 0 && !(use_guess && std::isfinite(guess_reject));
    const bool late = stats_late || guess_late || mixed_late;
    if (cn_f && !guess_late) return R->status = CCMG_EINVAL;  // (callers check first)
    if (e == hipSuccess && fmg_f1)
        e = launch_fstats_restrict(d_f, pitch, n, P->at<double>(lay.fstats), kStatBlocks, scal + S_FSUM,
                                   P->at<double>(lay.lev[1].f), lay.lev[1].pitch, s);
    else if (e == hipSuccess && !late)
        e = launch_fstats(d_f, pitch, n, P->at<double>(lay.fstats), kStatBlocks, scal + S_FSUM, s);
    // full multigrid start (FP64 solves without a guess, option CCMG_OPT_FMG):
    // its last launch also gives the starting residual, as a guess's would
    // (FP64 solves with the fused finest launch prolongate the FMG result
    // inside their first pre-smoothing launch; the start's own residual is
    // then not formed and rel_resid0 is NaN)
    const bool fmg = P->opt_fmg > 0 && !use_guess && !mixed;
    const bool fmg_fused = fmg && fused_eligible(P);
    if (e == hipSuccess && fmg && !fmg_fused)
        e = enqueue_fmg(P, d_f, pitch, d_phi, pitch, P->opt_fmg, P->opt_fmg, 0, nullptr, fmg_f1);
    const bool guess = use_guess || fmg;
    MixedState st = mixed_state(P, d_phi, pitch, !use_guess);
    if (e == hipSuccess && mixed) {
        e = enqueue_mixed_start(P, d_f, pitch, st, use_guess != 0, 0,  // r32, rho0 -> hist[0]
                                mixed_late ? P->hpin + CCMG_HISTORY : nullptr);
    } else if (e == hipSuccess && use_guess && !guess_late) {
        MarchArgs<double> a{};
        level_consts(P, 0, a);
        a.f = d_f;
        a.pf = pitch;
        a.phi_in = d_phi;
        a.pin = pitch;
        a.partial = P->at<double>(lay.normpart);
        int nt = 0;
        e = launch_march<double>(a, 0, true, false, POST_NORM, shape_for(n), s, &nt);
        if (e == hipSuccess)
            e = launch_cycle_end(P->at<double>(lay.normpart), nt, n, P->singular ? 1 : 0, scal + S_F2,
                                 P->p.rtol, P->hist(), scal + S_PHIMEAN, P->done(), P->drho, s);
    }
    if (e == hipSuccess && !late)
        e = hipMemcpyAsync(P->hpin + CCMG_HISTORY, scal, sizeof(double) * kScal, hipMemcpyDeviceToHost, s);
    Buf<double> fmg_l1{nullptr, 0};
    if (late) {
        // checked after the first cycle (below)
    } else if (fmg_fused) {
        // the full multigrid pass (workspace only) is queued before the host
        // waits for f's statistics: its many small launches are enqueued while
        // the device still works, and it runs while the host checks them
        if (e == hipSuccess) e = hipEventRecord(P->ev_sync[0], s);
        if (e == hipSuccess)
            e = enqueue_fmg(P, d_f, pitch, d_phi, pitch, P->opt_fmg, P->opt_fmg, -1, &fmg_l1, fmg_f1);
        if (e == hipSuccess) e = hipEventSynchronize(P->ev_sync[0]);
    } else if (e == hipSuccess) {
        e = hipStreamSynchronize(s);
    }
    if (e != hipSuccess) return R->status = CCMG_EHIP;
    const double *hs = P->hpin + CCMG_HISTORY;
    // f's statistics: kGoOn, or the status to return (phi = 0 for a zero f),
    // after the device work queued so far has finished
    constexpr int kGoOn = 1 << 20;
    auto check_f = [&]() -> int {
        int st = kGoOn;
        if (hs[S_FBAD] > 0 || !std::isfinite(hs[S_F2])) st = CCMG_ENONFINITE;
        else if (hs[S_F2] == 0.0) st = CCMG_OK;
        else if (P->singular && std::fabs(hs[S_FSUM]) > 1e-12 * hs[S_FABS]) st = CCMG_EINCOMPAT;
        if (st == kGoOn) return st;
        hipError_t x = hipSuccess;
        if (st == CCMG_OK)  // phi = 0 exactly (valid and ghost cells)
            x = hipMemset2DAsync(d_phi, sizeof(double) * pitch, 0, sizeof(double) * (n + 2), n + 2, s);
        if (x == hipSuccess) x = hipStreamSynchronize(s);
        return x == hipSuccess ? st : CCMG_EHIP;
    };
    if (!late) {
        const int st = check_f();
        if (st != kGoOn) return R->status = st;
    }

    const double rho0 = (fmg_fused || guess_late || mixed_late) ? NAN : (guess || mixed) ? P->hrho[0] : 1.0;
    R->rel_resid0 = rho0;
    R->history[0] = rho0;
    if (use_guess && std::isfinite(guess_reject) && !(rho0 <= guess_reject)) return R->status = kGuessRejected;
    if (!fmg_fused && !guess_late && !mixed_late && !std::isfinite(rho0)) return R->status = CCMG_ENONFINITE;
    int status = CCMG_NOT_CONVERGED;
    int cycles = 0;
    double rho = rho0;
    // MIXED: where the iterate is after each step (steps queued past convergence do nothing)
    std::vector<MixedState> after(P->p.max_cycles + 2, st);
    std::vector<int> inner_used(P->p.max_cycles + 2, 1);  // ... and its FP32 V-cycles
    // FP64 with fused finest launches: the driver's state after each cycle
    const bool fused = !mixed && fused_eligible(P);
    const double keep = P->opt_fused_keep;
    FusedCtx fx{Buf<double>{d_phi, pitch}, false, !guess, 0, Buf<double>{nullptr, 0}, Buf<double>{nullptr, 0}};
    if (fmg_fused) fx.first_ec = fmg_l1;
    fx.first_stats = late;
    fx.first_norm = guess_late;
    fx.cn_f = cn_f;
    fx.stats_host = P->hpin + CCMG_HISTORY;
    fx.allow_recompute = P->p.max_cycles >= 2 && (P->opt_visit == 2 || (P->opt_visit == 1 && P->fused0));
    std::vector<FusedCtx> fafter(P->p.max_cycles + 2, fx);
    if (rho0 <= P->p.rtol) {
        status = CCMG_OK;
    } else if (P->p.max_cycles > 0) {
        const double *shift = P->singular ? scal + S_PHIMEAN : nullptr;
        std::vector<double> rhos(P->p.max_cycles + 2, 0.0);
        // (a start whose residual was not formed predicts like the zero start)
        rhos[0] = std::isfinite(rho0) ? rho0 : 1.0;
        int checked = 0;  // cycles whose residual the host has read
        const int inner_max = mixed ? mixed_inner_max(P) : 1;
        std::vector<int> &inner = inner_used;
        // residual of cycle j extrapolated from the last two that were read;
        // before two are known, a lower bound: no V-cycle here contracts the
        // residual by more than 100x
        auto predict = [&](int j) -> double {
            const int m = checked;
            if (m < 1 || !(rhos[m - 1] > 0.0)) return rhos[m] * std::pow(0.01, (double)(j - m));
            return rhos[m] * std::pow(rhos[m] / rhos[m - 1], (double)(j - m));
        };
        // MIXED with several FP32 cycles per step: the per-cycle contraction of
        // the last step read, the residual it predicts at the start of step j,
        // and the inner cycles that step j needs to reach the tolerance (at
        // most inner_max).  The first step runs 2 cycles and step 2 is queued
        // only once its residual is known: contraction rates range from about
        // 0.1 (Poisson) to below 1e-6 (strongly diagonal Helmholtz), and a
        // blind guess either way costs whole cycles.  One a-priori bound is
        // used: a red-black sweep of a diagonally dominant operator contracts
        // the error by at least gamma = |4 beta / h^2| / |alpha + 4 beta / h^2|
        // (max norm), so when gamma^(2 (nu1 + nu2)) <= 1e-3 a cycle's
        // smoothing alone is worth three digits (its coarse correction, as
        // measured, only adds to that) and the first step runs one cycle.
        auto mixed_rate = [&]() -> double {
            const int m = checked;
            if (m < 1 || !(rhos[m - 1] > 0.0) || !(rhos[m] > 0.0)) return 0.1;
            const double r = std::pow(rhos[m] / rhos[m - 1], 1.0 / inner[m]);
            return (r > 0.0 && r < 0.9) ? r : 0.9;
        };
        auto mixed_pred = [&](int j) -> double {  // residual after step j - 1
            const double rate = mixed_rate();
            double r = rhos[checked];
            for (int i = checked + 1; i < j; ++i) r *= std::pow(rate, inner[i]);
            return r;
        };
        const int first_inner = [&] {
            const double h = P->lay.lev[0].h, c4 = 4.0 * P->p.beta / (h * h);
            const double gamma = std::fabs(c4) / std::fabs(P->p.alpha + c4);
            const bool diagonal = std::fabs(P->p.alpha + c4) > std::fabs(c4) &&
                                  std::pow(gamma, 2.0 * (P->p.nu1 + P->p.nu2)) <= 1e-3;
            return diagonal ? 1 : std::min(2, inner_max);
        }();
        auto inner_for = [&](int j) -> int {
            if (inner_max <= 1) return 1;
            if (j == 1 || checked == 0) return first_inner;
            const double r = mixed_pred(j);
            if (!(r > P->p.rtol)) return 1;
            const int need = (int)std::ceil(std::log(P->p.rtol / r) / std::log(mixed_rate()));
            if (need == inner_max + 1) return need;  // one more cycle than the cap ends the solve
            return std::max(1, std::min(inner_max, need));
        };
        auto cycle_event = [&](int k) { return k >= 2 ? P->ev_cyc[k & 1] : P->ev_sync[k & 1]; };
        auto enqueue = [&](int k) -> hipError_t {  // cycle / step k (1-based) -> hist[k]
            hipError_t x;
            P->tcycle = k;
            if (mixed) {
                inner[k] = inner_for(k);
                x = inner[k] >= 2 ? enqueue_mixed_step_inner(P, d_f, pitch, st, P->done(), k, inner[k])
                                  : enqueue_mixed_step(P, d_f, pitch, st, P->done(), k);
                after[k] = st;
            } else if (fused) {
                // the end of cycle k also pre-smooths cycle k+1 unless k is
                // expected to be the last; its post-smoothed iterate is kept
                // while k may be the last
                const double pred = predict(k);
                const bool end_fused = k < P->p.max_cycles && !(pred <= 0.5 * P->p.rtol && checked >= 2);
                // the extrapolation is trusted once three residuals are known;
                // before that (short solves from a good guess contract faster
                // than their first cycles show) the window is at least 100x
                const double kf = (keep == 0.0 || checked >= 3) ? keep : std::max(keep, 100.0);
                const bool with_mid = !std::isfinite(pred) || pred <= kf * P->p.rtol;
                x = enqueue_fused_cycle(P, fx, d_f, pitch, Buf<double>{d_phi, pitch}, k, end_fused, with_mid);
                fafter[k] = fx;
            } else {
                x = enqueue_vcycle64(P, d_f, pitch, d_phi, pitch, k == 1 && !guess, shift, true, k);
            }
            if (x == hipSuccess) x = hipEventRecord(cycle_event(k), s);
            return x;
        };
        // Cycle k+1 is queued before cycle k's residual is read, so the GPU
        // never waits for the host; if cycle k converges, k+1 runs as no-ops
        // (each launch still costs a dispatch).  When the last two residuals
        // predict that cycle k converges, k+1 is queued only after the check.
        e = enqueue(1);
        int queued = 1;
        for (int k = 1; e == hipSuccess; ++k) {
            if (queued == k && k < P->p.max_cycles) {
                const bool check_first =  // queue k+1 only after reading k
                    (mixed && inner_max > 1)
                        ? (k == 1 || mixed_pred(k + 1) <= 0.5 * P->p.rtol)
                        : (((guess_late || mixed_late) && k == 1) ||  // (the start's residual comes with cycle 1's)
                           (k >= 3 && rhos[k - 2] > 0.0 && rhos[k - 1] * (rhos[k - 1] / rhos[k - 2]) <= 0.5 * P->p.rtol));
                if (!check_first) {
                    e = enqueue(k + 1);
                    queued = k + 1;
                }
            }
            if (e != hipSuccess) break;
            e = hipEventSynchronize(cycle_event(k));
            if (e != hipSuccess) break;
            if (late && k == 1) {  // f's statistics (and the guess's residual) came with the first cycle
                const int st = check_f();
                if (st != kGoOn) {
                    std::memset(R, 0, sizeof(*R));
                    return R->status = st;
                }
                if (guess_late || mixed_late) {
                    const double r0 = P->hrho[0];
                    R->rel_resid0 = r0;
                    R->history[0] = r0;
                    rhos[0] = r0;
                    if (!std::isfinite(r0)) {  // (the device skipped the cycle)
                        e = hipStreamSynchronize(s);
                        return R->status = e == hipSuccess ? CCMG_ENONFINITE : CCMG_EHIP;
                    }
                    if (r0 <= P->p.rtol) {  // the guess meets the tolerance: the cycle did nothing
                        rho = r0;
                        status = CCMG_OK;
                        break;
                    }
                }
            }
            rho = P->hrho[k];  // written by the step's last kernel (host-mapped)
            R->history[k] = rho;
            rhos[k] = rho;
            checked = k;
            cycles = k;
            if (!std::isfinite(rho)) {
                status = CCMG_ENONFINITE;
                break;
            }
            if (rho <= P->p.rtol) {
                status = CCMG_OK;
                break;
            }
            if (k >= P->p.max_cycles) break;
            if (queued == k) {  // the prediction was wrong: queue the next cycle now
                e = enqueue(k + 1);
                queued = k + 1;
            }
        }
        if (e != hipSuccess) return R->status = CCMG_EHIP;
        if (fused && cycles > 0) {
            const FusedCtx &fc = fafter[cycles];
            if (fc.res.p) {
                e = copy_valid(d_phi, pitch, fc.res.p, fc.res.pitch, n, s);
            } else {
                // the last cycle ended in a fused launch whose post-smoothed
                // iterate was not kept (it was not expected to be the last):
                // take the next cycle's pre-smoothed iterate (two more sweeps)
                // with its own residual, and continue plainly if that is short
                const int slot = std::min(cycles + 1, CCMG_HISTORY - 1);
                e = copy_valid(d_phi, pitch, fc.next.p, fc.next.pitch, n, s);
                if (e == hipSuccess) e = launch_set_int(P->done(), 1, 0, s);
                MarchArgs<double> a{};
                level_consts(P, 0, a);
                a.f = d_f;
                a.pf = pitch;
                a.phi_in = d_phi;
                a.pin = pitch;
                a.partial = P->at<double>(lay.normpart);
                int nt = 0;
                if (e == hipSuccess) e = launch_march<double>(a, 0, true, false, POST_NORM, shape_for(n), s, &nt);
                if (e == hipSuccess)
                    e = launch_cycle_end(P->at<double>(lay.normpart), nt, n, P->singular ? 1 : 0, scal + S_F2,
                                         P->p.rtol, P->hist() + slot, scal + S_PHIMEAN, P->done(), P->drho + slot, s);
                if (e == hipSuccess) e = hipStreamSynchronize(s);
                if (e == hipSuccess) {
                    rho = P->hrho[slot];
                    if (!std::isfinite(rho)) status = CCMG_ENONFINITE;
                    else if (rho <= P->p.rtol) status = CCMG_OK;
                    else status = CCMG_NOT_CONVERGED;
                }
                for (int k = cycles + 1; e == hipSuccess && status == CCMG_NOT_CONVERGED && k <= P->p.max_cycles;
                     ++k) {
                    const int sl = std::min(k, CCMG_HISTORY - 1);
                    e = launch_set_int(P->done(), 1, 0, s);
                    if (e == hipSuccess) e = enqueue_vcycle64(P, d_f, pitch, d_phi, pitch, false, shift, true, sl);
                    if (e == hipSuccess) e = hipStreamSynchronize(s);
                    if (e != hipSuccess) break;
                    rho = P->hrho[sl];
                    R->history[sl] = rho;
                    cycles = k;
                    if (!std::isfinite(rho)) status = CCMG_ENONFINITE;
                    else if (rho <= P->p.rtol) status = CCMG_OK;
                }
            }
            if (e != hipSuccess) return R->status = CCMG_EHIP;
        }
    }
    if (mixed) {
        // the FP64 iterate of the last step that ran (or the guess / zero)
        const MixedState &fin = cycles > 0 ? after[cycles] : after[0];
        if (fin.q_zero) e = hipMemset2DAsync(d_phi, sizeof(double) * pitch, 0, sizeof(double) * (n + 2), n + 2, s);
        else e = copy_valid(d_phi, pitch, fin.q, fin.pq, n, s);
        if (e != hipSuccess) return R->status = CCMG_EHIP;
        int total = 0;
        for (int k = 1; k <= cycles; ++k) total += inner_used[k];
        R->inner_cycles = total;
    }
    // output: zero-mean representative for singular problems, ghost cells filled
    e = launch_fill_ghosts_f64(d_phi, pitch, n, P->p.bc, P->singular ? scal + S_PHIMEAN : nullptr, s);
    if (e == hipSuccess) e = hipEventRecord(P->ev_t1, s);
    if (e == hipSuccess) e = hipEventSynchronize(P->ev_t1);
    if (e != hipSuccess) return R->status = CCMG_EHIP;
    float ms = 0.f;
    hipEventElapsedTime(&ms, P->ev_t0, P->ev_t1);
    P->tcycle = 0;
    if (P->timer.on) P->tcollect(cycles);  // every launch has finished
    R->ms = ms;
    R->cycles = cycles;
    R->rel_resid = rho;
    R->status = status;
    return status;
}

extern "C" {

int ccmg_solve(ccmg_plan *P, const double *d_f, double *d_phi, ptrdiff_t pitch, int use_guess,
               ccmg_result *out) {
    return solve_impl(P, d_f, d_phi, pitch, use_guess, out, INFINITY);
}

int ccmg_fmg(ccmg_plan *P, const double *d_f, double *d_phi, ptrdiff_t pitch, int ncyc_top, int ncyc) {
    if (!P || !d_f || !d_phi || P->p.prec != CCMG_FP64) return CCMG_EINVAL;
    if (ncyc_top < 1 || ncyc_top > 16 || ncyc < 0 || ncyc > 16) return CCMG_EINVAL;
    if (check_pitch(P, 0, pitch) != CCMG_OK) return CCMG_EINVAL;
    hipError_t e = enqueue_fmg(P, d_f, pitch, d_phi, pitch, ncyc_top, ncyc, -1);
    if (e == hipSuccess) e = launch_fill_ghosts_f64(d_phi, pitch, P->lay.lev[0].n, P->p.bc, nullptr, P->stream);
    return hip_status(e);
}

// ---- single steps -----------------------------------------------------------
int ccmg_fill_ghosts(ccmg_plan *P, int level, double *d_a, ptrdiff_t pitch) {
    if (!P || !d_a) return CCMG_EINVAL;
    if (check_pitch(P, level, pitch) != CCMG_OK) return CCMG_EINVAL;
    return hip_status(launch_fill_ghosts_f64(d_a, pitch, P->lay.lev[level].n, P->p.bc, nullptr, P->stream));
}

int ccmg_smooth(ccmg_plan *P, int level, int iters, const double *d_f, const double *d_phi_in,
                double *d_phi_out, ptrdiff_t pitch) {
    if (!P || !d_f || !d_phi_in || !d_phi_out || d_phi_in == d_phi_out) return CCMG_EINVAL;
    if (iters < 1 || iters > 2 || check_pitch(P, level, pitch) != CCMG_OK) return CCMG_EINVAL;
    MarchArgs<double> a{};
    level_consts(P, level, a);
    a.f = d_f;
    a.pf = pitch;
    a.phi_in = d_phi_in;
    a.pin = pitch;
    a.phi_out = d_phi_out;
    a.pout = pitch;
    int nt;
    return hip_status(launch_march<double>(a, iters, true, false, POST_NONE, shape_for(a.n), P->stream, &nt));
}

int ccmg_residual(ccmg_plan *P, int level, const double *d_f, const double *d_phi, double *d_r,
                  ptrdiff_t pitch) {
    if (!P || !d_f || !d_phi || !d_r) return CCMG_EINVAL;
    if (check_pitch(P, level, pitch) != CCMG_OK) return CCMG_EINVAL;
    MarchArgs<double> a{};
    level_consts(P, level, a);
    a.f = d_f;
    a.pf = pitch;
    a.phi_in = d_phi;
    a.pin = pitch;
    a.aux = d_r;
    a.paux = pitch;
    int nt;
    return hip_status(launch_march<double>(a, 0, true, false, POST_RESID, shape_for(a.n), P->stream, &nt));
}

int ccmg_restrict_residual(ccmg_plan *P, int level, const double *d_f, const double *d_phi, ptrdiff_t pitch,
                           double *d_fc, ptrdiff_t pitch_c) {
    if (!P || !d_f || !d_phi || !d_fc) return CCMG_EINVAL;
    if (check_pitch(P, level, pitch) != CCMG_OK || check_pitch(P, level + 1, pitch_c) != CCMG_OK)
        return CCMG_EINVAL;
    MarchArgs<double> a{};
    level_consts(P, level, a);
    a.f = d_f;
    a.pf = pitch;
    a.phi_in = d_phi;
    a.pin = pitch;
    a.aux = d_fc;
    a.paux = pitch_c;
    a.partial = P->at<double>(P->lay.normpart);
    int nt;
    return hip_status(
        launch_march<double>(a, 0, true, false, POST_RESTRICT, shape_for(a.n), P->stream, &nt));
}

int ccmg_restrict(ccmg_plan *P, int level, const double *d_fine, ptrdiff_t pitch, double *d_coarse,
                  ptrdiff_t pitch_c) {
    if (!P || !d_fine || !d_coarse) return CCMG_EINVAL;
    if (check_pitch(P, level, pitch) != CCMG_OK || check_pitch(P, level + 1, pitch_c) != CCMG_OK)
        return CCMG_EINVAL;
    const int nc = P->lay.lev[level + 1].n;
    // the coarse array must not overlap the fine one
    const char *f0 = reinterpret_cast<const char *>(d_fine);
    const char *f1 = f0 + sizeof(double) * (size_t)(P->lay.lev[level].n + 2) * (size_t)pitch;
    const char *c0 = reinterpret_cast<const char *>(d_coarse);
    const char *c1 = c0 + sizeof(double) * (size_t)(nc + 2) * (size_t)pitch_c;
    if (c0 < f1 && f0 < c1) return CCMG_EINVAL;
    return hip_status(launch_restrict(d_fine, pitch, d_coarse, pitch_c, nc, P->stream));
}

int ccmg_prolong_add(ccmg_plan *P, int level, const double *d_ec, ptrdiff_t pitch_c, const double *d_phi_in,
                     double *d_phi_out, ptrdiff_t pitch) {
    if (!P || !d_ec || !d_phi_in || !d_phi_out || d_phi_in == d_phi_out) return CCMG_EINVAL;
    if (check_pitch(P, level, pitch) != CCMG_OK || check_pitch(P, level + 1, pitch_c) != CCMG_OK)
        return CCMG_EINVAL;
    MarchArgs<double> a{};
    level_consts(P, level, a);
    a.f = d_phi_in;  // f is read but unused by a pure prolongation
    a.pf = pitch;
    a.phi_in = d_phi_in;
    a.pin = pitch;
    a.phi_out = d_phi_out;
    a.pout = pitch;
    a.ec = d_ec;
    a.pc = pitch_c;
    int nt;
    return hip_status(launch_march<double>(a, 0, true, true, POST_NONE, shape_for(a.n), P->stream, &nt));
}

}  // extern "C"
