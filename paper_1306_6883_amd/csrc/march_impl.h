// march_impl.h -- fused row-march kernel: the hot path of every V-cycle level.
// (Included by the march_*.hip files, each of which instantiates a subset.)
//
// One wavefront owns a tile of the level: 128 consecutive columns (two per
// lane: x = X0 + 2*lane and X0 + 2*lane + 1) and a band of rows.  It walks
// the band one row at a time, keeping a short window of rows in registers,
// and runs a skewed pipeline over that window:
//
//     load row t  ->  [prolongation of the coarse correction into row t]
//     red sweep of iteration 1 on row t-1, black sweep on row t-2,
//     red sweep of iteration 2 on row t-3, black sweep on row t-4, ...
//     -> store the relaxed row t-2*NU
//     -> residual of row t-2*NU-1 -> four-cell restriction / norm / residual store
//
// Each stage only needs the previous stage's values on the rows directly
// above and below, so this is exactly red-black Gauss-Seidel (pyro paper,
// Sec. 3.3): the red cells of a row see the old black neighbours, the black
// cells see the new red ones.  The tile's outer columns and rows are a halo
// that is recomputed redundantly by the neighbouring tile; what a tile writes
// is independent of how the level is cut into tiles.
//
// Boundary conditions are applied where a neighbour is read: for a Dirichlet
// or Neumann side the ghost is -/+ the cell's own current value (the paper's
// homogeneous ghost rules, refreshed before each colour); periodic tiles load
// the wrapped rows and columns, so the halo *is* the periodic image.
//
// Bytes per cell and launch: read f, read phi (unless it starts at zero),
// write phi, plus a quarter cell of coarse rhs (restriction) or coarse
// correction (prolongation).  Every other intermediate lives in registers.
//
// Variants that recompute instead of reading back (internal.h, enum Post):
// POST_VISIT and POST_FUSED0 start with the pre-smoothing from zero (stages
// 1-4, on f alone), then prolongate into row t-4 and go on with their other
// stages, so the launch that ran that pre-smoothing earlier need not store
// it; POST_CNPRE forms its right-hand side phi + beta Lap phi from the
// loaded rows instead of loading f.  A first launch of a solve can also sum
// f's statistics and the residual of the loaded iterate (fstat_part,
// in_norm_part) from the loads it makes anyway.
//
// The output never aliases the input (phi_in != phi_out): a neighbour tile may
// still read the old values of rows this tile has finished.
#pragma once
#include <type_traits>

#include "internal.h"

// Products are fused into additions only within one expression, as written
// (a * b + c): never across statements.  A value kept in a register from an
// earlier stage then takes part in later sums exactly as it would after a
// round trip through memory, so the fused, visit and separate-launch forms
// of a cycle give the same bits for any operator.
#pragma clang fp contract(on)

namespace ccmg {

// ---- cross-lane moves (DPP wavefront shifts) --------------------------------
// from_left: lane l receives lane l-1's value; from_right: lane l+1's.
// The edge lanes (0 for from_left, 63 for from_right) receive 0; they are
// halo lanes by construction.
__device__ __forceinline__ double from_left(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x138, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_right(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0x130, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float from_left(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_right(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}

// Sum over the 64 lanes with a fixed butterfly: every lane gets the same bits.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Element offset of row r (>= 0) of an array with pitch p.  The host admits
// only arrays of fewer than 2^31 elements ((n + 2) * pitch), so the product
// fits 32 bits: one scalar multiply per row address instead of a 64-bit one.
__device__ __forceinline__ unsigned row_off(int r, long p) { return (unsigned)r * (unsigned)p; }

// Total of `count` partial sums, formed in a fixed order (deterministic):
// each lane adds every 64th value in turn, then the lanes are combined.  The
// values are loaded 16 at a time (predicated) before they are added in that
// order, so a few thousand partials cost a few memory round trips, not one
// per 64.
__device__ __forceinline__ double sum_partials(const double *p, int count) {
    const int lane = threadIdx.x & 63;
    constexpr int B = 16;
    double s = 0.0;
    for (int i = lane; i < count; i += B * 64) {
        double v[B];
#pragma unroll
        for (int k = 0; k < B; ++k) v[k] = i + 64 * k < count ? p[i + 64 * k] : 0.0;
#pragma unroll
        for (int k = 0; k < B; ++k)
            if (i + 64 * k < count) s += v[k];
    }
    return wave_sum(s);
}

// Compile-time loop: f(integral_constant<int, B>), ..., f(integral_constant<int, E-1>).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// ---- compile-time shape of a march variant ----------------------------------
template <int NU, bool PROLONG, int POST>
struct Cfg {
    // VISIT: pre-smoothing stages 1 .. 4 from zero, the prolongation,
    // post-smoothing stages 5 .. 8; no residual.  FUSED0: the same four
    // stages and prolongation, then POST_FUSED's stages, norm and residual.
    static constexpr bool VISIT = POST == POST_VISIT;
    static constexpr bool FUSED0 = POST == POST_FUSED0;
    static constexpr int PRE0 = (VISIT || FUSED0) ? 4 : 0;  // stages before the prolongation
    static constexpr bool RES = POST != POST_NONE && !VISIT;  // a residual stage follows the relaxation
    static constexpr int LAGR = RES ? 2 * NU + 1 : 0;  // residual stage
    static constexpr int LAST = RES ? LAGR : 2 * NU;   // last stage
    // halo columns: one per stage, two (one lane) for the prolongation slope
    // (VISIT: the slope's two columns lie within the pre-smoothing's four, so
    // the halo has a column to spare; FUSED0 counts them there too)
    static constexpr int HX = FUSED0 ? march_halo_x(NU, false, RES) : march_halo_x(NU, PROLONG, RES);
    static constexpr int HY = (LAST + 1) & ~1;  // halo rows (even: rows start on red parity)
    static constexpr int W = LAST >= 11 ? 18 : (LAST >= 7 ? 14 : 10);  // register window (rows), even
    static constexpr int D = W - LAST - 2;      // prefetch distance (rows)
    static constexpr int WC = W / 2;            // coarse-row window
    static constexpr int DC = WC - 3;           // coarse prefetch distance
    static constexpr int OUTW = 128 - 2 * HX;  // output columns per tile
    // Rows are stored as 16-byte aligned pairs (cells x0 - 1, x0 of lane x0),
    // which needs the column on either side of the output to be correct too:
    // true when the halo has a column to spare beyond the last stage.
    static constexpr bool PAIRST = HX >= 2 * NU + ((PROLONG && !PRE0) ? 2 : 0) + 1;
    static_assert(D >= 1 && DC >= 0, "window too small");
    static_assert(!VISIT || (NU == 4 && PROLONG), "a visit runs 2 + 2 iterations around the prolongation");
    static_assert(!FUSED0 || (NU == 6 && PROLONG), "FUSED0 runs 2 + 2 + 2 iterations");
};

// Per-wave description of the tile, computed once by the kernel entry.
struct Tile {
    int n, nm, nc;
    int xo0, x0, xl, I, Il;   // output column start; lane columns; loads; coarse column
    bool px, py, wedge, eedge, cwedge, ceedge, outl;
    bool st2;                 // aligned row store of cells x0 - 1, x0 (see march_tile)
    int y0, y1, ys, ye;       // output rows [y0, y1); march rows [ys, ye)
};

// The row march of one tile.  XB / YB: the tile touches a Dirichlet or Neumann
// side in x / y, so neighbour reads there must apply the ghost rule; interior
// tiles (most of them) skip every boundary select.
template <typename T, int NU, bool LOADPHI, bool PROLONG, int POST, bool XB, bool YB>
__device__ __forceinline__ void march_tile(const MarchArgs<T> &a, const Tile &tl, const int tile) {
    using C = Cfg<NU, PROLONG, POST>;
    constexpr int W = C::W, D = C::D, WC = C::WC, DC = C::DC;
    // POST_CNPRE: POST_RESTRICT with f formed from the loaded iterate
    constexpr bool CNF = POST == POST_CNPRE;
    constexpr bool RESTR = POST == POST_RESTRICT || CNF;
    const int lane = threadIdx.x & 63;
    const int nm = tl.nm, nc = tl.nc;
    const bool py = tl.py;
    const int ys = tl.ys, ye = tl.ye, y0 = tl.y0, y1 = tl.y1;
    // row y is one of the tile's output rows: one unsigned compare of
    // wave-uniform values
    const unsigned nrows = (unsigned)(y1 - y0);
    auto inrow = [&](int y) { return (unsigned)(y - y0) < nrows; };
    // Store one row of the tile, two values per lane (cells x0, x0 + 1), into
    // row base `o` (element 1 + x holds cell x).  PAIRST variants re-pair the
    // cells so that every lane writes cells x0 - 1 and x0 as one 16-byte
    // aligned store (a misaligned one is split in two by the memory path):
    // each tile writes its output columns and one correct column either side,
    // which the neighbouring tile writes with the same bits; on a periodic x
    // side that column is the ghost, written with its periodic image.  Tiles
    // on a Dirichlet or Neumann x side keep to their own columns.  Call with
    // the whole wavefront active (cross-lane move).
    auto store_row = [&](auto *o, const auto v0, const auto v1) {
        if constexpr (C::PAIRST && !XB) {
            const auto vl = from_left(v1);
            if (tl.st2) {
                o[tl.x0] = vl;
                o[tl.x0 + 1] = v0;
            }
        } else if (tl.outl) {
            o[1 + tl.x0] = v0;
            o[2 + tl.x0] = v1;
        }
    };
    const T sxl = a.bc[CCMG_XLO] == CCMG_BC_DIRICHLET ? T(-1) : T(1);
    const T sxh = a.bc[CCMG_XHI] == CCMG_BC_DIRICHLET ? T(-1) : T(1);
    const T syl = a.bc[CCMG_YLO] == CCMG_BC_DIRICHLET ? T(-1) : T(1);
    const T syh = a.bc[CCMG_YHI] == CCMG_BC_DIRICHLET ? T(-1) : T(1);
    const T cc = a.cc, invd = a.invd;

    const bool subf = a.fmean_part != nullptr;
    const bool subp = LOADPHI && a.phi_shift != nullptr;
    T fsub = T(0), psub = T(0);
    double psub64 = 0.0;  // POST_IR: the shift applies to the FP64 iterate, in FP64
    if (subf) {
        const int cnt = a.fmean_count_ptr ? *a.fmean_count_ptr : a.fmean_count;
        fsub = T(sum_partials(a.fmean_part, cnt) / ((double)tl.n * (double)tl.n));
    }
    if (subp) {
        psub64 = *a.phi_shift;
        psub = T(psub64);
    }

    const int lo = 1 + tl.xl;        // element offset of this lane's first column in a row
    const int co = 1 + tl.Il;        // ... of its coarse column

    T P0[W], P1[W], F0[W], F1[W], Cw[WC];
#pragma unroll
    for (int k = 0; k < W; ++k) P0[k] = P1[k] = F0[k] = F1[k] = T(0);
#pragma unroll
    for (int k = 0; k < WC; ++k) Cw[k] = T(0);
    // POST_IR: FP64 iterate (Q) and right-hand side (G) rows, same slots as P / F
    constexpr bool IR = POST == POST_IR;
    constexpr int WQ = IR ? W : 1;
    double Q0[WQ], Q1[WQ], G0[WQ], G1[WQ];
#pragma unroll
    for (int k = 0; k < WQ; ++k) Q0[k] = Q1[k] = G0[k] = G1[k] = 0.0;
    double acc2 = 0.0;

    // Loads are unconditional (a conditional load into the window would force
    // the compiler to wait for it): rows past the end of the band re-read the
    // band's last row, whose values only ever reach halo rows.
    auto load_row = [&](int y, T &p0, T &p1, T &f0, T &f1) {
        y = min(y, ye - 1);
        const int yy = py ? (y & nm) : y;
        if constexpr (!CNF) {  // (CNPRE forms f from phi)
            const T *fr = a.f + row_off(yy + 1, a.pf);
            f0 = fr[lo];
            f1 = fr[lo + 1];
        }
        if (LOADPHI) {
            const T *pr = a.phi_in + row_off(yy + 1, a.pin);
            p0 = pr[lo];
            p1 = pr[lo + 1];
        }
    };
    auto load_row64 = [&](int y, double &q0, double &q1, double &g0, double &g1) {
        y = min(y, ye - 1);
        const int yy = py ? (y & nm) : y;
        const double *qr = a.q_in + row_off(yy + 1, a.pq_in);
        const double *gr = a.g + row_off(yy + 1, a.pg);
        q0 = qr[lo];
        q1 = qr[lo + 1];
        g0 = gr[lo];
        g1 = gr[lo + 1];
    };
    auto load_coarse = [&](int J, T &c) {
        const int Jl = py ? (J & (nc - 1)) : (J < 0 ? 0 : (J >= nc ? nc - 1 : J));
        c = (a.ec + row_off(Jl + 1, a.pc))[co];
    };

    double acc0 = 0.0, acc1 = 0.0;
    T rprev0 = T(0), rprev1 = T(0);
    // POST_RESTRICT / POST_R32 with fstat_part: statistics of f over the output cells
    constexpr bool FSTATS = RESTR || POST == POST_R32;
    const bool fst = FSTATS && a.fstat_part != nullptr;
    double fs = 0.0, fa = 0.0, f2 = 0.0, fbad = 0.0;
    // POST_RESTRICT from a loaded iterate with in_norm_part: the residual
    // norm sums of the iterate as loaded, and the loaded values of the row
    // below the one whose residual is taken (stage 1 has already changed
    // that row in its window slot)
    const bool innorm = RESTR && LOADPHI && a.in_norm_part != nullptr;
    double accI0 = 0.0, accI1 = 0.0;
    T SI0 = T(0), SI1 = T(0);
    // POST_FUSED (and FUSED0): norm sums after the post-smoothing, and that
    // state of the previous row (the row below the one whose residual is taken)
    constexpr bool FUSED = POST == POST_FUSED || POST == POST_FUSED0;
    static_assert(POST != POST_FUSED || NU == 4, "the fused launch runs 2 + 2 iterations");
    double accN0 = 0.0, accN1 = 0.0;
    T SA[2] = {T(0), T(0)}, SB[2] = {T(0), T(0)};
    // VISIT: the pre-smoothed row below the one being pre-smoothed
    T SV0 = T(0), SV1 = T(0);

    static_for<0, D>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        load_row(ys + k, P0[k], P1[k], F0[k], F1[k]);
        if constexpr (IR) load_row64(ys + k, Q0[k], Q1[k], G0[k], G1[k]);
    });
    // Coarse rows sit in a ring: coarse row R in slot (R - ys/2 + 1) mod WC.
    // The prolongation of fine row y reads coarse rows y/2 - 1 .. y/2 + 1; it
    // runs on row t at step t, or (VISIT) on row t - NU after the
    // pre-smoothing, so there the ring starts two coarse rows lower.
    constexpr int CLAG = C::PRE0 / 2;
    if constexpr (PROLONG) {
        static_for<0, DC + 2>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            load_coarse((ys >> 1) - 1 - CLAG + q, Cw[(q - CLAG + WC) % WC]);
        });
    }

    const int tend = ye + C::LAST;
    // One step of the march (row t = tb + k).  YBR: apply the y ghost rules.
    // A y-side tile needs them only in the blocks of W steps whose rows reach
    // y = 0 or y = n - 1 (the stages lag at most LAST rows behind t; the
    // prolongation reads one coarse row on either side of row t); elsewhere
    // its selects would all keep the neighbour, so the interior step is the
    // same arithmetic with fewer instructions.
    auto step = [&](auto kc, auto ybc, const int tb) {
            constexpr int k = decltype(kc)::value;
            constexpr bool YBR = decltype(ybc)::value;
            const int t = tb + k;
            // 1. prefetch
            {
                constexpr int kd = (k + D) % W;
                load_row(t + D, P0[kd], P1[kd], F0[kd], F1[kd]);
                if constexpr (IR) load_row64(t + D, Q0[kd], Q1[kd], G0[kd], G1[kd]);
            }
            if constexpr (PROLONG) {
                if constexpr ((k & 1) == 0)
                    load_coarse((t >> 1) + 1 - CLAG + DC, Cw[((k >> 1) + 2 - CLAG + DC) % WC]);
            }
            // 2. finish the load of row t: mean shifts, prolongation (done for
            // every step: past the band it only touches halo slots)
            // (fsub and psub are 0 when there is no shift: x - 0 is x, bit for
            // bit, and costs less than selecting between the two)
            F0[k] -= fsub;
            F1[k] -= fsub;
            if constexpr (IR) {
                if (a.q_zero) {
                    Q0[k] = 0.0;
                    Q1[k] = 0.0;
                } else if (subp) {
                    Q0[k] -= psub64;
                    Q1[k] -= psub64;
                }
            }
            if (LOADPHI) {
                if constexpr (!IR) {
                    P0[k] -= psub;
                    P1[k] -= psub;
                }
            } else {
                P0[k] = T(0);
                P1[k] = T(0);
            }
            // prolongation of the coarse correction into row t - CLAG * 2
            // (slot kq): e + slopes, the cell's quarter offsets
            auto prolong = [&]() {
                constexpr int kq = (k - 2 * CLAG + 2 * W) % W;
                const int J = (t - 2 * CLAG) >> 1;
                T cm = Cw[((k >> 1) - CLAG + 0 + WC) % WC];
                const T c0 = Cw[((k >> 1) - CLAG + 1 + WC) % WC];
                T cp = Cw[((k >> 1) - CLAG + 2 + WC) % WC];
                if constexpr (YBR) {
                    if (J - 1 < 0) cm = syl * cm;    // coarse ghost row below
                    if (J + 1 >= nc) cp = syh * cp;  // coarse ghost row above
                }
                T ew = from_left(c0), ee = from_right(c0);
                if constexpr (XB) {
                    if (tl.cwedge) ew = sxl * c0;
                    if (tl.ceedge) ee = sxh * c0;
                }
                const T mx = T(0.5) * (ee - ew);
                const T my = T(0.5) * (cp - cm);
                const T dy = (k & 1) ? T(0.25) : T(-0.25);  // row t - 2 CLAG has t's parity
                P0[kq] = P0[kq] + ((c0 + T(-0.25) * mx) + dy * my);
                P1[kq] = P1[kq] + ((c0 + T(0.25) * mx) + dy * my);
            };
            if constexpr (PROLONG && C::PRE0 == 0) prolong();
            // 2a. CNPRE: f of row t-1 = phi + beta Lap phi of the loaded
            // iterate (rows t and t-1 are still as loaded; row t-2 from the
            // copy kept one step ago), Lap as differences from the centre in
            // the order east, west, north, south; stored for the later launches
            if constexpr (CNF) {
                const int y = t - 1;
                constexpr int kk = (k - 1 + W) % W;
                const T p0 = P0[kk], p1 = P1[kk];
                T w0 = from_left(P1[kk]);
                T e1 = from_right(P0[kk]);
                if constexpr (XB) {
                    if (tl.wedge) w0 = sxl * p0;
                    if (tl.eedge) e1 = sxh * p1;
                }
                T n0 = P0[k], n1 = P1[k], s0 = SI0, s1 = SI1;
                if constexpr (YBR) {
                    if (y == nm) {
                        n0 = syh * p0;
                        n1 = syh * p1;
                    }
                    if (y == 0) {
                        s0 = syl * p0;
                        s1 = syl * p1;
                    }
                }
                const T ih2 = a.ih2;
                const T lap0 = ((((p1 - p0) + (w0 - p0)) + (n0 - p0)) + (s0 - p0)) * ih2;
                const T lap1 = ((((e1 - p1) + (p0 - p1)) + (n1 - p1)) + (s1 - p1)) * ih2;
                F0[kk] = p0 + a.cn_beta * lap0;
                F1[kk] = p1 + a.cn_beta * lap1;
                if (inrow(y)) store_row(a.cn_f + row_off(y + 1, a.pcnf), F0[kk], F1[kk]);
                if (!innorm) {
                    SI0 = p0;
                    SI1 = p1;
                }
            }
            // 2b. residual of row t-1 as loaded (rows t and t-1 still are;
            // row t-2 from the copy kept one step ago)
            if constexpr (RESTR && LOADPHI) {
                if (innorm) {
                    const int y = t - 1;
                    constexpr int kk = (k - 1 + W) % W;
                    const T p0 = P0[kk], p1 = P1[kk];
                    T w0 = from_left(P1[kk]);
                    T e1 = from_right(P0[kk]);
                    if constexpr (XB) {
                        if (tl.wedge) w0 = sxl * p0;
                        if (tl.eedge) e1 = sxh * p1;
                    }
                    T n0 = P0[k], n1 = P1[k], s0 = SI0, s1 = SI1;
                    if constexpr (YBR) {
                        if (y == nm) {
                            n0 = syh * p0;
                            n1 = syh * p1;
                        }
                        if (y == 0) {
                            s0 = syl * p0;
                            s1 = syl * p1;
                        }
                    }
                    if (inrow(y) && tl.outl) {
                        const T ih2 = a.ih2;
                        const T lap0 = ((((p1 - p0) + (w0 - p0)) + (n0 - p0)) + (s0 - p0)) * ih2;
                        const T lap1 = ((((e1 - p1) + (p0 - p1)) + (n1 - p1)) + (s1 - p1)) * ih2;
                        const T r0 = F0[kk] - (a.alpha * p0 - a.beta * lap0);
                        const T r1 = F1[kk] - (a.alpha * p1 - a.beta * lap1);
                        accI0 += (double)r0 * (double)r0 + (double)r1 * (double)r1;
                        accI1 += (double)p0 + (double)p1;
                    }
                    SI0 = p0;
                    SI1 = p1;
                }
            }
            // 3. relaxation stages: stage s works on row t - s; odd s = red, even s = black.
            // Unconditional: a stage on a row outside [ys, ye) writes a slot that
            // either is reloaded before it is read again (rows below ys) or only
            // feeds halo rows (rows at or past ye).
            auto stage = [&](auto sc) {
                constexpr int s = decltype(sc)::value;
                const int y = t - s;
                constexpr int kk = (k - s + 2 * W) % W;
                constexpr int km = (k - s - 1 + 2 * W) % W;
                constexpr int kp = (k - s + 1 + 2 * W) % W;
                // red cells: (x + y) even; column 0 has x even; row parity = (k - s) & 1
                constexpr int col = ((s & 1) ? ((k - s) & 1) : (1 - ((k - s) & 1)));
                if constexpr (col == 0) {
                    const T self = P0[kk];
                    const T e = P1[kk];
                    T w = from_left(P1[kk]);
                    if constexpr (XB) {
                        if (tl.wedge) w = sxl * self;
                    }
                    T nn = P0[kp], ss = P0[km];
                    if constexpr (C::PRE0 > 0 && s == C::PRE0) ss = SV0;  // row below, before its prolongation
                    if constexpr (YBR) {
                        if (y == nm) nn = syh * self;
                        if (y == 0) ss = syl * self;
                    }
                    P0[kk] = (F0[kk] + cc * (((e + w) + nn) + ss)) * invd;
                } else {
                    const T self = P1[kk];
                    const T w = P0[kk];
                    T e = from_right(P0[kk]);
                    if constexpr (XB) {
                        if (tl.eedge) e = sxh * self;
                    }
                    T nn = P1[kp], ss = P1[km];
                    if constexpr (C::PRE0 > 0 && s == C::PRE0) ss = SV1;  // row below, before its prolongation
                    if constexpr (YBR) {
                        if (y == nm) nn = syh * self;
                        if (y == 0) ss = syl * self;
                    }
                    P1[kk] = (F1[kk] + cc * (((e + w) + nn) + ss)) * invd;
                }
            };
            if constexpr (FUSED) {
                // FUSED0: stages 1-4 recompute the pre-smoothing of row t-4
                // from zero, whose values are kept for the next step's stage 4
                // (as in a visit) before the prolongation adds to them.  Then
                // (B = 0 or 4) stages B+1 .. B+4 finish the post-smoothing of
                // row t-B-4; before stage B+5 touches row t-B-5, take the
                // residual norm of row t-B-5 (rows t-B-6 .. t-B-4 all after
                // stage B+4; row t-B-6 from the copy saved one step ago) and
                // store / save it
                constexpr int B = C::PRE0;
                if constexpr (B > 0) {
                    static_for<1, B + 1>(stage);
                    constexpr int kq = (k - B + 2 * W) % W;
                    SV0 = P0[kq];
                    SV1 = P1[kq];
                    prolong();
                }
                static_for<B + 1, B + 5>(stage);
                {
                    const int y = t - B - 5;
                    constexpr int kk = (k - B - 5 + 2 * W) % W;
                    constexpr int kp = (k - B - 4 + 2 * W) % W;
                    constexpr int sv = (k + B + 1) & 1;  // parity of row t-B-5 (t - k is even)
                    const T p0 = P0[kk], p1 = P1[kk];
                    T w0 = from_left(P1[kk]);
                    T e1 = from_right(P0[kk]);
                    if constexpr (XB) {
                        if (tl.wedge) w0 = sxl * p0;
                        if (tl.eedge) e1 = sxh * p1;
                    }
                    T n0 = P0[kp], n1 = P1[kp], s0 = SA[1 - sv], s1 = SB[1 - sv];
                    if constexpr (YBR) {
                        if (y == nm) {
                            n0 = syh * p0;
                            n1 = syh * p1;
                        }
                        if (y == 0) {
                            s0 = syl * p0;
                            s1 = syl * p1;
                        }
                    }
                    if (inrow(y)) {
                        if (tl.outl) {
                            const T ih2 = a.ih2;
                            const T lap0 = ((((p1 - p0) + (w0 - p0)) + (n0 - p0)) + (s0 - p0)) * ih2;
                            const T lap1 = ((((e1 - p1) + (p0 - p1)) + (n1 - p1)) + (s1 - p1)) * ih2;
                            const T r0 = F0[kk] - (a.alpha * p0 - a.beta * lap0);
                            const T r1 = F1[kk] - (a.alpha * p1 - a.beta * lap1);
                            accN0 += (double)r0 * (double)r0 + (double)r1 * (double)r1;
                            accN1 += (double)p0 + (double)p1;
                        }
                        if (a.phi_mid) store_row(a.phi_mid + row_off(y + 1, a.pmid), p0, p1);
                    }
                    SA[sv] = p0;
                    SB[sv] = p1;
                }
                static_for<B + 5, 2 * NU + 1>(stage);
            } else if constexpr (C::VISIT) {
                // stages 1 .. NU finish the pre-smoothing of row t - NU; its
                // values are kept (the last pre-smoothing stage of the next
                // row reads them) before the prolongation adds to them
                static_for<1, NU + 1>(stage);
                constexpr int kq = (k - NU + 2 * W) % W;
                SV0 = P0[kq];
                SV1 = P1[kq];
                prolong();
                static_for<NU + 1, 2 * NU + 1>(stage);
            } else {
                static_for<1, 2 * NU + 1>(stage);
            }
            // 4. store the finished row (POST_IR: add it to the FP64 iterate and store that)
            {
                const int y = t - 2 * NU;
                constexpr int kk = (k - 2 * NU + 2 * W) % W;
                if constexpr (IR) {
                    Q0[kk] += (double)P0[kk];
                    Q1[kk] += (double)P1[kk];
                    if (inrow(y)) store_row(a.q_out + row_off(y + 1, a.pq_out), Q0[kk], Q1[kk]);
                } else if ((FUSED || a.phi_out) && inrow(y)) {  // the fused launch always stores
                    store_row(a.phi_out + row_off(y + 1, a.pout), P0[kk], P1[kk]);
                }
            }
            // 5. residual of the finished rows and what is made from it
            if constexpr (IR) {
                const int y = t - C::LAGR;
                if (inrow(y)) {
                    constexpr int kk = (k - C::LAGR + 2 * W) % W;
                    constexpr int km = (k - C::LAGR - 1 + 2 * W) % W;
                    constexpr int kp = (k - C::LAGR + 1 + 2 * W) % W;
                    const double p0 = Q0[kk], p1 = Q1[kk];
                    double w0 = from_left(Q1[kk]);
                    double e1 = from_right(Q0[kk]);
                    if constexpr (XB) {
                        if (tl.wedge) w0 = (double)sxl * p0;
                        if (tl.eedge) e1 = (double)sxh * p1;
                    }
                    double n0 = Q0[kp], n1 = Q1[kp], s0 = Q0[km], s1 = Q1[km];
                    if constexpr (YBR) {
                        if (y == nm) {
                            n0 = (double)syh * p0;
                            n1 = (double)syh * p1;
                        }
                        if (y == 0) {
                            s0 = (double)syl * p0;
                            s1 = (double)syl * p1;
                        }
                    }
                    const double ih2 = a.ih2_64;
                    const double lap0 = ((((p1 - p0) + (w0 - p0)) + (n0 - p0)) + (s0 - p0)) * ih2;
                    const double lap1 = ((((e1 - p1) + (p0 - p1)) + (n1 - p1)) + (s1 - p1)) * ih2;
                    const double r0 = G0[kk] - (a.alpha64 * p0 - a.beta64 * lap0);
                    const double r1 = G1[kk] - (a.alpha64 * p1 - a.beta64 * lap1);
                    const float q0 = (float)r0, q1 = (float)r1;
                    store_row(a.r_out + row_off(y + 1, a.pr), q0, q1);
                    if (tl.outl) {
                        acc0 += r0 * r0 + r1 * r1;
                        acc1 += p0 + p1;
                        acc2 += (double)q0 + (double)q1;
                    }
                }
            } else if constexpr (C::RES) {
                const int y = t - C::LAGR;
                if (inrow(y)) {
                    constexpr int kk = (k - C::LAGR + 2 * W) % W;
                    constexpr int km = (k - C::LAGR - 1 + 2 * W) % W;
                    constexpr int kp = (k - C::LAGR + 1 + 2 * W) % W;
                    const T p0 = P0[kk], p1 = P1[kk];
                    T w0 = from_left(P1[kk]);
                    T e1 = from_right(P0[kk]);
                    if constexpr (XB) {
                        if (tl.wedge) w0 = sxl * p0;
                        if (tl.eedge) e1 = sxh * p1;
                    }
                    T n0 = P0[kp], n1 = P1[kp], s0 = P0[km], s1 = P1[km];
                    if constexpr (YBR) {
                        if (y == nm) {
                            n0 = syh * p0;
                            n1 = syh * p1;
                        }
                        if (y == 0) {
                            s0 = syl * p0;
                            s1 = syl * p1;
                        }
                    }
                    const T ih2 = a.ih2;
                    const T lap0 = ((((p1 - p0) + (w0 - p0)) + (n0 - p0)) + (s0 - p0)) * ih2;
                    const T lap1 = ((((e1 - p1) + (p0 - p1)) + (n1 - p1)) + (s1 - p1)) * ih2;
                    const T r0 = F0[kk] - (a.alpha * p0 - a.beta * lap0);
                    const T r1 = F1[kk] - (a.alpha * p1 - a.beta * lap1);
                    if constexpr (FSTATS) {
                        if (fst && tl.outl) {
                            auto add = [&](double v) {
                                if (!isfinite(v)) {
                                    fbad += 1.0;
                                } else {
                                    fs += v;
                                    fa += fabs(v);
                                    f2 += v * v;
                                }
                            };
                            add((double)F0[kk]);
                            add((double)F1[kk]);
                        }
                    }
                    if constexpr (RESTR || FUSED) {
                        if constexpr ((k - C::LAGR) & 1) {  // odd row: close the 2x2 block
                            const T v = T(0.25) * (((rprev0 + rprev1) + r0) + r1);
                            if (tl.outl) {
                                (a.aux + row_off((y >> 1) + 1, a.paux))[1 + (tl.x0 >> 1)] = v;
                                acc0 += (double)v;
                            }
                        } else {
                            rprev0 = r0;
                            rprev1 = r1;
                        }
                    } else if constexpr (POST == POST_NORM) {
                        if (tl.outl) {
                            acc0 += (double)r0 * (double)r0 + (double)r1 * (double)r1;
                            acc1 += (double)p0 + (double)p1;
                        }
                    } else if constexpr (POST == POST_R32) {
                        const float q0 = (float)r0, q1 = (float)r1;
                        store_row(a.r_out + row_off(y + 1, a.pr), q0, q1);
                        if (tl.outl) {
                            acc0 += (double)r0 * (double)r0 + (double)r1 * (double)r1;
                            acc1 += (double)p0 + (double)p1;
                            acc2 += (double)q0 + (double)q1;
                        }
                    } else {  // POST_RESID
                        if (tl.outl) {
                            T *o = a.aux + row_off(y + 1, a.paux);
                            o[1 + tl.x0] = r0;
                            o[2 + tl.x0] = r1;
                        }
                    }
                }
            }
    };
    // three runs of blocks (the first and last empty unless YB): near y = 0,
    // between, near y = n - 1
    int tb = ys;
    if constexpr (YB) {
        for (; tb < tend && tb <= C::LAST + 2; tb += W)
            static_for<0, W>([&](auto kc) { step(kc, std::true_type{}, tb); });
    }
    for (; tb < tend && (!YB || tb + W + 2 < nm); tb += W)
        static_for<0, W>([&](auto kc) { step(kc, std::false_type{}, tb); });
    if constexpr (YB) {
        for (; tb < tend; tb += W)
            static_for<0, W>([&](auto kc) { step(kc, std::true_type{}, tb); });
    }

    if constexpr (RESTR || FUSED) {
        const double s = wave_sum(acc0);
        if (lane == 0) a.partial[tile] = s;
        if (innorm) {
            const double q0 = wave_sum(accI0), q1 = wave_sum(accI1);
            if (lane == 0) {
                a.in_norm_part[2 * tile] = q0;
                a.in_norm_part[2 * tile + 1] = q1;
            }
        }
        if (fst) {
            const double q0 = wave_sum(fs), q1 = wave_sum(fa), q2 = wave_sum(f2), q3 = wave_sum(fbad);
            if (lane == 0) {
                a.fstat_part[4 * tile + 0] = q0;
                a.fstat_part[4 * tile + 1] = q1;
                a.fstat_part[4 * tile + 2] = q2;
                a.fstat_part[4 * tile + 3] = q3;
            }
        }
        if constexpr (FUSED) {
            const double s0 = wave_sum(accN0), s1 = wave_sum(accN1);
            if (lane == 0 && a.partial_norm) {
                a.partial_norm[2 * tile] = s0;
                a.partial_norm[2 * tile + 1] = s1;
            }
        }
    } else if constexpr (POST == POST_NORM || POST == POST_IR || POST == POST_R32) {
        const double s0 = wave_sum(acc0), s1 = wave_sum(acc1);
        double s2 = 0.0;
        if constexpr (POST != POST_NORM) s2 = wave_sum(acc2);
        if (lane == 0) {
            a.partial[2 * tile] = s0;
            a.partial[2 * tile + 1] = s1;
            if constexpr (POST != POST_NORM) a.partial3[tile] = s2;
        }
        if constexpr (POST == POST_R32) {
            if (fst) {
                const double q0 = wave_sum(fs), q1 = wave_sum(fa), q2 = wave_sum(f2), q3 = wave_sum(fbad);
                if (lane == 0) {
                    a.fstat_part[4 * tile + 0] = q0;
                    a.fstat_part[4 * tile + 1] = q1;
                    a.fstat_part[4 * tile + 2] = q2;
                    a.fstat_part[4 * tile + 3] = q3;
                }
            }
        }
    }
}

// One tile of one level: derive the tile geometry from the launch arguments and
// run the row march, specialised on whether the tile meets a Dirichlet /
// Neumann side.  `a` may live in the kernel arguments or in global memory.
template <typename T, int NU, bool LOADPHI, bool PROLONG, int POST>
__device__ __forceinline__ void march_one(const MarchArgs<T> &a, const int tile) {
    using C = Cfg<NU, PROLONG, POST>;
    const int lane = threadIdx.x & 63;
    if (a.skip && *a.skip) return;
    // interior strips first (row-major: a band's strips are consecutive
    // tiles), then the edge strips' shorter bands
    const int reg = a.echunks ? a.strips - 2 : a.strips;
    const int nreg = reg * a.chunks;
    int strip, ya, yh;
    if (tile < nreg) {
        strip = (a.echunks ? 1 : 0) + tile % reg;
        yh = a.ty;
        ya = (tile / reg) * yh;
    } else {
        const int e = tile - nreg;
        strip = (e & 1) ? a.strips - 1 : 0;
        yh = a.ety;
        ya = (e >> 1) * yh;
    }

    Tile tl;
    tl.n = a.n;
    tl.nm = a.n - 1;
    tl.nc = a.n >> 1;
    tl.px = a.bc[CCMG_XLO] == CCMG_BC_PERIODIC;
    tl.py = a.bc[CCMG_YLO] == CCMG_BC_PERIODIC;
    // columns: lane owns x0, x0 + 1 (x0 even)
    tl.xo0 = strip * a.outw;
    const int X0 = tl.xo0 - C::HX;
    tl.x0 = X0 + 2 * lane;
    const bool inx = tl.px || (tl.x0 >= 0 && tl.x0 < tl.n);
    tl.xl = tl.px ? (tl.x0 & tl.nm) : (inx ? tl.x0 : 0);  // out-of-domain lanes read column 0
    tl.wedge = !tl.px && tl.x0 == 0;
    tl.eedge = !tl.px && tl.x0 + 1 == tl.nm;
    tl.outl = tl.x0 >= tl.xo0 && tl.x0 < tl.xo0 + a.outw && tl.x0 >= 0 && tl.x0 < tl.n;
    // aligned row stores: columns [xo0 - 1, min(xo0 + outw, n)] (-1 and n:
    // the ghosts of a periodic x side), i.e. lanes x0 in [xo0, min(xo0 + outw, n)]
    tl.st2 = tl.x0 >= tl.xo0 && tl.x0 <= min(tl.xo0 + a.outw, tl.n);
    tl.I = tl.x0 >> 1;
    tl.Il = PROLONG ? (tl.px ? (tl.I & (tl.nc - 1)) : min(max(tl.I, 0), tl.nc - 1)) : 0;
    tl.cwedge = !tl.px && tl.I == 0;
    tl.ceedge = !tl.px && tl.I == tl.nc - 1;
    // rows
    tl.y0 = ya;
    tl.y1 = min(ya + yh, tl.n);
    tl.ys = tl.py ? tl.y0 - C::HY : max(tl.y0 - C::HY, 0);
    tl.ye = tl.py ? tl.y1 + C::HY : min(tl.y1 + C::HY, tl.n);

    // the producer of per-tile partial sums publishes how many tiles it has
    if (a.count_out && tile == 0 && lane == 0) *a.count_out = a.ntiles;

    // does any lane / row of the tile meet a Dirichlet or Neumann side?
    const bool xb = !tl.px && (X0 <= 0 || X0 + 128 >= tl.n - 1);
    const bool yb = !tl.py && (tl.ys == 0 || tl.ye == tl.n);
    if (xb) {
        if (yb) march_tile<T, NU, LOADPHI, PROLONG, POST, true, true>(a, tl, tile);
        else march_tile<T, NU, LOADPHI, PROLONG, POST, true, false>(a, tl, tile);
    } else {
        if (yb) march_tile<T, NU, LOADPHI, PROLONG, POST, false, true>(a, tl, tile);
        else march_tile<T, NU, LOADPHI, PROLONG, POST, false, false>(a, tl, tile);
    }
}

template <typename T, int NU, bool LOADPHI, bool PROLONG, int POST>
__global__ __launch_bounds__(256) void k_march(const MarchArgs<T> a) {
    const int wpb = blockDim.x >> 6;
    // The wave index is uniform across the wavefront; saying so keeps every row
    // decision in scalar registers and scalar branches.
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // XCD-aware order: consecutive workgroup ids go to different XCDs, so give
    // each XCD a contiguous run of tiles (neighbouring tiles share halo rows in L2).
    const int lb = (blockIdx.x & 7) * a.groups_per_xcd + (blockIdx.x >> 3);
    const int tile = lb * wpb + wib;
    if (tile >= a.ntiles) return;  // whole wavefront leaves; no barriers anywhere
    march_one<T, NU, LOADPHI, PROLONG, POST>(a, tile);
}

// Persistent form for batches: the waves walk a list of (level descriptor,
// tile) items that spans many independent problems.
template <typename T, int NU, bool LOADPHI, bool PROLONG, int POST>
__global__ __launch_bounds__(256) void k_march_list(const MarchArgs<T> *__restrict__ descs,
                                                     const WorkItem *__restrict__ items, int nitems) {
    const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = gridDim.x * (blockDim.x >> 6);
    for (int it = blockIdx.x * (blockDim.x >> 6) + wib; it < nitems; it += nw) {
        const WorkItem wi = items[it];
        march_one<T, NU, LOADPHI, PROLONG, POST>(descs[wi.desc], wi.tile);
    }
}

// ---- host side ---------------------------------------------------------------
template <typename T, int NU, bool LOADPHI, bool PROLONG, int POST>
static hipError_t go(const MarchArgs<T> &a0, MarchShape sh, hipStream_t s, int *nt) {
    MarchArgs<T> a = a0;
    a.outw = Cfg<NU, PROLONG, POST>::OUTW;
    a.ty = sh.ty;
    a.strips = (a.n + a.outw - 1) / a.outw;
    a.chunks = (a.n + a.ty - 1) / a.ty;
    a.ntiles = a.strips * a.chunks;
    a.ety = a.ty;
    a.echunks = 0;
    if (a.bc[CCMG_XLO] != CCMG_BC_PERIODIC && a.strips >= 3 && a.ty >= kEdgeSplitMinTy) {
        a.ety = edge_band_rows(a.ty);
        a.echunks = (a.n + a.ety - 1) / a.ety;
        a.ntiles = (a.strips - 2) * a.chunks + 2 * a.echunks;
    }
    if (nt) *nt = a.ntiles;
    const int wpb = sh.wpb;
    const int blocks = (a.ntiles + wpb - 1) / wpb;
    a.groups_per_xcd = (blocks + 7) / 8;
    const int grid = 8 * a.groups_per_xcd;
    hipLaunchKernelGGL((k_march<T, NU, LOADPHI, PROLONG, POST>), dim3(grid), dim3(64 * wpb), 0, s, a);
    return hipGetLastError();
}

// Launch one march variant with NU fused iterations (instantiated per NU and T
// in the march_*.hip files).
template <typename T, int NU>
hipError_t dispatch_nu(const MarchArgs<T> &a, bool load_phi, bool prolong, int post,
                              MarchShape sh, hipStream_t s, int *nt) {
    if (prolong) {
        if (!load_phi) {
            // the prolongation alone into a zero field (full multigrid), with
            // or without the residual norm of the result
            if constexpr (NU == 0) {
                if (post == POST_NONE) return go<T, 0, false, true, POST_NONE>(a, sh, s, nt);
                if (post == POST_NORM) return go<T, 0, false, true, POST_NORM>(a, sh, s, nt);
            }
            // ... or followed by the pre-smoothing and restriction (the first
            // cycle of an FP64 solve from a full multigrid start)
            if constexpr (NU == 2 && std::is_same<T, double>::value) {
                if (post == POST_RESTRICT) return go<T, 2, false, true, POST_RESTRICT>(a, sh, s, nt);
            }
            return hipErrorInvalidValue;
        }
        if (post == POST_NONE) return go<T, NU, true, true, POST_NONE>(a, sh, s, nt);
        if (post == POST_NORM) return go<T, NU, true, true, POST_NORM>(a, sh, s, nt);
        if constexpr (std::is_same<T, float>::value) {
            if (post == POST_IR) return go<T, NU, true, true, POST_IR>(a, sh, s, nt);
        }
        return hipErrorInvalidValue;
    }
    if constexpr (std::is_same<T, double>::value) {
        if (post == POST_R32) {
            if (load_phi) return go<T, NU, true, false, POST_R32>(a, sh, s, nt);
            return go<T, NU, false, false, POST_R32>(a, sh, s, nt);
        }
    }
    if constexpr (std::is_same<T, float>::value) {
        // the FP64 update after a cycle that ran entirely in the one-workgroup tail
        if (post == POST_IR && load_phi && NU == 0) return go<T, NU, true, false, POST_IR>(a, sh, s, nt);
    }
    if (load_phi) {
        switch (post) {
            case POST_NONE: return go<T, NU, true, false, POST_NONE>(a, sh, s, nt);
            case POST_RESTRICT: return go<T, NU, true, false, POST_RESTRICT>(a, sh, s, nt);
            case POST_NORM: return go<T, NU, true, false, POST_NORM>(a, sh, s, nt);
            case POST_RESID: return go<T, NU, true, false, POST_RESID>(a, sh, s, nt);
        }
    } else {
        switch (post) {
            case POST_NONE: return go<T, NU, false, false, POST_NONE>(a, sh, s, nt);
            case POST_RESTRICT: return go<T, NU, false, false, POST_RESTRICT>(a, sh, s, nt);
            case POST_NORM: return go<T, NU, false, false, POST_NORM>(a, sh, s, nt);
            default: break;
        }
    }
    return hipErrorInvalidValue;
}

// Work-list launch of one variant (see k_march_list); `waves` wavefronts in
// workgroups of four.
template <typename T, int NU, bool LOADPHI, bool PROLONG, int POST>
hipError_t launch_list_variant(const MarchArgs<T> *descs, const WorkItem *items, int nitems, int waves,
                               hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    const int blocks = (waves + 3) / 4;
    hipLaunchKernelGGL((k_march_list<T, NU, LOADPHI, PROLONG, POST>), dim3(blocks), dim3(256), 0, s, descs, items,
                       nitems);
    return hipGetLastError();
}

}  // namespace ccmg
