// march.hip -- fused row-march kernel: the hot path of every V-cycle level.
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
// The output never aliases the input (phi_in != phi_out): a neighbour tile may
// still read the old values of rows this tile has finished.
#include <type_traits>

#include "internal.h"

namespace ccmg {

// ---- cross-lane moves (DPP wavefront shifts) --------------------------------
// from_left: lane l receives lane l-1's value; from_right: lane l+1's.
// Edge lanes keep their own value (they are halo lanes by construction).
__device__ __forceinline__ double from_left(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_right(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false);
    hi = __builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float from_left(float v) {
    int x = __float_as_int(v);
    x = __builtin_amdgcn_update_dpp(x, x, 0x138, 0xf, 0xf, false);
    return __int_as_float(x);
}
__device__ __forceinline__ float from_right(float v) {
    int x = __float_as_int(v);
    x = __builtin_amdgcn_update_dpp(x, x, 0x130, 0xf, 0xf, false);
    return __int_as_float(x);
}

// Sum over the 64 lanes with a fixed butterfly: every lane gets the same bits.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Total of `count` partial sums, formed in a fixed order (deterministic).
__device__ __forceinline__ double sum_partials(const double *p, int count) {
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    for (int i = lane; i < count; i += 64) s += p[i];
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
    static constexpr int LAGR = POST ? 2 * NU + 1 : 0;  // residual stage
    static constexpr int LAST = POST ? LAGR : 2 * NU;   // last stage
    // halo columns: one per stage, two (one lane) for the prolongation slope
    static constexpr int HXC = 2 * NU + (POST ? 1 : 0) + (PROLONG ? 2 : 0);
    static constexpr int HX = (HXC + 1) & ~1;
    static constexpr int HY = (LAST + 1) & ~1;  // halo rows (even: rows start on red parity)
    static constexpr int W = 10;                // register window (rows), even
    static constexpr int D = W - LAST - 2;      // prefetch distance (rows)
    static constexpr int WC = W / 2;            // coarse-row window
    static constexpr int DC = WC - 3;           // coarse prefetch distance
    static constexpr int OUTW = 128 - 2 * HX;   // output columns per tile
    static_assert(D >= 1 && DC >= 0, "window too small");
};

template <typename T, int NU, bool LOADPHI, bool PROLONG, int POST>
__global__ __launch_bounds__(256) void k_march(const MarchArgs<T> a) {
    using C = Cfg<NU, PROLONG, POST>;
    constexpr int W = C::W, D = C::D, WC = C::WC, DC = C::DC;

    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    // XCD-aware order: consecutive workgroup ids go to different XCDs, so give
    // each XCD a contiguous run of tiles (neighbouring tiles share halo rows in L2).
    const int lb = (blockIdx.x & 7) * a.groups_per_xcd + (blockIdx.x >> 3);
    const int tile = lb * wpb + (threadIdx.x >> 6);
    if (tile >= a.ntiles) return;  // whole wavefront leaves; no barriers below
    if (a.skip && *a.skip) return;
    const int strip = tile % a.strips, chunk = tile / a.strips;

    const int n = a.n, nm = n - 1;
    const bool px = a.bc[CCMG_XLO] == CCMG_BC_PERIODIC;
    const bool py = a.bc[CCMG_YLO] == CCMG_BC_PERIODIC;
    const T sxl = a.bc[CCMG_XLO] == CCMG_BC_DIRICHLET ? T(-1) : T(1);
    const T sxh = a.bc[CCMG_XHI] == CCMG_BC_DIRICHLET ? T(-1) : T(1);
    const T syl = a.bc[CCMG_YLO] == CCMG_BC_DIRICHLET ? T(-1) : T(1);
    const T syh = a.bc[CCMG_YHI] == CCMG_BC_DIRICHLET ? T(-1) : T(1);

    // columns
    const int xo0 = strip * a.outw;
    const int x0 = xo0 - C::HX + 2 * lane;
    const bool inx = px || (x0 >= 0 && x0 < n);
    const int xl = px ? (x0 & nm) : (inx ? x0 : 0);
    const bool wedge = !px && x0 == 0;        // column 0's west neighbour is a ghost
    const bool eedge = !px && x0 + 1 == nm;   // column 1's east neighbour is a ghost
    const bool outl = x0 >= xo0 && x0 < xo0 + a.outw && x0 >= 0 && x0 < n;

    // rows
    const int y0 = chunk * a.ty, y1 = min(y0 + a.ty, n);
    const int ys = py ? y0 - C::HY : max(y0 - C::HY, 0);
    const int ye = py ? y1 + C::HY : min(y1 + C::HY, n);

    const T cc = a.cc, invd = a.invd;
    T fsub = T(0), psub = T(0);
    if (a.fmean_part) fsub = T(sum_partials(a.fmean_part, a.fmean_count) / ((double)n * (double)n));
    if (LOADPHI && a.phi_shift) psub = T(*a.phi_shift);

    // coarse columns (prolongation): one coarse cell per lane
    const int nc = n >> 1;
    const int I = x0 >> 1;
    const bool inc = PROLONG && (px || (I >= 0 && I < nc));
    const int Il = PROLONG ? (px ? (I & (nc - 1)) : (inc ? I : 0)) : 0;
    const bool cwedge = !px && I == 0, ceedge = !px && I == nc - 1;

    T P0[W], P1[W], F0[W], F1[W], Cw[WC];
#pragma unroll
    for (int k = 0; k < W; ++k) P0[k] = P1[k] = F0[k] = F1[k] = T(0);
#pragma unroll
    for (int k = 0; k < WC; ++k) Cw[k] = T(0);

    auto load_row = [&](int y, T &p0, T &p1, T &f0, T &f1) {
        const int yy = py ? (y & nm) : y;
        const T *fr = a.f + (long)(yy + 1) * a.pf + 1 + xl;
        f0 = fr[0];
        f1 = fr[1];
        if (LOADPHI) {
            const T *pr = a.phi_in + (long)(yy + 1) * a.pin + 1 + xl;
            p0 = pr[0];
            p1 = pr[1];
        }
    };
    auto load_coarse = [&](int J, T &c) {
        if (!py && (J < -1 || J > nc)) return;
        const int Jl = py ? (J & (nc - 1)) : (J < 0 ? 0 : (J >= nc ? nc - 1 : J));
        c = a.ec[(long)(Jl + 1) * a.pc + 1 + Il];
    };

    // accumulators for the post-processing
    double acc0 = 0.0, acc1 = 0.0;
    T rprev0 = T(0), rprev1 = T(0);

    // prologue loads
    static_for<0, D>([&](auto kc) {
        constexpr int k = decltype(kc)::value;
        if (ys + k < ye) load_row(ys + k, P0[k], P1[k], F0[k], F1[k]);
    });
    if constexpr (PROLONG) {
        static_for<0, DC + 2>([&](auto qc) {
            constexpr int q = decltype(qc)::value;
            load_coarse((ys >> 1) - 1 + q, Cw[q]);
        });
    }

    const int tend = ye + C::LAST;
    for (int tb = ys; tb < tend; tb += W) {
        static_for<0, W>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            const int t = tb + k;
            // 1. prefetch
            if (t + D < ye) {
                constexpr int kd = (k + D) % W;
                load_row(t + D, P0[kd], P1[kd], F0[kd], F1[kd]);
            }
            if constexpr (PROLONG) {
                if ((k & 1) == 0) load_coarse((t >> 1) + 1 + DC, Cw[((k >> 1) + 2 + DC) % WC]);
            }
            // 2. finish the load of row t: masks, mean shifts, prolongation
            if (t < ye) {
                F0[k] = inx ? F0[k] - fsub : T(0);
                F1[k] = inx ? F1[k] - fsub : T(0);
                if (LOADPHI) {
                    P0[k] = inx ? P0[k] - psub : T(0);
                    P1[k] = inx ? P1[k] - psub : T(0);
                } else {
                    P0[k] = T(0);
                    P1[k] = T(0);
                }
                if constexpr (PROLONG) {
                    const int J = t >> 1;
                    T cm = Cw[((k >> 1) + 0) % WC];
                    T c0 = Cw[((k >> 1) + 1) % WC];
                    T cp = Cw[((k >> 1) + 2) % WC];
                    if (!py) {
                        if (J - 1 < 0) cm = syl * cm;
                        if (J + 1 >= nc) cp = syh * cp;
                    }
                    if (!inc) cm = c0 = cp = T(0);
                    T ew = from_left(c0), ee = from_right(c0);
                    if (cwedge) ew = sxl * c0;
                    if (ceedge) ee = sxh * c0;
                    const T mx = T(0.5) * (ee - ew);
                    const T my = T(0.5) * (cp - cm);
                    const T dy = (k & 1) ? T(0.25) : T(-0.25);
                    P0[k] = P0[k] + ((c0 + T(-0.25) * mx) + dy * my);
                    P1[k] = P1[k] + ((c0 + T(0.25) * mx) + dy * my);
                }
            }
            // 3. relaxation stages: stage s works on row t - s; odd s = red, even s = black
            static_for<1, 2 * NU + 1>([&](auto sc) {
                constexpr int s = decltype(sc)::value;
                const int y = t - s;
                if (y >= ys && y < ye) {
                    constexpr int kk = (k - s + 2 * W) % W;
                    constexpr int km = (k - s - 1 + 2 * W) % W;
                    constexpr int kp = (k - s + 1 + 2 * W) % W;
                    // red cells: (x + y) even; column 0 has x even; row parity = (k - s) & 1
                    constexpr int col = ((s & 1) ? ((k - s) & 1) : (1 - ((k - s) & 1)));
                    if constexpr (col == 0) {
                        const T self = P0[kk];
                        T e = P1[kk];
                        T w = from_left(P1[kk]);
                        if (wedge) w = sxl * self;
                        T nn = P0[kp], ss = P0[km];
                        if (!py) {
                            if (y == nm) nn = syh * self;
                            if (y == 0) ss = syl * self;
                        }
                        P0[kk] = (F0[kk] + cc * (((e + w) + nn) + ss)) * invd;
                    } else {
                        const T self = P1[kk];
                        T w = P0[kk];
                        T e = from_right(P0[kk]);
                        if (eedge) e = sxh * self;
                        T nn = P1[kp], ss = P1[km];
                        if (!py) {
                            if (y == nm) nn = syh * self;
                            if (y == 0) ss = syl * self;
                        }
                        P1[kk] = (F1[kk] + cc * (((e + w) + nn) + ss)) * invd;
                    }
                }
            });
            // 4. store the finished row
            {
                const int y = t - 2 * NU;
                constexpr int kk = (k - 2 * NU + 2 * W) % W;
                if (a.phi_out && y >= y0 && y < y1 && outl) {
                    T *o = a.phi_out + (long)(y + 1) * a.pout + 1 + x0;
                    o[0] = P0[kk];
                    o[1] = P1[kk];
                }
            }
            // 5. residual of the finished rows and what is made from it
            if constexpr (POST != POST_NONE) {
                const int y = t - C::LAGR;
                if (y >= y0 && y < y1) {
                    constexpr int kk = (k - C::LAGR + 2 * W) % W;
                    constexpr int km = (k - C::LAGR - 1 + 2 * W) % W;
                    constexpr int kp = (k - C::LAGR + 1 + 2 * W) % W;
                    const T p0 = P0[kk], p1 = P1[kk];
                    T w0 = from_left(P1[kk]);
                    T e1 = from_right(P0[kk]);
                    if (wedge) w0 = sxl * p0;
                    if (eedge) e1 = sxh * p1;
                    T n0 = P0[kp], n1 = P1[kp], s0 = P0[km], s1 = P1[km];
                    if (!py) {
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
                    if constexpr (POST == POST_RESTRICT) {
                        if ((k - C::LAGR) & 1) {  // odd row: close the 2x2 block
                            const T v = T(0.25) * (((rprev0 + rprev1) + r0) + r1);
                            if (outl) {
                                a.aux[(long)((y >> 1) + 1) * a.paux + 1 + (x0 >> 1)] = v;
                                acc0 += (double)v;
                            }
                        } else {
                            rprev0 = r0;
                            rprev1 = r1;
                        }
                    } else if constexpr (POST == POST_NORM) {
                        if (outl) {
                            acc0 += (double)r0 * (double)r0 + (double)r1 * (double)r1;
                            acc1 += (double)p0 + (double)p1;
                        }
                    } else {  // POST_RESID
                        if (outl) {
                            T *o = a.aux + (long)(y + 1) * a.paux + 1 + x0;
                            o[0] = r0;
                            o[1] = r1;
                        }
                    }
                }
            }
        });
    }

    if constexpr (POST == POST_RESTRICT) {
        const double s = wave_sum(acc0);
        if (lane == 0) a.partial[tile] = s;
    } else if constexpr (POST == POST_NORM) {
        const double s0 = wave_sum(acc0), s1 = wave_sum(acc1);
        if (lane == 0) {
            a.partial[2 * tile] = s0;
            a.partial[2 * tile + 1] = s1;
        }
    }
}

// ---- host side ---------------------------------------------------------------
template <int NU, bool PROLONG, int POST>
static int outw_of() { return Cfg<NU, PROLONG, POST>::OUTW; }

int march_outw(int nu, bool prolong, int post) {
    const int hxc = 2 * nu + (post ? 1 : 0) + (prolong ? 2 : 0);
    return 128 - 2 * ((hxc + 1) & ~1);
}
int march_halo_y(int nu, int post) {
    const int last = post ? 2 * nu + 1 : 2 * nu;
    return (last + 1) & ~1;
}

template <typename T, int NU, bool LOADPHI, bool PROLONG, int POST>
static hipError_t go(const MarchArgs<T> &a0, MarchShape sh, hipStream_t s, int *nt) {
    MarchArgs<T> a = a0;
    a.outw = Cfg<NU, PROLONG, POST>::OUTW;
    a.ty = sh.ty;
    a.strips = (a.n + a.outw - 1) / a.outw;
    a.chunks = (a.n + a.ty - 1) / a.ty;
    a.ntiles = a.strips * a.chunks;
    if (nt) *nt = a.ntiles;
    const int wpb = sh.wpb;
    const int blocks = (a.ntiles + wpb - 1) / wpb;
    a.groups_per_xcd = (blocks + 7) / 8;
    const int grid = 8 * a.groups_per_xcd;
    hipLaunchKernelGGL((k_march<T, NU, LOADPHI, PROLONG, POST>), dim3(grid), dim3(64 * wpb), 0, s, a);
    return hipGetLastError();
}

template <typename T, int NU>
static hipError_t dispatch_nu(const MarchArgs<T> &a, bool load_phi, bool prolong, int post,
                              MarchShape sh, hipStream_t s, int *nt) {
    if (prolong) {
        if (!load_phi) return hipErrorInvalidValue;
        if (post == POST_NONE) return go<T, NU, true, true, POST_NONE>(a, sh, s, nt);
        if (post == POST_NORM) return go<T, NU, true, true, POST_NORM>(a, sh, s, nt);
        return hipErrorInvalidValue;
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

template <typename T>
hipError_t launch_march(const MarchArgs<T> &a, int nu, bool load_phi, bool prolong, int post,
                        MarchShape shape, hipStream_t s, int *nt) {
    if (shape.ty < 2 || (shape.ty & 1) || shape.wpb < 1 || shape.wpb > 4) return hipErrorInvalidValue;
    switch (nu) {
        case 0: return dispatch_nu<T, 0>(a, load_phi, prolong, post, shape, s, nt);
        case 1: return dispatch_nu<T, 1>(a, load_phi, prolong, post, shape, s, nt);
        case 2: return dispatch_nu<T, 2>(a, load_phi, prolong, post, shape, s, nt);
    }
    return hipErrorInvalidValue;
}

template hipError_t launch_march<double>(const MarchArgs<double> &, int, bool, bool, int, MarchShape,
                                         hipStream_t, int *);
template hipError_t launch_march<float>(const MarchArgs<float> &, int, bool, bool, int, MarchShape,
                                        hipStream_t, int *);

}  // namespace ccmg
