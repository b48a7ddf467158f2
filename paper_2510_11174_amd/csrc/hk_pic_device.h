// Device helpers shared by the particle and conversion kernels (internal).
#pragma once
#include "hk_internal.h"

namespace hkdev {

constexpr int FT = TILE + 2;       // field tile edge: cells -1 .. TILE
constexpr int FT3 = FT * FT * FT;
constexpr int JT = TILE + 3;       // current tile edge: nodes -1 .. TILE+1
constexpr int JT3 = JT * JT * JT;

// cell -> (i, j, k) without integer division: (c + 1/2) / n is at least
// 1/(2n) away from an integer, far beyond the FP64 rounding of the product.
__device__ inline void cell_ijk(const GridP &g, int cell, int &i, int &j, int &k) {
    const double inx = 1.0 / (double)g.nx, iny = 1.0 / (double)g.ny;
    int r = (int)(((double)cell + 0.5) * inx);
    i = cell - r * g.nx;
    k = (int)(((double)r + 0.5) * iny);
    j = r - k * g.ny;
}

__device__ inline int tile_of(const GridP &g, int cell) {
    int ci = cell % g.nx, r = cell / g.nx;
    int cj = r % g.ny, ck = r / g.ny;
    return (ci >> TLOG) + g.ntx * ((cj >> TLOG) + g.nty * (ck >> TLOG));
}

// CIC weights of a node-type (o) and a half-type (o - 1/2) sample along one
// axis, as an LDS index (field tile origin at cell -1) and fraction.
struct AxisW {
    int in_, ih;
    real fn, fh;
};
__device__ inline AxisW axis_weights(int l, real o) {
    AxisW a;
    a.in_ = l + 1;
    a.fn = o;
    if (o >= (real)0.5) { a.ih = l + 1; a.fh = o - (real)0.5; }
    else { a.ih = l; a.fh = o + (real)0.5; }
    return a;
}

__device__ inline real tri(const real *F, int i, int j, int k, real fx, real fy, real fz) {
    const int b = i + FT * (j + FT * k);
    real acc = 0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                real wgt = (a ? fx : 1 - fx) * (bb ? fy : 1 - fy) * (c ? fz : 1 - fz);
                acc += wgt * F[b + a + FT * (bb + FT * c)];
            }
    return acc;
}

// Esirkepov shape factors along one axis for a move from offset o to X1 = o +
// delta (relative to the old cell), written in terms of the displacement so
// that slow particles keep full relative precision.  Window nodes base..base+2
// relative to the old cell; base is -1 when the particle crossed downwards.
struct AxisS {
    int base;
    real S0[3], DS[3];
};
__device__ inline AxisS axis_shapes(real o, real X1) {
    AxisS s;
    if (X1 >= (real)1) {                // crossed up: nodes 0, 1, 2
        real e = X1 - (real)1;
        s.base = 0;
        s.S0[0] = (real)1 - o; s.S0[1] = o; s.S0[2] = 0;
        s.DS[0] = -((real)1 - o); s.DS[1] = ((real)1 - e) - o; s.DS[2] = e;
    } else if (X1 < (real)0) {          // crossed down: nodes -1, 0, 1
        real e = -X1;
        s.base = -1;
        s.S0[0] = 0; s.S0[1] = (real)1 - o; s.S0[2] = o;
        s.DS[0] = e; s.DS[1] = o - e; s.DS[2] = -o;
    } else {                            // stayed: nodes 0, 1, 2
        real d = X1 - o;
        s.base = 0;
        s.S0[0] = (real)1 - o; s.S0[1] = o; s.S0[2] = 0;
        s.DS[0] = -d; s.DS[1] = d; s.DS[2] = 0;
    }
    return s;
}

// Deposit the Esirkepov current of one particle into the LDS J tile.  (lx, ly,
// lz) is the old cell inside the tile; cx = q w / dV * dx / dt (per axis).
__device__ inline void esirkepov_lds(real *sJ, int lx, int ly, int lz, const AxisS &X,
                                     const AxisS &Y, const AxisS &Z, real cx, real cy, real cz) {
    const real third = (real)(1.0 / 3.0), half = (real)0.5;
    const int ox = lx + X.base + 1, oy = ly + Y.base + 1, oz = lz + Z.base + 1;
    // Jx on faces a = 0, 1 (prefix of W_x along x)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            real fyz = Y.S0[b] * Z.S0[c] + half * Y.DS[b] * Z.S0[c] + half * Y.S0[b] * Z.DS[c] +
                       third * Y.DS[b] * Z.DS[c];
            real acc = 0;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                acc -= cx * (X.DS[a] * fyz);
                if (acc != (real)0)
                    atomicAdd(&sJ[0 * JT3 + (ox + a) + JT * ((oy + b) + JT * (oz + c))], acc);
            }
        }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            real fxz = X.S0[a] * Z.S0[c] + half * X.DS[a] * Z.S0[c] + half * X.S0[a] * Z.DS[c] +
                       third * X.DS[a] * Z.DS[c];
            real acc = 0;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                acc -= cy * (Y.DS[b] * fxz);
                if (acc != (real)0)
                    atomicAdd(&sJ[1 * JT3 + (ox + a) + JT * ((oy + b) + JT * (oz + c))], acc);
            }
        }
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            real fxy = X.S0[a] * Y.S0[b] + half * X.DS[a] * Y.S0[b] + half * X.S0[a] * Y.DS[b] +
                       third * X.DS[a] * Y.DS[b];
            real acc = 0;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                acc -= cz * (Z.DS[c] * fxy);
                if (acc != (real)0)
                    atomicAdd(&sJ[2 * JT3 + (ox + a) + JT * ((oy + b) + JT * (oz + c))], acc);
            }
        }
}

// Current accumulator type of the LDS tile.  On gfx950 an LDS float atomic
// add is serialized per lane (about 3 cycles per active lane) while a 64-bit
// integer add costs a few cycles per wavefront, so the FP32 build deposits
// the current in 64-bit fixed point: each workgroup picks a scale from its
// largest |q w| so that one particle's largest contribution is 2^40 units;
// integer sums are exact and independent of order.  The FP64 build keeps
// FP64 atomics (it is the precision reference, not the fast path).
#ifdef HK_DOUBLE
typedef double jacc_t;
__device__ inline void jadd(jacc_t *p, real v, real) { atomicAdd(p, v); }
__device__ inline double jval(jacc_t v, double) { return v; }
#else
typedef unsigned long long jacc_t;
// round-to-nearest float -> int64 for |x| < 2^51: adding 1.5 * 2^52 leaves
// the integer in the low mantissa bits of the double
__device__ inline long long round_to_i64(double x) {
    const double magic = 6755399441055744.0;
    return __double_as_longlong(x + magic) - __double_as_longlong(magic);
}
__device__ inline void jadd(jacc_t *p, real v, real inv_scale) {
    long long q = round_to_i64((double)(v * inv_scale));
    if (q) atomicAdd(p, (unsigned long long)q);
}
__device__ inline double jval(jacc_t v, double scale) { return (double)(long long)v * scale; }
#endif
constexpr float JFIX_UNITS = 1099511627776.0f;   // 2^40

// Esirkepov current of one particle added to an LDS tile of accumulators.
__device__ inline void esirkepov_acc(jacc_t *sJ, int lx, int ly, int lz, const AxisS &X,
                                     const AxisS &Y, const AxisS &Z, real cx, real cy, real cz,
                                     real inv_scale) {
    const real third = (real)(1.0 / 3.0), half = (real)0.5;
    const int ox = lx + X.base + 1, oy = ly + Y.base + 1, oz = lz + Z.base + 1;
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            real fyz = Y.S0[b] * Z.S0[c] + half * Y.DS[b] * Z.S0[c] + half * Y.S0[b] * Z.DS[c] +
                       third * Y.DS[b] * Z.DS[c];
            real acc = 0;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                acc -= cx * (X.DS[a] * fyz);
                if (acc != (real)0)
                    jadd(&sJ[0 * JT3 + (ox + a) + JT * ((oy + b) + JT * (oz + c))], acc, inv_scale);
            }
        }
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            real fxz = X.S0[a] * Z.S0[c] + half * X.DS[a] * Z.S0[c] + half * X.S0[a] * Z.DS[c] +
                       third * X.DS[a] * Z.DS[c];
            real acc = 0;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                acc -= cy * (Y.DS[b] * fxz);
                if (acc != (real)0)
                    jadd(&sJ[1 * JT3 + (ox + a) + JT * ((oy + b) + JT * (oz + c))], acc, inv_scale);
            }
        }
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            real fxy = X.S0[a] * Y.S0[b] + half * X.DS[a] * Y.S0[b] + half * X.S0[a] * Y.DS[b] +
                       third * X.DS[a] * Y.DS[b];
            real acc = 0;
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                acc -= cz * (Z.DS[c] * fxy);
                if (acc != (real)0)
                    jadd(&sJ[2 * JT3 + (ox + a) + JT * ((oy + b) + JT * (oz + c))], acc, inv_scale);
            }
        }
}

__device__ inline real below_one() {
#ifdef HK_DOUBLE
    return 0.99999999999999988898;
#else
    return 0.99999994f;
#endif
}


// ------------------------------------------------------------------ QED lookups
// Table position of chi: the tables cover log10 chi in [-3, 3] in 255 steps;
// chi is clamped to that range.
__device__ inline void qed_chi_pos(double chi, int &i, double &f) {
    double x = (log10(chi) + 3.0) * (double)(QED_NCHI - 1) / 6.0;
    x = fmin(fmax(x, 0.0), (double)(QED_NCHI - 1));
    i = min((int)x, QED_NCHI - 2);
    f = x - i;
}
// Spectrum total W(chi), linear in log10 chi.
__device__ inline double qed_total(const double *W, double chi) {
    int i; double f;
    qed_chi_pos(chi, i, f);
    return (1.0 - f) * W[i] + f * W[i + 1];
}
// Energy fraction delta for the uniform draw r: bilinear in (log10 chi, u) on
// the table of x, then delta = x^3 / (x^3 + (1 - x)^3).
__device__ inline double qed_fraction(const double *X, double chi, double r) {
    int i; double f;
    qed_chi_pos(chi, i, f);
    double y = fmin(fmax(r * QED_NU - 0.5, 0.0), (double)(QED_NU - 1));
    const int j = min((int)y, QED_NU - 2);
    const double g = y - j;
    const double *a = X + (size_t)i * QED_NU, *b = a + QED_NU;
    const double x = (1.0 - f) * ((1.0 - g) * a[j] + g * a[j + 1]) + f * ((1.0 - g) * b[j] + g * b[j + 1]);
    const double x3 = x * x * x, y3 = (1.0 - x) * (1.0 - x) * (1.0 - x);
    return x3 / (x3 + y3);
}
// Quantum parameter of a lepton (momentum u) or photon (momentum k, photon = 1):
// (energy / a_s) sqrt(|E + v x B|^2 - (v.E)^2), v the velocity.
__device__ inline double qed_chi(double a_s, double ex, double ey, double ez, double bx, double by,
                                 double bz, double ux, double uy, double uz, bool photon) {
    const double p = sqrt(ux * ux + uy * uy + uz * uz);
    if (!(p > 0.0)) return 0.0;
    const double en = photon ? p : sqrt(1.0 + p * p);
    const double vx = ux / en, vy = uy / en, vz = uz / en;
    const double fx = ex + vy * bz - vz * by, fy = ey + vz * bx - vx * bz, fz = ez + vx * by - vy * bx;
    const double ve = vx * ex + vy * ey + vz * ez;
    const double q2 = fx * fx + fy * fy + fz * fz - ve * ve;
    return en / a_s * sqrt(fmax(q2, 0.0));
}

// One slot per requesting lane in ctr, one atomic per wave.  Every lane of
// the wave calls it.
__device__ inline int wave_slot(int *ctr, bool want) {
    const uint64_t m = __ballot(want);
    if (!m) return -1;
    const int lane = __lane_id();
    const int leader = __ffsll((long long)m) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(ctr, __popcll(m));
    base = __shfl(base, leader);
    return want ? base + __popcll(m & ((1ull << lane) - 1ull)) : -1;
}

// Work items of the per-tile particle kernels.  A tile of n particles forms
// ceil(n / c) items of c = tile_chunk(n, cmin) consecutive bin slots (the last
// one shorter), at most TILE_SPLIT of them.  A planner lists the items by
// decreasing size, and workgroups take them in order from a global ticket, so
// dense tiles start first and every compute unit, whichever XCD it sits on,
// pulls the next item when it frees a slot.  (Block i of a launch goes to XCD
// i mod 8: a dense sheet of tiles at one x index would land on one XCD.)
constexpr int TILE_SPLIT = 16;
__device__ inline int tile_chunk(int n, int cmin) {
    return max(cmin, ((n + TILE_SPLIT - 1) / TILE_SPLIT + 511) / 512 * 512);
}
// Thread 0 takes the workgroup's item from ticket ctl[ticket]; (-1, 0) when
// the list (ctl[0] items) is exhausted.
__device__ inline int2 take_item(const int2 *items, int *ctl, int ticket) {
    const int k = atomicAdd(&ctl[ticket], 1);
    return k < ctl[0] ? items[k] : make_int2(-1, 0);
}

}  // namespace hkdev
