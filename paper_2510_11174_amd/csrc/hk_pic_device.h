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

// Reciprocal and square root: the hardware's (1 ulp) in FP32, correctly
// rounded in FP64.  The FP32 square roots here take arguments >= 1 (Lorentz
// factors), where the correctly rounded FP32 sequence would only add
// denormal scaling and a final ulp fix-up.
__device__ inline float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double rcp_(double x) { return 1.0 / x; }
__device__ inline float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ inline double sqrt_(double x) { return sqrt(x); }

// Trilinear interpolation as three rounds of linear interpolation (x, y, z).
__device__ inline real tri(const real *F, int i, int j, int k, real fx, real fy, real fz) {
    const real *p = F + i + FT * (j + FT * k);
    const real c00 = p[0] + fx * (p[1] - p[0]);
    const real c10 = p[FT] + fx * (p[FT + 1] - p[FT]);
    const real c01 = p[FT * FT] + fx * (p[FT * FT + 1] - p[FT * FT]);
    const real c11 = p[FT * FT + FT] + fx * (p[FT * FT + FT + 1] - p[FT * FT + FT]);
    const real c0 = c00 + fy * (c10 - c00), c1 = c01 + fy * (c11 - c01);
    return c0 + fz * (c1 - c0);
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
    // crossed up: nodes 0, 1, 2 with e = X1 - 1; crossed down: nodes -1, 0, 1
    // with e = -X1; stayed: nodes 0, 1, 2 with d = X1 - o.  Selects, not
    // branches: the lanes of a wave take different cases.
    const bool up = X1 >= (real)1, dn = X1 < (real)0;
    const real e = up ? X1 - (real)1 : -X1, d = X1 - o, q = (real)1 - o;
    AxisS s;
    s.base = dn ? -1 : 0;
    s.S0[0] = dn ? (real)0 : q;
    s.S0[1] = dn ? q : o;
    s.S0[2] = dn ? o : (real)0;
    s.DS[0] = up ? -q : (dn ? e : -d);
    s.DS[1] = up ? ((real)1 - e) - o : (dn ? o - e : d);
    s.DS[2] = up ? e : (dn ? -o : (real)0);
    return s;
}

// A lane's move crosses a cell face along this axis (its shape window then
// uses the third node, and two longitudinal faces carry current).
__device__ inline bool crosses(real X1) { return X1 >= (real)1 || X1 < (real)0; }

// Bits 0, 1, 2: some active lane of the wave crosses along x, y, z.  The
// value is the same on every lane and lives in a scalar register.
__device__ inline unsigned wave_crossings(real X1, real Y1, real Z1) {
    const unsigned f = (__ballot(crosses(X1)) ? 1u : 0u) | (__ballot(crosses(Y1)) ? 2u : 0u) |
                       (__ballot(crosses(Z1)) ? 4u : 0u);
    return __builtin_amdgcn_readfirstlane(f);
}

// Current accumulator type of the LDS tile.  On gfx950 an LDS float atomic
// add is serialized per lane (about 3 cycles per active lane) while a 64-bit
// integer add costs a few cycles per wavefront, so the FP32 build deposits
// the current in 64-bit fixed point: the unit is a power of two 2^e chosen
// per species (jdep_exp) so that one particle's largest contribution, from
// the species' weight bound, is at most 2^30 units; integer sums are exact
// and independent of order, and a tile's sums move to the global
// accumulator (unit 2^-JG_BITS) by a left shift, exactly.  The FP64 build
// keeps FP64 atomics (it is the precision reference, not the fast path).
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
constexpr float JFIX_UNITS = 1099511627776.0f;   // 2^40 (moment sums)

// Exponent e of a species' deposit unit 2^e: the largest contribution jmax is
// at most 2^(e + 30) units' worth; e >= -JG_BITS keeps the conversion to the
// global unit a left shift.
__device__ inline int jdep_exp(double jmax) {
    if (!(jmax > 0.0)) return -JG_BITS;
    int e;
    const double m = frexp(jmax, &e);   // jmax = m 2^e, m in [0.5, 1): jmax <= 2^e
    (void)m;
    return max(e - 30, -JG_BITS);
}

// The push deposits in 32-bit units: one particle's largest current
// contribution is 2^30 units, so every contribution converts with one FP32 ->
// int32 rounding and is added to the 64-bit LDS sum (no overflow for any
// count of particles a tile can hold).
constexpr float JDEP_UNITS = 1073741824.0f;   // 2^30
#ifdef HK_DOUBLE
__device__ inline void jput(jacc_t *p, real v) {
    if (v != (real)0) atomicAdd(p, v);
}
#else
// v_cvt_rpi_i32_f32 rounds to the nearest integer (halves up) in one
// instruction, where rint and a conversion take two
__device__ inline int round_i32(float v) {
    int q;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(q) : "v"(v));
    return q;
}
__device__ inline void jput(jacc_t *p, real v) {   // v in units
    const int q = round_i32(v);
    if (q) atomicAdd(p, (unsigned long long)(long long)q);
}
#endif

// Tile sums and single contributions into the global accumulator.
#ifdef HK_DOUBLE
__device__ inline void jg_flush(jglob_t *p, jacc_t v, int) {
    if (v != 0.0) atomicAdd(p, v);
}
__device__ inline void jg_put(jglob_t *p, double v) {
    if (v != 0.0) atomicAdd(p, v);
}
#else
// v: a tile sum in units 2^e; shift = e + JG_BITS >= 0 (two's complement:
// the shifted bits are the signed product, modulo 2^64 like every sum here)
__device__ inline void jg_flush(jglob_t *p, jacc_t v, int shift) {
    if (v) atomicAdd(p, v << shift);
}
// one contribution in physical units, rounded once to the global unit
__device__ inline void jg_put(jglob_t *p, double v) {
    const long long q = __double2ll_rn(v * (double)(1ull << JG_BITS));
    if (q) atomicAdd(p, (unsigned long long)q);
}
#endif

// Esirkepov current of one particle (linear shapes, a 3-node window per
// axis) added to the LDS accumulators.  With A = S0 + DS / 2 and B = S0 / 2 +
// DS / 3 per axis, the transverse weight of an x face (b, c) is
// S0z_c Ay_b + DSz_c By_b (likewise for y and z faces), and the face current
// is minus the running sum of the longitudinal shape change, times q w / dV
// * dx / dt (cx, cy, cz: in units in the FP32 build).  The running sum over
// the last node of the window is zero, so two faces per line carry current.
// A lane that does not cross a face along an axis has zero shape on the
// window's third node and a zero second face (DS0 + DS1 = 0 exactly) along
// it: bits 0, 1, 2 of wf (the same on every lane of the wave) say whether
// any lane crossed along x, y, z; the terms that are zero on every lane are
// skipped, which leaves 12 of the 54 when none did.
__device__ inline void esirkepov_acc(jacc_t *sJ, int lx, int ly, int lz, const AxisS &X,
                                     const AxisS &Y, const AxisS &Z, real cx, real cy, real cz,
                                     unsigned wf) {
    const bool wx = wf & 1u, wy = wf & 2u, wz = wf & 4u;
    const real third = (real)(1.0 / 3.0), half = (real)0.5;
    real Ax[3], Bx[3], Ay[3], By[3], Az[3], Bz[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        Ax[k] = X.S0[k] + half * X.DS[k]; Bx[k] = half * X.S0[k] + third * X.DS[k];
        Ay[k] = Y.S0[k] + half * Y.DS[k]; By[k] = half * Y.S0[k] + third * Y.DS[k];
        Az[k] = Z.S0[k] + half * Z.DS[k]; Bz[k] = half * Z.S0[k] + third * Z.DS[k];
    }
    // window origin in the tile: constant offsets from here on
    jacc_t *o = sJ + (lx + X.base + 1) + JT * ((ly + Y.base + 1) + JT * (lz + Z.base + 1));
    const real kx0 = -cx * X.DS[0], kx1 = -cx * (X.DS[0] + X.DS[1]);
    const real ky0 = -cy * Y.DS[0], ky1 = -cy * (Y.DS[0] + Y.DS[1]);
    const real kz0 = -cz * Z.DS[0], kz1 = -cz * (Z.DS[0] + Z.DS[1]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (c == 2 && !wz) break;
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            if (b == 2 && !wy) break;
            const real f = Z.S0[c] * Ay[b] + Z.DS[c] * By[b];
            jput(o + 0 * JT3 + 0 + JT * (b + JT * c), kx0 * f);
            if (wx) jput(o + 0 * JT3 + 1 + JT * (b + JT * c), kx1 * f);
        }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (c == 2 && !wz) break;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (a == 2 && !wx) break;
            const real f = Z.S0[c] * Ax[a] + Z.DS[c] * Bx[a];
            jput(o + 1 * JT3 + a + JT * (0 + JT * c), ky0 * f);
            if (wy) jput(o + 1 * JT3 + a + JT * (1 + JT * c), ky1 * f);
        }
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        if (b == 2 && !wy) break;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (a == 2 && !wx) break;
            const real f = Y.S0[b] * Ax[a] + Y.DS[b] * Bx[a];
            jput(o + 2 * JT3 + a + JT * (b + JT * 0), kz0 * f);
            if (wz) jput(o + 2 * JT3 + a + JT * (b + JT * 1), kz1 * f);
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

// An FP32 upper bound of chi: |E + v x B| <= |E| + |B| for |v| <= 1, so chi <=
// energy (|E| + |B|) / a_s.  Below the QED floor with a 2% margin for the
// rounding of this bound, chi (in FP64) is below it too and no event, nor
// any change of the optical depth, can happen: the FP64 evaluation is skipped.
__device__ inline bool qed_chi_below_floor(float a_s, float ex, float ey, float ez, float bx, float by,
                                           float bz, float ux, float uy, float uz, bool photon, float floor_) {
    // hardware square roots (1 ulp each): the margin covers them
    const float p2 = ux * ux + uy * uy + uz * uz;
    const float en = __builtin_amdgcn_sqrtf(photon ? p2 : 1.0f + p2);
    const float f = __builtin_amdgcn_sqrtf(ex * ex + ey * ey + ez * ez) +
                    __builtin_amdgcn_sqrtf(bx * bx + by * by + bz * bz);
    return en * f * 1.02f < floor_ * a_s;
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
// decreasing size and block b of the launch takes item b: blocks go to the 8
// XCDs in turn and each XCD starts its blocks in order, so every XCD gets an
// even share of the dense tiles and starts with them.  (One block per tile in
// tile order would put a dense sheet of tiles at one x index, whose indices
// agree mod 8, on one XCD.)  No global ticket: a counter that every block
// bumps serializes at one L2 address, about 10 ns per block.
constexpr int TILE_SPLIT = 16;
__device__ inline int tile_chunk(int n, int cmin) {
    return max(cmin, ((n + TILE_SPLIT - 1) / TILE_SPLIT + 511) / 512 * 512);
}
// Item b of a plan with ctl[0] items; (-1, 0) past the end.
__device__ inline int2 plan_item(const int2 *items, const int *ctl, int b) {
    return b < ctl[0] ? items[b] : make_int2(-1, 0);
}
// Kernels without a plan (tile, part items in tile order): block b of a grid
// of 8 q blocks takes item (b mod 8) q + b / 8, so XCD x handles the
// contiguous item range [x q, (x + 1) q), a slab of whole tile rows in z.
__device__ inline int xcd_item(int b, int nblocks) {
    const int q = nblocks >> 3;
    return (b & 7) * q + (b >> 3);
}

}  // namespace hkdev
