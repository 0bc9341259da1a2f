// Matrix-core (MFMA) apply of the stored 80-offset operator to blocks of up
// to twelve right-hand sides: FP16 operands, FP32 accumulation.
//
// The off-diagonal part of Eq. def_pref is a sum over offsets n of
// [lambda_k + rho_k sum_mu n_mu gamma_mu] W(x,x+n) psi(x+n).  The spin matrix
// is moved out of the sum by splitting it into five colour contractions with
// scalar weights,
//   X_0 = sum_n lambda_k W_n psi(x+n),   X_mu = sum_n rho_k n_mu W_n psi(x+n),
// so that D psi = (lambda_0 + m) psi + X_0 + sum_mu gamma_mu X_mu.  Per site
// the five sums are one real matrix product:
//   rows       (channel c = 0..4, colour a, re/im)          30 of 32
//   reduction  (offset n, colour b, re/im)                    6 of 8 per offset
//   columns    (right-hand side r, spin s)                   16 per tile
// computed with v_mfma_f32_16x16x32_f16: the A operand is the weighted
// transporter (weights per channel and offset, in FP16, normalised by the
// largest |lambda_k| or |rho_k|), the B operand is psi(x+n) in FP16 scaled by
// a power of two per right-hand side, the products accumulate in FP32.  Every
// right-hand side of a site shares one transporter load, and no spin algebra
// is done per offset; the gamma matrices act once per site on X_mu.
//
// Work layout: a workgroup owns a 4 x 2 tile of (x, y) at fixed z and walks
// t over a chunk.  For each t it needs psi on the planes (z-1..z+1) x
// (t-1..t+1) over the tile and a one-site halo: a ring of nine planes in LDS
// (FP16, all right-hand sides of the block), three of which are replaced per
// step, loaded into registers during the previous step.  Eight wavefronts,
// two per SIMD so that one issues while the other waits, each compute one
// site per step: 20 reduction steps of four offsets, six MFMAs each (2 row
// tiles x 3 column tiles), then an epilogue through LDS that applies the
// gamma matrices, rescales and adds the diagonal term in FP32.
//
// The transporters come from a site-major FP16 store (bri_pack_w_mfma):
// for each site the 80 offsets in the order of the 80-offset store, each a
// row-major 3x3 complex matrix (2880 B per site), so that a lane's three
// entries of one row are one 12-byte load.  The spinors are site-major too,
// [V][nrhs][12] FP32 complex: the records of all right-hand sides of a halo
// point are one contiguous run, so staging a plane reads whole cache lines
// and writes the output in runs of 96 B per right-hand side.  k_transpose
// converts from and to the SoA layout of the other kernels.
#include <cmath>
#include <cstddef>

#include "abi_internal.h"
#include "kernels.h"

namespace bri {
namespace mfma {

constexpr int TX = 4, TY = 2, HX = TX + 2, HY = TY + 2, RP = HX * HY;  // 24 halo-tile points
constexpr int RPP = RP + 1;  // odd point stride of the LDS ring (conflict-free column reads)
constexpr int NTHR = 512;
constexpr int NWAVE = NTHR / 64;
constexpr int SPW = TX * TY / NWAVE;  // consecutive sites of a tile row per wavefront (1)
constexpr int NTB = 3;  // column tiles (4 right-hand sides each) per workgroup
constexpr int NPT = 80;        // offsets
constexpr int KSTEPS = NPT / 4;  // reduction steps of four offsets
constexpr int WSITE = NPT * 9;   // complex transporter entries per site

typedef _Float16 h2 __attribute__((ext_vector_type(2)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef uint32_t u4 __attribute__((ext_vector_type(4)));

// offset component mu (0..3 = x, y, z, t) of store index p (0..79)
__host__ __device__ constexpr int comp(int p, int mu) {
    const int i = p < 40 ? p : p + 1;  // index over the 81 points, centre = 40
    const int d = mu == 0 ? 1 : mu == 1 ? 3 : mu == 2 ? 9 : 27;
    return (i / d) % 3 - 1;
}

struct Args {
    Geom g;
    int ntx, nty, ntc, tlen, nrhs;  // nrhs: right-hand sides of a site record (12 complex each)
    int gx, gy, gz;                 // tiles per block group in x, y, z (divisors of ntx, nty, Lz)
    const uint32_t *Wm;     // site-major FP16 store, one complex per 32-bit word
    const float2 *in;       // site-major: [V][nrhs][12]
    float2 *out;
    const double *bound2;   // per right-hand side (stride bstride): >= max |component|^2 of in
    int bstride;
    double *nrm;            // optional: per (right-hand side, workgroup of its block) partial |out|^2
    float diag, slam, srho;  // lambda_0 + m; channel normalisations
    float lam[5], rho[5];    // lambda_k / slam, rho_k / srho (k = 1..4; rho negated for D^dag)
};

// select by k in 1..4 without indexing the argument array (a run-time index
// into a kernel argument would copy the argument block to scratch)
__device__ __forceinline__ float pick(const float (&v)[5], int k) {
    return k == 1 ? v[1] : k == 2 ? v[2] : k == 3 ? v[3] : v[4];
}

__device__ __forceinline__ uint32_t bits(h2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ h2 hv(uint32_t v) { return __builtin_bit_cast(h2, v); }

__device__ __forceinline__ int wrap(int v, int L) { return v < 0 ? v + L : v >= L ? v - L : v; }

template <int NT>
struct Smem {
    static constexpr int RN = 16 * NT;          // records (r, s) per point
    uint2 b01[9 * RN * RPP];                    // colours 0, 1 of a record (2 x FP16 complex)
    uint32_t b2[9 * RN * RPP];                  // colour 2
    float2 scr[NWAVE][16][16];                  // per-wavefront epilogue tile pair (re, im)
    // per (t mod 3, reduction step, lane): FP16 coefficient of the lane's A
    // row << 16 | ring record of the lane's B column for the step's offset
    uint32_t ktab[3][KSTEPS][64];
    float scl[4 * NT], iscl[4 * NT];
    // per halo point of a plane set (z-1..z+1 x the 6 x 4 halo tile): byte
    // offset of its site record (from the block's first right-hand side)
    // within a t plane, and its ring index (z plane, point)
    uint2 ptab[3 * RP];
};

template <int NT>
__global__ __launch_bounds__(NTHR) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_apply_mfma(const Args a) {
    constexpr int RN = Smem<NT>::RN;
    constexpr int NPTS = 3 * RP;             // halo points of one plane set (three z planes)
    constexpr int CPP = 3 * RN / 2;          // 16-byte chunks (two complex numbers) of a point's records
    constexpr int PS = NTHR / CPP;           // points staged side by side (a thread keeps its chunk)
    constexpr int KMAX = (NPTS + PS - 1) / PS;  // points per staging thread
    constexpr int NB = SPW;                   // staging batches per plane set (one per site)
    constexpr int KB = (KMAX + NB - 1) / NB;  // points of a batch
    __shared__ Smem<NT> sm;

    // kernel-argument fields as locals: the lambdas below capture by
    // reference, and a captured kernel argument would be copied to scratch
    const int Lx = a.g.L[0], Ly = a.g.L[1], Lz = a.g.L[2], Lt = a.g.L[3];
    // 64-bit bases are wave-uniform (scalar registers); the lanes add
    // 32-bit byte offsets (the host bounds a t plane of the fields by 4 GiB)
    const char *__restrict__ in = (const char *)a.in;
    char *__restrict__ out = (char *)a.out;
    const char *__restrict__ Wm = (const char *)a.Wm;
    const float diag = a.diag, slam = a.slam, srho = a.srho;
    const uint32_t recb = (uint32_t)a.nrhs * 96u;  // bytes of a site record (nrhs x 12 complex FP32)
    const size_t planeb = (size_t)a.g.V / Lt * recb;  // bytes of a t plane
    const float lamw[5] = {0.0f, a.lam[1], a.lam[2], a.lam[3], a.lam[4]};
    const float rhow[5] = {0.0f, a.rho[1], a.rho[2], a.rho[3], a.rho[4]};
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wavefront index (uniform)

    // right-hand-side block fastest: the blocks of a tile run back to back
    // on one XCD and share the transporter rows through its L2; then the
    // tiles of a gx x gy x gz group, so that the workgroups an XCD runs at
    // one time are neighbours in x, y and z and share their halo planes
    // through its L2
    const int nrb = (a.nrhs + 4 * NT - 1) / (4 * NT);
    int rest = xcd_block(blockIdx.x, gridDim.x);
    const int rb = rest % nrb;
    rest /= nrb;
    const int iwg = rest;  // workgroup within the right-hand-side block (partial norm index)
    const int ix = rest % a.gx;
    rest /= a.gx;
    const int iy = rest % a.gy;
    rest /= a.gy;
    const int iz = rest % a.gz;
    rest /= a.gz;
    const int bx = (rest % (a.ntx / a.gx)) * a.gx + ix;
    rest /= a.ntx / a.gx;
    const int by = (rest % (a.nty / a.gy)) * a.gy + iy;
    rest /= a.nty / a.gy;
    const int z = (rest % (Lz / a.gz)) * a.gz + iz;
    const int tc = rest / (Lz / a.gz);
    const int t0 = tc * a.tlen, t1 = min(t0 + a.tlen, Lt);
    const int r0 = rb * 4 * NT, nr = min(4 * NT, a.nrhs - r0);
    const int x0 = bx * TX, y0 = by * TY;

    // per right-hand side: psi is scaled by 2^(14 - e) with 2^e > its largest component
    if (tid < 4 * NT) {
        float s = 1.0f;
        if (tid < nr) {
            const double b2 = a.bound2[(size_t)(r0 + tid) * a.bstride];
            if (b2 > 0.0 && b2 < INFINITY) {
                int e;
                frexp(sqrt(b2), &e);
                e = min(max(e, -100), 128);
                s = ldexpf(1.0f, 14 - e);
            }
        }
        sm.scl[tid] = s;
        sm.iscl[tid] = 1.0f / s;
    }

    for (int p = tid; p < NPTS; p += NTHR) {
        const int pz = p / RP, rp = p % RP, hx = rp % HX, hy = rp / HX;
        // the halo tile can reach past the lattice by more than one extent
        // when Lx or Ly is smaller than the tile: a full modulo
        const int xx = (x0 + hx - 1 + Lx) % Lx, yy = (y0 + hy - 1 + Ly) % Ly, zz = (z + pz - 1 + Lz) % Lz;
        const uint32_t s3 = (uint32_t)xx + (uint32_t)Lx * ((uint32_t)yy + (uint32_t)Ly * (uint32_t)zz);
        sm.ptab[p] = make_uint2(s3 * recb + (uint32_t)r0 * 96u, (uint32_t)(pz * RN * RPP + rp));
    }

    // ---- lane constants of the MFMA operands, as an LDS table
    const int grp = lane >> 4, row = lane & 15;  // A/B: lane group (offset of the step), row or column
    const int acol = row < 15 ? row / 5 : 0;     // colour a of the A row (row 15 is padding)
    for (int i = tid; i < 3 * KSTEPS * 64; i += NTHR) {
        const int m = i / (KSTEPS * 64), q = (i / 64) % KSTEPS, l = i % 64;
        const int lg = l >> 4, lr = l & 15;
        const int p = 4 * q + lg;
        const int nx = comp(p, 0), ny = comp(p, 1), nz = comp(p, 2), nt = comp(p, 3);
        // FP16 weight of the lane's A row: channel 0 lambda_k, channel mu + 1 rho_k n_mu
        const int k = (nx != 0) + (ny != 0) + (nz != 0) + (nt != 0), ch = lr % 5;
        const float nmu = ch == 1 ? (float)nx : ch == 2 ? (float)ny : ch == 3 ? (float)nz : (float)nt;
        const float wgt = ch == 0 ? pick(lamw, k) : pick(rhow, k) * nmu;
        const uint32_t c = lr < 15 ? (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)wgt) : 0u;
        const int slot = (m + nt + 3) % 3;  // ring slot of the plane t + n_t
        const int li = ((slot * 3 + nz + 1) * RN + lr) * RPP + (1 + nx) + HX * (1 + ny);
        sm.ktab[m][q][l] = (c << 16) | (uint32_t)li;
    }
    const uint32_t awoff = (uint32_t)(grp * 9 + acol * 3);  // A: this lane's row of the step's first offset

    // ---- the wavefront's SPW sites (consecutive x of one tile row), walking t
    const int kx0 = (SPW * w) % TX, ky = (SPW * w) / TX;
    const int ys = y0 + ky, xs0 = x0 + kx0;
    const int nval = ys < Ly ? max(0, min(SPW, Lx - xs0)) : 0;  // valid sites of the wavefront
    const int srp0 = kx0 + HX * ky;  // halo-tile point of site 0 minus the offset (1, 1)
    // sites past the lattice (ragged tiles) are computed on a clamped site
    // and not stored, so that the walk has no branches
    const int ysc = min(ys, Ly - 1);
    auto site_of = [&](int i, int t) __attribute__((always_inline)) {
        return (size_t)min(xs0 + i, Lx - 1) + (size_t)Lx * (ysc + (size_t)Ly * (z + (size_t)Lz * t));
    };

    // epilogue lane (one column tile at a time): colour a = lane / 16, rhs r' = (lane % 16) / 4, spin s = lane % 4
    const int ea = lane >> 4, er4 = (lane >> 2) & 3, es = lane & 3;

    // ---- staging of one plane set (z-1..z+1 at time tt) in NB batches:
    // loads into registers, conversion to scaled FP16, stores into the ring.
    // A thread keeps one 16-byte chunk of a point's records (two complex
    // numbers of one right-hand side: 12 complex numbers, six chunks, per
    // right-hand side) and takes every PS-th halo point, so that the lanes of
    // a load cover whole cache lines of a site record.  Every load is issued
    // (straight-line code, so the compiler counts outstanding loads exactly):
    // points past the plane set read point 0 and are not stored, chunks of
    // absent right-hand sides read a present one and are scaled by zero.
    const int sch = tid % CPP, sp0 = tid / CPP;  // the thread's chunk and first point
    const int sr = sch / 6;                      // its right-hand side in the block
    const uint32_t rofs = (uint32_t)(min(sr, nr - 1) * 6 + sch % 6) * 16u;  // chunk within the block's records
    // LDS byte address of the chunk's complex number h (0, 1) in ring record
    // (0, 0) and the bytes per ring record of its array: colours 0, 1 in b01,
    // colour 2 in b2
    uint32_t lofs[2], lstr[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int k = 2 * (sch % 6) + h, rec = 4 * sr + k / 3, col = k % 3;  // spin k / 3
        constexpr uint32_t b01 = offsetof(Smem<NT>, b01), b2 = offsetof(Smem<NT>, b2);
        lstr[h] = col < 2 ? 8u : 4u;
        lofs[h] = (col < 2 ? b01 + 4u * col : b2) + (uint32_t)rec * RPP * lstr[h];
    }
    float ssc = 0.0f;  // the chunk's scale (zero for an absent right-hand side), set after the scales are stored
    float4 pre[KB];
    uint32_t preh[KMAX][2];
    auto point_of = [&](int k) __attribute__((always_inline)) {
        const int p = sp0 + PS * k;
        return p < NPTS ? p : 0;
    };
    auto load_batch = [&](int tt, auto B) __attribute__((always_inline)) {
        constexpr int k0 = decltype(B)::value * KB, k1 = k0 + KB < KMAX ? k0 + KB : KMAX;
        const int tw = ((tt % Lt) + Lt) % Lt;
        const char *pl = in + (size_t)tw * planeb;  // uniform
#pragma unroll
        for (int k = k0; k < k1; ++k) pre[k - k0] = *(const float4 *)(pl + (sm.ptab[point_of(k)].x + rofs));
    };
    auto convert_batch = [&](auto B) __attribute__((always_inline)) {
        constexpr int k0 = decltype(B)::value * KB, k1 = k0 + KB < KMAX ? k0 + KB : KMAX;
#pragma unroll
        for (int k = k0; k < k1; ++k) {
            const float4 v = pre[k - k0];
            preh[k][0] = bits(h2{(_Float16)(v.x * ssc), (_Float16)(v.y * ssc)});
            preh[k][1] = bits(h2{(_Float16)(v.z * ssc), (_Float16)(v.w * ssc)});
        }
    };
    // batch b: convert batch b - 1, issue batch b; b = NB converts the last
    auto stage_step = [&](int tt, auto B) __attribute__((always_inline)) {
        constexpr int b = decltype(B)::value;
        if constexpr (b > 0) convert_batch(ic<b - 1>{});
        if constexpr (b < NB) load_batch(tt, ic<b>{});
    };
    auto store_planes = [&](int tt) __attribute__((always_inline)) {
        const uint32_t sbase = (uint32_t)(((tt % 3) + 3) % 3) * (3 * RN * RPP);
#pragma unroll
        for (int k = 0; k < KMAX; ++k) {
            const int p = sp0 + PS * k;
            if (p < NPTS && sp0 < PS) {  // (threads past PS x CPP only load)
                const uint32_t li = sbase + sm.ptab[p].y;
#pragma unroll
                for (int h = 0; h < 2; ++h)
                    *(uint32_t *)((char *)&sm + (lofs[h] + li * lstr[h])) = preh[k][h];
            }
        }
    };

    // ---- per-site transporter rows and psi(x) for the diagonal term; the
    // rows of the next site are loaded into the registers of the rows just
    // consumed, one reduction step at a time (unconditionally, see above)
    uint32_t wa[KSTEPS][3];
    float2 px[NT];
    const uint32_t awb = awoff * 4u;  // byte offset of the lane's row in a site's transporters
    auto load_rows = [&](size_t site, int q) __attribute__((always_inline)) {
        const char *ws = Wm + site * (WSITE * 4);  // uniform
#pragma unroll
        for (int b = 0; b < 3; ++b)
            wa[q][b] = __builtin_nontemporal_load((const uint32_t *)(ws + (awb + (uint32_t)(q * 144 + 4 * b))));
    };
    // byte offset of the epilogue lane's output (column tile j) in a site record
    auto out_ofs = [&](int j) __attribute__((always_inline)) {
        return (uint32_t)((r0 + min(4 * j + er4, nr - 1)) * 12 + 3 * es + min(ea, 2)) * 8u;
    };
    auto load_px = [&](size_t site) __attribute__((always_inline)) {
        const char *is = in + site * recb;  // uniform
#pragma unroll
        for (int j = 0; j < NT; ++j) px[j] = *(const float2 *)(is + out_ofs(j));
    };

    // ---- one site at time t: 20 reduction steps, then the epilogue (stored
    // when the site is valid).  Offsets are ordered by n_t, so steps 0..QA
    // are the last to read plane t - 1 (step QA also reads plane t).  After
    // step QA one workgroup barrier serves the whole t step: every wavefront
    // is then past plane t - 1, whose ring slot takes plane t + 2 (loaded
    // into registers during the previous t step, converted and stored now),
    // and the stores of plane t + 1 made at the previous step are visible
    // before the steps that read it.  Then the loads of plane t + 3 are
    // issued, to be stored at the next step.  Every load is issued on every
    // step, also past the end of a chunk (not needed, stored harmlessly):
    // with no branch around the loads their registers need no copies, which
    // would wait for them at once.
    static_assert(SPW == 1 && NB == 1, "one site per wavefront and t step");
    constexpr int QA = 6;  // offsets 0..26 (4 QA + 3) have n_t = -1
    static_assert(comp(4 * QA + 2, 3) == -1 && comp(4 * QA + 3, 3) == 0 && comp(4 * QA + 4, 3) == 0,
                  "reduction steps ordered by n_t");
    int tm = 0;  // t mod 3 (table of the current t)
    const bool want_nrm = a.nrm != nullptr;
    double nacc[NT];  // the lane's |out|^2 per column tile (its right-hand side 4 j + er4)
#pragma unroll
    for (int j = 0; j < NT; ++j) nacc[j] = 0.0;
    auto compute_site = [&](size_t site, int srp, size_t next, bool valid, int t) __attribute__((always_inline)) {
        f4 acc[2][NT];
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int j = 0; j < NT; ++j) acc[m][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
        const uint32_t(*kt)[64] = sm.ktab[tm];
        // B operands of a step: psi(x + n) for the step's four offsets, all
        // column tiles; read from LDS two steps ahead into three static
        // buffers (step mod 3), the padding word of every operand zeroed once
        constexpr int BD = 3;  // B buffers
        u4 Bb[BD][NT];
        u4 A0 = u4{0u, 0u, 0u, 0u}, A1 = u4{0u, 0u, 0u, 0u};
#pragma unroll
        for (int h = 0; h < BD; ++h)
#pragma unroll
            for (int j = 0; j < NT; ++j) Bb[h][j] = u4{0u, 0u, 0u, 0u};
        auto read_b = [&](uint32_t k, u4 (&B)[NT]) {
            const int li = (int)(k & 0xffffu) + srp;
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const uint2 u = sm.b01[li + 16 * j * RPP];
                B[j].x = u.x;
                B[j].y = u.y;
                B[j].z = sm.b2[li + 16 * j * RPP];
            }
        };
        // table words of steps q, q + 1, q + 2 (each step reads the one of q + 3)
        uint32_t kw[BD];
#pragma unroll
        for (int h = 0; h < BD; ++h) kw[h] = kt[h][lane];
        read_b(kw[0], Bb[0]);
        read_b(kw[1], Bb[1]);
#pragma unroll
        for (int q = 0; q < KSTEPS; ++q) {
            u4(&B)[NT] = Bb[q % BD];
            const uint32_t kq = kw[q % BD];
            if (q + 2 < KSTEPS) read_b(kw[(q + 2) % BD], Bb[(q + 2) % BD]);  // operands two steps ahead
            if (q + BD < KSTEPS) kw[q % BD] = kt[q + BD][lane];
            const h2 m1 = hv((kq >> 16) * 0x10001u);  // (c, c)
            const h2 m0 = h2{m1.x, -m1.y};
            const h2 w0 = hv(wa[q][0]), w1 = hv(wa[q][1]), w2 = hv(wa[q][2]);
            A0.x = bits(w0 * m0);  // (c Re W, -c Im W)
            A0.y = bits(w1 * m0);
            A0.z = bits(w2 * m0);
            A1.x = bits(w0.yx * m1);  // (c Im W, c Re W)
            A1.y = bits(w1.yx * m1);
            A1.z = bits(w2.yx * m1);
            load_rows(next, q);
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const h8 Bj = __builtin_bit_cast(h8, B[j]);
                acc[0][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, A0), Bj, acc[0][j], 0, 0, 0);
                acc[1][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(h8, A1), Bj, acc[1][j], 0, 0, 0);
            }
            if (q == QA) {
                // (the B reads issued so far beyond this step are of planes t, t + 1)
                __syncthreads();
                convert_batch(ic<0>{});
                store_planes(t + 2);
                load_batch(t + 3, ic<0>{});
            }
            __builtin_amdgcn_sched_barrier(0);  // keep the steps in order (bounded register use)
        }
        // epilogue per column tile: accumulator rows 4 (lane / 16) + e, column
        // lane % 16; row = 5 a + c, column = 4 r' + s
        float2(*scr)[16] = sm.scr[w];
        // chiral basis, (gamma_mu X)(s) = phase X(partner): gamma_x (-i, -i, i, i), gamma_y (-1, 1, 1, -1),
        // gamma_z (-i, i, i, -i), gamma_t (1, 1, 1, 1); as signs of i X (x, z) and of X (y), branch-free
        const int sxy = 3 - es, szt = es ^ 2;  // gamma_x, gamma_y pair s with 3 - s; gamma_z, gamma_t with s ^ 2
        const float sx = es < 2 ? -1.0f : 1.0f;
        const float syz = (es == 0 || es == 3) ? -1.0f : 1.0f;
        const int cb = 4 * er4;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
#pragma unroll
            for (int e = 0; e < 4; ++e) scr[4 * grp + e][row] = make_float2(acc[0][j][e], acc[1][j][e]);
            __builtin_amdgcn_wave_barrier();
            const int r = 4 * j + er4;
            if (valid && lane < 48 && r < nr) {
                const float2 X0 = scr[5 * ea + 0][cb + es];
                const float2 X1 = scr[5 * ea + 1][cb + sxy];
                const float2 X2 = scr[5 * ea + 2][cb + sxy];
                const float2 X3 = scr[5 * ea + 3][cb + szt];
                const float2 X4 = scr[5 * ea + 4][cb + szt];
                // i X = (-X.y, X.x)
                const float gre = -sx * X1.y + syz * X2.x - syz * X3.y + X4.x;
                const float gim = sx * X1.x + syz * X2.y + syz * X3.x + X4.y;
                const float is = sm.iscl[r];
                float2 o;
                o.x = fmaf(slam * X0.x + srho * gre, is, diag * px[j].x);
                o.y = fmaf(slam * X0.y + srho * gim, is, diag * px[j].y);
                // the 48 lanes of a column tile write 384 contiguous bytes of
                // the site record
                *(float2 *)(out + site * recb + out_ofs(j)) = o;
                if (want_nrm) nacc[j] = fma((double)o.y, (double)o.y, fma((double)o.x, (double)o.x, nacc[j]));
            }
            __builtin_amdgcn_wave_barrier();
        }
        load_px(next);
    };

    // ---- t walk; the wavefront's sites in order (site 0, t), (site 1, t), (site 0, t + 1), ...
    {
        const size_t first = site_of(0, t0);
#pragma unroll
        for (int q = 0; q < KSTEPS; ++q) load_rows(first, q);
        load_px(first);
    }
    __syncthreads();  // scales, tables
    ssc = sr < nr ? sm.scl[sr] : 0.0f;
    for (int k = 0; k < 3; ++k) {
        static_for<0, NB + 1>([&](auto B) __attribute__((always_inline)) { stage_step(t0 - 1 + k, B); });
        store_planes(t0 - 1 + k);
    }
    load_batch(t0 + 2, ic<0>{});  // stored during the first step
    __syncthreads();
    for (int t = t0; t < t1; ++t) {
        tm = t % 3;
        // next site of the chain (after the last t of the chunk: this site
        // again, so that every load is issued)
        const size_t next = site_of(0, t + 1 < t1 ? t + 1 : t);
        compute_site(site_of(0, t), srp0, next, nval > 0, t);
    }
    if (want_nrm) {
        // |out|^2 per right-hand side: over the 12 lanes of a (column tile,
        // rhs) pair (spin: lane bits 0-1, colour: bits 4-5; lanes 48-63 hold
        // zero), then over the wavefronts in order, in fixed order throughout
        double *ws = (double *)&sm.scr[w][0][0];  // this wavefront's epilogue tile, free now
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            double v = nacc[j];
            v += __shfl_xor(v, 1);
            v += __shfl_xor(v, 2);
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if ((lane & 0x33) == 0) ws[4 * j + er4] = v;
        }
        __syncthreads();
        if (tid < 4 * NT && tid < nr) {
            double sum = 0.0;
            for (int v = 0; v < NWAVE; ++v) sum += ((const double *)&sm.scr[v][0][0])[tid];
            const size_t nwg = gridDim.x / nrb;
            double *o = a.nrm + 2 * ((size_t)(r0 + tid) * nwg + iwg);
            o[0] = sum;
            o[1] = 0.0;
        }
    }
}

// ---------------------------------------------------------------- store
// one workgroup per 16 sites: the 80 x 9 entries are gathered through LDS
// (coalesced reads of the [offset][9][V] store, coalesced writes of the
// site-major rows)
template <typename WS>
__device__ __forceinline__ uint32_t to_h2(WS v, bool conj) {
    const float re = (float)v.x, im = (float)v.y;
    const h2 h = h2{(_Float16)re, (_Float16)(conj ? -im : im)};
    return __builtin_bit_cast(uint32_t, h);
}
template <>
__device__ __forceinline__ uint32_t to_h2<__half2>(__half2 v, bool conj) {
    const float2 f = __half22float2(v);
    const h2 h = h2{(_Float16)f.x, (_Float16)(conj ? -f.y : f.y)};
    return __builtin_bit_cast(uint32_t, h);
}

template <typename WS, int NOFF>
__global__ __launch_bounds__(256) void k_pack(Geom g, const WS *__restrict__ W, uint32_t *__restrict__ Wm) {
    constexpr int S = 16;
    __shared__ uint32_t buf[S * WSITE];
    const int V = g.V;
    const int s0 = blockIdx.x * S;
    const int ns = min(S, V - s0);
    for (int i = threadIdx.x; i < S * WSITE; i += blockDim.x) {
        const int s = i % S, pe = i / S;
        if (s >= ns) continue;
        const int p = pe / 9, e = pe % 9;
        const int x = s0 + s;
        uint32_t v;
        if (NOFF == 80) {
            v = to_h2(W[(size_t)pe * V + x], false);
        } else {
            const int i81 = p < 40 ? p : p + 1;
            if (i81 > 40) {
                v = to_h2(W[((size_t)(i81 - 41) * 9 + e) * V + x], false);
            } else {
                // W(x, x+n) = W(x+n, x)^dag, stored at x+n under offset -n
                int c[4], r = x;
                for (int mu = 0; mu < 4; ++mu) {
                    c[mu] = r % g.L[mu];
                    r /= g.L[mu];
                }
                int y = 0;
                for (int mu = 3; mu >= 0; --mu) y = y * g.L[mu] + wrap(c[mu] + comp(p, mu), g.L[mu]);
                const int a_ = e / 3, b_ = e % 3;
                v = to_h2(W[((size_t)(39 - i81) * 9 + 3 * b_ + a_) * V + y], true);
            }
        }
        buf[s * WSITE + pe] = v;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < ns * WSITE; i += blockDim.x) Wm[(size_t)s0 * WSITE + i] = buf[i];
}

// ---------------------------------------------------------------- site-major spinors
// SoA [nrhs][12][V] <-> site-major [V][nrhs][12] (FP32 complex), through LDS
// in blocks of 32 sites x 96 components (8 right-hand sides), so that both
// sides are read and written in contiguous pieces.  The forward direction
// can also give bound2 (as k_absmax2).
constexpr int TS = 32, TC = 96;
template <bool TO_SITES>
__global__ __launch_bounds__(256) void k_transpose(int V, int ncomp, const float2 *__restrict__ src,
                                                   float2 *__restrict__ dst, unsigned long long *__restrict__ bound2) {
    __shared__ float2 tile[TC][TS + 1];
    const int s0 = blockIdx.x * TS, c0 = blockIdx.y * TC;
    const int ns = min(TS, V - s0), nc = min(TC, ncomp - c0);
    for (int i = threadIdx.x; i < TC * TS; i += blockDim.x) {
        if (TO_SITES) {
            const int c = i / TS, s = i % TS;  // 32 consecutive sites of one plane
            if (c < nc && s < ns) tile[c][s] = src[(size_t)(c0 + c) * V + s0 + s];
        } else {
            const int s = i / TC, c = i % TC;  // consecutive components of one site
            if (c < nc && s < ns) tile[c][s] = src[(size_t)(s0 + s) * ncomp + c0 + c];
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < TC * TS; i += blockDim.x) {
        if (TO_SITES) {
            const int s = i / TC, c = i % TC;
            if (c < nc && s < ns) dst[(size_t)(s0 + s) * ncomp + c0 + c] = tile[c][s];
        } else {
            const int c = i / TS, s = i % TS;
            if (c < nc && s < ns) dst[(size_t)(c0 + c) * V + s0 + s] = tile[c][s];
        }
    }
    if (TO_SITES && bound2) {
        // thread (k, s): right-hand side c0 / 12 + k at site s0 + s; max over its 24 reals
        const int k = threadIdx.x / TS, s = threadIdx.x % TS;
        float m = 0.0f;
        if (12 * k < nc && s < ns)
            for (int c = 0; c < 12; ++c) m = fmaxf(m, fmaxf(fabsf(tile[12 * k + c][s].x), fabsf(tile[12 * k + c][s].y)));
        for (int o = 16; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));  // within the 32 lanes of k
        if (s == 0 && 12 * k < nc) {
            // the bound only grows: once it covers this block's value, as it
            // soon does on most blocks, no atomic is needed (a stale read
            // only costs a redundant one)
            const unsigned long long d = (unsigned long long)__double_as_longlong((double)m * (double)m);
            unsigned long long *b = bound2 + c0 / 12 + k;
            if (__hip_atomic_load(b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < d) atomicMax(b, d);
        }
    }
}

// ---------------------------------------------------------------- bounds
// bound2[r] = (max over the real components of psi_r of |v|)^2, by an
// unsigned maximum on the bits of the non-negative doubles (order-independent)
__global__ void k_zero_u64(unsigned long long *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}
__global__ __launch_bounds__(256) void k_absmax2(const float *__restrict__ in, size_t per_rhs,
                                                 unsigned long long *__restrict__ out) {
    const int r = blockIdx.y;
    const float *p = in + (size_t)r * per_rhs;
    float m = 0.0f;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < per_rhs; i += (size_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(p[i]));
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if ((threadIdx.x & 63) == 0) {
        const double d = (double)m * (double)m;
        atomicMax(out + r, (unsigned long long)__double_as_longlong(d));
    }
}

}  // namespace mfma

hipError_t pack_w_mfma(const Geom &g, const void *W, int wp, int noff, void *Wm, hipStream_t st) {
    const int blocks = (g.V + 15) / 16;
    uint32_t *o = (uint32_t *)Wm;
#define BRI_PACK(WS)                                                                                 \
    do {                                                                                             \
        if (noff == 80)                                                                              \
            hipLaunchKernelGGL((mfma::k_pack<WS, 80>), dim3(blocks), dim3(256), 0, st, g, (const WS *)W, o); \
        else                                                                                         \
            hipLaunchKernelGGL((mfma::k_pack<WS, 40>), dim3(blocks), dim3(256), 0, st, g, (const WS *)W, o); \
    } while (0)
    if (wp == 0)
        BRI_PACK(double2);
    else if (wp == 1)
        BRI_PACK(float2);
    else
        BRI_PACK(__half2);
#undef BRI_PACK
    return hipGetLastError();
}

hipError_t spinor_bound2(const Geom &g, int nrhs, const float2 *in, double *bound2, hipStream_t st) {
    unsigned long long *o = (unsigned long long *)bound2;
    hipLaunchKernelGGL(mfma::k_zero_u64, dim3((nrhs + 63) / 64), dim3(64), 0, st, o, nrhs);
    const size_t per = (size_t)g.V * 24;
    size_t bx = (per + 255) / 256;
    if (bx > 512) bx = 512;
    hipLaunchKernelGGL(mfma::k_absmax2, dim3((unsigned)bx, (unsigned)nrhs), dim3(256), 0, st, (const float *)in, per, o);
    return hipGetLastError();
}

hipError_t spinor_sites(const Geom &g, int nrhs, const float2 *src, float2 *dst, bool to_sites, double *bound2,
                        hipStream_t st) {
    const int ncomp = 12 * nrhs;
    const dim3 grid((g.V + mfma::TS - 1) / mfma::TS, (ncomp + mfma::TC - 1) / mfma::TC);
    unsigned long long *b = (unsigned long long *)bound2;
    if (to_sites && b) hipLaunchKernelGGL(mfma::k_zero_u64, dim3((nrhs + 63) / 64), dim3(64), 0, st, b, nrhs);
    if (to_sites)
        hipLaunchKernelGGL(mfma::k_transpose<true>, grid, dim3(256), 0, st, g.V, ncomp, src, dst, b);
    else
        hipLaunchKernelGGL(mfma::k_transpose<false>, grid, dim3(256), 0, st, g.V, ncomp, src, dst, nullptr);
    return hipGetLastError();
}

static int mfma_tlen(const Geom &g, int tlen) {
    return tlen > 0 ? (tlen < g.L[3] ? tlen : g.L[3]) : (g.L[3] < 64 ? g.L[3] : 64);
}

long long mfma_workgroups(const Geom &g, int tlen) {
    const int tl = mfma_tlen(g, tlen);
    return (long long)((g.L[0] + mfma::TX - 1) / mfma::TX) * ((g.L[1] + mfma::TY - 1) / mfma::TY) * g.L[2] *
           ((g.L[3] + tl - 1) / tl);
}

hipError_t apply_mfma(const Geom &g, const void *Wm, const float2 *in, float2 *out, int nrhs, double diag,
                      const double *table, bool dag, const double *bound2, int bstride, int tlen, hipStream_t st,
                      double *nrm) {
    mfma::Args a{};
    a.g = g;
    a.ntx = (g.L[0] + mfma::TX - 1) / mfma::TX;
    a.nty = (g.L[1] + mfma::TY - 1) / mfma::TY;
    a.tlen = mfma_tlen(g, tlen);
    a.ntc = (g.L[3] + a.tlen - 1) / a.tlen;
    a.nrhs = nrhs;
    // block groups of up to 2 x 4 x 4 tiles (32 workgroups, one per CU of an XCD)
    auto group = [](int n, int want) {
        while (want > 1 && n % want) want /= 2;
        return want;
    };
    a.gx = group(a.ntx, 2);
    a.gy = group(a.nty, 4);
    a.gz = group(g.L[2], 4);
    a.Wm = (const uint32_t *)Wm;
    a.in = in;
    a.out = out;
    a.bound2 = bound2;
    a.bstride = bstride;
    a.nrm = nrm;
    a.diag = (float)diag;
    double lam[5], rho[5], sl = 0.0, sr = 0.0;
    for (int k = 1; k <= 4; ++k) {
        lam[k] = table ? table[k] : lam_k(k);
        rho[k] = (table ? table[4 + k] : rho_k(k)) * (dag ? -1.0 : 1.0);
        sl = std::fmax(sl, std::fabs(lam[k]));
        sr = std::fmax(sr, std::fabs(rho[k]));
    }
    if (sl == 0.0) sl = 1.0;
    if (sr == 0.0) sr = 1.0;
    a.slam = (float)sl;
    a.srho = (float)sr;
    for (int k = 1; k <= 4; ++k) {
        a.lam[k] = (float)(lam[k] / sl);
        a.rho[k] = (float)(rho[k] / sr);
    }
    // the kernel adds 32-bit byte offsets within a t plane of the spinor fields
    if ((size_t)g.V / g.L[3] * (size_t)nrhs * 96 > 0xffffffffull) return hipErrorInvalidValue;
    const int nrb = (nrhs + 4 * mfma::NTB - 1) / (4 * mfma::NTB);
    const long long blocks = (long long)a.ntx * a.nty * g.L[2] * a.ntc * nrb;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(mfma::k_apply_mfma<mfma::NTB>, dim3((unsigned)blocks), dim3(mfma::NTHR), 0, st, a);
    return hipGetLastError();
}

}  // namespace bri

using namespace bri;

extern "C" {

bri_status bri_pack_w_mfma(bri_dims d, const void *W, bri_prec w_prec, int32_t n_offsets, void *W_mfma,
                           void *stream) {
    g_last_error.clear();
    Geom g;
    if (!dims_ok(d, &g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (!prec_ok(w_prec)) return fail(BRI_E_ARG, "invalid precision");
    if (n_offsets != 40 && n_offsets != 80) return fail(BRI_E_ARG, "n_offsets must be 40 or 80");
    if (!aligned(W) || !aligned(W_mfma)) return fail(BRI_E_ARG, "null or misaligned (16 B) pointer");
    const size_t wb = (size_t)g.V * 9 * n_offsets * cbytes(w_prec);
    if (overlap(W, wb, W_mfma, (size_t)g.V * BRI_MFMA_W_BYTES_PER_SITE)) return fail(BRI_E_ARG, "W and W_mfma overlap");
    return hip_check(pack_w_mfma(g, W, (int)w_prec, n_offsets, W_mfma, (hipStream_t)stream), "pack (matrix-core store)");
}

bri_status bri_spinor_bound2(bri_dims d, int32_t nrhs, const float *psi, double *bound2, void *stream) {
    g_last_error.clear();
    Geom g;
    if (!dims_ok(d, &g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (nrhs < 1 || nrhs > 65535) return fail(BRI_E_ARG, "nrhs must be in [1, 65535]");
    if (!aligned(psi) || !aligned(bound2)) return fail(BRI_E_ARG, "null or misaligned (16 B) pointer");
    return hip_check(spinor_bound2(g, nrhs, (const float2 *)psi, bound2, (hipStream_t)stream), "spinor bound");
}

bri_status bri_spinor_to_sites(bri_dims d, int32_t nrhs, const float *psi, float *psi_sites, double *bound2,
                               void *stream) {
    g_last_error.clear();
    Geom g;
    if (!dims_ok(d, &g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (nrhs < 1 || nrhs > 65535) return fail(BRI_E_ARG, "nrhs must be in [1, 65535]");
    if (!aligned(psi) || !aligned(psi_sites) || (bound2 && !aligned(bound2)))
        return fail(BRI_E_ARG, "null or misaligned (16 B) pointer");
    const size_t sb = (size_t)g.V * 12 * nrhs * 8;
    if (overlap(psi, sb, psi_sites, sb)) return fail(BRI_E_ARG, "psi and psi_sites overlap");
    return hip_check(spinor_sites(g, nrhs, (const float2 *)psi, (float2 *)psi_sites, true, bound2, (hipStream_t)stream),
                     "spinor to site-major");
}

bri_status bri_spinor_from_sites(bri_dims d, int32_t nrhs, const float *psi_sites, float *psi, void *stream) {
    g_last_error.clear();
    Geom g;
    if (!dims_ok(d, &g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (nrhs < 1 || nrhs > 65535) return fail(BRI_E_ARG, "nrhs must be in [1, 65535]");
    if (!aligned(psi) || !aligned(psi_sites)) return fail(BRI_E_ARG, "null or misaligned (16 B) pointer");
    const size_t sb = (size_t)g.V * 12 * nrhs * 8;
    if (overlap(psi, sb, psi_sites, sb)) return fail(BRI_E_ARG, "psi and psi_sites overlap");
    return hip_check(spinor_sites(g, nrhs, (const float2 *)psi_sites, (float2 *)psi, false, nullptr, (hipStream_t)stream),
                     "spinor from site-major");
}

bri_status bri_apply_mfma(bri_dims d, const void *W_mfma, double mass, const float *in, float *out, int32_t nrhs,
                          int32_t dagger, const double *coef, const double *bound2, void *stream) {
    g_last_error.clear();
    Geom g;
    if (!dims_ok(d, &g)) return fail(BRI_E_ARG, "invalid lattice extents");
    if (nrhs < 1 || nrhs > 65535) return fail(BRI_E_ARG, "nrhs must be in [1, 65535]");
    if (dagger != 0 && dagger != 1) return fail(BRI_E_ARG, "dagger must be 0 or 1");
    if (!aligned(W_mfma) || !aligned(in) || !aligned(out) || !aligned(bound2))
        return fail(BRI_E_ARG, "null or misaligned (16 B) pointer");
    const size_t sb = (size_t)g.V * 12 * nrhs * 8;
    if (overlap(in, sb, out, sb)) return fail(BRI_E_ARG, "in and out overlap");
    if (sb / g.L[3] > 0xffffffffull) return fail(BRI_E_UNSUPPORTED, "a t plane of the spinor field exceeds 4 GiB");
    const double diag = (coef ? coef[0] : lam_k(0)) + mass;
    return hip_check(apply_mfma(g, W_mfma, (const float2 *)in, (float2 *)out, nrhs, diag, coef, dagger != 0, bound2, 1,
                                0, (hipStream_t)stream),
                     "apply (matrix cores)");
}

}  // extern "C"
