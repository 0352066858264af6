// lbm_core.hip -- gfx950 kernels of the binary-fluid lattice Boltzmann update
// (arXiv:1702.04487, Methods Eqs. 3-10; actuation of Fig. 1; wetting walls and
// "fully developed" rows of Results, "Reproducing the experiment").
//
// Storage: one buffer = 14 float planes of ny rows x pitch columns (pitch a
// multiple of 64) plus one 16-bit plane:
//   planes 0..8   f_i - w_i n0 (D2Q9 distributions shifted by their rest
//                 value, which keeps the low-order bits of the small velocity
//                 signal in FP32);
//   planes 9..13  g_0..g_4 (D2Q5);
//   16-bit plane  bfloat16 of g_0 - float(g_0): g_0 carries +-phi* and is the
//                 only population whose FP32 rounding would quantise phi.
// Two buffers A (current, pre-collision) and B (next) alternate.
//
// Velocities c_0=(0,0) c_1=(1,0) c_2=(0,1) c_3=(-1,0) c_4=(0,-1)
// c_5=(1,1) c_6=(-1,1) c_7=(-1,-1) c_8=(1,-1); D2Q5 = c_0..c_4.
// Wall mask bytes: 0 fluid, 1 inner wall, 2 outer wall; inside the kernels 3
// marks a row beyond an open lattice edge.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm_core.h"

namespace ij {

// ---------------------------------------------------------------- device math

__device__ __forceinline__ float bf16_to_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// round-to-nearest-even to bfloat16 (finite inputs)
__device__ __forceinline__ uint16_t float_to_bf16(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// phi = sum_i g_i (Eq. 9's zeroth moment) in double from the five stored
// populations and the low-order part of g_0
__device__ __forceinline__ double phi_of(float g0, float g1, float g2, float g3, float g4, float lo)
{
    return ((((double)g1 + (double)g2) + ((double)g3 + (double)g4)) + (double)lo) + (double)g0;
}

// Wetting ghost of a solid node (Results, contact-angle wall; Cahn wetting):
// mean of phi over its fluid axis neighbours (E, N, W, S order), or over its
// fluid diagonal neighbours (NE, NW, SW, SE) when it has none on the axes,
// plus the offset 2 Omega phi*/W of its wall class.
// v[k], m[k]: raw phi and mask of the neighbour in direction k+1 (1..8).
__device__ __forceinline__ double ghost_value(const double (&v)[8], const uint8_t (&m)[8], double wet)
{
    double sum = 0.0;
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (m[k] == 0) { sum += v[k]; ++cnt; }
    if (cnt == 0) {
#pragma unroll
        for (int k = 4; k < 8; ++k)
            if (m[k] == 0) { sum += v[k]; ++cnt; }
    }
    return cnt ? sum / (double)cnt + wet : 0.0;
}

struct Macro {
    float n, dn, ux, uy, jx, jy;  // dn = n - n0 = sum of the shifted f
    double phi, mu;
};

// Macroscopic quantities of a fluid node from its distributions and the phi
// stencil st[k] = phi~(x + c_k) (phi at fluid nodes, wetting ghost at solids):
//  - n = sum f (the mean density of Eq. 1), phi = st[0] (Eq. 7);
//  - isotropic nine-point gradient and Laplacian (from neighbour
//    differences, so no O(phi) terms cancel);
//  - mu = 4 beta phi (phi^2 - phi*^2) - kappa lap(phi) (phi^4 free energy);
//  - F = mu grad(phi) + F_b (Eq. 4) and n u = sum c f + F/2.
__device__ __forceinline__ void node_macro(const KParams& P, const float (&f)[9], const double (&st)[9],
                                           float fb, Macro& m, double& Fx, double& Fy)
{
    const double phi = st[0];
    const double gx = (st[1] - st[3]) * (1.0 / 3.0) + ((st[5] - st[7]) + (st[8] - st[6])) * (1.0 / 12.0);
    const double gy = (st[2] - st[4]) * (1.0 / 3.0) + ((st[5] - st[7]) + (st[6] - st[8])) * (1.0 / 12.0);
    const double lap = ((((st[1] - phi) + (st[3] - phi)) + ((st[2] - phi) + (st[4] - phi))) * 4.0 +
                        (((st[5] - phi) + (st[7] - phi)) + ((st[6] - phi) + (st[8] - phi)))) * (1.0 / 6.0);
    const double mu = P.beta4 * phi * ((phi - P.phi_star) * (phi + P.phi_star)) - P.kappa * lap;
    Fx = mu * gx;
    Fy = mu * gy + (double)fb;
    const float dn = (((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7]))) + f[8];
    const float n = P.n0 + dn;
    const float jx = (f[1] - f[3]) + ((f[5] - f[6]) + (f[8] - f[7]));
    const float jy = (f[2] - f[4]) + ((f[5] - f[8]) + (f[6] - f[7]));
    const float inv_n = 1.f / n;
    m.n = n;
    m.dn = dn;
    m.phi = phi;
    m.jx = jx;
    m.jy = jy;
    m.mu = mu;
    // j and -F/2 nearly cancel at a resting interface: add them in double
    m.ux = (float)((double)jx + 0.5 * Fx) * inv_n;
    m.uy = (float)((double)jy + 0.5 * Fy) * inv_n;
}

// Collision of one fluid node: f* (BGK + the Guo source of Eq. 4, equilibrium
// of Eqs. 5-6; f shifted by w_i n0) and h = g* - (1-q) g with g* the BGK
// relaxation of Eq. 8 towards the equilibrium of Eqs. 9-10 (rest index 0
// carries B = 1, A = -2 Gamma mu).  The rest population of g does not move:
// its new value h_0 + (1-q) g_0 = g_0 + (g_eq_0 - g_0)/tau_phi is returned
// as the pair (g0_hi, g0_lo), with g_eq_0 - g_0 = (g_1+..+g_4) - 2 Gamma mu.
__device__ __forceinline__ void node_collide(const KParams& P, const float (&f)[9], const float (&g)[5],
                                             float lo, const double (&st)[9], float fb, float (&fs)[9],
                                             float (&h)[5], float& g0_hi, uint16_t& g0_lo, Macro& m)
{
    double Fxd, Fyd;
    node_macro(P, f, st, fb, m, Fxd, Fyd);
    const float Fx = (float)Fxd, Fy = (float)Fyd;
    const float ux = m.ux, uy = m.uy, n = m.n, dn = m.dn;
    const float phi = (float)m.phi, mu = (float)m.mu;

    // per-phase relaxation: tau = tau_amb + C (tau_ink - tau_amb)
    const float C = fminf(fmaxf(0.5f * (phi * P.inv_phi_star + 1.f), 0.f), 1.f);
    const float om = 1.f / (P.tau_amb + C * P.dtau);
    const float pref = 1.f - 0.5f * om;
    const float keep = 1.f - om;

    const float phimu = (float)(m.phi * m.mu);
    const float uu15 = 1.5f * (ux * ux + uy * uy);
    const float uF3 = 3.f * (ux * Fx + uy * Fy);
    const float a0 = dn - 3.75f * phimu; // A_0 - n0
    const float ai = dn + 3.f * phimu;   // A_i - n0, i >= 1

    {
        const float feq = (4.f / 9.f) * (a0 - n * uu15);
        const float S = pref * (4.f / 9.f) * (-uF3);
        fs[0] = keep * f[0] + om * feq + S;
    }
#define IJ_DIR(i, w, cu_, cF_)                                                        \
    {                                                                                 \
        const float cu = (cu_), cF = (cF_);                                          \
        const float feq = (w) * (ai + n * (3.f * cu - uu15 + 4.5f * cu * cu));       \
        const float S = pref * (w) * (3.f * cF - uF3 + 9.f * cu * cF);               \
        fs[i] = keep * f[i] + om * feq + S;                                          \
    }
    IJ_DIR(1, 1.f / 9.f, ux, Fx)
    IJ_DIR(2, 1.f / 9.f, uy, Fy)
    IJ_DIR(3, 1.f / 9.f, -ux, -Fx)
    IJ_DIR(4, 1.f / 9.f, -uy, -Fy)
    IJ_DIR(5, 1.f / 36.f, ux + uy, Fx + Fy)
    IJ_DIR(6, 1.f / 36.f, uy - ux, Fy - Fx)
    IJ_DIR(7, 1.f / 36.f, -(ux + uy), -(Fx + Fy))
    IJ_DIR(8, 1.f / 36.f, ux - uy, Fx - Fy)
#undef IJ_DIR

    // order parameter: h_i = g_i (1 - 1/tau_phi - (1-q)) + g_eq_i / tau_phi
    const float gmu = P.gamma_f * mu;
    const float keepg = 1.f - P.omega_phi_f - P.omq;
    const float cphi = P.c_half_q * phi;
    h[0] = 0.f;
    h[1] = keepg * g[1] + P.omega_phi_f * (0.5f * gmu + cphi * ux);
    h[2] = keepg * g[2] + P.omega_phi_f * (0.5f * gmu + cphi * uy);
    h[3] = keepg * g[3] + P.omega_phi_f * (0.5f * gmu - cphi * ux);
    h[4] = keepg * g[4] + P.omega_phi_f * (0.5f * gmu - cphi * uy);
    const double d0 = P.omega_phi * ((((double)g[1] + (double)g[2]) + ((double)g[3] + (double)g[4])) -
                                     2.0 * P.gamma * m.mu);
    const double G = ((double)g[0] + (double)lo) + d0;
    g0_hi = (float)G;
    g0_lo = float_to_bf16((float)(G - (double)g0_hi));
}

// Equilibria at rest density n0 (initial state): shifted f_eq; g_eq with the
// rest population as a (hi, lo) pair.
__device__ __forceinline__ void node_equilibrium(const KParams& P, double phi, double mu, float ux, float uy,
                                                 float (&fe)[9], float (&ge)[5], uint16_t& g0_lo)
{
    const float n = P.n0;
    const float phimu = (float)(phi * mu);
    const float uu15 = 1.5f * (ux * ux + uy * uy);
    const float a0 = -3.75f * phimu;
    const float ai = 3.f * phimu;
    fe[0] = (4.f / 9.f) * (a0 - n * uu15);
#define IJ_EQ(i, w, cu_)                                                          \
    {                                                                             \
        const float cu = (cu_);                                                  \
        fe[i] = (w) * (ai + n * (3.f * cu - uu15 + 4.5f * cu * cu));             \
    }
    IJ_EQ(1, 1.f / 9.f, ux)
    IJ_EQ(2, 1.f / 9.f, uy)
    IJ_EQ(3, 1.f / 9.f, -ux)
    IJ_EQ(4, 1.f / 9.f, -uy)
    IJ_EQ(5, 1.f / 36.f, ux + uy)
    IJ_EQ(6, 1.f / 36.f, uy - ux)
    IJ_EQ(7, 1.f / 36.f, -(ux + uy))
    IJ_EQ(8, 1.f / 36.f, ux - uy)
#undef IJ_EQ
    const float gmu = P.gamma_f * (float)mu;
    const float cphi = P.c_half_q * (float)phi;
    const double G0 = phi - 2.0 * P.gamma * mu;
    ge[0] = (float)G0;
    g0_lo = float_to_bf16((float)(G0 - (double)ge[0]));
    ge[1] = 0.5f * gmu + cphi * ux;
    ge[2] = 0.5f * gmu + cphi * uy;
    ge[3] = 0.5f * gmu - cphi * ux;
    ge[4] = 0.5f * gmu - cphi * uy;
}

__device__ __forceinline__ int wrapx(int x, int nx) { return x < 0 ? x + nx : (x >= nx ? x - nx : x); }

// Row index seen by a stencil: periodic wrap, or the mirror rule at an open edge.
__device__ __forceinline__ int stencil_row(int y, const KParams& P)
{
    if (y < 0) return P.bc_open ? 0 : y + P.ny;
    if (y >= P.ny) return P.bc_open ? P.ny - 1 : y - P.ny;
    return y;
}

// Mask of (x, y) with x wrapped; rows beyond an open edge are "outside" (3).
__device__ __forceinline__ uint8_t mask_at(const KParams& P, const uint8_t* wall, int x, int y)
{
    x = wrapx(x, P.nx);
    if (y < 0 || y >= P.ny) {
        if (P.bc_open) return 3;
        y = y < 0 ? y + P.ny : y - P.ny;
    }
    return wall[(unsigned)y * P.pitch + x];
}

__device__ __forceinline__ const uint16_t* lo_plane(const float* A, const KParams& P)
{
    return reinterpret_cast<const uint16_t*>(A + (size_t)kFloatPlanes * P.plane);
}
__device__ __forceinline__ uint16_t* lo_plane(float* A, const KParams& P)
{
    return reinterpret_cast<uint16_t*>(A + (size_t)kFloatPlanes * P.plane);
}

// Direction table of the streaming step.
template <int I> struct Dir;
template <> struct Dir<1> { static constexpr int dx = 1, dy = 0, opp = 3; };
template <> struct Dir<2> { static constexpr int dx = 0, dy = 1, opp = 4; };
template <> struct Dir<3> { static constexpr int dx = -1, dy = 0, opp = 1; };
template <> struct Dir<4> { static constexpr int dx = 0, dy = -1, opp = 2; };
template <> struct Dir<5> { static constexpr int dx = 1, dy = 1, opp = 7; };
template <> struct Dir<6> { static constexpr int dx = -1, dy = 1, opp = 8; };
template <> struct Dir<7> { static constexpr int dx = -1, dy = -1, opp = 5; };
template <> struct Dir<8> { static constexpr int dx = 1, dy = -1, opp = 6; };

struct StreamCtx {
    const KParams* P;
    float* B;
    int x, y;
    unsigned own;  // y * pitch + x
};

// Stream one post-collision population of node (x, y): to x + c_I, or back
// into the node itself as the opposite population when x + c_I is solid
// (halfway bounce-back); dropped when x + c_I lies beyond an open row.  For g
// (IS_G) the value written is h + (1-q) g_old with g_old the pre-collision
// value of the slot written (Eq. 8 reads g_i(x + c_i, t) at the
// destination); the caller passes both candidates.  When the slot written is
// an unknown incoming population of the row next to an open row, the same
// value also goes to the open row ("fully developed": its unknown
// populations equal those of the row inside it).
// dest_mask() is the wall mask at x + c_I; open_fluid(top, dx) tells whether
// the open row (bottom: 0, top: 1) is fluid at column x + dx.
template <int I, bool IS_G, typename MaskFn, typename OpenFn>
__device__ __forceinline__ void stream_one(const StreamCtx& c, float hv, float g_dest, float g_self,
                                           MaskFn dest_mask, OpenFn open_fluid)
{
    constexpr int DX = Dir<I>::dx, DY = Dir<I>::dy, OPP = Dir<I>::opp;
    const KParams& P = *c.P;
    int ty = c.y + DY;
    if (DY != 0 && (ty < 0 || ty >= P.ny)) {
        if (P.bc_open) return;
        ty = ty < 0 ? ty + P.ny : ty - P.ny;
    }
    const int tx = wrapx(c.x + DX, P.nx);
    const bool fl = dest_mask() == 0;
    const int d = fl ? I : OPP;
    const int wx = fl ? tx : c.x, wy = fl ? ty : c.y;
    const unsigned woff = fl ? ((unsigned)ty * P.pitch + tx) : c.own;
    const float v = IS_G ? hv + P.omq * (fl ? g_dest : g_self) : hv;
    const int pl = IS_G ? 9 + d : d;
    c.B[(size_t)pl * P.plane + woff] = v;
    if (P.bc_open) {
        const int cyd = fl ? DY : -DY;
        if (cyd > 0 && wy == 1 && open_fluid(0, fl ? DX : 0))
            c.B[(size_t)pl * P.plane + wx] = v;
        if (cyd < 0 && wy == P.ny - 2 && open_fluid(1, fl ? DX : 0))
            c.B[(size_t)pl * P.plane + (unsigned)(P.ny - 1) * P.pitch + wx] = v;
    }
}

// ------------------------------------------------------ reference path kernels

// raw phi at fluid nodes into the phi field (solid entries untouched)
__global__ void k_phi_from_g(KParams P, const float* __restrict__ A, const uint8_t* __restrict__ wall,
                             double* __restrict__ phi)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= P.nx) return;
    const unsigned k = (unsigned)y * P.pitch + x;
    if (wall[k]) return;
    const float* g = A + (size_t)9 * P.plane;
    phi[k] = phi_of(g[k], g[(size_t)P.plane + k], g[2 * (size_t)P.plane + k], g[3 * (size_t)P.plane + k],
                    g[4 * (size_t)P.plane + k], bf16_to_float(lo_plane(A, P)[k]));
}

// wetting ghosts on the list of solid nodes that touch fluid
__global__ void k_ghost(KParams P, const int2* __restrict__ list, int n, const uint8_t* __restrict__ wall,
                        double* __restrict__ phi)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int x = list[i].x, y = list[i].y;
    const int dx[8] = {1, 0, -1, 0, 1, -1, -1, 1};
    const int dy[8] = {0, 1, 0, -1, 1, 1, -1, -1};
    double v[8];
    uint8_t m[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        m[k] = mask_at(P, wall, x + dx[k], y + dy[k]);
        v[k] = 0.0;
        if (m[k] == 0) {
            const int xx = wrapx(x + dx[k], P.nx);
            int yy = y + dy[k];
            yy = yy < 0 ? yy + P.ny : (yy >= P.ny ? yy - P.ny : yy);
            v[k] = phi[(unsigned)yy * P.pitch + xx];
        }
    }
    const unsigned k0 = (unsigned)y * P.pitch + x;
    phi[k0] = ghost_value(v, m, P.wet[wall[k0]]);
}

__device__ __forceinline__ void load_stencil(const KParams& P, const double* __restrict__ phi, int x, int y,
                                             double (&st)[9])
{
    const int xe = wrapx(x + 1, P.nx), xw = wrapx(x - 1, P.nx);
    const int yn = stencil_row(y + 1, P), ys = stencil_row(y - 1, P);
    const unsigned r0 = (unsigned)y * P.pitch, rn = (unsigned)yn * P.pitch, rs = (unsigned)ys * P.pitch;
    st[0] = phi[r0 + x];
    st[1] = phi[r0 + xe];
    st[2] = phi[rn + x];
    st[3] = phi[r0 + xw];
    st[4] = phi[rs + x];
    st[5] = phi[rn + xe];
    st[6] = phi[rn + xw];
    st[7] = phi[rs + xw];
    st[8] = phi[rs + xe];
}

// Reference collide-stream: one node per thread, phi~ from the phi field,
// masks and the destination's pre-collision g read from memory.
__global__ void k_collide_ref(KParams P, const float* __restrict__ A, float* __restrict__ B,
                              const uint8_t* __restrict__ wall, const double* __restrict__ phi)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= P.nx) return;
    const unsigned k = (unsigned)y * P.pitch + x;
    if (wall[k]) return;
    float f[9], g[5], fs[9], h[5];
    double st[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = A[(size_t)i * P.plane + k];
#pragma unroll
    for (int i = 0; i < 5; ++i) g[i] = A[(size_t)(9 + i) * P.plane + k];
    const float lo = bf16_to_float(lo_plane(A, P)[k]);
    load_stencil(P, phi, x, y, st);
    Macro m;
    float g0h;
    uint16_t g0l;
    node_collide(P, f, g, lo, st, y < P.force_rows ? P.fb : 0.f, fs, h, g0h, g0l, m);

    B[k] = fs[0];
    B[(size_t)9 * P.plane + k] = g0h;
    lo_plane(B, P)[k] = g0l;
    const StreamCtx c{&P, B, x, y, k};
    auto open_fluid = [&](int top, int dx) {
        const int cx = wrapx(x + dx, P.nx);
        return wall[top ? (unsigned)(P.ny - 1) * P.pitch + cx : (unsigned)cx] == 0;
    };
    // pre-collision g at (x + dx, y + dy), wrapped (only read when that node is fluid)
    auto gold = [&](int i, int dx, int dy) -> float {
        if (P.bc_open && (y + dy < 0 || y + dy >= P.ny)) return 0.f;
        int ty = y + dy;
        ty = ty < 0 ? ty + P.ny : (ty >= P.ny ? ty - P.ny : ty);
        return A[(size_t)(9 + i) * P.plane + (unsigned)ty * P.pitch + wrapx(x + dx, P.nx)];
    };
#define IJ_MASK(DX, DY) [&]() { return mask_at(P, wall, x + (DX), y + (DY)); }
    stream_one<1, false>(c, fs[1], 0.f, 0.f, IJ_MASK(1, 0), open_fluid);
    stream_one<2, false>(c, fs[2], 0.f, 0.f, IJ_MASK(0, 1), open_fluid);
    stream_one<3, false>(c, fs[3], 0.f, 0.f, IJ_MASK(-1, 0), open_fluid);
    stream_one<4, false>(c, fs[4], 0.f, 0.f, IJ_MASK(0, -1), open_fluid);
    stream_one<5, false>(c, fs[5], 0.f, 0.f, IJ_MASK(1, 1), open_fluid);
    stream_one<6, false>(c, fs[6], 0.f, 0.f, IJ_MASK(-1, 1), open_fluid);
    stream_one<7, false>(c, fs[7], 0.f, 0.f, IJ_MASK(-1, -1), open_fluid);
    stream_one<8, false>(c, fs[8], 0.f, 0.f, IJ_MASK(1, -1), open_fluid);
    stream_one<1, true>(c, h[1], gold(1, 1, 0), g[3], IJ_MASK(1, 0), open_fluid);
    stream_one<2, true>(c, h[2], gold(2, 0, 1), g[4], IJ_MASK(0, 1), open_fluid);
    stream_one<3, true>(c, h[3], gold(3, -1, 0), g[1], IJ_MASK(-1, 0), open_fluid);
    stream_one<4, true>(c, h[4], gold(4, 0, -1), g[2], IJ_MASK(0, -1), open_fluid);
#undef IJ_MASK
}

// ----------------------------------------------------- fused collide-stream
//
// One workgroup owns a strip of BW = 64*NW columns and a block of rows and
// marches up the rows.  Per row it (1) forms raw phi of row r+2 (from g and
// the g_0 remainder, loaded one iteration ahead) in an LDS ring with two
// halo columns each side, (2) turns row r+1 into phi~ (wetting ghosts at
// solid nodes), (3) collides row r (its distributions also loaded one
// iteration ahead) with the nine-point stencil from LDS and streams it.  phi
// never goes through HBM: per fluid node the kernel reads the 14
// distributions and the 16-bit g_0 remainder once and writes them once.  The
// pre-collision g of the destination (the (1-q) term of Eq. 8) comes from
// the row registers or the LDS ring, never from memory.
template <int NW>
__global__ __launch_bounds__(64 * NW) void k_collide_fused(KParams P, const float* __restrict__ A,
                                                           float* __restrict__ B,
                                                           const uint8_t* __restrict__ wall,
                                                           int rows_per_block, int n_strips,
                                                           int n_rowblocks)
{
    constexpr int BW = 64 * NW;
    constexpr int RING = 8;
    __shared__ double s_raw[RING][BW + 4];
    __shared__ uint8_t s_m[RING][BW + 4];
    __shared__ float s_g1[RING][BW + 4];  // g_1 and g_3 of each raw row: the
    __shared__ float s_g3[RING][BW + 4];  // (1-q) terms of the x-neighbours
    __shared__ double s_pt[4][BW + 2];

    // consecutive tiles of a strip are vertical neighbours; keep runs of them
    // on one XCD (workgroups are dealt round-robin over the 8 XCDs)
    const int ntiles = n_strips * n_rowblocks;
    int tile = blockIdx.x;
    if ((ntiles & 7) == 0) tile = (blockIdx.x & 7) * (ntiles >> 3) + (blockIdx.x >> 3);
    const int strip = tile / n_rowblocks;
    const int rb = tile - strip * n_rowblocks;
    const int x0 = strip * BW;
    const int wv = min(BW, P.nx - x0);
    const int y0 = rb * rows_per_block;
    const int y1 = min(P.ny, y0 + rows_per_block);
    const int t = threadIdx.x;
    const bool active = t < wv;
    const int x = x0 + t;
    const int hx = t < 2 ? x0 - 2 + t : x0 + wv + (t - 2);   // halo column of threads 0..3
    const int hidx = t < 2 ? t : wv + 2 + (t - 2);
    const int hxw = wrapx(hx, P.nx);

    const float* Ag = A + (size_t)9 * P.plane;
    const uint16_t* Alo = lo_plane(A, P);

    // raw-row registers: row rr (newest), rr-1, rr-2 (= collide row)
    float g2[5], g1[5], gc[5], lo2 = 0.f, lo1 = 0.f, loc = 0.f, g4prev = 0.f;
    uint8_t m2 = 3, m1 = 3;
#pragma unroll
    for (int i = 0; i < 5; ++i) { g2[i] = 0.f; g1[i] = 0.f; gc[i] = 0.f; }
    // loads issued one iteration ahead
    float pg[5], plo = 0.f, hg[5], hlo = 0.f, pf[9];
    uint8_t pm = 3, hm = 3;
#pragma unroll
    for (int i = 0; i < 9; ++i) pf[i] = 0.f;

    auto fetch_raw = [&](int rr) {
        int ry = rr;
        bool on = true;
        if (ry < 0 || ry >= P.ny) {
            if (P.bc_open) on = false;
            else ry = ry < 0 ? ry + P.ny : ry - P.ny;
        }
        pm = 3;
#pragma unroll
        for (int i = 0; i < 5; ++i) pg[i] = 0.f;
        plo = 0.f;
        if (on && active) {
            const unsigned k = (unsigned)ry * P.pitch + x;
            pm = wall[k];
            if (pm == 0) {
#pragma unroll
                for (int i = 0; i < 5; ++i) pg[i] = Ag[(size_t)i * P.plane + k];
                plo = bf16_to_float(Alo[k]);
            }
        }
        hm = 3;
#pragma unroll
        for (int i = 0; i < 5; ++i) hg[i] = 0.f;
        hlo = 0.f;
        if (on && t < 4) {
            const unsigned k = (unsigned)ry * P.pitch + hxw;
            hm = wall[k];
            if (hm == 0) {
#pragma unroll
                for (int i = 0; i < 5; ++i) hg[i] = Ag[(size_t)i * P.plane + k];
                hlo = bf16_to_float(Alo[k]);
            }
        }
    };

    const int nk = (y1 - y0) + 4;
    fetch_raw(y0 - 2);
    for (int kk = 0; kk < nk; ++kk) {
        const int rr = y0 - 2 + kk;
        const int rc = rr - 2;
        const int slot = rr & (RING - 1);
        g4prev = gc[4];
#pragma unroll
        for (int i = 0; i < 5; ++i) { gc[i] = g1[i]; g1[i] = g2[i]; g2[i] = pg[i]; }
        loc = lo1;
        lo1 = lo2;
        lo2 = plo;
        const uint8_t mc = m1;  // mask of the collide row rc
        m1 = m2;
        m2 = pm;
        const float hg1 = hg[1], hg3 = hg[3];
        const double hraw = hm == 0 ? phi_of(hg[0], hg[1], hg[2], hg[3], hg[4], hlo) : 0.0;
        const uint8_t hmm = hm;
        float fc[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) fc[i] = pf[i];
        // issue the next iteration's loads before working on this one: the
        // raw row rr+1 and the distributions of the next collide row rc+1,
        // whose mask m1 is already known
        if (kk + 1 < nk) {
            fetch_raw(rr + 1);
            if (rc + 1 >= y0 && rc + 1 < y1 && active && m1 == 0) {
                const unsigned k = (unsigned)(rc + 1) * P.pitch + x;
#pragma unroll
                for (int i = 0; i < 9; ++i) pf[i] = A[(size_t)i * P.plane + k];
            }
        }

        // (1) raw phi and mask of row rr
        if (active) {
            s_raw[slot][t + 2] = m2 == 0 ? phi_of(g2[0], g2[1], g2[2], g2[3], g2[4], lo2) : 0.0;
            s_m[slot][t + 2] = m2;
            s_g1[slot][t + 2] = g2[1];
            s_g3[slot][t + 2] = g2[3];
        }
        if (t < 4) {
            s_raw[slot][hidx] = hraw;
            s_m[slot][hidx] = hmm;
            s_g1[slot][hidx] = hg1;
            s_g3[slot][hidx] = hg3;
        }
        __syncthreads();

        // (2) phi~ of row rr-1
        if (kk >= 1) {
            const int rg = rr - 1;
            const int sc = rg & (RING - 1), sn = (rg + 1) & (RING - 1), ss = (rg - 1) & (RING - 1);
            auto phit = [&](int j) -> double {
                const uint8_t m0 = s_m[sc][j];
                if (m0 == 0) return s_raw[sc][j];
                if (m0 == 3) return 0.0;
                double v[8];
                uint8_t mm[8];
                mm[0] = s_m[sc][j + 1]; v[0] = s_raw[sc][j + 1];
                mm[1] = s_m[sn][j];     v[1] = s_raw[sn][j];
                mm[2] = s_m[sc][j - 1]; v[2] = s_raw[sc][j - 1];
                mm[3] = s_m[ss][j];     v[3] = s_raw[ss][j];
                mm[4] = s_m[sn][j + 1]; v[4] = s_raw[sn][j + 1];
                mm[5] = s_m[sn][j - 1]; v[5] = s_raw[sn][j - 1];
                mm[6] = s_m[ss][j - 1]; v[6] = s_raw[ss][j - 1];
                mm[7] = s_m[ss][j + 1]; v[7] = s_raw[ss][j + 1];
                return ghost_value(v, mm, P.wet[m0]);
            };
            if (active) s_pt[rg & 3][t + 1] = phit(t + 2);
            if (t < 2) {
                const int j = t == 0 ? 1 : wv + 2;
                s_pt[rg & 3][t == 0 ? 0 : wv + 1] = phit(j);
            }
        }
        __syncthreads();

        // (3) collide and stream row rr-2
        if (kk >= 2 && rc >= y0 && active && mc == 0) {
            const int rn = (P.bc_open && rc == P.ny - 1) ? rc : rc + 1;
            const int rs = (P.bc_open && rc == 0) ? rc : rc - 1;
            const int pc = rc & 3, pn = rn & 3, ps = rs & 3;
            const int j = t + 1;
            double st[9];
            st[0] = s_pt[pc][j];
            st[1] = s_pt[pc][j + 1];
            st[2] = s_pt[pn][j];
            st[3] = s_pt[pc][j - 1];
            st[4] = s_pt[ps][j];
            st[5] = s_pt[pn][j + 1];
            st[6] = s_pt[pn][j - 1];
            st[7] = s_pt[ps][j - 1];
            st[8] = s_pt[ps][j + 1];
            float fs[9], h[5], g0h;
            uint16_t g0l;
            Macro mac;
            node_collide(P, fc, gc, loc, st, rc < P.force_rows ? P.fb : 0.f, fs, h, g0h, g0l, mac);

            const unsigned own = (unsigned)rc * P.pitch + x;
            B[own] = fs[0];
            B[(size_t)9 * P.plane + own] = g0h;
            lo_plane(B, P)[own] = g0l;
            const StreamCtx c{&P, B, x, rc, own};
            const int jm = t + 2;
            const int sc = rc & (RING - 1), sn = (rc + 1) & (RING - 1), ss = (rc - 1) & (RING - 1);
            // rows 0 and ny-1 are in the ring whenever a copy into them occurs
            auto open_fluid = [&](int top, int dx) {
                const int row = top ? P.ny - 1 : 0;
                return s_m[row & (RING - 1)][jm + dx] == 0;
            };
#define IJ_M(SLOT, DXX) [&]() { return s_m[SLOT][jm + (DXX)]; }
            stream_one<1, false>(c, fs[1], 0.f, 0.f, IJ_M(sc, 1), open_fluid);
            stream_one<2, false>(c, fs[2], 0.f, 0.f, IJ_M(sn, 0), open_fluid);
            stream_one<3, false>(c, fs[3], 0.f, 0.f, IJ_M(sc, -1), open_fluid);
            stream_one<4, false>(c, fs[4], 0.f, 0.f, IJ_M(ss, 0), open_fluid);
            stream_one<5, false>(c, fs[5], 0.f, 0.f, IJ_M(sn, 1), open_fluid);
            stream_one<6, false>(c, fs[6], 0.f, 0.f, IJ_M(sn, -1), open_fluid);
            stream_one<7, false>(c, fs[7], 0.f, 0.f, IJ_M(ss, -1), open_fluid);
            stream_one<8, false>(c, fs[8], 0.f, 0.f, IJ_M(ss, 1), open_fluid);
            stream_one<1, true>(c, h[1], s_g1[sc][jm + 1], gc[3], IJ_M(sc, 1), open_fluid);
            stream_one<2, true>(c, h[2], g1[2], gc[4], IJ_M(sn, 0), open_fluid);
            stream_one<3, true>(c, h[3], s_g3[sc][jm - 1], gc[1], IJ_M(sc, -1), open_fluid);
            stream_one<4, true>(c, h[4], g4prev, gc[2], IJ_M(ss, 0), open_fluid);
#undef IJ_M
        }
    }
}

// ------------------------------------------------------------ init / moments

// raw phi of the initial state at fluid nodes: from phi itself, or
// phi = phi* tanh(2 d / W) from a signed distance d (the equilibrium profile)
__global__ void k_set_phi(KParams P, const float* __restrict__ src, int from_distance,
                          const uint8_t* __restrict__ wall, double* __restrict__ phi)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= P.nx) return;
    const unsigned k = (unsigned)y * P.pitch + x;
    if (wall[k]) return;
    const double v = (double)src[(size_t)y * P.nx + x];
    phi[k] = from_distance ? P.phi_star * tanh(2.0 * v * P.inv_width) : v;
}

// f = f_eq(n0, u), g = g_eq(phi, u) with mu from the phi~ field
__global__ void k_init_eq(KParams P, float* __restrict__ A, const uint8_t* __restrict__ wall,
                          const double* __restrict__ phi, const float* __restrict__ ux,
                          const float* __restrict__ uy)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= P.nx) return;
    const unsigned k = (unsigned)y * P.pitch + x;
    float fe[9], ge[5];
    uint16_t g0l = 0;
    if (wall[k]) {
#pragma unroll
        for (int i = 0; i < 9; ++i) fe[i] = 0.f;
#pragma unroll
        for (int i = 0; i < 5; ++i) ge[i] = 0.f;
    } else {
        double st[9];
        load_stencil(P, phi, x, y, st);
        const double ph = st[0];
        const double lap = ((((st[1] - ph) + (st[3] - ph)) + ((st[2] - ph) + (st[4] - ph))) * 4.0 +
                            (((st[5] - ph) + (st[7] - ph)) + ((st[6] - ph) + (st[8] - ph)))) * (1.0 / 6.0);
        const double mu = P.beta4 * ph * ((ph - P.phi_star) * (ph + P.phi_star)) - P.kappa * lap;
        const size_t kin = (size_t)y * P.nx + x;
        node_equilibrium(P, ph, mu, ux ? ux[kin] : 0.f, uy ? uy[kin] : 0.f, fe, ge, g0l);
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) A[(size_t)i * P.plane + k] = fe[i];
#pragma unroll
    for (int i = 0; i < 5; ++i) A[(size_t)(9 + i) * P.plane + k] = ge[i];
    lo_plane(A, P)[k] = g0l;
}

// n, phi, u at every node (0 at solids) into caller arrays [ny][nx]
__global__ void k_moments(KParams P, const float* __restrict__ A, const uint8_t* __restrict__ wall,
                          const double* __restrict__ phi, float* __restrict__ on, float* __restrict__ ophi,
                          float* __restrict__ oux, float* __restrict__ ouy)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= P.nx) return;
    const unsigned k = (unsigned)y * P.pitch + x;
    const size_t ko = (size_t)y * P.nx + x;
    float n = 0.f, ph = 0.f, vx = 0.f, vy = 0.f;
    if (!wall[k]) {
        float f[9];
        double st[9], Fx, Fy;
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = A[(size_t)i * P.plane + k];
        load_stencil(P, phi, x, y, st);
        Macro m;
        node_macro(P, f, st, y < P.force_rows ? P.fb : 0.f, m, Fx, Fy);
        n = m.n;
        ph = (float)m.phi;
        vx = m.ux;
        vy = m.uy;
    }
    if (on) on[ko] = n;
    if (ophi) ophi[ko] = ph;
    if (oux) oux[ko] = vx;
    if (ouy) ouy[ko] = vy;
}

// distributions <-> caller layout [q][ny][nx] (f without the w_i n0 shift;
// g_0 as float(hi + lo); writing g_0 clears the remainder)
__global__ void k_state_io(KParams P, float* __restrict__ A, float* __restrict__ ext, int to_ext, int is_f)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    const int i = blockIdx.z;
    if (x >= P.nx) return;
    const float w[9] = {4.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f,
                        1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
    const unsigned kp = (unsigned)y * P.pitch + x;
    const size_t k = (size_t)(is_f ? i : 9 + i) * P.plane + kp;
    const size_t ke = (size_t)i * P.nx * P.ny + (size_t)y * P.nx + x;
    uint16_t* lo = lo_plane(A, P);
    if (is_f) {
        const float shift = w[i] * P.n0;
        if (to_ext)
            ext[ke] = A[k] + shift;
        else
            A[k] = ext[ke] - shift;
    } else if (i == 0) {
        if (to_ext) {
            ext[ke] = (float)((double)A[k] + (double)bf16_to_float(lo[kp]));
        } else {
            A[k] = ext[ke];
            lo[kp] = 0;
        }
    } else {
        if (to_ext)
            ext[ke] = A[k];
        else
            A[k] = ext[ke];
    }
}

// ---------------------------------------------------------------- diagnostics
//
// Pass 1: one workgroup per row.  Row ink count (phi > 0, rows >= row0) and
// summed u_y; partial sums of n, phi, momentum (double), max |u| and the
// count of non-finite nodes.
constexpr int DIAG_THREADS = 256;

__global__ __launch_bounds__(DIAG_THREADS) void k_diag_rows(KParams P, const float* __restrict__ A,
                                                           const uint8_t* __restrict__ wall,
                                                           const double* __restrict__ phi, int row0,
                                                           DiagRow* __restrict__ rows)
{
    const int y = blockIdx.x;
    double sn = 0, sp = 0, sjx = 0, sjy = 0, suy = 0;
    float umax = 0.f;
    int cnt = 0, bad = 0;
    for (int x = threadIdx.x; x < P.nx; x += DIAG_THREADS) {
        const unsigned k = (unsigned)y * P.pitch + x;
        if (wall[k]) continue;
        float f[9];
        double st[9], Fx, Fy;
#pragma unroll
        for (int i = 0; i < 9; ++i) f[i] = A[(size_t)i * P.plane + k];
        load_stencil(P, phi, x, y, st);
        Macro m;
        node_macro(P, f, st, y < P.force_rows ? P.fb : 0.f, m, Fx, Fy);
        sn += (double)m.n;
        sp += m.phi;
        sjx += (double)m.jx;
        sjy += (double)m.jy;
        const float um = sqrtf(m.ux * m.ux + m.uy * m.uy);
        if (!isfinite(m.n) || !isfinite(m.phi) || !isfinite(um))
            ++bad;
        else
            umax = fmaxf(umax, um);
        if (y >= row0 && m.phi > 0.0) {
            ++cnt;
            suy += (double)m.uy;
        }
    }
    __shared__ double sh[6][DIAG_THREADS];
    __shared__ int shi[2][DIAG_THREADS];
    const int t = threadIdx.x;
    sh[0][t] = sn; sh[1][t] = sp; sh[2][t] = sjx; sh[3][t] = sjy; sh[4][t] = suy; sh[5][t] = umax;
    shi[0][t] = cnt; shi[1][t] = bad;
    __syncthreads();
    for (int s = DIAG_THREADS / 2; s > 0; s >>= 1) {
        if (t < s) {
            for (int q = 0; q < 5; ++q) sh[q][t] += sh[q][t + s];
            sh[5][t] = fmax(sh[5][t], sh[5][t + s]);
            shi[0][t] += shi[0][t + s];
            shi[1][t] += shi[1][t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        DiagRow r;
        r.mass_n = sh[0][0];
        r.mass_phi = sh[1][0];
        r.mom_x = sh[2][0];
        r.mom_y = sh[3][0];
        r.uy = sh[4][0];
        r.max_u = sh[5][0];
        r.count = shi[0][0];
        r.bad = shi[1][0];
        rows[y] = r;
    }
}

// Pass 2.  Sums over rows in a fixed order.  Ink segments (maximal runs of
// rows with ink in [row0, ny)) are found in parallel: each thread scans a
// contiguous chunk of rows and summarises it as its first run, its last run
// and the statistics of the runs strictly between them (those are complete
// segments); one thread then walks the chunk summaries in row order, joining
// runs that continue across chunk boundaries.  Segments are closed in order
// of their first row, so ties on size resolve to the lowest one, as in a
// sequential scan.  The run that starts at row0 touches the nozzle exit and
// is not a drop; other runs with at least a_min ink nodes are.
struct RunSum {
    int a, b;     // rows [a, b)
    long long c;  // ink nodes
    double u;     // summed u_y
};

__global__ __launch_bounds__(DIAG_THREADS) void k_diag_finish(int ny, int row0, int a_min, int64_t step,
                                                             const DiagRow* __restrict__ rows,
                                                             SampleRec* __restrict__ out)
{
    __shared__ double sh[4][DIAG_THREADS];
    __shared__ double smax[DIAG_THREADS];
    __shared__ long long sbad[DIAG_THREADS];
    __shared__ RunSum s_first[DIAG_THREADS], s_last[DIAG_THREADS], s_best[DIAG_THREADS];
    __shared__ int s_nruns[DIAG_THREADS];
    __shared__ long long s_ndet[DIAG_THREADS];
    const int t = threadIdx.x;
    double a = 0, b = 0, c = 0, d = 0, mx = 0;
    long long bad = 0;
    for (int y = t; y < ny; y += DIAG_THREADS) {
        a += rows[y].mass_n;
        b += rows[y].mass_phi;
        c += rows[y].mom_x;
        d += rows[y].mom_y;
        mx = fmax(mx, rows[y].max_u);
        bad += rows[y].bad;
    }
    sh[0][t] = a; sh[1][t] = b; sh[2][t] = c; sh[3][t] = d; smax[t] = mx; sbad[t] = bad;

    const int span = ny - row0;
    const int chunk = (span + DIAG_THREADS - 1) / DIAG_THREADS;
    const int ya = row0 + t * chunk, yb = min(ny, ya + chunk);
    RunSum first{-1, -1, 0, 0.0}, pend{-1, -1, 0, 0.0}, best{-1, -1, 0, 0.0};
    int nr = 0;
    long long ndet = 0;
    int y = ya;
    while (y < yb) {
        if (rows[y].count <= 0) {
            ++y;
            continue;
        }
        RunSum r{y, y, 0, 0.0};
        while (y < yb && rows[y].count > 0) {
            r.c += rows[y].count;
            r.u += rows[y].uy;
            ++y;
        }
        r.b = y;
        if (nr == 0) first = r;
        if (nr >= 2 && pend.c >= a_min) {  // pend lies strictly inside the chunk
            ++ndet;
            if (pend.c > best.c) best = pend;
        }
        pend = r;
        ++nr;
    }
    s_first[t] = first;
    s_last[t] = pend;
    s_best[t] = best;
    s_nruns[t] = nr;
    s_ndet[t] = ndet;
    __syncthreads();
    for (int s = DIAG_THREADS / 2; s > 0; s >>= 1) {
        if (t < s) {
            for (int q = 0; q < 4; ++q) sh[q][t] += sh[q][t + s];
            smax[t] = fmax(smax[t], smax[t + s]);
            sbad[t] += sbad[t + s];
        }
        __syncthreads();
    }
    if (t != 0) return;
    long long nd = 0;
    RunSum top{-1, -1, 0, 0.0};
    auto close = [&](const RunSum& r) {
        if (r.a != row0 && r.c >= a_min) {
            ++nd;
            if (r.c > top.c) top = r;
        }
    };
    RunSum open{-1, -1, 0, 0.0};
    bool has_open = false;
    for (int k = 0; k < DIAG_THREADS; ++k) {
        const int ka = row0 + k * chunk;
        if (ka >= ny) break;
        const int kb = min(ny, ka + chunk);
        if (s_nruns[k] == 0) {
            if (has_open) {
                close(open);
                has_open = false;
            }
            continue;
        }
        const RunSum f = s_first[k];
        if (has_open && f.a == ka) {
            open.b = f.b;
            open.c += f.c;
            open.u += f.u;
        } else {
            if (has_open) close(open);
            open = f;
            has_open = true;
        }
        if (open.b < kb) {
            close(open);
            has_open = false;
        }
        if (s_ndet[k] > 0) {
            nd += s_ndet[k];
            if (s_best[k].c > top.c) top = s_best[k];
        }
        if (s_nruns[k] >= 2) {
            const RunSum l = s_last[k];
            if (l.b == kb) {
                open = l;
                has_open = true;
            } else {
                close(l);
            }
        }
    }
    if (has_open) close(open);
    SampleRec r;
    r.step = step;
    r.mass_n = sh[0][0];
    r.mass_phi = sh[1][0];
    r.mom_x = sh[2][0];
    r.mom_y = sh[3][0];
    r.max_u = smax[0];
    r.nan_count = sbad[0];
    r.n_detached = nd;
    r.largest_count = top.c;
    r.largest_uy = top.u;
    r.largest_top = top.c > 0 ? top.b - 1 : -1;
    *out = r;
}

// ------------------------------------------------------------------ launchers

static inline dim3 row_grid(const KParams& P, int tpb) { return dim3((P.nx + tpb - 1) / tpb, P.ny, 1); }

hipError_t launch_phi_ghost(const KParams& P, const float* A, const uint8_t* wall, double* phi,
                            const int2* ghost_list, int n_ghost, hipStream_t st)
{
    hipLaunchKernelGGL(k_phi_from_g, row_grid(P, 256), dim3(256), 0, st, P, A, wall, phi);
    if (n_ghost > 0)
        hipLaunchKernelGGL(k_ghost, dim3((n_ghost + 255) / 256), dim3(256), 0, st, P, ghost_list, n_ghost,
                           wall, phi);
    return hipGetLastError();
}

hipError_t launch_collide_ref(const KParams& P, const float* A, float* B, const uint8_t* wall,
                              const double* phi, hipStream_t st)
{
    hipLaunchKernelGGL(k_collide_ref, row_grid(P, 256), dim3(256), 0, st, P, A, B, wall, phi);
    return hipGetLastError();
}

hipError_t launch_collide_fused(const KParams& P, const float* A, float* B, const uint8_t* wall,
                                int waves_x, int rows_per_block, hipStream_t st)
{
    const int bw = 64 * waves_x;
    const int n_strips = (P.nx + bw - 1) / bw;
    const int n_rb = (P.ny + rows_per_block - 1) / rows_per_block;
    const dim3 grid(n_strips * n_rb);
    switch (waves_x) {
    case 1:
        hipLaunchKernelGGL(k_collide_fused<1>, grid, dim3(64), 0, st, P, A, B, wall, rows_per_block, n_strips, n_rb);
        break;
    case 2:
        hipLaunchKernelGGL(k_collide_fused<2>, grid, dim3(128), 0, st, P, A, B, wall, rows_per_block, n_strips, n_rb);
        break;
    case 4:
        hipLaunchKernelGGL(k_collide_fused<4>, grid, dim3(256), 0, st, P, A, B, wall, rows_per_block, n_strips, n_rb);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_init(const KParams& P, float* A, const uint8_t* wall, double* phi, const float* src,
                       int from_distance, const float* ux, const float* uy, const int2* ghost_list,
                       int n_ghost, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_phi, row_grid(P, 256), dim3(256), 0, st, P, src, from_distance, wall, phi);
    if (n_ghost > 0)
        hipLaunchKernelGGL(k_ghost, dim3((n_ghost + 255) / 256), dim3(256), 0, st, P, ghost_list, n_ghost,
                           wall, phi);
    hipLaunchKernelGGL(k_init_eq, row_grid(P, 256), dim3(256), 0, st, P, A, wall, phi, ux, uy);
    return hipGetLastError();
}

hipError_t launch_moments(const KParams& P, const float* A, const uint8_t* wall, const double* phi, float* n,
                          float* ph, float* ux, float* uy, hipStream_t st)
{
    hipLaunchKernelGGL(k_moments, row_grid(P, 256), dim3(256), 0, st, P, A, wall, phi, n, ph, ux, uy);
    return hipGetLastError();
}

hipError_t launch_state_io(const KParams& P, float* A, float* f_ext, float* g_ext, int to_ext, hipStream_t st)
{
    const dim3 b(256);
    if (f_ext)
        hipLaunchKernelGGL(k_state_io, dim3((P.nx + 255) / 256, P.ny, 9), b, 0, st, P, A, f_ext, to_ext, 1);
    if (g_ext)
        hipLaunchKernelGGL(k_state_io, dim3((P.nx + 255) / 256, P.ny, 5), b, 0, st, P, A, g_ext, to_ext, 0);
    return hipGetLastError();
}

hipError_t launch_diag(const KParams& P, const float* A, const uint8_t* wall, const double* phi, int row0,
                       int a_min, int64_t step, DiagRow* rows, SampleRec* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_diag_rows, dim3(P.ny), dim3(DIAG_THREADS), 0, st, P, A, wall, phi, row0, rows);
    hipLaunchKernelGGL(k_diag_finish, dim3(1), dim3(DIAG_THREADS), 0, st, P.ny, row0, a_min, step, rows, out);
    return hipGetLastError();
}

} // namespace ij
