// lbm_core.hip -- gfx950 kernels of the binary-fluid lattice Boltzmann update
// (arXiv:1702.04487, Methods Eqs. 3-10; actuation of Fig. 1; wetting walls and
// "fully developed" rows of Results, "Reproducing the experiment").
//
// Storage: one buffer holds, for each lattice row y, a block of 14 rows of
// pitch floats (pitch = nx rounded up to 64) and then one row of pitch
// 16-bit words; the block of row y starts at float y * rs, rs = 14.5 pitch.
// Population i of node (x, y) sits at y rs + i pitch + x, so everything a
// lattice row holds is one contiguous region of memory (one stream per
// lattice row, not 15 streams planes apart):
//   i = 0..8      f_i - w_i n0 (D2Q9 distributions shifted by their rest
//                 value, which keeps the low-order bits of the small velocity
//                 signal in FP32);
//   i = 9..13     g_0..g_4 (D2Q5);
//   16-bit row    bfloat16 of g_0 - float(g_0): g_0 carries +-phi* and is the
//                 only population whose FP32 rounding would quantise phi.
// Two buffers A (current, pre-collision) and B (next) alternate.
//
// Velocities c_0=(0,0) c_1=(1,0) c_2=(0,1) c_3=(-1,0) c_4=(0,-1)
// c_5=(1,1) c_6=(-1,1) c_7=(-1,-1) c_8=(1,-1); D2Q5 = c_0..c_4.
// Wall mask bytes: 0 fluid, 1 inner wall, 2 outer wall; inside the kernels 3
// marks a row beyond an open lattice edge.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include <algorithm>

#include "bf16_split.h"
#include "lbm_core.h"

namespace ij {

// ---------------------------------------------------------------- device math

using ij_bf16::bf16_to_float;
using ij_bf16::float_to_bf16;

// phi = sum_i g_i (Eq. 9's zeroth moment) in double from the five stored
// populations and the low-order part of g_0
__device__ __forceinline__ double phi_of(float g0, float g1, float g2, float g3, float g4, float lo)
{
    return ((((double)g1 + (double)g2) + ((double)g3 + (double)g4)) + (double)lo) + (double)g0;
}

// Accesses through the global address space (at a uniform base plus a
// 32-bit byte offset, or at an element index).  A pointer read from a case
// record is generic to the compiler; generic (flat) accesses need a 64-bit
// address per lane and are counted with the scalar loads, so that waiting for
// one waits for the other.  Every buffer here is in global memory.
typedef __attribute__((address_space(1))) char gchar_t;
__device__ __forceinline__ float gld(const float* base, unsigned bo)
{
    return *reinterpret_cast<const __attribute__((address_space(1))) float*>((const gchar_t*)base + bo);
}
__device__ __forceinline__ uint16_t gldh(const uint16_t* base, unsigned bo)
{
    return *reinterpret_cast<const __attribute__((address_space(1))) uint16_t*>((const gchar_t*)base + bo);
}
__device__ __forceinline__ void gst(float* base, unsigned bo, float v)
{
    *reinterpret_cast<__attribute__((address_space(1))) float*>((gchar_t*)base + bo) = v;
}
__device__ __forceinline__ void gsth(uint16_t* base, unsigned bo, uint16_t v)
{
    *reinterpret_cast<__attribute__((address_space(1))) uint16_t*>((gchar_t*)base + bo) = v;
}

template <class T>
__device__ __forceinline__ T gat(const T* p, size_t i)
{
    return reinterpret_cast<const __attribute__((address_space(1))) T*>((const gchar_t*)p)[i];
}
template <class T>
__device__ __forceinline__ void gput(T* p, size_t i, T v)
{
    reinterpret_cast<__attribute__((address_space(1))) T*>((gchar_t*)p)[i] = v;
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
    return gat(wall, (unsigned)y * P.pitch + x);
}

// index of population i of node (x, y) in a buffer
__device__ __forceinline__ size_t pidx(const KParams& P, int i, int x, int y)
{
    return (size_t)(unsigned)y * P.rs + (unsigned)(i * P.pitch + x);
}

// the 16-bit g_0 remainders of lattice row y (after its 14 float rows)
__device__ __forceinline__ const uint16_t* lo_row(const float* A, const KParams& P, int y)
{
    return reinterpret_cast<const uint16_t*>(A + (size_t)(unsigned)y * P.rs + (size_t)kFloatPlanes * P.pitch);
}
__device__ __forceinline__ uint16_t* lo_row(float* A, const KParams& P, int y)
{
    return reinterpret_cast<uint16_t*>(A + (size_t)(unsigned)y * P.rs + (size_t)kFloatPlanes * P.pitch);
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
    const float v = IS_G ? hv + P.omq * (fl ? g_dest : g_self) : hv;
    const int pl = IS_G ? 9 + d : d;
    gput(c.B, pidx(P, pl, wx, wy), v);
    if (P.bc_open) {
        const int cyd = fl ? DY : -DY;
        if (cyd > 0 && wy == 1 && open_fluid(0, fl ? DX : 0))
            gput(c.B, pidx(P, pl, wx, 0), v);
        if (cyd < 0 && wy == P.ny - 2 && open_fluid(1, fl ? DX : 0))
            gput(c.B, pidx(P, pl, wx, P.ny - 1), v);
    }
}

// Streaming of a population that changes column (c_x != 0) inside one
// wave, with aligned stores.  Push semantics are kept: the value v of node
// (x, y) still lands in x + c_i, or bounces back into (x, y) when x + c_i is
// solid, or is dropped beyond an open row; but the store into column x + c_i
// is issued by the lane that owns that column, which receives the value vin
// of its neighbour x - c_i (through LDS), so every row of a plane is written
// by whole cache lines.  Only the lane at the wave edge pushes its value
// across the edge itself.  For g, g_recv is the pre-collision g_I of the
// receiving slot (the lane's own node, c_y = 0 for the g directions that
// move in x), g_self the own g of the opposite direction (bounce-back) and
// g_edge the pre-collision g_I of the node across the wave edge.
struct ShiftCtx {
    const KParams* P;
    float* B;
    int t, lane, wv, x, y;
    bool active, own_fluid;
};

template <int I, bool IS_G, typename MaskRel, typename OpenFn>
__device__ __forceinline__ void stream_shifted(const ShiftCtx& c, float v, float vin, float g_recv, float g_self,
                                               float g_edge, MaskRel mask_rel, OpenFn open_fluid)
{
    constexpr int DX = Dir<I>::dx, DY = Dir<I>::dy, OPP = Dir<I>::opp;
    const KParams& P = *c.P;
    int ty = c.y + DY;
    bool in_lat = true;
    if (DY != 0 && (ty < 0 || ty >= P.ny)) {
        if (P.bc_open) in_lat = false;
        else ty = ty < 0 ? ty + P.ny : ty - P.ny;
    }
    const int pl = IS_G ? 9 + I : I;
    auto put = [&](int plane_idx, int cyd, int wx, int wy, int dxo, float val) {
        gput(c.B, pidx(P, plane_idx, wx, wy), val);
        if (P.bc_open) {
            if (cyd > 0 && wy == 1 && open_fluid(0, dxo)) gput(c.B, pidx(P, plane_idx, wx, 0), val);
            if (cyd < 0 && wy == P.ny - 2 && open_fluid(1, dxo)) gput(c.B, pidx(P, plane_idx, wx, P.ny - 1), val);
        }
    };
    // receive: this lane's column at row y + DY, pushed from column x - DX
    const int src_lane = c.lane - DX, src_t = c.t - DX;
    const bool src_in_wave = src_lane >= 0 && src_lane < 64 && src_t >= 0 && src_t < c.wv;
    if (c.active && in_lat && src_in_wave && mask_rel(0, -DX) == 0 && mask_rel(DY, 0) == 0)
        put(pl, DY, c.x, ty, 0, IS_G ? vin + P.omq * g_recv : vin);
    // own push: bounce-back, or across the wave edge
    if (c.own_fluid && in_lat) {
        const bool tgt_fluid = mask_rel(DY, DX) == 0;
        const int dst_lane = c.lane + DX, dst_t = c.t + DX;
        const bool dst_in_wave = dst_lane >= 0 && dst_lane < 64 && dst_t >= 0 && dst_t < c.wv;
        if (!tgt_fluid)
            put(IS_G ? 9 + OPP : OPP, -DY, c.x, c.y, 0, IS_G ? v + P.omq * g_self : v);
        else if (!dst_in_wave)
            put(pl, DY, wrapx(c.x + DX, P.nx), ty, DX, IS_G ? v + P.omq * g_edge : v);
    }
}

// ------------------------------------------------------ reference path kernels

// raw phi at fluid nodes into the phi field (solid entries untouched)
__device__ __forceinline__ void phi_node(const KParams& P, const float* __restrict__ A,
                                         const uint8_t* __restrict__ wall, double* __restrict__ phi, int x, int y)
{
    const unsigned k = (unsigned)y * P.pitch + x;
    if (gat(wall, k)) return;
    gput(phi, k, phi_of(gat(A, pidx(P, 9, x, y)), gat(A, pidx(P, 10, x, y)), gat(A, pidx(P, 11, x, y)),
                        gat(A, pidx(P, 12, x, y)), gat(A, pidx(P, 13, x, y)), bf16_to_float(gat(lo_row(A, P, y), x))));
}

__global__ void k_phi_from_g(KParams P, const float* __restrict__ A, const uint8_t* __restrict__ wall,
                             double* __restrict__ phi)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x < P.nx) phi_node(P, A, wall, phi, x, blockIdx.y);
}

// wetting ghosts on the list of solid nodes that touch fluid
__device__ __forceinline__ void ghost_node(const KParams& P, int2 node, const uint8_t* __restrict__ wall,
                                           double* __restrict__ phi)
{
    const int x = node.x, y = node.y;
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
            v[k] = gat(phi, (unsigned)yy * P.pitch + xx);
        }
    }
    const unsigned k0 = (unsigned)y * P.pitch + x;
    gput(phi, k0, ghost_value(v, m, P.wet[gat(wall, k0)]));
}

__global__ void k_ghost(KParams P, const int2* __restrict__ list, int n, const uint8_t* __restrict__ wall,
                        double* __restrict__ phi)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ghost_node(P, list[i], wall, phi);
}

__device__ __forceinline__ void load_stencil(const KParams& P, const double* __restrict__ phi, int x, int y,
                                             double (&st)[9])
{
    const int xe = wrapx(x + 1, P.nx), xw = wrapx(x - 1, P.nx);
    const int yn = stencil_row(y + 1, P), ys = stencil_row(y - 1, P);
    const unsigned r0 = (unsigned)y * P.pitch, rn = (unsigned)yn * P.pitch, rs = (unsigned)ys * P.pitch;
    st[0] = gat(phi, r0 + x);
    st[1] = gat(phi, r0 + xe);
    st[2] = gat(phi, rn + x);
    st[3] = gat(phi, r0 + xw);
    st[4] = gat(phi, rs + x);
    st[5] = gat(phi, rn + xe);
    st[6] = gat(phi, rn + xw);
    st[7] = gat(phi, rs + xw);
    st[8] = gat(phi, rs + xe);
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
    for (int i = 0; i < 9; ++i) f[i] = A[pidx(P, i, x, y)];
#pragma unroll
    for (int i = 0; i < 5; ++i) g[i] = A[pidx(P, 9 + i, x, y)];
    const float lo = bf16_to_float(lo_row(A, P, y)[x]);
    load_stencil(P, phi, x, y, st);
    Macro m;
    float g0h;
    uint16_t g0l;
    node_collide(P, f, g, lo, st, y < P.force_rows ? P.fb : 0.f, fs, h, g0h, g0l, m);

    B[pidx(P, 0, x, y)] = fs[0];
    B[pidx(P, 9, x, y)] = g0h;
    lo_row(B, P, y)[x] = g0l;
    const StreamCtx c{&P, B, x, y};
    auto open_fluid = [&](int top, int dx) {
        const int cx = wrapx(x + dx, P.nx);
        return wall[top ? (unsigned)(P.ny - 1) * P.pitch + cx : (unsigned)cx] == 0;
    };
    // pre-collision g at (x + dx, y + dy), wrapped (only read when that node is fluid)
    auto gold = [&](int i, int dx, int dy) -> float {
        if (P.bc_open && (y + dy < 0 || y + dy >= P.ny)) return 0.f;
        int ty = y + dy;
        ty = ty < 0 ? ty + P.ny : (ty >= P.ny ? ty - P.ny : ty);
        return A[pidx(P, 9 + i, wrapx(x + dx, P.nx), ty)];
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
// the g_0 remainder) in an LDS ring with two halo columns each side, (2)
// turns row r+1 into phi~ (wetting ghosts at solid nodes), (3) collides row
// r with the nine-point stencil from LDS and streams it.  phi never goes
// through HBM: per fluid node the kernel reads the 14 distributions and the
// 16-bit g_0 remainder once and writes them once.
//
// Memory-level parallelism: the loads of a raw row and of a collide row are
// issued two iterations before their use into two alternating register sets
// (the loop is unrolled by two, so no register copies wait on them), and no
// branch depends on a value still in flight: raw rows are loaded whatever
// their mask and masked afterwards; the decision to load a collide row uses
// masks and row flags already in LDS.
//
// Stores are aligned: a population that changes column is handed to the
// lane that owns the destination column (a wave shift for rows without
// solid nodes, LDS otherwise); only the wave-edge lanes store across the
// edge.  Rows are "plain" when the geometry puts no solid node in rows
// r-1..r+1 of the strip and its halo and no open row within reach (a static
// per-(strip,row) table built on the host).  The PLAIN instantiation
// collides and streams only plain rows, with a branch-free store sequence;
// the other instantiation runs over the tiles that contain other rows and
// collides only those, with every slot decided by the masks (bounce-back,
// open-row copies).  Each fluid node is collided by exactly one of the two
// launches.  Tiles are numbered row-block major, so that the workgroups
// resident at one time cover whole rows of the planes.

// The value held by lane - 1 (from_left) or lane + 1 (from_right) of the
// wave (DPP wave shifts); the lane at the wave edge gets its own value back.
__device__ __forceinline__ float from_left(float v)
{
    const int b = __float_as_int(v);
    return __int_as_float(__builtin_amdgcn_update_dpp(b, b, 0x138, 0xf, 0xf, false));   // wave_shr:1
}
__device__ __forceinline__ float from_right(float v)
{
    const int b = __float_as_int(v);
    return __int_as_float(__builtin_amdgcn_update_dpp(b, b, 0x130, 0xf, 0xf, false));   // wave_shl:1
}

// Diagnostics sample terms.  Every path that takes a sample (the separate
// pass, or a step that samples its input state) reduces the same per-node
// terms in the same order: a butterfly over the 64 columns of each piece
// (64-column block of a row), then the pieces of the row in order.  Samples
// are therefore bit for bit the same whichever path took them.
struct SampleTerms {
    double n = 0.0, phi = 0.0, jx = 0.0, jy = 0.0, uy = 0.0;
    float u = 0.f;
    int cnt = 0, bad = 0;
};

__device__ __forceinline__ void sample_node(const Macro& m, bool ink_row, SampleTerms& d)
{
    d.n = (double)m.n;
    d.phi = m.phi;
    d.jx = (double)m.jx;
    d.jy = (double)m.jy;
    const float um = sqrtf(m.ux * m.ux + m.uy * m.uy);
    // the guard's count: a non-finite value, or a density that is not
    // positive (the mean density n of Eq. 1 must stay above zero)
    if (!isfinite(m.n) || !isfinite(m.phi) || !isfinite(um) || !(m.n > 0.f))
        d.bad = 1;
    else
        d.u = um;
    if (ink_row && m.phi > 0.0) {
        d.cnt = 1;
        d.uy = (double)m.uy;
    }
}

// sum over the 64 lanes of the wave (every lane takes part and gets the sum)
__device__ __forceinline__ DiagRow sample_piece(SampleTerms d)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        d.n += __shfl_xor(d.n, o);
        d.phi += __shfl_xor(d.phi, o);
        d.jx += __shfl_xor(d.jx, o);
        d.jy += __shfl_xor(d.jy, o);
        d.uy += __shfl_xor(d.uy, o);
        d.u = fmaxf(d.u, __shfl_xor(d.u, o));
        d.cnt += __shfl_xor(d.cnt, o);
        d.bad += __shfl_xor(d.bad, o);
    }
    DiagRow r;
    r.mass_n = d.n;
    r.mass_phi = d.phi;
    r.mom_x = d.jx;
    r.mom_y = d.jy;
    r.uy = d.uy;
    r.max_u = (double)d.u;
    r.count = d.cnt;
    r.bad = d.bad;
    return r;
}

__device__ __forceinline__ void sample_add(DiagRow& r, const DiagRow& q)
{
    r.mass_n += q.mass_n;
    r.mass_phi += q.mass_phi;
    r.mom_x += q.mom_x;
    r.mom_y += q.mom_y;
    r.uy += q.uy;
    r.max_u = fmax(r.max_u, q.max_u);
    r.count += q.count;
    r.bad += q.bad;
}

// One tile (strip, rows [y0, y1)) of the fused update.  fb is the body force
// of the step.  Shared by the single-lattice and the batched kernels; it
// starts with a barrier so that a workgroup may run several tiles in a row.
template <int NW, bool PLAIN, bool SAMPLE = false>
__device__ __forceinline__ void collide_tile(const KParams& P, float fb, const float* __restrict__ A,
                                             float* __restrict__ B, const uint8_t* __restrict__ wall,
                                             const uint8_t* __restrict__ plain_rows, int strip, int x0, int y0,
                                             int y1, DiagRow* __restrict__ parts = nullptr, bool down = false)
{
    constexpr int BW = 64 * NW;
    // raw rows rr - 3 dir .. rr are in use while row rr is processed; the last
    // reader of a slot finishes before the barrier that ends the row
    constexpr int RING = 4;
    __shared__ double s_raw[RING][BW + 4];
    __shared__ uint8_t s_m[RING][BW + 4];
    __shared__ float s_g[5][RING][BW + 4];   // pre-collision g of each raw row
    __shared__ uint16_t s_lo[RING][BW];      // g_0 remainder bits of each raw row
    __shared__ double s_pt[4][BW + 2];
    __shared__ float s_out[PLAIN ? 1 : 12][BW + 2];   // post-collision f_1..f_8, h_1..h_4 of the row
    __shared__ uint8_t s_mine[kMaxRowsPerBlock];      // rows of the block this launch collides

    __syncthreads();   // LDS of a previous tile of this workgroup is free
    const int wv = min(BW, P.nx - x0);
    const int t = threadIdx.x;
    const int lane = t & 63;
    const bool active = t < wv;
    const int x = x0 + t;
    const int hidx = t < 2 ? t : wv + 2 + (t - 2);   // LDS column of the halo of threads 0..3

    for (int i = t; i < y1 - y0; i += BW)
        s_mine[i] = (gat(plain_rows, (size_t)strip * P.ny + y0 + i) != 0) == PLAIN;

    // row bases (uniform over the workgroup: 64-bit) and 32-bit byte offsets
    // of population i of column xx within a row
    auto arow = [&](int yy) { return A + (size_t)(unsigned)yy * P.rs; };
    auto brow = [&](int yy) { return B + (size_t)(unsigned)yy * P.rs; };
    auto boff = [&](int i, int xx) -> unsigned { return ((unsigned)i * (unsigned)P.pitch + (unsigned)xx) << 2; };
    auto ldf = [](const float* base, unsigned bo) { return gld(base, bo); };
    auto stf = [](float* base, unsigned bo, float v) { gst(base, bo, v); };

    // two register sets for loads in flight: raw rows (g, remainder bits,
    // mask; halo columns) and collide rows (f)
    float rg[2][5], hg[2][5], rf[2][9];
    uint16_t rlo[2], hlo[2];
    uint8_t rm[2], hm[2];
    bool ron[2];
    // every lane loads at an in-bounds column: lanes past the lattice edge
    // reuse the last column, and every lane loads the halo column of lane
    // t % 4 (only lanes 0..3 keep it)
    const int xc = active ? x : P.nx - 1;
    const int hq = t & 3;
    const int hx = wrapx(hq < 2 ? x0 - 2 + hq : x0 + wv + (hq - 2), P.nx);

    // Loads are issued without any branch around them, at in-bounds
    // addresses, so that the number of memory operations issued after a
    // fetch is known at its use and the wait there is partial.
    auto fetch_raw = [&](int rr, float (&g)[5], uint16_t& lo, uint8_t& m, float (&gh)[5], uint16_t& loh,
                         uint8_t& mh, bool& on) {
        int ry = rr;
        on = true;
        if (ry < 0 || ry >= P.ny) {
            if (P.bc_open) { on = false; ry = 0; }
            else ry = ry < 0 ? ry + P.ny : ry - P.ny;
        }
        const unsigned k = (unsigned)ry * P.pitch + xc;
        const unsigned kh = (unsigned)ry * P.pitch + hx;
        const float* Ar = arow(ry);
        m = gat(wall, k);
        mh = gat(wall, kh);
#pragma unroll
        for (int i = 0; i < 5; ++i) g[i] = ldf(Ar, boff(9 + i, xc));
#pragma unroll
        for (int i = 0; i < 5; ++i) gh[i] = ldf(Ar, boff(9 + i, hx));
        lo = gat(lo_row(A, P, ry), xc);
        loh = gat(lo_row(A, P, ry), hx);
    };

    // rows y0-2 .. y1+1 pass through the ring, upwards, or downwards when
    // `down` is set; the count is rounded up to an even number (the extra
    // iteration collides nothing).  Every ring slot and stencil neighbour is
    // addressed by absolute row, so the direction changes only the order of
    // the rows.  Vertically adjacent tiles that walk towards each other read
    // their shared halo rows at about the same time, from L2.
    const int nk = ((y1 - y0) + 5) & ~1;
    const int dir = down ? -1 : 1;
    const int rfirst = down ? y1 + 1 : y0 - 2;

    // iteration kk: raw row rr = rfirst + dir kk, phi~ row rr - dir, collide
    // row rc = rr - 2 dir; register set S = kk % 2
    auto body = [&](auto Sc, int kk) {
        constexpr int S = decltype(Sc)::value;
        const int rr = rfirst + dir * kk;
        const int rc = rr - 2 * dir;
        const int slot = rr & (RING - 1);

        // (1) raw row rr into the LDS ring (non-fluid entries zeroed)
        {
            const uint8_t m = ron[S] && active ? rm[S] : 3;
            if (active) {
                const bool fl = m == 0;
                s_m[slot][t + 2] = m;
                s_raw[slot][t + 2] =
                    fl ? phi_of(rg[S][0], rg[S][1], rg[S][2], rg[S][3], rg[S][4], bf16_to_float(rlo[S])) : 0.0;
#pragma unroll
                for (int i = 0; i < 5; ++i) s_g[i][slot][t + 2] = fl ? rg[S][i] : 0.f;
                s_lo[slot][t] = fl ? rlo[S] : (uint16_t)0;
            }
            if (t < 4) {
                const uint8_t mh = ron[S] ? hm[S] : 3;
                const bool fl = mh == 0;
                s_m[slot][hidx] = mh;
                s_raw[slot][hidx] =
                    fl ? phi_of(hg[S][0], hg[S][1], hg[S][2], hg[S][3], hg[S][4], bf16_to_float(hlo[S])) : 0.0;
                s_g[1][slot][hidx] = fl ? hg[S][1] : 0.f;
                s_g[3][slot][hidx] = fl ? hg[S][3] : 0.f;
            }
        }
        // the raw row two iterations ahead reuses set S (past the last row
        // the block needs, the loads repeat that row: cache hits, unused)
        fetch_raw(min(max(rr + 2 * dir, y0 - 2), y1 + 1), rg[S], rlo[S], rm[S], hg[S], hlo[S], hm[S], ron[S]);
        __syncthreads();

        // (2) phi~ of row rr - dir
        if (kk >= 1) {
            const int rgw = rr - dir;
            const int sc = rgw & (RING - 1), sn = (rgw + 1) & (RING - 1), ss = (rgw - 1) & (RING - 1);
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
                return ghost_value(v, mm, m0 == 1 ? P.wet[1] : P.wet[2]);   // no indexed kernarg load
            };
            if (active) s_pt[rgw & 3][t + 1] = phit(t + 2);
            if (t < 2) {
                const int j = t == 0 ? 1 : wv + 2;
                s_pt[rgw & 3][t == 0 ? 0 : wv + 1] = phit(j);
            }
        }
        __syncthreads();

        // (3) collide and stream row rc (the condition is uniform over the
        // workgroup: every lane reaches the barriers below)
        if (kk >= 4 && rc >= y0 && rc < y1 && s_mine[rc - y0]) {
            const int jm = t + 2, jo = t + 1;
            const int sc = rc & (RING - 1), sn = (rc + 1) & (RING - 1), ss = (rc - 1) & (RING - 1);
            const bool own_fluid = active && s_m[sc][jm] == 0;
            float fs[9], h[5];
#pragma unroll
            for (int i = 0; i < 9; ++i) fs[i] = 0.f;
#pragma unroll
            for (int i = 0; i < 5; ++i) h[i] = 0.f;
            SampleTerms dterm;   // this node's share of a diagnostics sample (SAMPLE only)
            if (own_fluid) {
                const int rn = (P.bc_open && rc == P.ny - 1) ? rc : rc + 1;
                const int rs = (P.bc_open && rc == 0) ? rc : rc - 1;
                const int pc = rc & 3, pn = rn & 3, ps = rs & 3;
                double st[9];
                st[0] = s_pt[pc][jo];
                st[1] = s_pt[pc][jo + 1];
                st[2] = s_pt[pn][jo];
                st[3] = s_pt[pc][jo - 1];
                st[4] = s_pt[ps][jo];
                st[5] = s_pt[pn][jo + 1];
                st[6] = s_pt[pn][jo - 1];
                st[7] = s_pt[ps][jo - 1];
                st[8] = s_pt[ps][jo + 1];
                float gcur[5];
#pragma unroll
                for (int i = 0; i < 5; ++i) gcur[i] = s_g[i][sc][jm];
                float g0h;
                uint16_t g0l;
                Macro mac;
                node_collide(P, rf[S], gcur, bf16_to_float(s_lo[sc][t]), st, rc < P.force_rows ? fb : 0.f, fs,
                             h, g0h, g0l, mac);
                if constexpr (SAMPLE) sample_node(mac, rc >= P.diag_row0, dterm);
                float* Bc = brow(rc);
                stf(Bc, boff(0, x), fs[0]);
                stf(Bc, boff(9, x), g0h);
                gput(lo_row(B, P, rc), x, g0l);
                if constexpr (!PLAIN) {
#pragma unroll
                    for (int i = 1; i < 9; ++i) s_out[i - 1][jo] = fs[i];
#pragma unroll
                    for (int i = 1; i < 5; ++i) s_out[7 + i][jo] = h[i];
                }
            }
            if constexpr (PLAIN) {
                // every node of rows rc-1..rc+1 is fluid; the populations
                // moving in x come from the neighbouring lanes
                const float l1 = from_left(fs[1]), l5 = from_left(fs[5]), l8 = from_left(fs[8]);
                const float lh1 = from_left(h[1]);
                const float r3 = from_right(fs[3]), r6 = from_right(fs[6]), r7 = from_right(fs[7]);
                const float rh3 = from_right(h[3]);
                if (active) {
                    const int yn = rc + 1 >= P.ny ? rc + 1 - P.ny : rc + 1;   // periodic wrap
                    const int ys = rc == 0 ? P.ny - 1 : rc - 1;
                    float* Bc = brow(rc);
                    float* Bn = brow(yn);
                    float* Bs = brow(ys);
                    stf(Bn, boff(2, x), fs[2]);
                    stf(Bs, boff(4, x), fs[4]);
                    stf(Bn, boff(11, x), h[2] + P.omq * s_g[2][sn][jm]);
                    stf(Bs, boff(13, x), h[4] + P.omq * s_g[4][ss][jm]);
                    if (lane >= 1) {                       // pusher x-1 is in this wave
                        stf(Bc, boff(1, x), l1);
                        stf(Bn, boff(5, x), l5);
                        stf(Bs, boff(8, x), l8);
                        stf(Bc, boff(10, x), lh1 + P.omq * s_g[1][sc][jm]);
                    }
                    if (lane < 63 && t + 1 < wv) {         // pusher x+1 is in this wave
                        stf(Bc, boff(3, x), r3);
                        stf(Bn, boff(6, x), r6);
                        stf(Bs, boff(7, x), r7);
                        stf(Bc, boff(12, x), rh3 + P.omq * s_g[3][sc][jm]);
                    }
                    // the lanes at the wave edges store across them
                    if (lane == 63 || t + 1 >= wv) {
                        const int xe = wrapx(x + 1, P.nx);
                        stf(Bc, boff(1, xe), fs[1]);
                        stf(Bn, boff(5, xe), fs[5]);
                        stf(Bs, boff(8, xe), fs[8]);
                        stf(Bc, boff(10, xe), h[1] + P.omq * s_g[1][sc][jm + 1]);
                    }
                    if (lane == 0) {
                        const int xw = wrapx(x - 1, P.nx);
                        stf(Bc, boff(3, xw), fs[3]);
                        stf(Bn, boff(6, xw), fs[6]);
                        stf(Bs, boff(7, xw), fs[7]);
                        stf(Bc, boff(12, xw), h[3] + P.omq * s_g[3][sc][jm - 1]);
                    }
                }
            } else {
                __syncthreads();
                // masks decide every slot
                auto open_fluid = [&](int top, int dx) {
                    // rows 0 and ny-1 are in the ring whenever a copy into them occurs
                    const int row = top ? P.ny - 1 : 0;
                    return s_m[row & (RING - 1)][jm + dx] == 0;
                };
                auto mask_rel = [&](int dy, int dx) { return s_m[(rc + dy) & (RING - 1)][jm + dx]; };
                if (own_fluid) {
                    const StreamCtx c{&P, B, x, rc};
                    stream_one<2, false>(c, fs[2], 0.f, 0.f, [&]() { return mask_rel(1, 0); }, open_fluid);
                    stream_one<4, false>(c, fs[4], 0.f, 0.f, [&]() { return mask_rel(-1, 0); }, open_fluid);
                    stream_one<2, true>(c, h[2], s_g[2][sn][jm], s_g[4][sc][jm], [&]() { return mask_rel(1, 0); },
                                        open_fluid);
                    stream_one<4, true>(c, h[4], s_g[4][ss][jm], s_g[2][sc][jm], [&]() { return mask_rel(-1, 0); },
                                        open_fluid);
                }
                const ShiftCtx sx{&P, B, t, lane, wv, x, rc, active, own_fluid};
                stream_shifted<1, false>(sx, fs[1], s_out[0][jo - 1], 0.f, 0.f, 0.f, mask_rel, open_fluid);
                stream_shifted<3, false>(sx, fs[3], s_out[2][jo + 1], 0.f, 0.f, 0.f, mask_rel, open_fluid);
                stream_shifted<5, false>(sx, fs[5], s_out[4][jo - 1], 0.f, 0.f, 0.f, mask_rel, open_fluid);
                stream_shifted<6, false>(sx, fs[6], s_out[5][jo + 1], 0.f, 0.f, 0.f, mask_rel, open_fluid);
                stream_shifted<7, false>(sx, fs[7], s_out[6][jo + 1], 0.f, 0.f, 0.f, mask_rel, open_fluid);
                stream_shifted<8, false>(sx, fs[8], s_out[7][jo - 1], 0.f, 0.f, 0.f, mask_rel, open_fluid);
                stream_shifted<1, true>(sx, h[1], s_out[8][jo - 1], s_g[1][sc][jm], s_g[3][sc][jm],
                                        s_g[1][sc][jm + 1], mask_rel, open_fluid);
                stream_shifted<3, true>(sx, h[3], s_out[10][jo + 1], s_g[3][sc][jm], s_g[1][sc][jm],
                                        s_g[3][sc][jm - 1], mask_rel, open_fluid);
            }
            if constexpr (SAMPLE) {
                // the wave's 64 columns of row rc are piece x0 / 64 + wave;
                // a wave past the lattice edge writes nothing
                const DiagRow r = sample_piece(dterm);
                if (lane == 0 && t < wv) parts[(size_t)((x0 >> 6) + (t >> 6)) * P.ny + rc] = r;
            }
        }
        // the distributions of collide row rc + 2 dir into set S; for rows this
        // launch does not collide the loads go to a row of the block that is
        // (or is about to be) in the cache, and are unused
        {
            const int rf2 = rc + 2 * dir;
            const int rcl = min(max(rf2, y0), y1 - 1);
            const float* Ar = arow(rcl);
#pragma unroll
            for (int i = 0; i < 9; ++i) rf[S][i] = ldf(Ar, boff(i, xc));
        }
        // the ring slot of row rr - 3 dir is reused next: with one wave the
        // wave barrier keeps the compiler from moving the next row's LDS
        // writes above this row's last reads (the hardware keeps LDS
        // accesses of a wave in order)
        if (NW > 1)
            __syncthreads();
        else
            __builtin_amdgcn_wave_barrier();
    };

#pragma unroll
    for (int i = 0; i < 9; ++i) rf[0][i] = rf[1][i] = 0.f;
    fetch_raw(rfirst, rg[0], rlo[0], rm[0], hg[0], hlo[0], hm[0], ron[0]);
    fetch_raw(rfirst + dir, rg[1], rlo[1], rm[1], hg[1], hlo[1], hm[1], ron[1]);
    __syncthreads();   // s_mine
    for (int kk = 0; kk < nk; kk += 2) {
        body(std::integral_constant<int, 0>{}, kk);
        body(std::integral_constant<int, 1>{}, kk + 1);
    }
}

// A double held by lane - 1 (from_left) or lane + 1 (from_right): DPP wave
// shifts of both halves; the lane at the wave edge gets its own value back.
__device__ __forceinline__ double dfrom_left(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x138, 0xf, 0xf, false),
                            __builtin_amdgcn_update_dpp(lo, lo, 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ double dfrom_right(double v)
{
    const int lo = __double2loint(v), hi = __double2hiint(v);
    return __hiloint2double(__builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xf, 0xf, false),
                            __builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xf, 0xf, false));
}

// Plain rows without a walk: the row kernel.  Each wave updates the 64
// columns of one row of one piece on its own (no LDS, no barrier).  A plain
// row has no solid node in rows y-1..y+1 of its strip and halo and no open
// row within reach, so phi~ is the raw phi = sum g of those rows and every
// population streams to a fluid node.  Each lane loads f of its node and g
// (with the g_0 remainder) of its column in rows y-1, y, y+1; the stencil
// takes the neighbouring columns' phi by lane shifts, and the edge lanes
// take the halo columns (x0 - 1 and the column past the piece), which the
// wave reads with uniform (scalar) loads.  Streaming is that of the walked
// kernel's plain rows (aligned stores: lane shifts hand the x-moving
// populations to the lane that owns the destination column); the edge lanes
// store across the piece edge with the halo column's old g.  The rows above
// and below are read again by the waves of those rows at about the same
// time, so the halo rows come from the cache: per node the kernel moves the
// 14 populations in and out once.  Workgroups are numbered row-major (strip
// fastest), the order in which the populations of a row lie in memory; a
// workgroup of NW waves covers a strip of 64 NW columns.
// One wave: the 64 columns from x0 (< nx) of the plain row y, with the
// body force fb of the step.
template <bool SAMPLE, bool AS_GLOBAL = false>
__device__ __forceinline__ void collide_row_wave(const KParams& P, float fb, const float* __restrict__ A,
                                                 float* __restrict__ B, int y, int x0, DiagRow* __restrict__ parts)
{
    const int lane = threadIdx.x & 63;
    const int wv = min(64, P.nx - x0);
    const bool active = lane < wv;
    const int x = x0 + lane;
    const int xc = active ? x : P.nx - 1;   // lanes past the edge load the last column (unused)
    const int ys = y == 0 ? P.ny - 1 : y - 1, yn = y + 1 == P.ny ? 0 : y + 1;   // periodic (plain rows)
    const int xl = x0 == 0 ? P.nx - 1 : x0 - 1;                // halo columns (uniform)
    const int xr = x0 + wv == P.nx ? 0 : x0 + wv;

    // population rows of the three lattice rows (uniform bases), one lane offset
    const float* As = A + (size_t)(unsigned)ys * P.rs;
    const float* Ac = A + (size_t)(unsigned)y * P.rs;
    const float* An = A + (size_t)(unsigned)yn * P.rs;
    const unsigned pch = (unsigned)P.pitch;
    // 32-bit byte offset of this lane's column (one per lane, shared by every
    // access); the population rows are uniform bases
    const unsigned xo = (unsigned)xc << 2, xo2 = (unsigned)xc << 1;
    // AS_GLOBAL: A and B were read from memory (a case record), so the
    // accesses name the global address space themselves
    auto ldf = [](const float* base, unsigned bo) {
        if constexpr (AS_GLOBAL) return gld(base, bo);
        else return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + bo);
    };
    auto ldh = [](const uint16_t* base, unsigned bo) {
        if constexpr (AS_GLOBAL) return gldh(base, bo);
        else return *reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(base) + bo);
    };
    auto at = [](const auto* base, size_t i) {
        if constexpr (AS_GLOBAL) return gat(base, i);
        else return base[i];
    };
    float f[9], gs[5], gc[5], gn[5];
    uint16_t los, loc, lon;
#pragma unroll
    for (int i = 0; i < 9; ++i) f[i] = ldf(Ac + i * pch, xo);
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        gs[i] = ldf(As + (9 + i) * pch, xo);
        gc[i] = ldf(Ac + (9 + i) * pch, xo);
        gn[i] = ldf(An + (9 + i) * pch, xo);
    }
    los = ldh(lo_row(A, P, ys), xo2);
    loc = ldh(lo_row(A, P, y), xo2);
    lon = ldh(lo_row(A, P, yn), xo2);
    // halo columns: uniform addresses
    auto halo_phi = [&](const float* R, int yy, int hx) {
        return phi_of(at(R, 9 * pch + hx), at(R, 10 * pch + hx), at(R, 11 * pch + hx), at(R, 12 * pch + hx),
                      at(R, 13 * pch + hx), bf16_to_float(at(lo_row(A, P, yy), hx)));
    };
    const double pls = halo_phi(As, ys, xl), plc = halo_phi(Ac, y, xl), pln = halo_phi(An, yn, xl);
    const double prs = halo_phi(As, ys, xr), prc = halo_phi(Ac, y, xr), prn = halo_phi(An, yn, xr);
    const float g1r = at(Ac, 10 * pch + xr);   // pre-collision g_1 of the column past the piece, row y
    const float g3l = at(Ac, 12 * pch + xl);   // pre-collision g_3 of the column before it

    const double ps = phi_of(gs[0], gs[1], gs[2], gs[3], gs[4], bf16_to_float(los));
    const double pc = phi_of(gc[0], gc[1], gc[2], gc[3], gc[4], bf16_to_float(loc));
    const double pn = phi_of(gn[0], gn[1], gn[2], gn[3], gn[4], bf16_to_float(lon));
    const bool ledge = lane == 0, redge = lane == wv - 1;
    double st[9];
    st[0] = pc;
    st[2] = pn;
    st[4] = ps;
    {
        const double l_s = dfrom_left(ps), l_c = dfrom_left(pc), l_n = dfrom_left(pn);
        const double r_s = dfrom_right(ps), r_c = dfrom_right(pc), r_n = dfrom_right(pn);
        st[1] = redge ? prc : r_c;
        st[3] = ledge ? plc : l_c;
        st[5] = redge ? prn : r_n;
        st[6] = ledge ? pln : l_n;
        st[7] = ledge ? pls : l_s;
        st[8] = redge ? prs : r_s;
    }

    float fs[9], h[5], g0h = 0.f;
    uint16_t g0l = 0;
    SampleTerms dterm;
#pragma unroll
    for (int i = 0; i < 9; ++i) fs[i] = 0.f;
#pragma unroll
    for (int i = 0; i < 5; ++i) h[i] = 0.f;
    if (active) {
        Macro mac;
        node_collide(P, f, gc, bf16_to_float(loc), st, y < P.force_rows ? fb : 0.f, fs, h, g0h, g0l, mac);
        if constexpr (SAMPLE) sample_node(mac, y >= P.diag_row0, dterm);
    }
    // the populations moving in x come from the neighbouring lanes
    const float l1 = from_left(fs[1]), l5 = from_left(fs[5]), l8 = from_left(fs[8]);
    const float lh1 = from_left(h[1]);
    const float r3 = from_right(fs[3]), r6 = from_right(fs[6]), r7 = from_right(fs[7]);
    const float rh3 = from_right(h[3]);
    if (active) {
        auto stf = [](float* base, unsigned bo, float v) {
            if constexpr (AS_GLOBAL) gst(base, bo, v);
            else *reinterpret_cast<float*>(reinterpret_cast<char*>(base) + bo) = v;
        };
        float* Bs = B + (size_t)(unsigned)ys * P.rs;
        float* Bc = B + (size_t)(unsigned)y * P.rs;
        float* Bn = B + (size_t)(unsigned)yn * P.rs;
        const unsigned wo = (unsigned)x << 2;
        stf(Bc, wo, fs[0]);
        stf(Bc + 9 * pch, wo, g0h);
        if constexpr (AS_GLOBAL) gsth(lo_row(B, P, y), (unsigned)x << 1, g0l);
        else *reinterpret_cast<uint16_t*>(reinterpret_cast<char*>(lo_row(B, P, y)) + ((unsigned)x << 1)) = g0l;
        stf(Bn + 2 * pch, wo, fs[2]);
        stf(Bs + 4 * pch, wo, fs[4]);
        stf(Bn + 11 * pch, wo, h[2] + P.omq * gn[2]);
        stf(Bs + 13 * pch, wo, h[4] + P.omq * gs[4]);
        if (!ledge) {                          // pusher x-1 is in this wave
            stf(Bc + 1 * pch, wo, l1);
            stf(Bn + 5 * pch, wo, l5);
            stf(Bs + 8 * pch, wo, l8);
            stf(Bc + 10 * pch, wo, lh1 + P.omq * gc[1]);
        } else {                               // lane 0 stores across the left edge
            const unsigned lo_ = (unsigned)xl << 2;
            stf(Bc + 3 * pch, lo_, fs[3]);
            stf(Bn + 6 * pch, lo_, fs[6]);
            stf(Bs + 7 * pch, lo_, fs[7]);
            stf(Bc + 12 * pch, lo_, h[3] + P.omq * g3l);
        }
        if (!redge) {                          // pusher x+1 is in this wave
            stf(Bc + 3 * pch, wo, r3);
            stf(Bn + 6 * pch, wo, r6);
            stf(Bs + 7 * pch, wo, r7);
            stf(Bc + 12 * pch, wo, rh3 + P.omq * gc[3]);
        } else {                               // the last lane stores across the right edge
            const unsigned ro_ = (unsigned)xr << 2;
            stf(Bc + 1 * pch, ro_, fs[1]);
            stf(Bn + 5 * pch, ro_, fs[5]);
            stf(Bs + 8 * pch, ro_, fs[8]);
            stf(Bc + 10 * pch, ro_, h[1] + P.omq * g1r);
        }
    }
    if constexpr (SAMPLE) {
        // this wave's 64 columns of row y are piece x0 / 64
        const DiagRow r = sample_piece(dterm);
        if (lane == 0) parts[(size_t)(x0 >> 6) * P.ny + y] = r;
    }
}

template <int NW, bool SAMPLE>
__global__ __launch_bounds__(64 * NW) void k_collide_rows(KParams P, const float* __restrict__ A,
                                                          float* __restrict__ B,
                                                          const uint8_t* __restrict__ plain_rows, int n_strips,
                                                          int y_first, DiagRow* __restrict__ parts)
{
    // XCD x (workgroup b % 8) takes the x-th contiguous run of the row-major
    // (row, strip) numbering, so that the rows a wave reads g from (y - 1 and
    // y + 1) are those its own XCD's L2 has just read or is about to read
    const unsigned n = gridDim.x, b = blockIdx.x, xcd = b & 7u;
    const unsigned tile = xcd * (n >> 3) + min(xcd, n & 7u) + (b >> 3);
    const int y = y_first + (int)(tile / (unsigned)n_strips);
    const int strip = (int)(tile - (unsigned)(y - y_first) * (unsigned)n_strips);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int x0 = (strip * NW + wave) * 64;   // first column of this wave's piece (uniform)
    if (y >= P.ny || x0 >= P.nx || !plain_rows[(size_t)strip * P.ny + y]) return;   // uniform over the wave
    collide_row_wave<SAMPLE>(P, P.fb, A, B, y, x0, parts);
}

// One lattice: the PLAIN launch covers every tile, numbered row-block major
// and dealt so that runs of consecutive tiles stay on one XCD (workgroups are
// dealt round-robin over the 8 XCDs, each with its own L2); the other launch
// takes the (strip, block, first column) pieces of tile_list.
template <int NW, bool PLAIN, bool SAMPLE = false>
__global__ __launch_bounds__(64 * NW) void k_collide_fused(KParams P, const float* __restrict__ A,
                                                           float* __restrict__ B,
                                                           const uint8_t* __restrict__ wall,
                                                           const uint8_t* __restrict__ plain_rows,
                                                           const int4* __restrict__ tile_list,
                                                           int rows_per_block, int n_strips,
                                                           int n_rowblocks, DiagRow* __restrict__ parts)
{
    if (PLAIN) {
        const int ntiles = n_strips * n_rowblocks;
        int tile = blockIdx.x;
        if ((ntiles & 7) == 0) tile = (blockIdx.x & 7) * (ntiles >> 3) + (blockIdx.x >> 3);
        const int rb = tile / n_strips;
        const int strip = tile - rb * n_strips;
        const int y0 = rb * rows_per_block;
        // odd row blocks walk down, towards the block above them
        collide_tile<NW, PLAIN, SAMPLE>(P, P.fb, A, B, wall, plain_rows, strip, strip * 64 * NW, y0,
                                        min(P.ny, y0 + rows_per_block), parts, (rb & 1) != 0);
    } else {
        const int4 tl = tile_list[blockIdx.x];   // (strip, first row, first column, rows)
        collide_tile<NW, PLAIN, SAMPLE>(P, P.fb, A, B, wall, plain_rows, tl.x, tl.z, tl.y, tl.y + tl.w, parts);
    }
}

// The plain launch over a list of tiles (those that hold a plain row),
// listed row-block major as (strip, first row, first column, rows): XCD x
// (workgroup b % 8) takes the x-th contiguous run of the list.  As in the
// full-grid launch, odd row blocks walk down.
template <int NW, bool SAMPLE = false>
__global__ __launch_bounds__(64 * NW) void k_collide_listed(KParams P, const float* __restrict__ A,
                                                            float* __restrict__ B,
                                                            const uint8_t* __restrict__ wall,
                                                            const uint8_t* __restrict__ plain_rows,
                                                            const int4* __restrict__ tile_list,
                                                            int rows_per_block, DiagRow* __restrict__ parts)
{
    const int n = gridDim.x, b = blockIdx.x, xcd = b & 7;
    const int4 tl = tile_list[xcd * (n >> 3) + min(xcd, n & 7) + (b >> 3)];
    collide_tile<NW, true, SAMPLE>(P, P.fb, A, B, wall, plain_rows, tl.x, tl.z, tl.y, tl.y + tl.w, parts,
                                   ((tl.y / rows_per_block) & 1) != 0);
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
    for (int i = 0; i < 9; ++i) A[pidx(P, i, x, y)] = fe[i];
#pragma unroll
    for (int i = 0; i < 5; ++i) A[pidx(P, 9 + i, x, y)] = ge[i];
    lo_row(A, P, y)[x] = g0l;
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
        for (int i = 0; i < 9; ++i) f[i] = A[pidx(P, i, x, y)];
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
// Distributions to or from unshifted [i][ny][nx] arrays.  Solid nodes carry
// no populations: they read as 0 and are not written.
__global__ void k_state_io(KParams P, float* __restrict__ A, const uint8_t* __restrict__ wall,
                           float* __restrict__ ext, int to_ext, int is_f)
{
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    const int i = blockIdx.z;
    if (x >= P.nx) return;
    if (wall[(unsigned)y * P.pitch + x] != 0) {
        if (to_ext) ext[(size_t)i * P.nx * P.ny + (size_t)y * P.nx + x] = 0.f;
        return;
    }
    const float w[9] = {4.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f, 1.f / 9.f,
                        1.f / 36.f, 1.f / 36.f, 1.f / 36.f, 1.f / 36.f};
    const size_t k = pidx(P, is_f ? i : 9 + i, x, y);
    const size_t ke = (size_t)i * P.nx * P.ny + (size_t)y * P.nx + x;
    uint16_t* lo = lo_row(A, P, y);
    if (is_f) {
        const float shift = w[i] * P.n0;
        if (to_ext)
            ext[ke] = A[k] + shift;
        else
            A[k] = ext[ke] - shift;
    } else if (i == 0) {
        if (to_ext) {
            ext[ke] = (float)((double)A[k] + (double)bf16_to_float(lo[x]));
        } else {
            A[k] = ext[ke];
            lo[x] = 0;
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
// summed u_y; sums of n, phi, momentum (double), max |u| and the count of
// non-finite nodes, reduced in the order of every sampling path (sample_piece,
// sample_add).
constexpr int DIAG_THREADS = 256;

__device__ __forceinline__ void diag_row(const KParams& P, float fb, const float* __restrict__ A,
                                         const uint8_t* __restrict__ wall, const double* __restrict__ phi,
                                         int row0, DiagRow* __restrict__ rows, int y)
{
    // pieces of 64 columns, one per wave at a time, 64 pieces per round; the
    // pieces of a round are added in order by thread 0
    constexpr int kRound = 64;
    __shared__ DiagRow s_piece[kRound];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int n_sub = (P.nx + 63) / 64;
    DiagRow acc{};
    for (int k0 = 0; k0 < n_sub; k0 += kRound) {
        const int k1 = min(n_sub, k0 + kRound);
        for (int k = k0 + wave; k < k1; k += DIAG_THREADS / 64) {   // uniform over the wave
            SampleTerms d;
            const int x = k * 64 + lane;
            if (x < P.nx) {
                const unsigned kk = (unsigned)y * P.pitch + x;
                if (!gat(wall, kk)) {
                    float f[9];
                    double st[9], Fx, Fy;
#pragma unroll
                    for (int i = 0; i < 9; ++i) f[i] = gat(A, pidx(P, i, x, y));
                    load_stencil(P, phi, x, y, st);
                    Macro m;
                    node_macro(P, f, st, y < P.force_rows ? fb : 0.f, m, Fx, Fy);
                    sample_node(m, y >= row0, d);
                }
            }
            const DiagRow r = sample_piece(d);
            if (lane == 0) s_piece[k - k0] = r;
        }
        __syncthreads();
        if (t == 0)
            for (int k = k0; k < k1; ++k) sample_add(acc, s_piece[k - k0]);
        __syncthreads();
    }
    if (t == 0) rows[y] = acc;
}

__global__ __launch_bounds__(DIAG_THREADS) void k_diag_rows(KParams P, const float* __restrict__ A,
                                                           const uint8_t* __restrict__ wall,
                                                           const double* __restrict__ phi, int row0,
                                                           DiagRow* __restrict__ rows)
{
    diag_row(P, P.fb, A, wall, phi, row0, rows, blockIdx.x);
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

// Thread 0 writes the record to *out and returns it (other threads return
// an unspecified record).
__device__ __forceinline__ SampleRec diag_finish(int ny, int row0, int a_min, int band, int64_t step,
                                                 const DiagRow* __restrict__ rows, SampleRec* __restrict__ out)
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
    SampleRec r{};
    if (t != 0) return r;
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
    r.largest_bottom = top.c > 0 ? top.a : -1;
    // head and tail of the largest drop: mean u_y of the ink in its top and
    // its bottom `band` rows (the drop's rows all hold ink)
    if (top.c > 0) {
        double hu = 0.0, tu = 0.0;
        long long hc = 0, tc = 0;
        for (int y = max(top.a, top.b - band); y < top.b; ++y) {
            hu += rows[y].uy;
            hc += rows[y].count;
        }
        for (int y = top.a; y < min(top.b, top.a + band); ++y) {
            tu += rows[y].uy;
            tc += rows[y].count;
        }
        r.head_uy = hu / (double)hc;
        r.tail_uy = tu / (double)tc;
    }
    *out = r;
    return r;
}

__global__ __launch_bounds__(DIAG_THREADS) void k_diag_finish(int ny, int row0, int a_min, int band, int64_t step,
                                                             const DiagRow* __restrict__ rows,
                                                             SampleRec* __restrict__ out)
{
    (void)diag_finish(ny, row0, a_min, band, step, rows, out);
}

// ----------------------------------------------------------------- batches
//
// A batch holds independent lattices (cases) of different sizes and
// parameters.  One launch per kind of step work covers every case: the
// case records are in device memory, the current step is a device counter
// (advanced by k_batch_tick) and the driving force of each case is evaluated
// from it, so a captured graph of several steps replays correctly.  A case
// whose diagnostics sample fails the stability guard is switched off on the
// device (its state stays frozen; its samples are still recorded).

// Fig. 1 pulse of a case at step t (same selection as the host's).
__device__ __forceinline__ double case_pulse(const CaseRec& c, int64_t t)
{
    const int64_t period = c.t_pos + c.t_neg + c.t_idle;
    int64_t tt = t;
    if (c.periodic && period > 0) tt = t % period;
    if (tt < c.t_pos) return c.f_pos;
    if (tt < c.t_pos + c.t_neg) return -c.f_neg;
    return 0.0;
}

// Workgroup b runs tiles [b * per_wg, (b + 1) * per_wg) of the (case,
// strip, first row | rows << 16 | odd block << 30, first column) list, in
// order (neighbouring tiles of a case share their halo rows through the
// cache); a launch takes the tiles of its own width (64 * NW columns).  With
// one tile per workgroup, odd row blocks walk down, as in the single-lattice
// launch (consecutive workgroups then meet in their shared halo rows).
template <int NW, bool PLAIN, bool SAMPLE = false>
__global__ __launch_bounds__(64 * NW) void k_batch_collide(const CaseRec* __restrict__ cases,
                                                           const int4* __restrict__ tiles, int n_tiles,
                                                           int per_wg, int parity, const int* __restrict__ active)
{
    const bool single = per_wg == 1;
    const int i0 = blockIdx.x * per_wg, i1 = min(n_tiles, i0 + per_wg);
    for (int i = i0; i < i1; ++i) {
        const int4 tl = tiles[i];
        if (!active[tl.x]) continue;
        const CaseRec& R = cases[tl.x];
        const KParams P = R.P;   // P.fb: the case's body force of this step
        const int y0 = tl.z & 0xffff;
        const bool down = single && ((tl.z >> 30) & 1);
        collide_tile<NW, PLAIN, SAMPLE>(P, P.fb, R.buf[parity], R.buf[1 - parity], R.wall, R.plain, tl.y, tl.w,
                                        y0, y0 + ((tl.z >> 16) & 0x3fff), SAMPLE ? R.parts : nullptr, down);
    }
}

// The plain rows of every case of a batch: pieces (case, row, first column,
// nodes) of 64 columns of a plain strip of a row, one per wave (the update of
// collide_row_wave), listed case by case, row-major: workgroup g takes pieces
// NW g .. NW g + NW - 1, and XCD x (workgroup b % 8) takes the x-th contiguous
// range of workgroups, so that neighbouring rows of a case share one L2.
template <int NW, bool SAMPLE>
__global__ __launch_bounds__(64 * NW) void k_batch_rows(const CaseRec* __restrict__ cases,
                                                        const int4* __restrict__ pieces, int n_pieces, int parity,
                                                        const int* __restrict__ active)
{
    const unsigned n = gridDim.x, b = blockIdx.x, xcd = b & 7u;
    const unsigned g = xcd * (n >> 3) + min(xcd, n & 7u) + (b >> 3);
    const unsigned i = g * NW + (unsigned)__builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (i >= (unsigned)n_pieces) return;
    const int4 r = pieces[i];
    const CaseRec& R = cases[r.x];
    // the guard flag is read with the record: one round trip before the populations
    if (!active[r.x]) return;
    const KParams P = R.P;   // P.fb: the case's body force of this step
    collide_row_wave<SAMPLE, true>(P, P.fb, R.buf[parity], R.buf[1 - parity], r.y, r.z, SAMPLE ? R.parts : nullptr);
}

// One workgroup: the step counter moves on, a case the guard froze swaps
// its buffers (its state stays), and every case's body force of the new
// step goes to its record (the collide launches read it there instead of
// evaluating the pulse of Fig. 1 in every wave)
__global__ __launch_bounds__(1024) void k_batch_tick(int64_t* t_dev, CaseRec* __restrict__ cases, int n_cases,
                                                      const int* __restrict__ active)
{
    const int64_t t1 = t_dev[0] + 1;
    __syncthreads();   // every thread has read the counter before it moves
    if (threadIdx.x == 0) t_dev[0] = t1;
    for (int c = threadIdx.x; c < n_cases; c += blockDim.x) {
        if (!active[c]) {
            float* a = cases[c].buf[0];
            cases[c].buf[0] = cases[c].buf[1];
            cases[c].buf[1] = a;
        }
        cases[c].P.fb = (float)case_pulse(cases[c], t1);
    }
}

__global__ __launch_bounds__(1024) void k_batch_set_time(int64_t* t_dev, int64_t t, CaseRec* __restrict__ cases,
                                                          int n_cases)
{
    if (threadIdx.x == 0) t_dev[0] = t;
    for (int c = threadIdx.x; c < n_cases; c += blockDim.x) cases[c].P.fb = (float)case_pulse(cases[c], t);
}

// A sampling step takes each case's sample of its input state inside the
// collide launches (per 64-column piece and row, as the single-lattice step
// does).  Grid (pieces / 256, case): the partials are cleared first.
__global__ void k_batch_sample_clear(const CaseRec* __restrict__ cases)
{
    const CaseRec& R = cases[blockIdx.y];
    const size_t n = (size_t)((R.P.nx + 63) / 64) * R.P.ny;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) R.parts[i] = DiagRow{};
}

// grid (rows / 256, case): rows[y] = the partials of row y summed over the
// pieces in order.  A case the guard switched off keeps the rows of its
// failing sample (its state has not changed since), so its later records
// repeat that sample.
__global__ void k_batch_sample_rows(const CaseRec* __restrict__ cases, const int* __restrict__ active)
{
    const int c = blockIdx.y;
    const CaseRec& R = cases[c];
    const int y = blockIdx.x * blockDim.x + threadIdx.x;
    if (!active[c] || y >= R.P.ny) return;
    const int n_sub = (R.P.nx + 63) / 64;
    DiagRow r{};
    for (int k = 0; k < n_sub; ++k) sample_add(r, R.parts[(size_t)k * R.P.ny + y]);
    R.rows[y] = r;
}

// grid (case): the sample goes to the case's ring at n_rec[case], which is
// then advanced; a sample that fails the guard (non-finite nodes, or
// max |u| above the case's limit) switches the case off.
__global__ __launch_bounds__(DIAG_THREADS) void k_batch_diag_finish(const CaseRec* __restrict__ cases,
                                                                   const int64_t* __restrict__ t_dev,
                                                                   int64_t* __restrict__ n_rec,
                                                                   int* __restrict__ active)
{
    const int c = blockIdx.x;
    const CaseRec& R = cases[c];
    const int64_t k = n_rec[c];
    const SampleRec r = diag_finish(R.P.ny, R.row0, R.a_min, R.band, *t_dev, R.rows, R.ring + k);
    if (threadIdx.x == 0) {
        n_rec[c] = k + 1;
        if (r.nan_count > 0 || !(r.max_u <= R.u_limit)) active[c] = 0;
    }
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

template <bool SAMPLE>
hipError_t launch_collide_fused_t(const KParams& P, const float* A, float* B, const uint8_t* wall,
                                  const uint8_t* plain_rows, const int4* plain_tiles, int n_plain_tiles,
                                  const int4* general_tiles, int n_general_tiles, int waves_x, int rows_per_block,
                                  DiagRow* parts, hipStream_t st)
{
    const int bw = 64 * waves_x;
    const int n_strips = (P.nx + bw - 1) / bw;
    const int n_rb = (P.ny + rows_per_block - 1) / rows_per_block;
    if (rows_per_block == 1) {   // one row per workgroup, no walk: the row kernel
        const dim3 grid((unsigned)n_strips * (unsigned)P.ny);
        switch (waves_x) {
        case 1:
            hipLaunchKernelGGL((k_collide_rows<1, SAMPLE>), grid, dim3(64), 0, st, P, A, B, plain_rows, n_strips, 0,
                               parts);
            break;
        case 2:
            hipLaunchKernelGGL((k_collide_rows<2, SAMPLE>), grid, dim3(128), 0, st, P, A, B, plain_rows, n_strips,
                               0, parts);
            break;
        case 4:
            hipLaunchKernelGGL((k_collide_rows<4, SAMPLE>), grid, dim3(256), 0, st, P, A, B, plain_rows, n_strips,
                               0, parts);
            break;
        default:
            return hipErrorInvalidValue;
        }
    } else if (n_plain_tiles < 0) {   // every tile
        const dim3 grid(n_strips * n_rb);
        switch (waves_x) {
        case 1:
            hipLaunchKernelGGL((k_collide_fused<1, true, SAMPLE>), grid, dim3(64), 0, st, P, A, B, wall, plain_rows,
                               nullptr, rows_per_block, n_strips, n_rb, parts);
            break;
        case 2:
            hipLaunchKernelGGL((k_collide_fused<2, true, SAMPLE>), grid, dim3(128), 0, st, P, A, B, wall,
                               plain_rows, nullptr, rows_per_block, n_strips, n_rb, parts);
            break;
        case 4:
            hipLaunchKernelGGL((k_collide_fused<4, true, SAMPLE>), grid, dim3(256), 0, st, P, A, B, wall,
                               plain_rows, nullptr, rows_per_block, n_strips, n_rb, parts);
            break;
        default:
            return hipErrorInvalidValue;
        }
    } else if (n_plain_tiles > 0) {
        const dim3 grid(n_plain_tiles);
        switch (waves_x) {
        case 1:
            hipLaunchKernelGGL((k_collide_listed<1, SAMPLE>), grid, dim3(64), 0, st, P, A, B, wall, plain_rows,
                               plain_tiles, rows_per_block, parts);
            break;
        case 2:
            hipLaunchKernelGGL((k_collide_listed<2, SAMPLE>), grid, dim3(128), 0, st, P, A, B, wall, plain_rows,
                               plain_tiles, rows_per_block, parts);
            break;
        case 4:
            hipLaunchKernelGGL((k_collide_listed<4, SAMPLE>), grid, dim3(256), 0, st, P, A, B, wall, plain_rows,
                               plain_tiles, rows_per_block, parts);
            break;
        default:
            return hipErrorInvalidValue;
        }
    }
    // the general pieces are 64 columns wide: one wave each
    if (n_general_tiles > 0)
        hipLaunchKernelGGL((k_collide_fused<1, false, SAMPLE>), dim3(n_general_tiles), dim3(64), 0, st, P, A, B,
                           wall, plain_rows, general_tiles, 0, n_strips, n_rb, parts);
    return hipGetLastError();
}

hipError_t launch_collide_fused(const KParams& P, const float* A, float* B, const uint8_t* wall,
                                const uint8_t* plain_rows, const int4* plain_tiles, int n_plain_tiles,
                                const int4* general_tiles, int n_general_tiles, int waves_x, int rows_per_block,
                                DiagRow* sample_parts, hipStream_t st)
{
    if (rows_per_block < 1 || rows_per_block > kMaxRowsPerBlock || (n_plain_tiles > 0 && !plain_tiles))
        return hipErrorInvalidValue;
    if (sample_parts)
        return launch_collide_fused_t<true>(P, A, B, wall, plain_rows, plain_tiles, n_plain_tiles, general_tiles,
                                            n_general_tiles, waves_x, rows_per_block, sample_parts, st);
    return launch_collide_fused_t<false>(P, A, B, wall, plain_rows, plain_tiles, n_plain_tiles, general_tiles,
                                         n_general_tiles, waves_x, rows_per_block, nullptr, st);
}

__global__ void k_sample_clear(DiagRow* __restrict__ parts, size_t n)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) parts[i] = DiagRow{};
}

// rows[y] = the partials of row y summed over the pieces in order
__global__ void k_sample_rows(const DiagRow* __restrict__ parts, int n_sub, int ny, DiagRow* __restrict__ rows)
{
    const int y = blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= ny) return;
    DiagRow r{};
    for (int k = 0; k < n_sub; ++k) sample_add(r, parts[(size_t)k * ny + y]);
    rows[y] = r;
}

hipError_t launch_sample_clear(DiagRow* parts, size_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sample_clear, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, parts, n);
    return hipGetLastError();
}

int batch_resident_workgroups(int waves_x)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    hipError_t e = hipErrorInvalidValue;
    switch (waves_x) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_collide<1, true>, 64, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_collide<2, true>, 128, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_collide<4, true>, 256, 0); break;
    default: return 0;
    }
    return e == hipSuccess ? cus * per_cu : 0;
}

template <bool S>
static hipError_t launch_batch_rows_t(const BatchTiles& T, const CaseRec* cases, int parity, const int* active,
                                      int waves_x, hipStream_t st)
{
    if (T.n_rows > 0) {   // pieces: one per wave
        const unsigned n = (unsigned)T.n_rows;
        switch (waves_x) {
        case 1:
            hipLaunchKernelGGL((k_batch_rows<1, S>), dim3(n), dim3(64), 0, st, cases, T.rows, T.n_rows, parity,
                               active);
            break;
        case 2:
            hipLaunchKernelGGL((k_batch_rows<2, S>), dim3((n + 1) / 2), dim3(128), 0, st, cases, T.rows, T.n_rows,
                               parity, active);
            break;
        case 4:
            hipLaunchKernelGGL((k_batch_rows<4, S>), dim3((n + 3) / 4), dim3(256), 0, st, cases, T.rows, T.n_rows,
                               parity, active);
            break;
        default:
            return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_batch_rows(const BatchTiles& T, const CaseRec* cases, int parity, const int* active, int waves_x,
                             bool sample, hipStream_t st)
{
    if (parity & ~1) return hipErrorInvalidValue;
    return sample ? launch_batch_rows_t<true>(T, cases, parity, active, waves_x, st)
                  : launch_batch_rows_t<false>(T, cases, parity, active, waves_x, st);
}

// the walked plain tiles (one launch per strip width; persistent when the
// grid is smaller than the tile count), then the general pieces
template <bool S>
static hipError_t launch_batch_general_t(const BatchTiles& T, const CaseRec* cases, int parity, const int* active,
                                         int waves_x, hipStream_t st)
{
    auto runs = [&](int n, int grid, int& per_wg) {
        grid = n > 0 ? std::min(grid, n) : 0;
        per_wg = grid > 0 ? (n + grid - 1) / grid : 0;
        return per_wg > 0 ? (n + per_wg - 1) / per_wg : 0;
    };
    int pw = 0, pt = 0;
    const int gw = runs(T.n_wide, T.grid_wide, pw);
    const int gt = runs(T.n_tail, T.grid_tail, pt);
    if (gt > 0)
        hipLaunchKernelGGL((k_batch_collide<1, true, S>), dim3(gt), dim3(64), 0, st, cases, T.tail, T.n_tail, pt,
                           parity, active);
    if (gw > 0) {
        switch (waves_x) {
        case 1:
            hipLaunchKernelGGL((k_batch_collide<1, true, S>), dim3(gw), dim3(64), 0, st, cases, T.wide, T.n_wide, pw,
                               parity, active);
            break;
        case 2:
            hipLaunchKernelGGL((k_batch_collide<2, true, S>), dim3(gw), dim3(128), 0, st, cases, T.wide, T.n_wide, pw,
                               parity, active);
            break;
        case 4:
            hipLaunchKernelGGL((k_batch_collide<4, true, S>), dim3(gw), dim3(256), 0, st, cases, T.wide, T.n_wide, pw,
                               parity, active);
            break;
        default:
            return hipErrorInvalidValue;
        }
    }
    if (T.n_gen > 0)
        hipLaunchKernelGGL((k_batch_collide<1, false, S>), dim3(T.n_gen), dim3(64), 0, st, cases, T.gen, T.n_gen, 1,
                           parity, active);
    return hipGetLastError();
}

hipError_t launch_batch_general(const BatchTiles& T, const CaseRec* cases, int parity, const int* active,
                                int waves_x, bool sample, hipStream_t st)
{
    if (parity & ~1) return hipErrorInvalidValue;
    return sample ? launch_batch_general_t<true>(T, cases, parity, active, waves_x, st)
                  : launch_batch_general_t<false>(T, cases, parity, active, waves_x, st);
}

hipError_t launch_batch_collide(const BatchTiles& T, const CaseRec* cases, int parity, const int* active,
                                int waves_x, bool sample, hipStream_t st)
{
    const hipError_t e = launch_batch_rows(T, cases, parity, active, waves_x, sample, st);
    return e != hipSuccess ? e : launch_batch_general(T, cases, parity, active, waves_x, sample, st);
}

hipError_t launch_batch_tick(int64_t* t_dev, CaseRec* cases, int n_cases, const int* active, hipStream_t st)
{
    hipLaunchKernelGGL(k_batch_tick, dim3(1), dim3(1024), 0, st, t_dev, cases, n_cases, active);
    return hipGetLastError();
}

hipError_t launch_batch_set_time(int64_t* t_dev, int64_t t, CaseRec* cases, int n_cases, hipStream_t st)
{
    hipLaunchKernelGGL(k_batch_set_time, dim3(1), dim3(1024), 0, st, t_dev, t, cases, n_cases);
    return hipGetLastError();
}

hipError_t launch_batch_sample_begin(const CaseRec* cases, int n_cases, size_t max_parts, hipStream_t st)
{
    if (n_cases <= 0) return hipSuccess;
    if (n_cases > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_batch_sample_clear, dim3((unsigned)((max_parts + 255) / 256), n_cases), dim3(256), 0, st,
                       cases);
    return hipGetLastError();
}

hipError_t launch_batch_sample_end(const CaseRec* cases, int n_cases, int max_ny, const int64_t* t_dev, int64_t* n_rec,
                                   int* active, hipStream_t st)
{
    if (n_cases <= 0) return hipSuccess;
    if (n_cases > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_batch_sample_rows, dim3((max_ny + 255) / 256, n_cases), dim3(256), 0, st, cases, active);
    hipLaunchKernelGGL(k_batch_diag_finish, dim3(n_cases), dim3(DIAG_THREADS), 0, st, cases, t_dev, n_rec, active);
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

hipError_t launch_state_io(const KParams& P, float* A, const uint8_t* wall, float* f_ext, float* g_ext, int to_ext,
                           hipStream_t st)
{
    const dim3 b(256);
    if (f_ext)
        hipLaunchKernelGGL(k_state_io, dim3((P.nx + 255) / 256, P.ny, 9), b, 0, st, P, A, wall, f_ext, to_ext, 1);
    if (g_ext)
        hipLaunchKernelGGL(k_state_io, dim3((P.nx + 255) / 256, P.ny, 5), b, 0, st, P, A, wall, g_ext, to_ext, 0);
    return hipGetLastError();
}

hipError_t launch_diag(const KParams& P, const float* A, const uint8_t* wall, const double* phi, int row0,
                       int a_min, int band, int64_t step, DiagRow* rows, SampleRec* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_diag_rows, dim3(P.ny), dim3(DIAG_THREADS), 0, st, P, A, wall, phi, row0, rows);
    hipLaunchKernelGGL(k_diag_finish, dim3(1), dim3(DIAG_THREADS), 0, st, P.ny, row0, a_min, band, step, rows, out);
    return hipGetLastError();
}

hipError_t launch_sample_finish(const DiagRow* parts, int n_sub, int ny, int row0, int a_min, int band,
                                int64_t step, DiagRow* rows, SampleRec* out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sample_rows, dim3((unsigned)((ny + 255) / 256)), dim3(256), 0, st, parts, n_sub, ny, rows);
    hipLaunchKernelGGL(k_diag_finish, dim3(1), dim3(DIAG_THREADS), 0, st, ny, row0, a_min, band, step, rows, out);
    return hipGetLastError();
}

} // namespace ij
