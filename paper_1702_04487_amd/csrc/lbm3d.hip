// Three-dimensional form of the binary-fluid update (D3Q19 f, D3Q7 g) for
// round nozzles, and its C ABI (ij3_* in inkjet_lbm.h).
//
// Method: Methods, Eqs. 1-10 (mean density n, order parameter phi, BGK with
// the forcing of Eq. 4, the modified streaming of Eq. 8), the pulse of
// Results, "Actuation modeling" (Fig. 1), and the wetting walls of
// "Reproducing the experiment", written on three-dimensional lattices.
//
// Storage: two buffers of 26 float populations per node (f_0..f_18, then
// g_0..g_6) followed by one 16-bit plane.  The populations of one lattice
// row (fixed y, z) are 26 consecutive rows of pitch floats (nx rounded up to
// 64): population i of node x of row r = y*nz + z sits at (r*26 + i)*pitch +
// x, so a workgroup's 26 streams lie in one contiguous region of memory.
// The 16-bit plane, [y][z][pitch], holds the bfloat16 remainder of the rest
// population g_0 - float(g_0): g_0 carries +-phi*, and its float rounding
// alone, accumulated over the steps, would move phi and through mu the
// velocity field by more than the float rounding of every other population
// together.  The g_0 update is formed in double for the same reason.  The
// wall mask and phi are plain [y][z][pitch] arrays (node k = r*pitch + x).
// f is stored shifted by w_i n0 (the equilibrium of the mean density at
// rest), so that float carries the deviations that the collision works on.
// phi, its wetting ghosts, the stencils and mu are double precision.
//
// One step is two launches: the ghost phi of the solid nodes within reach of
// fluid (from their fluid neighbours' g), and one collide-and-push launch
// whose workgroups build the phi of their tile and its halo from g in LDS (a
// node collides f and g and pushes each post-collision population to its
// destination, or back into its own opposite slot at a solid).  With open
// rows a third launch copies the incoming populations of rows 0 and ny-1.
// phi is written to memory only at ghost nodes, and as a whole field only
// for readback (moments, diagnostics, the initial state).  HBM-bound: 26
// floats read and written per fluid node (208 B), plus the halo's g and the
// destinations' old g (mostly cache hits).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "bf16_split.h"
#include "checkpoint.h"
#include "inkjet_lbm.h"

namespace ij3 {

using ij_bf16::bf16_to_float;
using ij_bf16::split;

constexpr int Q = 19, QG = 7, NPL = Q + QG;
constexpr int CX[Q] = {0, 1, 0, -1, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 1, 0, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, -1, 1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1};
constexpr int OPP[Q] = {0, 3, 4, 1, 2, 6, 5, 9, 10, 7, 8, 13, 14, 11, 12, 17, 18, 15, 16};
// lattice weights: 1/3 at rest, 1/18 on the axes, 1/36 on the edges
__host__ __device__ constexpr float wt(int i) { return i == 0 ? 1.f / 3.f : (i < 7 ? 1.f / 18.f : 1.f / 36.f); }
__host__ __device__ constexpr double wtd(int i) { return i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0); }

constexpr int BX = 128, BZ = 4;   // workgroup: 128 x-lanes (two waves) by 4 z-rows

struct K3 {
    int nx, ny, nz, pitch;
    size_t plane;     // nodes, row padding included: ny * nz * pitch
    int bc_open, force_rows;
    double phi_star, n0, beta4, kappa, q, inv_tau_phid, gammad;
    double wet[3];    // ghost offsets 2 Omega phi* / W of wall classes 1, 2
    float omq, inv_tau_phi, gamma, inv_2q, tau_ink, tau_amb, n0f, inv_phi_star;
};

__device__ __forceinline__ int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }
// population i (0..18 f, 19..25 g) of node k (column x)
__device__ __forceinline__ size_t pidx(const K3& P, size_t k, int x, int i)
{
    return (k - (size_t)x) * NPL + (size_t)i * P.pitch + (size_t)x;
}
__device__ __forceinline__ size_t nodek(const K3& P, int x, int y, int z)
{
    return ((size_t)y * P.nz + z) * P.pitch + x;
}
// the g_0 remainder plane of a buffer, indexed by node k
__device__ __forceinline__ const uint16_t* lo3(const K3& P, const float* A)
{
    return reinterpret_cast<const uint16_t*>(A + (size_t)NPL * P.plane);
}
__device__ __forceinline__ uint16_t* lo3(const K3& P, float* A)
{
    return reinterpret_cast<uint16_t*>(A + (size_t)NPL * P.plane);
}

// row of a stencil neighbour: periodic, or mirrored onto the open row
__device__ __forceinline__ int stencil_row(const K3& P, int y)
{
    if (y >= 0 && y < P.ny) return y;
    if (P.bc_open) return y < 0 ? 0 : P.ny - 1;
    return wrapi(y, P.ny);
}

// phi = sum g of a fluid node (Eq. 9's zeroth moment), in double, with the
// remainder of g_0; every kernel that needs phi of a node forms it here
__device__ __forceinline__ double phi_of_g(const K3& P, const float* __restrict__ A, size_t k, int x)
{
    double s = 0.0;
#pragma unroll
    for (int i = 1; i < QG; ++i) s += (double)A[pidx(P, k, x, Q + i)];
    return (s + (double)bf16_to_float(lo3(P, A)[k])) + (double)A[pidx(P, k, x, Q)];
}

// phi = sum_i g_i at fluid nodes
__global__ __launch_bounds__(BX* BZ) void k3_phi(K3 P, const float* __restrict__ A,
                                                 const uint8_t* __restrict__ wall, double* __restrict__ phi)
{
    const int x = blockIdx.x * BX + threadIdx.x, z = blockIdx.y * BZ + threadIdx.y, y = blockIdx.z;
    if (x >= P.nx || z >= P.nz) return;
    const size_t k = nodek(P, x, y, z);
    if (wall[k]) return;
    phi[k] = phi_of_g(P, A, k, x);
}

// ghost phi of each listed solid node (x, y, z, wall class): the mean of its
// fluid axis neighbours, or of its fluid edge neighbours if it has none,
// plus the wetting offset of its class
__global__ void k3_ghost(K3 P, const int4* __restrict__ list, int n, const uint8_t* __restrict__ wall,
                         double* __restrict__ phi)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int4 L = list[e];
    double sum = 0.0;
    int cnt = 0;
    for (int pass = 0; pass < 2 && cnt == 0; ++pass) {
        const int i0 = pass == 0 ? 1 : 7, i1 = pass == 0 ? 7 : Q;
        for (int i = i0; i < i1; ++i) {
            const int yn = L.y + CY[i];
            if (yn < 0 || yn >= P.ny) {
                if (P.bc_open) continue;
            }
            const size_t kn = nodek(P, wrapi(L.x + CX[i], P.nx), wrapi(yn, P.ny), wrapi(L.z + CZ[i], P.nz));
            if (wall[kn]) continue;
            sum += phi[kn];
            ++cnt;
        }
    }
    phi[nodek(P, L.x, L.y, L.z)] = cnt ? sum / cnt + P.wet[L.w] : 0.0;
}

// the ghost of each listed solid node as k3_ghost computes it, with the
// fluid neighbours' phi summed from their g
__global__ void k3_ghost_g(K3 P, const int4* __restrict__ list, int n, const uint8_t* __restrict__ wall,
                           const float* __restrict__ A, double* __restrict__ phi)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int4 L = list[e];
    double sum = 0.0;
    int cnt = 0;
    for (int pass = 0; pass < 2 && cnt == 0; ++pass) {
        const int i0 = pass == 0 ? 1 : 7, i1 = pass == 0 ? 7 : Q;
        for (int i = i0; i < i1; ++i) {
            const int yn = L.y + CY[i];
            if (yn < 0 || yn >= P.ny) {
                if (P.bc_open) continue;
            }
            const int xn = wrapi(L.x + CX[i], P.nx);
            const size_t kn = nodek(P, xn, wrapi(yn, P.ny), wrapi(L.z + CZ[i], P.nz));
            if (wall[kn]) continue;
            sum += phi_of_g(P, A, kn, xn);
            ++cnt;
        }
    }
    phi[nodek(P, L.x, L.y, L.z)] = cnt ? sum / cnt + P.wet[L.w] : 0.0;
}

// phi, its gradient and Laplacian (isotropic D3Q19 sums) and mu at a fluid node
struct Phi3 {
    double phi, mu, gx, gy, gz;
};
__device__ __forceinline__ Phi3 phi_fields(const K3& P, const double* __restrict__ phi, int x, int y, int z)
{
    Phi3 r;
    const double ph = phi[nodek(P, x, y, z)];
    double sx = 0.0, sy = 0.0, sz = 0.0, sl = 0.0;
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const double pn = phi[nodek(P, wrapi(x + CX[i], P.nx), stencil_row(P, y + CY[i]), wrapi(z + CZ[i], P.nz))];
        const double wp = wtd(i) * pn;
        if (CX[i]) sx += CX[i] * wp;
        if (CY[i]) sy += CY[i] * wp;
        if (CZ[i]) sz += CZ[i] * wp;
        sl += wtd(i) * (pn - ph);
    }
    r.phi = ph;
    r.gx = 3.0 * sx;
    r.gy = 3.0 * sy;
    r.gz = 3.0 * sz;
    r.mu = P.beta4 * ph * ((ph - P.phi_star) * (ph + P.phi_star)) - P.kappa * (6.0 * sl);
    return r;
}

// a load at a uniform base plus a 32-bit byte offset per lane (one address
// register per lane instead of a 64-bit pair)
__device__ __forceinline__ float ld_at(const float* __restrict__ base, unsigned bo)
{
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) + bo);
}

// collide every fluid node and push its populations (Eqs. 3, 4, 8).
// The workgroup first stages phi (sum g at fluid nodes, the ghost at solid
// ones) and the wall bytes of its tile and a one-node halo (three y-slices)
// in LDS: the stencil and the destination checks then read LDS instead of
// issuing 36 scattered loads per node.
constexpr int HX = BX + 2, HZ = BZ + 2, HN = 3 * HZ * HX;
constexpr uint8_t kBeyond = 255;   // LDS wall byte of a node beyond an open row

// a staging coordinate one step outside [0, n) wrapped back; coordinates
// further out belong to no fluid node's stencil (the unused tail of a
// partial tile) and are clamped in bounds
__device__ __forceinline__ int wrap_stage(int a, int n)
{
    a = a < 0 ? a + n : (a >= n ? a - n : a);
    return a < n ? a : n - 1;
}

// (six waves per SIMD, three workgroups per CU: the register budget this asks
// for keeps the destinations' old g loaded early at the cost of a few spilled
// registers, measured faster than five waves without spills)
__global__ __launch_bounds__(BX* BZ) __attribute__((amdgpu_waves_per_eu(6))) void k3_collide(K3 P, const float* __restrict__ A, float* __restrict__ B,
                                                     const uint8_t* __restrict__ wall,
                                                     const double* __restrict__ phi, float fb)
{
    __shared__ double s_phi[HN];
    __shared__ uint8_t s_w[HN];
    int bx = blockIdx.x, bz = blockIdx.y, y = blockIdx.z;
    {
        // workgroups b and b + 8 (one XCD, one after the other) take the two
        // tiles of an x-pair, so the x-halo lines they share meet in one L2
        const unsigned nxt = gridDim.x, nzt = gridDim.y;
        const unsigned b = blockIdx.x + nxt * (blockIdx.y + nzt * blockIdx.z);
        const unsigned total = nxt * nzt * gridDim.z;
        if (nxt == 2 && (total & 15) == 0) {
            const unsigned t = (b >> 4) * 16 + (b & 7) * 2 + ((b >> 3) & 1);
            bx = (int)(t % nxt);
            const unsigned r = t / nxt;
            bz = (int)(r % nzt);
            y = (int)(r / nzt);
        }
    }
    const int x0 = bx * BX, z0 = bz * BZ;
    const int tid = threadIdx.y * BX + threadIdx.x;
    const size_t rlen = (size_t)NPL * P.pitch;   // floats of one lattice row's 26 populations
    const uint16_t* loA = lo3(P, A);
    // the halo tile: entry e = (slice dy, z-row ez, column ex), x = x0 - 1 + ex.
    // Each thread takes entries tid, tid + 512, ...: first the coordinates
    // and wall bytes of all of them, then the loads of all of them (the g
    // rows of a fluid entry, the ghost phi of a solid one), then the sums,
    // so that the loads of its entries are in flight together
    constexpr int NS = (HN + BX * BZ - 1) / (BX * BZ);
    size_t rsk[NS];
    int xk[NS];
    uint8_t wk[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const int e = tid + k * BX * BZ;
        if (e >= HN) break;
        const int hr = e / HX, ex = e - hr * HX;
        const int dy = hr / HZ, ez = hr - dy * HZ;
        const int yy = y - 1 + dy;
        const int zz = wrap_stage(z0 - 1 + ez, P.nz);
        const int xx = wrap_stage(x0 - 1 + ex, P.nx);
        const bool beyond = (yy < 0 || yy >= P.ny) && P.bc_open;
        rsk[k] = (size_t)((unsigned)stencil_row(P, yy) * (unsigned)P.nz + (unsigned)zz);
        xk[k] = xx;
        wk[k] = wall[rsk[k] * P.pitch + xx];
        // short of an open edge the stencil row is the node's own row (wrapped
        // when periodic), so its wall byte is the destination check's too
        s_w[e] = beyond ? kBeyond : wk[k];
    }
    float gk[NS][QG];
    uint16_t lk[NS];
    double pk[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        if (tid + k * BX * BZ >= HN) break;
        if (wk[k]) {
            pk[k] = phi[rsk[k] * P.pitch + xk[k]];
        } else {
            const float* row = A + rsk[k] * rlen;
            const unsigned xo = (unsigned)xk[k] << 2, pb = (unsigned)P.pitch << 2;
#pragma unroll
            for (int i = 0; i < QG; ++i) gk[k][i] = ld_at(row, (unsigned)(Q + i) * pb + xo);
            lk[k] = loA[rsk[k] * P.pitch + xk[k]];
        }
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const int e = tid + k * BX * BZ;
        if (e >= HN) break;
        if (wk[k]) {
            s_phi[e] = pk[k];
        } else {
            // the order of phi_of_g: g_1 .. g_6, the remainder, then g_0
            double sum = 0.0;
#pragma unroll
            for (int i = 1; i < QG; ++i) sum += (double)gk[k][i];
            s_phi[e] = (sum + (double)bf16_to_float(lk[k])) + (double)gk[k][0];
        }
    }
    __syncthreads();
    // a wave's 64 lanes lie along x at one z: the node's lattice row, and
    // with it every row address below, is uniform over the wave
    const int zl = __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    const int x = x0 + threadIdx.x, z = z0 + zl;
    const int lc = (HZ + zl + 1) * HX + threadIdx.x + 1;   // LDS index of this node (middle slice)
    if (x >= P.nx || z >= P.nz || s_w[lc]) return;
    const size_t k = nodek(P, x, y, z);
    const size_t r0 = (size_t)((unsigned)y * (unsigned)P.nz + (unsigned)z);
    const float* Ar = A + r0 * rlen;
    const unsigned pb = (unsigned)P.pitch << 2, xo = (unsigned)x << 2;   // byte offsets within the row
    float f[Q], g[QG];
#pragma unroll
    for (int i = 0; i < Q; ++i) f[i] = ld_at(Ar, (unsigned)i * pb + xo);
#pragma unroll
    for (int i = 0; i < QG; ++i) g[i] = ld_at(Ar, (unsigned)(Q + i) * pb + xo);
    // the old g_i at each destination (Eq. 8 keeps (1-q) of it), loaded with
    // the node's own populations; every address is in the lattice (a solid
    // destination or one beyond an open row is loaded and not used)
    float gd[QG];
#pragma unroll
    for (int i = 1; i < QG; ++i) {
        const int xd = wrapi(x + CX[i], P.nx);
        gd[i] = A[pidx(P, nodek(P, xd, wrapi(y + CY[i], P.ny), wrapi(z + CZ[i], P.nz)), xd, Q + i)];
    }

    auto lds = [&](int i) { return lc + CY[i] * (HZ * HX) + CZ[i] * HX + CX[i]; };
    Phi3 ph;
    {
        const double p0 = s_phi[lc];
        double sx = 0.0, sy = 0.0, sz = 0.0, sl = 0.0;
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const double pn = s_phi[lds(i)];
            const double wp = wtd(i) * pn;
            if (CX[i]) sx += CX[i] * wp;
            if (CY[i]) sy += CY[i] * wp;
            if (CZ[i]) sz += CZ[i] * wp;
            sl += wtd(i) * (pn - p0);
        }
        ph.phi = p0;
        ph.gx = 3.0 * sx;
        ph.gy = 3.0 * sy;
        ph.gz = 3.0 * sz;
        ph.mu = P.beta4 * p0 * ((p0 - P.phi_star) * (p0 + P.phi_star)) - P.kappa * (6.0 * sl);
    }
    double Fx = ph.mu * ph.gx, Fy = ph.mu * ph.gy, Fz = ph.mu * ph.gz;
    if (y < P.force_rows) Fy += (double)fb;
    const float fx = (float)Fx, fy = (float)Fy, fz = (float)Fz;

    // moments of the shifted populations: dn = n - n0, j = sum c f
    float dn = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        dn += f[i];
        if (CX[i]) jx += CX[i] * f[i];
        if (CY[i]) jy += CY[i] * f[i];
        if (CZ[i]) jz += CZ[i] * f[i];
    }
    const float n = P.n0f + dn;
    const float inv_n = 1.f / n;
    // j and -F/2 nearly cancel at a resting interface: add them in double
    const float ux = (float)((double)jx + 0.5 * Fx) * inv_n, uy = (float)((double)jy + 0.5 * Fy) * inv_n,
                uz = (float)((double)jz + 0.5 * Fz) * inv_n;
    const float phif = (float)ph.phi;
    float C = (phif * P.inv_phi_star + 1.f) * 0.5f;
    C = fminf(fmaxf(C, 0.f), 1.f);
    const float tau = P.tau_amb + C * (P.tau_ink - P.tau_amb);
    const float inv_tau = 1.f / tau;
    const float pref = 1.f - 0.5f * inv_tau;
    const float pm = (float)(ph.phi * ph.mu);
    const float uu = ux * ux + uy * uy + uz * uz;
    const float uF = ux * fx + uy * fy + uz * fz;

    // the destination of each population; a solid destination bounces back
    // into the node's own opposite slot; beyond an open row it is dropped
    // (the open-row launch refills those populations)
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const float cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
        const float cF = CX[i] * fx + CY[i] * fy + CZ[i] * fz;
        const float a = i == 0 ? dn - 6.f * pm : dn + 3.f * pm;   // A_i - n0
        // the weight is applied in double: in float 1/3 rounds 4x more
        // (relatively) than 1/18 and 1/36, and the equilibrium would then
        // create mass and momentum in proportion to phi mu at interfaces
        const float feq =
            (float)(wtd(i) * ((double)a + (double)n * (double)(3.f * cu + 4.5f * cu * cu - 1.5f * uu)));
        const float S = pref * wt(i) * 3.f * ((cF - uF) + 3.f * cu * cF);
        const float fs = f[i] + (feq - f[i]) * inv_tau + S;
        if (i == 0) {
            B[pidx(P, k, x, 0)] = fs;
            continue;
        }
        const uint8_t wd = s_w[lds(i)];
        if (wd == kBeyond) continue;
        if (wd) {
            B[pidx(P, k, x, OPP[i])] = fs;
        } else {
            const int xd = wrapi(x + CX[i], P.nx);
            B[pidx(P, nodek(P, xd, wrapi(y + CY[i], P.ny), wrapi(z + CZ[i], P.nz)), xd, i)] = fs;
        }
    }

    // g: equilibrium of Eqs. 9-10 on D3Q7, h = g* - (1-q) g, and the
    // destination keeps (1-q) of its own old value (Eq. 8).  The rest
    // population stays: its new value h_0 + (1-q) g_0 = g_0 + (g_eq_0 -
    // g_0)/tau_phi, with g_eq_0 - g_0 = (g_1 + .. + g_6) - 3 Gamma mu, is
    // formed in double and stored as float plus remainder.
    {
        double sg = 0.0;
#pragma unroll
        for (int i = 1; i < QG; ++i) sg += (double)g[i];
        const double G = ((double)g[0] + (double)bf16_to_float(lo3(P, A)[k])) +
                         P.inv_tau_phid * (sg - 3.0 * P.gammad * ph.mu);
        float hi;
        uint16_t lo;
        split(G, hi, lo);
        B[pidx(P, k, x, Q)] = hi;
        lo3(P, B)[k] = lo;
    }
    const float gmu = P.gamma * (float)ph.mu;
#pragma unroll
    for (int i = 1; i < QG; ++i) {
        const float cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
        const float geq = 0.5f * gmu + phif * cu * P.inv_2q;
        const float gs = g[i] + (geq - g[i]) * P.inv_tau_phi;
        const float h = gs - P.omq * g[i];
        const uint8_t wd = s_w[lds(i)];
        if (wd == kBeyond) continue;
        if (wd) {
            B[pidx(P, k, x, Q + OPP[i])] = h + P.omq * g[OPP[i]];
        } else {
            const int xd = wrapi(x + CX[i], P.nx);
            const size_t pd = pidx(P, nodek(P, xd, wrapi(y + CY[i], P.ny), wrapi(z + CZ[i], P.nz)), xd, Q + i);
            B[pd] = h + P.omq * gd[i];
        }
    }
}

// open rows: the incoming populations of rows 0 and ny-1 from the adjacent
// interior row ("fully developed")
__global__ void k3_open(K3 P, float* __restrict__ B, const uint8_t* __restrict__ wall)
{
    const int x = blockIdx.x * BX + threadIdx.x, z = blockIdx.y * BZ + threadIdx.y;
    if (x >= P.nx || z >= P.nz) return;
    const bool top = blockIdx.z == 1;
    const size_t k = nodek(P, x, top ? P.ny - 1 : 0, z);
    const size_t kin = nodek(P, x, top ? P.ny - 2 : 1, z);
    if (wall[k]) return;
#pragma unroll
    for (int i = 0; i < Q; ++i)
        if (top ? CY[i] < 0 : CY[i] > 0) {
            B[pidx(P, k, x, i)] = B[pidx(P, kin, x, i)];
            if (i < QG) B[pidx(P, k, x, Q + i)] = B[pidx(P, kin, x, Q + i)];
        }
}

// initial phi: from phi itself or from a signed distance (tanh profile)
__global__ void k3_set_phi(K3 P, const float* __restrict__ src, int from_distance, double inv_w,
                           const uint8_t* __restrict__ wall, double* __restrict__ phi)
{
    const int x = blockIdx.x * BX + threadIdx.x, z = blockIdx.y * BZ + threadIdx.y, y = blockIdx.z;
    if (x >= P.nx || z >= P.nz) return;
    const size_t k = nodek(P, x, y, z);
    if (wall[k]) return;
    const double v = (double)src[((size_t)y * P.nz + z) * P.nx + x];
    phi[k] = from_distance ? P.phi_star * tanh(2.0 * v * inv_w) : v;
}

// f = f_eq(n0, u), g = g_eq(phi, u) with mu of the initial phi
__global__ void k3_init_eq(K3 P, float* __restrict__ A, const uint8_t* __restrict__ wall,
                           const double* __restrict__ phi, const float* __restrict__ uxs,
                           const float* __restrict__ uys, const float* __restrict__ uzs)
{
    const int x = blockIdx.x * BX + threadIdx.x, z = blockIdx.y * BZ + threadIdx.y, y = blockIdx.z;
    if (x >= P.nx || z >= P.nz) return;
    const size_t k = nodek(P, x, y, z);
    if (wall[k]) {
        for (int i = 0; i < NPL; ++i) A[pidx(P, k, x, i)] = 0.f;
        lo3(P, A)[k] = 0;
        return;
    }
    const size_t ke = ((size_t)y * P.nz + z) * P.nx + x;
    const float ux = uxs ? uxs[ke] : 0.f, uy = uys ? uys[ke] : 0.f, uz = uzs ? uzs[ke] : 0.f;
    const Phi3 ph = phi_fields(P, phi, x, y, z);
    const float pm = (float)(ph.phi * ph.mu), n = P.n0f, uu = ux * ux + uy * uy + uz * uz;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const float cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
        const float a = i == 0 ? -6.f * pm : 3.f * pm;
        A[pidx(P, k, x, i)] = (float)(wtd(i) * ((double)a + (double)n * (double)(3.f * cu + 4.5f * cu * cu - 1.5f * uu)));
    }
    const float gmu = P.gamma * (float)ph.mu, phif = (float)ph.phi;
    float g0;
    uint16_t g0lo;
    split(ph.phi - 3.0 * P.gammad * ph.mu, g0, g0lo);
    A[pidx(P, k, x, Q)] = g0;
    lo3(P, A)[k] = g0lo;
#pragma unroll
    for (int i = 1; i < QG; ++i) {
        const float cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
        A[pidx(P, k, x, Q + i)] = 0.5f * gmu + phif * cu * P.inv_2q;
    }
}

// n, phi, u of a fluid node (current state; needs phi and its ghosts)
struct Mac3 {
    float n, phi, ux, uy, uz, jx, jy, jz;
};
__device__ __forceinline__ Mac3 node_macro(const K3& P, const float* __restrict__ A,
                                           const double* __restrict__ phi, int x, int y, int z, float fb)
{
    const size_t k = nodek(P, x, y, z);
    const Phi3 ph = phi_fields(P, phi, x, y, z);
    double Fx = ph.mu * ph.gx, Fy = ph.mu * ph.gy, Fz = ph.mu * ph.gz;
    if (y < P.force_rows) Fy += (double)fb;
    float dn = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const float f = A[pidx(P, k, x, i)];
        dn += f;
        if (CX[i]) jx += CX[i] * f;
        if (CY[i]) jy += CY[i] * f;
        if (CZ[i]) jz += CZ[i] * f;
    }
    Mac3 m;
    m.n = P.n0f + dn;
    m.phi = (float)ph.phi;
    const float inv_n = 1.f / m.n;
    m.ux = (float)((double)jx + 0.5 * Fx) * inv_n;
    m.uy = (float)((double)jy + 0.5 * Fy) * inv_n;
    m.uz = (float)((double)jz + 0.5 * Fz) * inv_n;
    m.jx = jx;
    m.jy = jy;
    m.jz = jz;
    return m;
}

__global__ void k3_moments(K3 P, const float* __restrict__ A, const uint8_t* __restrict__ wall,
                           const double* __restrict__ phi, float fb, float* __restrict__ on,
                           float* __restrict__ ophi, float* __restrict__ oux, float* __restrict__ ouy,
                           float* __restrict__ ouz)
{
    const int x = blockIdx.x * BX + threadIdx.x, z = blockIdx.y * BZ + threadIdx.y, y = blockIdx.z;
    if (x >= P.nx || z >= P.nz) return;
    const size_t ke = ((size_t)y * P.nz + z) * P.nx + x;
    Mac3 m{};
    if (!wall[nodek(P, x, y, z)]) m = node_macro(P, A, phi, x, y, z, fb);
    if (on) on[ke] = m.n;
    if (ophi) ophi[ke] = m.phi;
    if (oux) oux[ke] = m.ux;
    if (ouy) ouy[ke] = m.uy;
    if (ouz) ouz[ke] = m.uz;
}

// distributions <-> caller arrays [i][ny][nz][nx]: the f planes (is_f, the
// stored shift removed) or the g planes (g_0 read as float(hi + remainder);
// writing g_0 clears its remainder)
__global__ void k3_state_io(K3 P, float* __restrict__ A, const uint8_t* __restrict__ wall,
                            float* __restrict__ ext, int to_ext, int is_f)
{
    const int x = blockIdx.x * BX + threadIdx.x, z = blockIdx.y * BZ + threadIdx.y, y = blockIdx.z;
    if (x >= P.nx || z >= P.nz) return;
    const size_t k = nodek(P, x, y, z);
    const size_t ne = (size_t)P.ny * P.nz * P.nx;
    const size_t ke = ((size_t)y * P.nz + z) * P.nx + x;
    const bool solid = wall[k] != 0;
    const int nq = is_f ? Q : QG, i0 = is_f ? 0 : Q;
    for (int i = 0; i < nq; ++i) {
        const float shift = is_f ? wt(i) * P.n0f : 0.f;
        const size_t pk = pidx(P, k, x, i0 + i);
        const bool rest_g = !is_f && i == 0;
        if (to_ext)
            ext[i * ne + ke] = solid ? 0.f
                                     : (rest_g ? (float)((double)A[pk] + (double)bf16_to_float(lo3(P, A)[k]))
                                               : A[pk] + shift);
        else if (!solid) {
            A[pk] = ext[i * ne + ke] - shift;
            if (rest_g) lo3(P, A)[k] = 0;
        }
    }
}

// per-row sums of the diagnostics, one workgroup per row (x-z slice),
// reduced in a fixed order
struct Row3 {
    double n, phi, jx, jy, jz, umax, bad, ink, uy;
};
constexpr int DT = 256;
__global__ __launch_bounds__(DT) void k3_rows(K3 P, const float* __restrict__ A, const uint8_t* __restrict__ wall,
                                              const double* __restrict__ phi, float fb, int row0,
                                              Row3* __restrict__ rows)
{
    const int y = blockIdx.x;
    Row3 a{};
    const int nn = P.nx * P.nz;
    for (int e = threadIdx.x; e < nn; e += DT) {
        const int z = e / P.nx, x = e - z * P.nx;
        if (wall[nodek(P, x, y, z)]) continue;
        const Mac3 m = node_macro(P, A, phi, x, y, z, fb);
        a.n += (double)m.n;
        a.phi += (double)m.phi;
        a.jx += (double)m.jx;
        a.jy += (double)m.jy;
        a.jz += (double)m.jz;
        const float um = sqrtf(m.ux * m.ux + m.uy * m.uy + m.uz * m.uz);
        if (!isfinite(m.n) || !isfinite(m.phi) || !isfinite(um) || !(m.n > 0.f))
            a.bad += 1.0;
        else
            a.umax = fmax(a.umax, (double)um);
        if (y >= row0 && m.phi > 0.f) {
            a.ink += 1.0;
            a.uy += (double)m.uy;
        }
    }
    __shared__ Row3 s[DT];
    s[threadIdx.x] = a;
    __syncthreads();
    for (unsigned h = DT / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            Row3& l = s[threadIdx.x];
            const Row3& r = s[threadIdx.x + h];
            l.n += r.n;
            l.phi += r.phi;
            l.jx += r.jx;
            l.jy += r.jy;
            l.jz += r.jz;
            l.umax = fmax(l.umax, r.umax);
            l.bad += r.bad;
            l.ink += r.ink;
            l.uy += r.uy;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) rows[y] = s[0];
}

// Droplet segments of a sample (Results: breakup, drop velocity): the rows
// y >= row0 split into maximal runs with ink; the run that starts at row0 is
// attached to the nozzle, every other run with at least a_min ink nodes is
// a detached drop.  For the largest (the lowest on a tie): its ink count,
// summed u_y, lowest and highest rows, and the mean u_y of its ink in its
// top and bottom `band` rows (head and tail).  One thread, rows in order.
__global__ void k3_drops(const Row3* __restrict__ rows, int ny, int row0, double a_min, int band,
                         ij3_drops* __restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int64_t n_det = 0;
    int ba = -1, bb = -1;
    double bc = 0.0, bu = 0.0;
    int y = row0;
    while (y < ny) {
        if (!(rows[y].ink > 0.0)) {
            ++y;
            continue;
        }
        const int a = y;
        double c = 0.0, u = 0.0;
        while (y < ny && rows[y].ink > 0.0) {
            c += rows[y].ink;
            u += rows[y].uy;
            ++y;
        }
        if (a != row0 && c >= a_min) {
            ++n_det;
            if (c > bc) {
                bc = c;
                bu = u;
                ba = a;
                bb = y;
            }
        }
    }
    ij3_drops d{};
    d.n_detached = n_det;
    d.largest_count = (int64_t)bc;
    d.largest_uy = bu;
    d.largest_bottom = ba;
    d.largest_top = ba >= 0 ? bb - 1 : -1;
    if (ba >= 0) {
        double hc = 0.0, hu = 0.0, tc = 0.0, tu = 0.0;
        for (int r = max(ba, bb - band); r < bb; ++r) {
            hc += rows[r].ink;
            hu += rows[r].uy;
        }
        for (int r = ba; r < min(bb, ba + band); ++r) {
            tc += rows[r].ink;
            tu += rows[r].uy;
        }
        d.head_uy = hu / hc;
        d.tail_uy = tu / tc;
    }
    *out = d;
}

// totals over the rows, summed in row order by one thread
__global__ void k3_finish(const Row3* __restrict__ rows, int ny, double* __restrict__ rec)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int y = 0; y < ny; ++y) {
        const Row3& r = rows[y];
        a[0] += r.n;
        a[1] += r.phi;
        a[2] += r.jx;
        a[3] += r.jy;
        a[4] += r.jz;
        a[5] = fmax(a[5], r.umax);
        a[6] += r.bad;
    }
    for (int i = 0; i < 7; ++i) rec[i] = a[i];
}

}  // namespace ij3

using namespace ij3;

struct ij3_sim {
    ij3_params p{};
    K3 K{};
    float* buf[2] = {nullptr, nullptr};
    uint8_t* wall = nullptr;
    double* phi = nullptr;
    int4* ghost = nullptr;
    int n_ghost = 0;
    Row3* rows = nullptr;
    double* rec = nullptr;     // 7 totals of the last sample
    ij3_drops* drops = nullptr;
    int cur = 0;
    int64_t t = 0;
    bool ready = false;
    uint64_t wall_hash = 0;   // of the host wall mask [ny][nz][nx]
    std::string err;
};

namespace {

std::string g_create_error;

ij_status fail(ij3_sim* s, ij_status code, const std::string& msg)
{
    if (s)
        s->err = msg;
    else
        g_create_error = msg;
    return code;
}

ij_status hip_fail(ij3_sim* s, hipError_t e, const char* what)
{
    return fail(s, IJ_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define IJ3_HIP(s, call)                                    \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return hip_fail(s, e_, #call); \
    } while (0)

double omega_of_theta(double theta_deg)
{
    // inverse of cos(theta) = [(1+Omega)^{3/2} - (1-Omega)^{3/2}] / 2
    const double s = std::sin(theta_deg * M_PI / 180.0);
    const double c = std::cos(std::acos(s * s) / 3.0);
    const double mag = 2.0 * std::sqrt(c * (1.0 - c));
    return theta_deg < 90.0 ? mag : (theta_deg > 90.0 ? -mag : 0.0);
}

double pulse(const ij3_params& p, int64_t t)
{
    const int64_t period = p.t_pos + p.t_neg + p.t_idle;
    int64_t tt = t;
    if (p.periodic_pulse && period > 0) tt = t % period;
    if (tt < p.t_pos) return p.f_pos;
    if (tt < p.t_pos + p.t_neg) return -p.f_neg;
    return 0.0;
}

// one distribution buffer: 26 float populations per node and the 16-bit g_0
// remainder plane
size_t buffer_bytes3(const K3& K) { return K.plane * (NPL * sizeof(float) + sizeof(uint16_t)); }

dim3 grid_of(const K3& K, int zdim) { return dim3((K.nx + BX - 1) / BX, (K.nz + BZ - 1) / BZ, zdim); }

ij_status validate(const ij3_params* p)
{
    if (!p) return fail(nullptr, IJ_ERR_INVALID_ARG, "params is NULL");
    if (p->nx < 3 || p->ny < 3 || p->nz < 3) return fail(nullptr, IJ_ERR_INVALID_ARG, "nx, ny, nz must be >= 3");
    if (p->nx > 65536 || p->ny > 65535 || p->nz > 65535)
        return fail(nullptr, IJ_ERR_INVALID_ARG, "nx <= 65536, ny and nz <= 65535");
    const double pitch = (double)((p->nx + 63) / 64 * 64);
    if (pitch * (double)p->ny * (double)p->nz * NPL >= 4294967296.0 * 8.0)
        return fail(nullptr, IJ_ERR_INVALID_ARG, "lattice too large");
    if (p->bc_y != IJ_BC_PERIODIC && p->bc_y != IJ_BC_OPEN) return fail(nullptr, IJ_ERR_INVALID_ARG, "bad bc_y");
    if (!(p->tau_ink > 0.5) || !(p->tau_amb > 0.5) || !(p->tau_phi > 0.5))
        return fail(nullptr, IJ_ERR_INVALID_ARG, "relaxation times must exceed 1/2");
    if (!(p->width > 0.0) || !(p->rho_amb > 0.0) || !(p->rho_ink > p->rho_amb) || !(p->sigma >= 0.0))
        return fail(nullptr, IJ_ERR_INVALID_ARG, "need width > 0, 0 < rho_amb < rho_ink, sigma >= 0");
    if (!(p->theta_inner >= 0.0 && p->theta_inner <= 180.0) || !(p->theta_outer >= 0.0 && p->theta_outer <= 180.0))
        return fail(nullptr, IJ_ERR_INVALID_ARG, "contact angles must lie in [0, 180]");
    if (p->t_pos < 0 || p->t_neg < 0 || p->t_idle < 0 || p->force_rows < 0)
        return fail(nullptr, IJ_ERR_INVALID_ARG, "negative pulse duration or force_rows");
    return IJ_OK;
}

}  // namespace

extern "C" {

ij_status ij3_create(const ij3_params* p, const uint8_t* wall, ij3_sim** out)
{
    if (!out) return fail(nullptr, IJ_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (ij_status st = validate(p)) return st;
    const int nx = (int)p->nx, ny = (int)p->ny, nz = (int)p->nz;
    const size_t nn = (size_t)nx * ny * nz;
    std::vector<uint8_t> w(nn, 0);
    if (wall) std::memcpy(w.data(), wall, nn);
    auto at = [&](int x, int y, int z) -> uint8_t { return w[((size_t)y * nz + z) * nx + x]; };
    for (size_t k = 0; k < nn; ++k)
        if (w[k] > 2) return fail(nullptr, IJ_ERR_INVALID_ARG, "wall classes are 0, 1, 2");
    if (p->bc_y == IJ_BC_OPEN)
        for (int z = 0; z < nz; ++z)
            for (int x = 0; x < nx; ++x)
                if ((!at(x, 0, z) && at(x, 1, z)) || (!at(x, ny - 1, z) && at(x, ny - 2, z)))
                    return fail(nullptr, IJ_ERR_INVALID_ARG, "a fluid node of an open row needs fluid inside it");

    ij3_sim* s = new ij3_sim();
    s->p = *p;
    s->wall_hash = ij_ckpt::fnv1a(w.data(), w.size());
    K3& K = s->K;
    K.nx = nx;
    K.ny = ny;
    K.nz = nz;
    K.pitch = (nx + 63) / 64 * 64;
    K.plane = (size_t)ny * nz * K.pitch;
    K.bc_open = p->bc_y == IJ_BC_OPEN;
    K.force_rows = (int)std::min<int64_t>(p->force_rows, ny);
    K.phi_star = 0.5 * (p->rho_ink - p->rho_amb);
    K.n0 = 0.5 * (p->rho_ink + p->rho_amb);
    const double ps2 = K.phi_star * K.phi_star;
    K.beta4 = 4.0 * (3.0 * p->sigma / (4.0 * p->width * ps2 * ps2));
    K.kappa = 3.0 * p->sigma * p->width / (8.0 * ps2);
    K.q = 1.0 / (p->tau_phi + 0.5);
    K.wet[0] = 0.0;
    K.wet[1] = 2.0 * omega_of_theta(p->theta_inner) * K.phi_star / p->width;
    K.wet[2] = 2.0 * omega_of_theta(p->theta_outer) * K.phi_star / p->width;
    K.inv_tau_phid = 1.0 / p->tau_phi;
    K.gammad = p->gamma;
    K.omq = (float)(1.0 - K.q);
    K.inv_tau_phi = (float)(1.0 / p->tau_phi);
    K.gamma = (float)p->gamma;
    K.inv_2q = (float)(1.0 / (2.0 * K.q));
    K.tau_ink = (float)p->tau_ink;
    K.tau_amb = (float)p->tau_amb;
    K.n0f = (float)K.n0;
    K.inv_phi_star = (float)(1.0 / K.phi_star);

    // solid nodes within reach of a fluid node's stencil get a ghost
    std::vector<int4> gl;
    for (int y = 0; y < ny; ++y)
        for (int z = 0; z < nz; ++z)
            for (int x = 0; x < nx; ++x) {
                if (!at(x, y, z)) continue;
                bool near = false;
                for (int i = 1; i < Q && !near; ++i) {
                    int yn = y + CY[i];
                    if (yn < 0 || yn >= ny) {
                        if (K.bc_open) continue;
                        yn = (yn + ny) % ny;
                    }
                    near = !at((x + CX[i] + nx) % nx, yn, (z + CZ[i] + nz) % nz);
                }
                if (near) gl.push_back(make_int4(x, y, z, at(x, y, z)));
            }
    s->n_ghost = (int)gl.size();

    const size_t bytes = buffer_bytes3(K);
    std::vector<uint8_t> wp(K.plane, 1);   // pitch padding reads as solid
    for (int y = 0; y < ny; ++y)
        for (int z = 0; z < nz; ++z)
            std::memcpy(&wp[((size_t)y * nz + z) * K.pitch], &w[((size_t)y * nz + z) * nx], nx);
    auto cleanup = [&](ij_status st, const std::string& msg) {
        ij3_destroy(s);
        return fail(nullptr, st, msg);
    };
    if (hipMalloc(&s->buf[0], bytes) != hipSuccess || hipMalloc(&s->buf[1], bytes) != hipSuccess ||
        hipMalloc(&s->wall, K.plane) != hipSuccess || hipMalloc(&s->phi, K.plane * sizeof(double)) != hipSuccess ||
        hipMalloc(&s->rows, (size_t)ny * sizeof(Row3)) != hipSuccess ||
        hipMalloc(&s->rec, 7 * sizeof(double)) != hipSuccess ||
        hipMalloc(&s->drops, sizeof(ij3_drops)) != hipSuccess ||
        (s->n_ghost && hipMalloc(&s->ghost, gl.size() * sizeof(int4)) != hipSuccess))
        return cleanup(IJ_ERR_OOM, "device allocation failed");
    if (hipMemcpy(s->wall, wp.data(), K.plane, hipMemcpyHostToDevice) != hipSuccess ||
        (s->n_ghost && hipMemcpy(s->ghost, gl.data(), gl.size() * sizeof(int4), hipMemcpyHostToDevice) != hipSuccess) ||
        hipMemset(s->buf[0], 0, bytes) != hipSuccess || hipMemset(s->buf[1], 0, bytes) != hipSuccess ||
        hipMemset(s->phi, 0, K.plane * sizeof(double)) != hipSuccess)
        return cleanup(IJ_ERR_DEVICE, "device copy failed");
    *out = s;
    return IJ_OK;
}

void ij3_destroy(ij3_sim* s)
{
    if (!s) return;
    (void)hipFree(s->buf[0]);
    (void)hipFree(s->buf[1]);
    (void)hipFree(s->wall);
    (void)hipFree(s->phi);
    (void)hipFree(s->ghost);
    (void)hipFree(s->rows);
    (void)hipFree(s->rec);
    (void)hipFree(s->drops);
    delete s;
}

const char* ij3_last_error(const ij3_sim* s) { return s ? s->err.c_str() : g_create_error.c_str(); }

}  // extern "C"

namespace {

// phi of the current state and its ghosts
ij_status refresh_phi(ij3_sim* s, hipStream_t st)
{
    const K3& K = s->K;
    hipLaunchKernelGGL(k3_phi, grid_of(K, K.ny), dim3(BX, BZ), 0, st, K, s->buf[s->cur], s->wall, s->phi);
    if (s->n_ghost)
        hipLaunchKernelGGL(k3_ghost, dim3((s->n_ghost + 255) / 256), dim3(256), 0, st, K, s->ghost, s->n_ghost,
                           s->wall, s->phi);
    IJ3_HIP(s, hipGetLastError());
    return IJ_OK;
}

}  // namespace

extern "C" {

ij_status ij3_init(ij3_sim* s, const float* src, int32_t from_distance, const float* ux, const float* uy,
                   const float* uz, void* stream)
{
    if (!s) return fail(nullptr, IJ_ERR_INVALID_ARG, "handle is NULL");
    if (!src) return fail(s, IJ_ERR_INVALID_ARG, "src is NULL");
    hipStream_t st = (hipStream_t)stream;
    const K3& K = s->K;
    s->cur = 0;
    hipLaunchKernelGGL(k3_set_phi, grid_of(K, K.ny), dim3(BX, BZ), 0, st, K, src, from_distance,
                       1.0 / s->p.width, s->wall, s->phi);
    if (s->n_ghost)
        hipLaunchKernelGGL(k3_ghost, dim3((s->n_ghost + 255) / 256), dim3(256), 0, st, K, s->ghost, s->n_ghost,
                           s->wall, s->phi);
    hipLaunchKernelGGL(k3_init_eq, grid_of(K, K.ny), dim3(BX, BZ), 0, st, K, s->buf[0], s->wall, s->phi, ux, uy, uz);
    IJ3_HIP(s, hipGetLastError());
    s->t = 0;
    s->ready = true;
    return IJ_OK;
}

ij_status ij3_step(ij3_sim* s, int64_t nsteps, void* stream)
{
    if (!s) return fail(nullptr, IJ_ERR_INVALID_ARG, "handle is NULL");
    if (!s->ready) return fail(s, IJ_ERR_STATE, "step before init");
    if (nsteps < 0) return fail(s, IJ_ERR_INVALID_ARG, "nsteps < 0");
    hipStream_t st = (hipStream_t)stream;
    const K3& K = s->K;
    for (int64_t n = 0; n < nsteps; ++n) {
        if (s->n_ghost)
            hipLaunchKernelGGL(k3_ghost_g, dim3((s->n_ghost + 255) / 256), dim3(256), 0, st, K, s->ghost,
                               s->n_ghost, s->wall, s->buf[s->cur], s->phi);
        const float fb = (float)pulse(s->p, s->t);
        hipLaunchKernelGGL(k3_collide, grid_of(K, K.ny), dim3(BX, BZ), 0, st, K, s->buf[s->cur],
                           s->buf[1 - s->cur], s->wall, s->phi, fb);
        if (K.bc_open)
            hipLaunchKernelGGL(k3_open, grid_of(K, 2), dim3(BX, BZ), 0, st, K, s->buf[1 - s->cur], s->wall);
        IJ3_HIP(s, hipGetLastError());
        s->cur = 1 - s->cur;
        s->t += 1;
    }
    return IJ_OK;
}

int64_t ij3_time(const ij3_sim* s) { return s ? s->t : -1; }

ij_status ij3_get_moments(ij3_sim* s, float* n, float* phi, float* ux, float* uy, float* uz, void* stream)
{
    if (!s) return fail(nullptr, IJ_ERR_INVALID_ARG, "handle is NULL");
    if (!s->ready) return fail(s, IJ_ERR_STATE, "no state yet");
    hipStream_t st = (hipStream_t)stream;
    if (ij_status e = refresh_phi(s, st)) return e;
    const K3& K = s->K;
    hipLaunchKernelGGL(k3_moments, grid_of(K, K.ny), dim3(BX, BZ), 0, st, K, s->buf[s->cur], s->wall, s->phi,
                       (float)pulse(s->p, s->t), n, phi, ux, uy, uz);
    IJ3_HIP(s, hipGetLastError());
    return IJ_OK;
}

ij_status ij3_get_state(ij3_sim* s, float* f, float* g, void* stream)
{
    if (!s) return fail(nullptr, IJ_ERR_INVALID_ARG, "handle is NULL");
    if (!s->ready) return fail(s, IJ_ERR_STATE, "no state yet");
    if (!f || !g) return fail(s, IJ_ERR_INVALID_ARG, "f and g are required");
    const K3& K = s->K;
    hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(k3_state_io, grid_of(K, K.ny), dim3(BX, BZ), 0, st, K, s->buf[s->cur], s->wall, f, 1, 1);
    hipLaunchKernelGGL(k3_state_io, grid_of(K, K.ny), dim3(BX, BZ), 0, st, K, s->buf[s->cur], s->wall, g, 1, 0);
    IJ3_HIP(s, hipGetLastError());
    return IJ_OK;
}

ij_status ij3_set_state(ij3_sim* s, const float* f, const float* g, int64_t t, void* stream)
{
    if (!s) return fail(nullptr, IJ_ERR_INVALID_ARG, "handle is NULL");
    if (!f || !g || t < 0) return fail(s, IJ_ERR_INVALID_ARG, "f and g are required, t >= 0");
    const K3& K = s->K;
    hipStream_t st = (hipStream_t)stream;
    const size_t bytes = buffer_bytes3(K);
    IJ3_HIP(s, hipMemsetAsync(s->buf[0], 0, bytes, st));
    hipLaunchKernelGGL(k3_state_io, grid_of(K, K.ny), dim3(BX, BZ), 0, st, K, s->buf[0], s->wall,
                       const_cast<float*>(f), 0, 1);
    hipLaunchKernelGGL(k3_state_io, grid_of(K, K.ny), dim3(BX, BZ), 0, st, K, s->buf[0], s->wall,
                       const_cast<float*>(g), 0, 0);
    IJ3_HIP(s, hipGetLastError());
    s->cur = 0;
    s->t = t;
    s->ready = true;
    return IJ_OK;
}

ij_status ij3_state_bytes(const ij3_sim* s, size_t* bytes)
{
    if (!s || !bytes) return IJ_ERR_INVALID_ARG;
    *bytes = sizeof(ij_ckpt::StateHeader) + buffer_bytes3(s->K);
    return IJ_OK;
}

ij_status ij3_save_state(ij3_sim* s, void* blob, size_t bytes, void* stream)
{
    if (!s) return fail(nullptr, IJ_ERR_INVALID_ARG, "handle is NULL");
    if (!blob) return fail(s, IJ_ERR_INVALID_ARG, "blob is NULL");
    if (!s->ready) return fail(s, IJ_ERR_STATE, "no state yet");
    const K3& K = s->K;
    const size_t payload = buffer_bytes3(K);
    if (bytes < sizeof(ij_ckpt::StateHeader) + payload)
        return fail(s, IJ_ERR_INVALID_ARG, "blob smaller than ij3_state_bytes");
    ij_ckpt::StateHeader h{};
    std::memcpy(h.magic, "IJ3STAT1", 8);
    h.nx = K.nx;
    h.ny = K.ny;
    h.nz = K.nz;
    h.pitch = K.pitch;
    h.t = s->t;
    h.wall_hash = s->wall_hash;
    h.payload = payload;
    std::memcpy(blob, &h, sizeof h);
    hipStream_t st = (hipStream_t)stream;
    IJ3_HIP(s, hipMemcpyAsync((char*)blob + sizeof h, s->buf[s->cur], payload, hipMemcpyDeviceToHost, st));
    IJ3_HIP(s, hipStreamSynchronize(st));
    return IJ_OK;
}

ij_status ij3_load_state(ij3_sim* s, const void* blob, size_t bytes, void* stream)
{
    if (!s) return fail(nullptr, IJ_ERR_INVALID_ARG, "handle is NULL");
    if (!blob || bytes < sizeof(ij_ckpt::StateHeader)) return fail(s, IJ_ERR_INVALID_ARG, "blob is NULL or too small");
    ij_ckpt::StateHeader h;
    std::memcpy(&h, blob, sizeof h);
    const K3& K = s->K;
    const size_t payload = buffer_bytes3(K);
    if (std::memcmp(h.magic, "IJ3STAT1", 8) != 0) return fail(s, IJ_ERR_INVALID_ARG, "not a 3-D checkpoint of this library");
    if (h.nx != K.nx || h.ny != K.ny || h.nz != K.nz || h.pitch != K.pitch || h.payload != payload)
        return fail(s, IJ_ERR_INVALID_ARG, "checkpoint of a different lattice size");
    if (h.wall_hash != s->wall_hash) return fail(s, IJ_ERR_INVALID_ARG, "checkpoint of a different wall mask");
    if (h.t < 0) return fail(s, IJ_ERR_INVALID_ARG, "negative step counter");
    if (bytes < sizeof h + payload) return fail(s, IJ_ERR_INVALID_ARG, "blob shorter than its payload");
    hipStream_t st = (hipStream_t)stream;
    IJ3_HIP(s, hipMemcpyAsync(s->buf[0], (const char*)blob + sizeof h, payload, hipMemcpyHostToDevice, st));
    IJ3_HIP(s, hipStreamSynchronize(st));
    s->cur = 0;
    s->t = h.t;
    s->ready = true;
    return IJ_OK;
}

ij_status ij3_sample(ij3_sim* s, int64_t row0, double* rec, int64_t* row_count, double* row_uy, int64_t a_min,
                     int64_t band, ij3_drops* drops, void* stream)
{
    if (!s) return fail(nullptr, IJ_ERR_INVALID_ARG, "handle is NULL");
    if (!s->ready) return fail(s, IJ_ERR_STATE, "no state yet");
    if (!rec) return fail(s, IJ_ERR_INVALID_ARG, "rec is NULL");
    if (drops && (a_min < 1 || band < 1)) return fail(s, IJ_ERR_INVALID_ARG, "a_min and band must be >= 1");
    hipStream_t st = (hipStream_t)stream;
    if (ij_status e = refresh_phi(s, st)) return e;
    const K3& K = s->K;
    const int r0 = (int)std::max<int64_t>(0, std::min<int64_t>(row0, K.ny));
    hipLaunchKernelGGL(k3_rows, dim3(K.ny), dim3(DT), 0, st, K, s->buf[s->cur], s->wall, s->phi,
                       (float)pulse(s->p, s->t), r0, s->rows);
    hipLaunchKernelGGL(k3_finish, dim3(1), dim3(64), 0, st, s->rows, K.ny, s->rec);
    if (drops)
        hipLaunchKernelGGL(k3_drops, dim3(1), dim3(64), 0, st, s->rows, K.ny, r0, (double)a_min,
                           (int)std::min<int64_t>(band, K.ny), s->drops);
    IJ3_HIP(s, hipGetLastError());
    std::vector<Row3> h(K.ny);
    IJ3_HIP(s, hipMemcpyAsync(h.data(), s->rows, h.size() * sizeof(Row3), hipMemcpyDeviceToHost, st));
    IJ3_HIP(s, hipMemcpyAsync(rec, s->rec, 7 * sizeof(double), hipMemcpyDeviceToHost, st));
    if (drops) IJ3_HIP(s, hipMemcpyAsync(drops, s->drops, sizeof(ij3_drops), hipMemcpyDeviceToHost, st));
    IJ3_HIP(s, hipStreamSynchronize(st));
    for (int y = 0; y < K.ny; ++y) {
        if (row_count) row_count[y] = (int64_t)h[y].ink;
        if (row_uy) row_uy[y] = h[y].uy;
    }
    return IJ_OK;
}

}  // extern "C"
