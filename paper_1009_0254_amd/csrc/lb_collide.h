// Device helpers shared by the step kernels (private): buffer-descriptor loads and stores
// of population rows, fast reciprocal and square root, and the collision of one node.
#pragma once

#include "lb_internal.h"
#include "lb_rng.h"

#include <math.h>

namespace lbf {

// The fused step addresses populations through buffer resources: one per lattice row (base =
// the row, range = its 9 nx elements), the lane's column as a 32-bit offset and the plane of
// population i as a scalar offset, so that no per-lane 64-bit address arithmetic is spent on
// the 18 accesses per node.  Stores carry the nontemporal cache policy.
typedef unsigned u32x2_t __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void *row, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(row), 0, (int)bytes, 0x00020000);
}
template <typename S> __device__ __forceinline__ S bld(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff);
template <> __device__ __forceinline__ float bld<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <> __device__ __forceinline__ double bld<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
constexpr int CPOL_NT = 2;
template <typename S> __device__ __forceinline__ void bst(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, S v);
template <> __device__ __forceinline__ void bst<float>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, CPOL_NT);
}
template <> __device__ __forceinline__ void bst<double>(__amdgpu_buffer_rsrc_t r, unsigned voff, unsigned soff, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, (int)voff, (int)soff, CPOL_NT);
}

template <typename R> __device__ __forceinline__ R frcp(R v);
template <> __device__ __forceinline__ float frcp<float>(float v) { return __builtin_amdgcn_rcpf(v); }
template <> __device__ __forceinline__ double frcp<double>(double v) { return 1.0 / v; }

// a + b rounded once, never contracted with the product that formed a (the re-shift of plain
// FP32 storage after the back-transform must round the same way in every kernel)
template <typename R> __device__ __forceinline__ R add_rn(R a, R b);
template <> __device__ __forceinline__ float add_rn<float>(float a, float b) { return __fadd_rn(a, b); }
template <> __device__ __forceinline__ double add_rn<double>(double a, double b) { return __dadd_rn(a, b); }

template <typename R> __device__ __forceinline__ R fsqrt(R v);
template <> __device__ __forceinline__ float fsqrt<float>(float v) { return __builtin_amdgcn_sqrtf(v); }
template <> __device__ __forceinline__ double fsqrt<double>(double v) { return sqrt(v); }

// density deviation rho - rho0 of nine pulled stored values (PLAIN: stored f_i, whose sum
// includes rho0 = sum_i fbar_i), in one fixed summation order
template <typename R, bool PLAIN> __device__ __forceinline__ R dens9(const R f[Q], const Consts<R> &c)
{
    R s = ((f[0] + (f[1] + f[2])) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8]));
    if (PLAIN) s -= c.rho0;
    return s;
}

// the 9-point stencils of a density deviation field around C (E = x+1, N = y+1, ...):
// the Laplacian of App. B, [4 (E + W + N + S) + (NE + NW + SW + SE) - 20 C] / 6, and the
// isotropic gradient 3 sum_i w_i c_i rho(r + c_i)
template <typename R>
__device__ __forceinline__ void stencil9(R C, R E, R Wv, R N, R NE, R NW, R Sv, R SE, R SW, R &lap, R &gx, R &gy)
{
#pragma clang fp contract(on)
    lap = (4 * ((E + Wv) + (N + Sv)) + ((NE + NW) + (SW + SE)) - 20 * C) * (R)(1.0 / 6.0);
    gx = (4 * (E - Wv) + (NE - NW) + (SE - SW)) * (R)(1.0 / 12.0);
    gy = (4 * (N - Sv) + (NE - SE) + (NW - SW)) * (R)(1.0 / 12.0);
}

// Uniform constants that the collision's FMAs meet beside another uniform operand: a vector
// instruction reads at most one scalar register (pair), so each such FMA would first move one of
// them into vector registers, per node.  Copied into vector registers once per kernel instead.
// The copy reads a scalar register: c must be the same for every lane of a wave (the step
// kernels take it from their tile's replica, one replica per wave).
template <typename R> struct VConsts {
    R dp3, A, k44x2, k49m, k99x125;
};
__device__ __forceinline__ uint32_t vreg32(uint32_t x)
{
    uint32_t r;
    asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
    return r;
}
template <typename R> __device__ __forceinline__ R vreg(R x);
template <> __device__ __forceinline__ float vreg<float>(float x)
{
    return __builtin_bit_cast(float, vreg32(__builtin_bit_cast(uint32_t, x)));
}
template <> __device__ __forceinline__ double vreg<double>(double x)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, x);
    const unsigned long long lo = vreg32((uint32_t)u), hi = vreg32((uint32_t)(u >> 32));
    return __builtin_bit_cast(double, lo | (hi << 32));
}
template <typename R> __device__ __forceinline__ VConsts<R> vconsts(const Consts<R> &c)
{
    return VConsts<R>{vreg<R>(c.dp3), vreg<R>(c.A), vreg<R>(c.k44x2), vreg<R>(c.k49m), vreg<R>(c.k99x125)};
}

// ------------------------------------------------------------------ the collision
// Deviations df_i = f_i - fbar_i from the rest state fbar = T^-1 m^eq(rho0, u = 0) in,
// post-collision deviations out.  The moments of df are m - mbar (mbar: rho0 and the rest
// values of e4, e9), and the equilibrium is formed as m^eq - mbar, so that near rest no
// value in the collision is O(1).  Stencil values are of drho = rho - rho0.  Returns
// status bits (LB_FLAG_*).
// CN: the replica set has correlated noise (noise == 2 possible)
template <typename R, bool CN>
__device__ __forceinline__ unsigned collide(R f[Q], R lap, R gx, R gy, const Consts<R> &c, const VConsts<R> &vk,
                                            uint32_t noise,
                                            uint32_t node, uint32_t rep, unsigned long long t, uint32_t k0,
                                            uint32_t k1, R xi4, R xi9)
{
    // a product and a sum fuse into one rounding only where they are written in one
    // expression, so that every kernel inlining the collision rounds it the same way (left
    // to the optimiser, fusion depends on the surrounding code)
#pragma clang fp contract(on)
    // m = T f (Table I rows, eq. Tmat), sharing the axis / diagonal partial sums
    const R sa = (f[1] + f[2]) + (f[3] + f[4]);
    const R sd = (f[5] + f[6]) + (f[7] + f[8]);
    const R drho = f[0] + sa + sd;
    const R ax = f[1] - f[3], ay = f[2] - f[4];
    const R d68 = f[5] - f[7], d97 = f[8] - f[6];
    const R jx = ax + d68 + d97;
    const R jy = ay + d68 - d97;
    const R m4 = -2 * f[0] + sa + 4 * sd;
    const R m5 = (f[1] + f[3]) - (f[2] + f[4]);
    const R m6 = (f[5] + f[7]) - (f[6] + f[8]);
    const R m7 = -ax + 2 * (d68 + d97);
    const R m8 = -ay + 2 * (d68 - d97);
    const R m9 = 2 * f[0] - 4 * sa + 8 * sd;

    unsigned st = 0;
    const R rho = c.rho0 + drho;
    if (!__builtin_isfinite(rho)) st |= 4u;
    const R irho = frcp<R>(rho);

    // local thermodynamics (Sec. II.A): pex = p0 - rho sigma_s^2 relative to its rest value,
    // from the exact Taylor expansion at rho0 in drho
    const R kap = c.kappa;
    const R pex = drho * (c.dp1 + drho * (c.dp2 + drho * (vk.dp3 + drho * c.dp4)));
    const R piso = pex - kap * rho * lap;

    // Table II (C_n = 0), minus the rest values mbar_4 = 6 pex(rho0), mbar_9 = -6 pex(rho0)
    const R jxx = jx * jx, jyy = jy * jy;
    const R gxx = gx * gx, gyy = gy * gy;
    const R jj = (jxx + jyy) * irho;
    const R e4 = 3 * jj + 6 * piso;
    const R e5 = (jxx - jyy) * irho + kap * (gxx - gyy);
    const R e6 = jx * jy * irho + kap * gx * gy;
    const R e9 = -6 * piso - 3 * kap * (gxx + gyy);

    // MRT relaxation m* = m + lambda (m - m^eq)
    const R lb = c.lam_b, ls = c.lam_s, lq = c.lam_q, le = c.lam_e;
    R s4 = m4 + lb * (m4 - e4);
    R s5 = m5 + ls * (m5 - e5);
    R s6 = m6 + ls * (m6 - e6);
    R s7 = m7 + lq * m7;
    R s8 = m8 + lq * m8;
    R s9 = m9 + le * (m9 - e9);

    if (CN && noise == 2) {
        // correlated noise: modes 4 and 9 from the filtered fields, modes 5..8 white at rho0
        // (normals scaled by sqrt(3 kT rho0))
        R nu[6];
        normals6s<R>(node, rep, t, k0, k1, c.sq0, nu);
        s4 += xi4;
        s9 += xi9;
        s5 += c.l55 * nu[1];
        s6 += c.l66 * nu[2];
        s7 += c.l77 * nu[3];
        s8 += c.l88 * nu[4];
    } else if (noise) {
        // xi = L nu, L L^T = Xi(0) at the local rho and c_s^2 (eq. noise-yeo at k = 0); the
        // normals come scaled by sqrt(rho kT / sigma_s^2)
        R rr = rho;
        if (!(rr > 0)) {
            st |= 2u;
            rr = 0;
        }
        const R xx = c.xr0 + (rr - c.rho0);
        const R cs2 = c.c0sq + rr * (vk.A + c.B3 * (xx * xx));
        const R a44 = vk.k44x2 + c.k44n3 * cs2;        // k44 (2 - 3 c_s^2)
        const R a49 = c.k49 * cs2 + vk.k49m;           // k49 (c_s^2 - 1/3)
        const R a99 = vk.k99x125 + c.k99n075 * cs2;    // k99 (5/4 - 3 c_s^2 / 4)
        R nu[6];
        normals6s<R>(node, rep, t, k0, k1, fsqrt<R>(rr * c.kT3), nu);
        R l44 = 0, l94 = 0;
        if (a44 > 0) {
            l44 = fsqrt<R>(a44);
            if (noise != 3) l94 = a49 * frcp<R>(l44);   // 3: the diagonal of Xi(0) only (Sec. IV)
        } else if (a44 < 0) {
            st |= 1u;
        }
        R p99 = a99 - l94 * l94;
        if (p99 < 0) {
            st |= 1u;
            p99 = 0;
        }
        const R l99 = fsqrt<R>(p99);
        s4 += l44 * nu[0];
        s5 += c.l55 * nu[1];
        s6 += c.l66 * nu[2];
        s7 += c.l77 * nu[3];
        s8 += c.l88 * nu[4];
        s9 += l94 * nu[0] + l99 * nu[5];
    }

    // f* = T^-1 m*, (T^-1)_ia = w_i T_ai / N_a with N = (1, 1/3, 1/3, 4, 4/9, 1/9, 2/3, 2/3, 16),
    // the factors w_i / N_a gathered per term:
    //   f1,3 = a + c5 +- bx, f2,4 = a - c5 +- by, a = drho/9 + (s4 - s9)/36, c5 = s5/4,
    //          bx = jx/3 - s7/6, by = jy/3 - s8/6
    //   f5..8 = dd +- g +- ex +- ey, dd = (drho + s4)/36 + s9/72, g = s6/4,
    //          ex = (jx + s7)/12 = (jx - 2 bx)/4, ey = (jy - 2 by)/4
    //   f0 = 4/9 drho - 2/9 s4 + 1/18 s9 = drho - 4 (a + dd)
    // The last two forms return the conserved moments exactly (sum_i f_i = f0 + 4 a + 4 dd,
    // sum_i c_ix f_i = 2 bx + 4 ex) up to the rounding of one subtraction; with rounded
    // constants 1/3, 1/12, 4/9 they would come back scaled by 1 + O(1e-8) every step, a drift of
    // mass and momentum that grows linearly with time in FP32.
    const R aa = drho * (R)(1.0 / 9.0) + (s4 - s9) * (R)(1.0 / 36.0);
    const R c5 = s5 * (R)0.25;
    const R bx = jx * (R)(1.0 / 3.0) + s7 * (R)(-1.0 / 6.0);
    const R by = jy * (R)(1.0 / 3.0) + s8 * (R)(-1.0 / 6.0);
    const R dd = (drho + s4) * (R)(1.0 / 36.0) + s9 * (R)(1.0 / 72.0);
    const R g = s6 * (R)0.25;
    const R ex = (jx - 2 * bx) * (R)0.25;
    const R ey = (jy - 2 * by) * (R)0.25;
    const R ap = aa + c5, am = aa - c5;
    const R dp = dd + g, dm = dd - g;
    const R u = ex + ey, v = ex - ey;
    f[0] = drho - 4 * (aa + dd);
    f[1] = ap + bx;
    f[2] = am + by;
    f[3] = ap - bx;
    f[4] = am - by;
    f[5] = dp + u;
    f[6] = dm - v;
    f[7] = dp - u;
    f[8] = dm + v;
    return st;
}

}  // namespace lbf
