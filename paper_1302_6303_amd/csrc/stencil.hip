// Stencil kernels of the NRD residual and its Jacobian action (paper Sec.
// 3.1-3.3, 4.1).  Restriction and ghost fill are in sync.hip, the transpose
// in adjoint.hip.
//
// Layout: per patch a ghosted block, x fastest; field f of a native vector
// starts at f * nl.  One workgroup processes one tile (a run of interior
// cells of one patch); the patch descriptor is wave-uniform and lives in
// scalar registers.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "kernels.h"

namespace nrd {

// ---------------------------------------------------------------------------
// face formulas
//
// Flux density through a face between lower cell a and upper cell b:
//   Phi_E = D_E (E_b - E_a) / h,  D_E = D_h / (1 + lam D_h g),
//   D_h = 2 T_f^3 / (3 (z_a^3 + z_b^3)),  g = |E_b - E_a| / (h (E_a + E_b)/2)
// folded into one division:
//   Phi_E = 2 T_f^3 S dE / (3 Z_f h S + 4 lam T_f^3 |dE|),  S = E_a + E_b.
//   Phi_T = kappa T_f^(5/2) (T_b - T_a) / h.
// Marshak face: inflow q = 2 D_b (4R - E_c) / (4 D_b + h), D_b = T_c^3/(3 z_c^3)
//   = 2 T^3 (4R - E) / (4 T^3 + 3 z^3 h).
// ---------------------------------------------------------------------------


__device__ __forceinline__ void face_flux(double Ea, double Eb, double Ta, double Tb,
                                          double za, double zb, double h, double ih,
                                          double kappa, double lam, double& fe,
                                          double& ft) {
    const double Tf = 0.5 * (Ta + Tb);
    const double Tf2 = Tf * Tf;
    const double Tf3 = Tf2 * Tf;
    const double S = Ea + Eb;
    const double dE = Eb - Ea;
    fe = (2.0 * Tf3 * S * dE) *
         rcp_nr(3.0 * (za + zb) * h * S + 4.0 * lam * Tf3 * fabs(dE));
    ft = kappa * Tf3 * rsqrt_nr(Tf) * (Tb - Ta) * ih;       // kappa Tf^(5/2) dT / h
}

__device__ __forceinline__ void face_flux_tan(double Ea, double Eb, double Ta, double Tb,
                                              double za, double zb, double dEa, double dEb,
                                              double dTa, double dTb, double h, double ih,
                                              double kappa, double lam, double& dfe,
                                              double& dft) {
    const double Tf = 0.5 * (Ta + Tb);
    const double dTf = 0.5 * (dTa + dTb);
    const double Tf2 = Tf * Tf;
    const double Tf3 = Tf2 * Tf;
    const double S = Ea + Eb;
    const double dS = dEa + dEb;
    const double dE = Eb - Ea;
    const double ddE = dEb - dEa;
    const double adE = fabs(dE);
    const double sg = (dE > 0.0) ? 1.0 : ((dE < 0.0) ? -1.0 : 0.0);
    const double Zh = 3.0 * (za + zb) * h;
    const double N = 2.0 * Tf3 * S * dE;
    const double iD = rcp_nr(Zh * S + 4.0 * lam * Tf3 * adE);
    const double phi = N * iD;
    const double dN = 2.0 * (3.0 * Tf2 * dTf * S * dE + Tf3 * (dS * dE + S * ddE));
    const double dDn = Zh * dS + 4.0 * lam * (3.0 * Tf2 * dTf * adE + Tf3 * sg * ddE);
    dfe = (dN - phi * dDn) * iD;
    const double sq = Tf * rsqrt_nr(Tf);
    dft = kappa * Tf * sq * (2.5 * dTf * (Tb - Ta) + Tf * (dTb - dTa)) * ih;
}

__device__ __forceinline__ double robin_q(double Ec, double Tc, double zc, double R,
                                          double h) {
    const double T3 = Tc * Tc * Tc;
    return 2.0 * T3 * (4.0 * R - Ec) * rcp_nr(4.0 * T3 + 3.0 * zc * h);
}

__device__ __forceinline__ double robin_q_tan(double Ec, double Tc, double zc, double R,
                                              double h, double dEc, double dTc) {
    const double T2 = Tc * Tc;
    const double T3 = T2 * Tc;
    const double iD = rcp_nr(4.0 * T3 + 3.0 * zc * h);
    const double q = 2.0 * T3 * (4.0 * R - Ec) * iD;
    const double dN = 6.0 * T2 * dTc * (4.0 * R - Ec) - 2.0 * T3 * dEc;
    return (dN - q * 12.0 * T2 * dTc) * iD;
}

// Cell terms of the residual (MODE 0) or of its derivative (MODE 1):
// coupling S = sigma (T^4 - E) = z^3 (T - E / T^3).
__device__ __forceinline__ void cell_out0(const ProbScalars& q, double E, double T, double z,
                                          double bE, double bT, double divE, double divT,
                                          double& oE, double& oT) {
    const double T3 = T * T * T;
    const double S = z * (T - E * rcp_nr(T3));
    oE = q.c0 * E - bE - q.dt * (divE + S);
    oT = q.c0 * T - bT - q.dt * (divT - S);
}
__device__ __forceinline__ void cell_out1(const ProbScalars& q, double E, double T, double z,
                                          double dE, double dT, double divE, double divT,
                                          double& oE, double& oT) {
    const double T3 = T * T * T;
    const double r3 = rcp_nr(T3);
    const double dS = z * ((1.0 + 3.0 * E * r3 * rcp_nr(T)) * dT - dE * r3);
    oE = q.c0 * dE - q.dt * (divE + dS);
    oT = q.c0 * dT - q.dt * (divT - dS);
}


static inline int nblocks(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

// ---------------------------------------------------------------------------
// residual (MODE 0) and Jacobian action (MODE 1), z-marching bricks
//
// Each thread owns one (i, j) column of a brick and walks k upward, carrying
// the centre plane and the flux through the shared z face in registers; the
// x and y neighbours are read from global memory, where the other columns of
// the workgroup have just brought them into L1.  A face bordering a covered
// cell is skipped on the non-covered side (flux matching supplies it).
// ---------------------------------------------------------------------------

template <int MODE>
__device__ __forceinline__ void face_any(const double* __restrict__ u,
                                         const double* __restrict__ v,
                                         const double* __restrict__ z3, int a, int b,
                                         int64_t nl, double h, double ih, double kappa,
                                         double lam, double& fe, double& ft) {
    if (MODE == 0)
        face_flux(u[a], u[b], u[a + nl], u[b + nl], z3[a], z3[b], h, ih, kappa, lam, fe, ft);
    else
        face_flux_tan(u[a], u[b], u[a + nl], u[b + nl], z3[a], z3[b], v[a], v[b], v[a + nl],
                      v[b + nl], h, ih, kappa, lam, fe, ft);
}

template <int MODE>
__device__ __forceinline__ double robin_any(double E, double T, double z, double R, double h,
                                            double dE, double dT) {
    return MODE == 0 ? robin_q(E, T, z, R, h) : robin_q_tan(E, T, z, R, h, dE, dT);
}

// Plane-marching variant.  A tile is a run of up to 256 consecutive cells of
// one z-plane of a patch (x fastest) and a range of planes.  Every face is
// evaluated once: a thread computes the low x and low y faces of its cell
// and the high z face; the high x / high y faces come from the neighbouring
// thread through LDS when that neighbour is in the tile (otherwise they are
// evaluated directly), and the z face is carried in registers to the next
// plane.  Physical faces are evaluated by the cell that owns them.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_stencil_z(
    const STile* __restrict__ tiles, int t0, const int32_t* __restrict__ map,
    const PatchInfo* __restrict__ P,
    const ProbScalars* __restrict__ ps, const int32_t* __restrict__ active,
    const uint8_t* __restrict__ ctype, const double* __restrict__ u,
    const double* __restrict__ v, const double* __restrict__ z3,
    const double* __restrict__ b, double* __restrict__ out, int64_t nl) {
    __shared__ double fxs[2][2][kBlock];
    __shared__ double fys[2][2][kBlock];
    const STile t = tiles[tile_index(map, t0)];
    if (active && !active[t.prob]) return;          // uniform over the workgroup
    const PatchInfo& p = P[t.patch];
    const ProbScalars& q = ps[t.prob];
    const double kappa = q.kappa, lam = q.lam;
    const int tid = threadIdx.x;
    const bool live = tid < t.cnt;
    const int nx = p.n[0], ny = p.n[1], nz = p.n[2];
    const int lin = t.s0 + (live ? tid : 0);
    const int i = lin % nx, j = lin / nx;
    const int sy = p.sy, sz = p.sz;
    const bool use_ct = p.flags & PF_CTYPE;
    const double hx = p.h[0], hy = p.h[1], hz = p.h[2];
    const double ihx = p.ih[0], ihy = p.ih[1], ihz = p.ih[2];
    const bool xlo_p = (p.phys & 1) && i == 0, xhi_p = ((p.phys >> 1) & 1) && i == nx - 1;
    const bool ylo_p = ((p.phys >> 2) & 1) && j == 0, yhi_p = ((p.phys >> 3) & 1) && j == ny - 1;
    const bool zlo_p = (p.phys >> 4) & 1, zhi_p = (p.phys >> 5) & 1;
    const bool x_lds = (i < nx - 1) && (tid + 1 < t.cnt);
    const bool y_lds = (tid + nx < t.cnt);
    int c = p.off + (i + 1) + sy * (j + 1) + sz * (t.k0 + 1);
    double czE = 0.0, czT = 0.0;
    if (live && !(t.k0 == 0 && zlo_p))
        face_any<MODE>(u, v, z3, c - sz, c, nl, hz, ihz, kappa, lam, czE, czT);
    int buf = 0;
    for (int k = t.k0; k < t.k1; ++k, c += sz, buf ^= 1) {
        double E = 0.0, T = 1.0, z = 1.0, dE = 0.0, dT = 0.0;
        double lxE = 0.0, lxT = 0.0, lyE = 0.0, lyT = 0.0, hzE = 0.0, hzT = 0.0;
        double lzE = 0.0, lzT = 0.0;
        if (live) {
            E = u[c];
            T = u[c + nl];
            z = z3[c];
            if (MODE) {
                dE = v[c];
                dT = v[c + nl];
            }
            if (xlo_p) {
                if (p.robin & 1) lxE = -robin_any<MODE>(E, T, z, q.R[0], hx, dE, dT);
            } else {
                face_any<MODE>(u, v, z3, c - 1, c, nl, hx, ihx, kappa, lam, lxE, lxT);
            }
            if (ylo_p) {
                if ((p.robin >> 2) & 1) lyE = -robin_any<MODE>(E, T, z, q.R[2], hy, dE, dT);
            } else {
                face_any<MODE>(u, v, z3, c - sy, c, nl, hy, ihy, kappa, lam, lyE, lyT);
            }
            if (k == nz - 1 && zhi_p) {
                if ((p.robin >> 5) & 1) hzE = robin_any<MODE>(E, T, z, q.R[5], hz, dE, dT);
            } else {
                face_any<MODE>(u, v, z3, c, c + sz, nl, hz, ihz, kappa, lam, hzE, hzT);
            }
            if (k == 0 && zlo_p) {
                if ((p.robin >> 4) & 1) lzE = -robin_any<MODE>(E, T, z, q.R[4], hz, dE, dT);
            } else {
                lzE = czE;
                lzT = czT;
            }
            czE = hzE;
            czT = hzT;
            fxs[buf][0][tid] = lxE;
            fxs[buf][1][tid] = lxT;
            fys[buf][0][tid] = lyE;
            fys[buf][1][tid] = lyT;
        }
        __syncthreads();
        if (!live) continue;
        double hxE = 0.0, hxT = 0.0, hyE = 0.0, hyT = 0.0;
        if (xhi_p) {
            if ((p.robin >> 1) & 1) hxE = robin_any<MODE>(E, T, z, q.R[1], hx, dE, dT);
        } else if (x_lds) {
            hxE = fxs[buf][0][tid + 1];
            hxT = fxs[buf][1][tid + 1];
        } else {
            face_any<MODE>(u, v, z3, c, c + 1, nl, hx, ihx, kappa, lam, hxE, hxT);
        }
        if (yhi_p) {
            if ((p.robin >> 3) & 1) hyE = robin_any<MODE>(E, T, z, q.R[3], hy, dE, dT);
        } else if (y_lds) {
            hyE = fys[buf][0][tid + nx];
            hyT = fys[buf][1][tid + nx];
        } else {
            face_any<MODE>(u, v, z3, c, c + sy, nl, hy, ihy, kappa, lam, hyE, hyT);
        }
        const int ct = use_ct ? ctype[c] : 0;
        if (ct & CT_COVERED) {
            out[c] = 0.0;
            out[c + nl] = 0.0;
            continue;
        }
        if (ct & (1 << 1)) lxE = lxT = 0.0;
        if (ct & (1 << 2)) hxE = hxT = 0.0;
        if (ct & (1 << 3)) lyE = lyT = 0.0;
        if (ct & (1 << 4)) hyE = hyT = 0.0;
        if (ct & (1 << 5)) lzE = lzT = 0.0;
        if (ct & (1 << 6)) hzE = hzT = 0.0;
        const double divE = (hxE - lxE) * ihx + (hyE - lyE) * ihy + (hzE - lzE) * ihz;
        const double divT = (hxT - lxT) * ihx + (hyT - lyT) * ihy + (hzT - lzT) * ihz;
        double oE, oT;
        if (MODE == 0)
            cell_out0(q, E, T, z, b[c], b[c + nl], divE, divT, oE, oT);
        else
            cell_out1(q, E, T, z, dE, dT, divE, divT, oE, oT);
        out[c] = oE;
        out[c + nl] = oT;
    }
}

// Wave-run variant.  Each wavefront of the workgroup owns a run of 63
// consecutive cells of the (x fastest) linear index of a z-plane and walks
// the planes k0 <= k < k1.  Lane l evaluates the low x face of its cell; the
// high x face of lane l < 63 is lane l+1's low face (cross-lane shuffle, no
// barrier), lane 63 only helps.  The y faces are evaluated per cell and the
// z face is carried in registers to the next plane.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_stencil_w(
    const STile* __restrict__ tiles, int t0, const int32_t* __restrict__ map,
    const PatchInfo* __restrict__ P,
    const ProbScalars* __restrict__ ps, const int32_t* __restrict__ active,
    const uint8_t* __restrict__ ctype, const double* __restrict__ u,
    const double* __restrict__ v, const double* __restrict__ z3,
    const double* __restrict__ b, double* __restrict__ out, int64_t nl) {
    const STile t = tiles[tile_index(map, t0)];
    if (active && !active[t.prob]) return;
    const PatchInfo& p = P[t.patch];
    const ProbScalars& q = ps[t.prob];
    const double kappa = q.kappa, lam = q.lam;
    const int lane = threadIdx.x & 63;
    const int pos = (threadIdx.x >> 6) * 63 + lane;        // within the tile's run
    const int nx = p.n[0], ny = p.n[1], nz = p.n[2];
    const int lin = t.s0 + pos;
    const bool exists = pos <= t.cnt && lin < nx * ny;     // helper lanes included
    const bool owned = lane < 63 && pos < t.cnt;
    const int i = lin % nx, j = lin / nx;
    const int sy = p.sy, sz = p.sz;
    const bool use_ct = p.flags & PF_CTYPE;
    const double hx = p.h[0], hy = p.h[1], hz = p.h[2];
    const double ihx = p.ih[0], ihy = p.ih[1], ihz = p.ih[2];
    const bool xlo_p = (p.phys & 1) && i == 0, xhi_p = ((p.phys >> 1) & 1) && i == nx - 1;
    const bool ylo_p = ((p.phys >> 2) & 1) && j == 0, yhi_p = ((p.phys >> 3) & 1) && j == ny - 1;
    const bool zlo_p = (p.phys >> 4) & 1, zhi_p = (p.phys >> 5) & 1;
    int c = p.off + (i + 1) + sy * (j + 1) + sz * (t.k0 + 1);
    double czE = 0.0, czT = 0.0;
    if (owned && !(t.k0 == 0 && zlo_p))
        face_any<MODE>(u, v, z3, c - sz, c, nl, hz, ihz, kappa, lam, czE, czT);
    for (int k = t.k0; k < t.k1; ++k, c += sz) {
        double E = 0.0, T = 1.0, z = 1.0, dE = 0.0, dT = 0.0;
        double lxE = 0.0, lxT = 0.0;
        if (exists) {
            E = u[c];
            T = u[c + nl];
            z = z3[c];
            if (MODE) {
                dE = v[c];
                dT = v[c + nl];
            }
            if (xlo_p) {
                if (p.robin & 1) lxE = -robin_any<MODE>(E, T, z, q.R[0], hx, dE, dT);
            } else {
                face_any<MODE>(u, v, z3, c - 1, c, nl, hx, ihx, kappa, lam, lxE, lxT);
            }
        }
        // high x face of lane l = low x face of lane l + 1
        double hxE = __shfl_down(lxE, 1, 64);
        double hxT = __shfl_down(lxT, 1, 64);
        if (!owned) continue;
        if (i == nx - 1) {
            hxE = hxT = 0.0;
            if (xhi_p) {
                if ((p.robin >> 1) & 1) hxE = robin_any<MODE>(E, T, z, q.R[1], hx, dE, dT);
            } else {
                face_any<MODE>(u, v, z3, c, c + 1, nl, hx, ihx, kappa, lam, hxE, hxT);
            }
        }
        double lyE = 0.0, lyT = 0.0, hyE = 0.0, hyT = 0.0, hzE = 0.0, hzT = 0.0;
        double lzE = 0.0, lzT = 0.0;
        if (ylo_p) {
            if ((p.robin >> 2) & 1) lyE = -robin_any<MODE>(E, T, z, q.R[2], hy, dE, dT);
        } else {
            face_any<MODE>(u, v, z3, c - sy, c, nl, hy, ihy, kappa, lam, lyE, lyT);
        }
        if (yhi_p) {
            if ((p.robin >> 3) & 1) hyE = robin_any<MODE>(E, T, z, q.R[3], hy, dE, dT);
        } else {
            face_any<MODE>(u, v, z3, c, c + sy, nl, hy, ihy, kappa, lam, hyE, hyT);
        }
        if (k == nz - 1 && zhi_p) {
            if ((p.robin >> 5) & 1) hzE = robin_any<MODE>(E, T, z, q.R[5], hz, dE, dT);
        } else {
            face_any<MODE>(u, v, z3, c, c + sz, nl, hz, ihz, kappa, lam, hzE, hzT);
        }
        if (k == 0 && zlo_p) {
            if ((p.robin >> 4) & 1) lzE = -robin_any<MODE>(E, T, z, q.R[4], hz, dE, dT);
        } else {
            lzE = czE;
            lzT = czT;
        }
        czE = hzE;
        czT = hzT;
        const int ct = use_ct ? ctype[c] : 0;
        if (ct & CT_COVERED) {
            out[c] = 0.0;
            out[c + nl] = 0.0;
            continue;
        }
        if (ct & (1 << 1)) lxE = lxT = 0.0;
        if (ct & (1 << 2)) hxE = hxT = 0.0;
        if (ct & (1 << 3)) lyE = lyT = 0.0;
        if (ct & (1 << 4)) hyE = hyT = 0.0;
        if (ct & (1 << 5)) lzE = lzT = 0.0;
        if (ct & (1 << 6)) hzE = hzT = 0.0;
        const double divE = (hxE - lxE) * ihx + (hyE - lyE) * ihy + (hzE - lzE) * ihz;
        const double divT = (hxT - lxT) * ihx + (hyT - lyT) * ihy + (hzT - lzT) * ihz;
        double oE, oT;
        if (MODE == 0)
            cell_out0(q, E, T, z, b[c], b[c + nl], divE, divT, oE, oT);
        else
            cell_out1(q, E, T, z, dE, dT, divE, divT, oE, oT);
        out[c] = oE;
        out[c + nl] = oT;
    }
}

// Flat variant: one thread per cell of a run of 256 interior cells (x
// fastest); all six faces of the cell are evaluated by that thread.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_stencil_flat(
    const Tile* __restrict__ tiles, int t0, const int32_t* __restrict__ map,
    const PatchInfo* __restrict__ P,
    const ProbScalars* __restrict__ ps, const int32_t* __restrict__ active,
    const uint8_t* __restrict__ ctype, const double* __restrict__ u,
    const double* __restrict__ v, const double* __restrict__ z3,
    const double* __restrict__ b, double* __restrict__ out, int64_t nl) {
    const Tile t = tiles[tile_index(map, t0)];
    if (active && !active[t.prob]) return;
    if ((int)threadIdx.x >= t.count) return;
    const PatchInfo& p = P[t.patch];
    const ProbScalars& q = ps[t.prob];
    int id[3];
    cell_coords(p, t.start + threadIdx.x, id[0], id[1], id[2]);
    const int c = native_index(p, id[0], id[1], id[2]);
    const int ct = (p.flags & PF_CTYPE) ? ctype[c] : 0;
    if (ct & CT_COVERED) {
        out[c] = 0.0;
        out[c + nl] = 0.0;
        return;
    }
    const int st[3] = {1, p.sy, p.sz};
    const double E = u[c], T = u[c + nl], z = z3[c];
    double dE = 0.0, dT = 0.0;
    if (MODE == 1) {
        dE = v[c];
        dT = v[c + nl];
    }
    const double kappa = q.kappa, lam = q.lam;
    double divE = 0.0, divT = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double h = p.h[d], ih = p.ih[d];
        double fe_lo = 0.0, ft_lo = 0.0, fe_hi = 0.0, ft_hi = 0.0;
        // low face
        if (id[d] == 0 && ((p.phys >> (2 * d)) & 1)) {
            if ((p.robin >> (2 * d)) & 1) {
                fe_lo = (MODE == 0) ? -robin_q(E, T, z, q.R[2 * d], h)
                                    : -robin_q_tan(E, T, z, q.R[2 * d], h, dE, dT);
            }
        } else if (!((ct >> (2 * d + 1)) & 1)) {
            const int a = c - st[d];
            if (MODE == 0)
                face_flux(u[a], E, u[a + nl], T, z3[a], z, h, ih, kappa, lam, fe_lo, ft_lo);
            else
                face_flux_tan(u[a], E, u[a + nl], T, z3[a], z, v[a], dE, v[a + nl], dT, h, ih,
                              kappa, lam, fe_lo, ft_lo);
        }
        // high face
        if (id[d] == p.n[d] - 1 && ((p.phys >> (2 * d + 1)) & 1)) {
            if ((p.robin >> (2 * d + 1)) & 1) {
                fe_hi = (MODE == 0) ? robin_q(E, T, z, q.R[2 * d + 1], h)
                                    : robin_q_tan(E, T, z, q.R[2 * d + 1], h, dE, dT);
            }
        } else if (!((ct >> (2 * d + 2)) & 1)) {
            const int bb = c + st[d];
            if (MODE == 0)
                face_flux(E, u[bb], T, u[bb + nl], z, z3[bb], h, ih, kappa, lam, fe_hi, ft_hi);
            else
                face_flux_tan(E, u[bb], T, u[bb + nl], z, z3[bb], dE, v[bb], dT, v[bb + nl], h,
                              ih, kappa, lam, fe_hi, ft_hi);
        }
        divE += (fe_hi - fe_lo) * ih;
        divT += (ft_hi - ft_lo) * ih;
    }
    double oE, oT;
    if (MODE == 0)
        cell_out0(q, E, T, z, b[c], b[c + nl], divE, divT, oE, oT);
    else
        cell_out1(q, E, T, z, dE, dT, divE, divT, oE, oT);
    out[c] = oE;
    out[c + nl] = oT;
}

// Staged-plane variant.  A tile is a run of up to 2 x 256 consecutive cells
// of one z-plane (x fastest) and a range of planes; thread t owns cells t and
// t + 256 of the run.  For every plane the workgroup copies the contiguous
// slice of the ghosted plane that covers the run and its x / y neighbours
// (E, T, z^3, plus the tangent in MODE 1) into LDS once, so every value is
// read from memory once per tile rather than once per face.  Each face is
// evaluated once: low x / low y faces by the cell, high ones from the
// neighbouring cell through LDS (evaluated directly when the neighbour is
// outside the run), the z face carried in registers to the next plane.  The
// next plane's slice is loaded into registers while the current faces are
// evaluated.
constexpr int kStageCPT = kStageCells / kBlock;    // cells per thread
static_assert(kStageCells == kStageCPT * kBlock, "whole cells per thread");
constexpr int kStagePer = (kStageLen + kBlock - 1) / kBlock;

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_stencil_s(
    const STile* __restrict__ tiles, int t0, const int32_t* __restrict__ map,
    const PatchInfo* __restrict__ P,
    const ProbScalars* __restrict__ ps, const int32_t* __restrict__ active,
    const uint8_t* __restrict__ ctype, const double* __restrict__ u,
    const double* __restrict__ v, const double* __restrict__ z3,
    const double* __restrict__ b, double* __restrict__ out, int64_t nl) {
    constexpr int NA = MODE ? 5 : 3;            // E, T, z^3 (, vE, vT)
    __shared__ double sl[NA][kStageLen];
    __shared__ double fl[4][kStageCells];       // low x E/T, low y E/T fluxes
    const STile t = tiles[tile_index(map, t0)];
    if (active && !active[t.prob]) return;      // uniform over the workgroup
    const PatchInfo& p = P[t.patch];
    const ProbScalars& q = ps[t.prob];
    const double kappa = q.kappa, lam = q.lam;
    const int tid = threadIdx.x;
    const int nx = p.n[0], ny = p.n[1], nz = p.n[2];
    const int sy = p.sy, sz = p.sz;
    const bool use_ct = p.flags & PF_CTYPE;
    const double hx = p.h[0], hy = p.h[1], hz = p.h[2];
    const double ihx = p.ih[0], ihy = p.ih[1], ihz = p.ih[2];
    const bool zlo_p = (p.phys >> 4) & 1, zhi_p = (p.phys >> 5) & 1;
    // the slice [g0, g0 + len) of a ghosted plane covers the run and its
    // x / y neighbours (host-checked: len <= kStageLen)
    const int la = t.s0, lb = t.s0 + t.cnt - 1;
    const int g0 = (la % nx + 1) + sy * (la / nx);
    const int len = (lb % nx + 1) + sy * (lb / nx + 2) - g0 + 1;
    const double* src[NA];
    src[0] = u;
    src[1] = u + nl;
    src[2] = z3;
    if (MODE) {
        src[NA - 2] = v;
        src[NA - 1] = v + nl;
    }
    // per cell (r = 0, 1): run index, coordinates, slice index, native index
    int ix[kStageCPT], jx[kStageCPT], sidx[kStageCPT], cn[kStageCPT];
    bool live[kStageCPT];
#pragma unroll
    for (int r = 0; r < kStageCPT; ++r) {
        const int idx = tid + r * kBlock;
        live[r] = idx < t.cnt;
        const int lin = t.s0 + (live[r] ? idx : 0);
        ix[r] = lin % nx;
        jx[r] = lin / nx;
        sidx[r] = (ix[r] + 1) + sy * (jx[r] + 1) - g0;
        cn[r] = p.off + (ix[r] + 1) + sy * (jx[r] + 1);   // plane offset added per k
    }
    // prologue: stage plane k0 directly
    {
        const int64_t base = p.off + (int64_t)sz * (t.k0 + 1) + g0;
#pragma unroll
        for (int a = 0; a < NA; ++a)
            for (int e = tid; e < len; e += kBlock) sl[a][e] = src[a][base + e];
    }
    __syncthreads();
    double oE[kStageCPT], oT[kStageCPT], oz[kStageCPT], odE[kStageCPT], odT[kStageCPT];          // own values, plane k
    double czE[kStageCPT], czT[kStageCPT];                               // low z face fluxes
#pragma unroll
    for (int r = 0; r < kStageCPT; ++r) {
        oE[r] = sl[0][sidx[r]];
        oT[r] = sl[1][sidx[r]];
        oz[r] = sl[2][sidx[r]];
        odE[r] = MODE ? sl[NA - 2][sidx[r]] : 0.0;
        odT[r] = MODE ? sl[NA - 1][sidx[r]] : 0.0;
        czE[r] = czT[r] = 0.0;
        if (!live[r]) continue;
        const int c = cn[r] + sz * (t.k0 + 1);
        if (t.k0 == 0 && zlo_p) {
            if ((p.robin >> 4) & 1) czE[r] = -robin_any<MODE>(oE[r], oT[r], oz[r], q.R[4], hz,
                                                              odE[r], odT[r]);
        } else {
            const int a = c - sz;
            if (MODE == 0)
                face_flux(u[a], oE[r], u[a + nl], oT[r], z3[a], oz[r], hz, ihz, kappa, lam,
                          czE[r], czT[r]);
            else
                face_flux_tan(u[a], oE[r], u[a + nl], oT[r], z3[a], oz[r], v[a], odE[r],
                              v[a + nl], odT[r], hz, ihz, kappa, lam, czE[r], czT[r]);
        }
    }
    for (int k = t.k0; k < t.k1; ++k) {
        // next plane's slice into registers (the ghost plane when k = nz - 1)
        double pre[NA][kStagePer];
        {
            const int64_t base = p.off + (int64_t)sz * (k + 2) + g0;
#pragma unroll
            for (int a = 0; a < NA; ++a)
#pragma unroll
                for (int w = 0; w < kStagePer; ++w) {
                    const int e = tid + w * kBlock;
                    pre[a][w] = (e < len) ? src[a][base + e] : 0.0;
                }
        }
        double bE[kStageCPT] = {}, bT[kStageCPT] = {};
        if (MODE == 0) {
#pragma unroll
            for (int r = 0; r < kStageCPT; ++r)
                if (live[r]) {
                    const int c = cn[r] + sz * (k + 1);
                    bE[r] = b[c];
                    bT[r] = b[c + nl];
                }
        }
        // phase A: faces from the staged plane k
        double lxE[kStageCPT], lxT[kStageCPT], lyE[kStageCPT], lyT[kStageCPT], hxE[kStageCPT],
            hxT[kStageCPT], hyE[kStageCPT], hyT[kStageCPT];
#pragma unroll
        for (int r = 0; r < kStageCPT; ++r) {
            lxE[r] = lxT[r] = lyE[r] = lyT[r] = hxE[r] = hxT[r] = hyE[r] = hyT[r] = 0.0;
            if (!live[r]) continue;
            const int idx = tid + r * kBlock;
            const int si = sidx[r];
            const int i = ix[r], j = jx[r];
            const double E = oE[r], T = oT[r], z = oz[r], dE = odE[r], dT = odT[r];
            auto face = [&](int sa, int sb, double h, double ih, double& fe, double& ft) {
                if (MODE == 0)
                    face_flux(sl[0][sa], sl[0][sb], sl[1][sa], sl[1][sb], sl[2][sa], sl[2][sb], h,
                              ih, kappa, lam, fe, ft);
                else
                    face_flux_tan(sl[0][sa], sl[0][sb], sl[1][sa], sl[1][sb], sl[2][sa],
                                  sl[2][sb], sl[NA - 2][sa], sl[NA - 2][sb], sl[NA - 1][sa],
                                  sl[NA - 1][sb], h, ih, kappa, lam, fe, ft);
            };
            if (i == 0 && (p.phys & 1)) {
                if (p.robin & 1) lxE[r] = -robin_any<MODE>(E, T, z, q.R[0], hx, dE, dT);
            } else {
                face(si - 1, si, hx, ihx, lxE[r], lxT[r]);
            }
            if (j == 0 && ((p.phys >> 2) & 1)) {
                if ((p.robin >> 2) & 1) lyE[r] = -robin_any<MODE>(E, T, z, q.R[2], hy, dE, dT);
            } else {
                face(si - sy, si, hy, ihy, lyE[r], lyT[r]);
            }
            if (i == nx - 1 && ((p.phys >> 1) & 1)) {
                if ((p.robin >> 1) & 1) hxE[r] = robin_any<MODE>(E, T, z, q.R[1], hx, dE, dT);
            } else if (!(i < nx - 1 && idx + 1 < t.cnt)) {
                face(si, si + 1, hx, ihx, hxE[r], hxT[r]);
            }
            if (j == ny - 1 && ((p.phys >> 3) & 1)) {
                if ((p.robin >> 3) & 1) hyE[r] = robin_any<MODE>(E, T, z, q.R[3], hy, dE, dT);
            } else if (!(idx + nx < t.cnt)) {
                face(si, si + sy, hy, ihy, hyE[r], hyT[r]);
            }
        }
        __syncthreads();
        // phase B: publish low fluxes, stage plane k + 1
#pragma unroll
        for (int r = 0; r < kStageCPT; ++r) {
            const int idx = tid + r * kBlock;
            fl[0][idx] = lxE[r];
            fl[1][idx] = lxT[r];
            fl[2][idx] = lyE[r];
            fl[3][idx] = lyT[r];
        }
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
            for (int w = 0; w < kStagePer; ++w) {
                const int e = tid + w * kBlock;
                if (e < len) sl[a][e] = pre[a][w];
            }
        __syncthreads();
        // phase C: high faces, z faces, cell terms
#pragma unroll
        for (int r = 0; r < kStageCPT; ++r) {
            const int idx = tid + r * kBlock;
            const int si = sidx[r];
            const double nE = sl[0][si], nT = sl[1][si], nz3 = sl[2][si];
            const double ndE = MODE ? sl[NA - 2][si] : 0.0;
            const double ndT = MODE ? sl[NA - 1][si] : 0.0;
            if (live[r]) {
                const int i = ix[r];
                const int c = cn[r] + sz * (k + 1);
                const double E = oE[r], T = oT[r], z = oz[r], dE = odE[r], dT = odT[r];
                if (i < nx - 1 && idx + 1 < t.cnt && !(i == nx - 1 && ((p.phys >> 1) & 1))) {
                    hxE[r] = fl[0][idx + 1];
                    hxT[r] = fl[1][idx + 1];
                }
                if (idx + nx < t.cnt && !(jx[r] == ny - 1 && ((p.phys >> 3) & 1))) {
                    hyE[r] = fl[2][idx + nx];
                    hyT[r] = fl[3][idx + nx];
                }
                double hzE = 0.0, hzT = 0.0;
                if (k == nz - 1 && zhi_p) {
                    if ((p.robin >> 5) & 1) hzE = robin_any<MODE>(E, T, z, q.R[5], hz, dE, dT);
                } else if (MODE == 0) {
                    face_flux(E, nE, T, nT, z, nz3, hz, ihz, kappa, lam, hzE, hzT);
                } else {
                    face_flux_tan(E, nE, T, nT, z, nz3, dE, ndE, dT, ndT, hz, ihz, kappa, lam,
                                  hzE, hzT);
                }
                double l_xE = lxE[r], l_xT = lxT[r], l_yE = lyE[r], l_yT = lyT[r];
                double h_xE = hxE[r], h_xT = hxT[r], h_yE = hyE[r], h_yT = hyT[r];
                double l_zE = czE[r], l_zT = czT[r];
                czE[r] = hzE;
                czT[r] = hzT;
                const int ct = use_ct ? ctype[c] : 0;
                if (ct & CT_COVERED) {
                    out[c] = 0.0;
                    out[c + nl] = 0.0;
                } else {
                    if (ct & (1 << 1)) l_xE = l_xT = 0.0;
                    if (ct & (1 << 2)) h_xE = h_xT = 0.0;
                    if (ct & (1 << 3)) l_yE = l_yT = 0.0;
                    if (ct & (1 << 4)) h_yE = h_yT = 0.0;
                    if (ct & (1 << 5)) l_zE = l_zT = 0.0;
                    if (ct & (1 << 6)) hzE = hzT = 0.0;
                    const double divE =
                        (h_xE - l_xE) * ihx + (h_yE - l_yE) * ihy + (hzE - l_zE) * ihz;
                    const double divT =
                        (h_xT - l_xT) * ihx + (h_yT - l_yT) * ihy + (hzT - l_zT) * ihz;
                    double rE, rT;
                    if (MODE == 0)
                        cell_out0(q, E, T, z, bE[r], bT[r], divE, divT, rE, rT);
                    else
                        cell_out1(q, E, T, z, dE, dT, divE, divT, rE, rT);
                    out[c] = rE;
                    out[c + nl] = rT;
                }
            }
            oE[r] = nE;
            oT[r] = nT;
            oz[r] = nz3;
            odE[r] = ndE;
            odT[r] = ndT;
        }
    }
}

// Flux matching: a coarse face bordering a finer level carries the mean of
// the four fine fluxes (Sec. 3.2.1).  The stencil skipped that face; add
// -dt * (+-mean) / h_c here.  One thread per coarse cell (no races).
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_reflux(
    const RefluxCell* __restrict__ rc, int n, const RefluxFace* __restrict__ rf,
    const PatchInfo* __restrict__ P, const ProbScalars* __restrict__ ps,
    const int32_t* __restrict__ active, const double* __restrict__ u,
    const double* __restrict__ v, const double* __restrict__ z3,
    double* __restrict__ out, int64_t nl) {
    // four lanes per coarse cell (the quad shares the cell's loop bounds)
    const int t = (blockIdx.x * blockDim.x + threadIdx.x) >> 2;
    const int k = threadIdx.x & 3;
    if (t >= n) return;
    const RefluxCell cell = rc[t];
    if (active && !active[cell.prob]) return;
    const ProbScalars& q = ps[cell.prob];
    double accE = 0.0, accT = 0.0;
    for (int e = cell.first; e < cell.first + cell.count; ++e) {
        const int face = rf[e].face;
        const int d = face >> 1;
        const bool hi = face & 1;
        const PatchInfo& fp = P[rf[e].fpatch];
        const double h = fp.h[d], ih = fp.ih[d];
        const int fi = rf[e].fine[k];
        const int g = fi + rf[e].gofs;
        const int a = hi ? g : fi;            // lower cell of the fine face
        const int b = hi ? fi : g;
        double fe, ft;
        if (MODE == 0)
            face_flux(u[a], u[b], u[a + nl], u[b + nl], z3[a], z3[b], h, ih, q.kappa, q.lam,
                      fe, ft);
        else
            face_flux_tan(u[a], u[b], u[a + nl], u[b + nl], z3[a], z3[b], v[a], v[b],
                          v[a + nl], v[b + nl], h, ih, q.kappa, q.lam, fe, ft);
        const double se = quad_sum(fe), st = quad_sum(ft);
        const double sgn = hi ? 1.0 : -1.0;
        const double ihc = 0.5 * ih;          // coarse h = 2 fine h
        accE += sgn * 0.25 * se * ihc;
        accT += sgn * 0.25 * st * ihc;
    }
    if (k == 0) {
        out[cell.c] -= q.dt * accE;
        out[cell.c + nl] -= q.dt * accT;
    }
}

static void residual_launch(const Dev& D, hipStream_t s, int t0, int nt, const int32_t* map,
                            const double* u, const double* b, double* F) {
    if (nt <= 0) return;
    if (D.bricks == 3)
        k_stencil_s<0><<<nt, kBlock, 0, s>>>(D.stiles, t0, map, D.patches, D.ps, D.active,
                                             D.ctype, u, nullptr, D.z3, b, F, D.nl);
    else if (D.bricks == 1)
        k_stencil_z<0><<<nt, kBlock, 0, s>>>(D.stiles, t0, map, D.patches, D.ps, D.active,
                                             D.ctype, u, nullptr, D.z3, b, F, D.nl);
    else if (D.bricks == 2)
        k_stencil_w<0><<<nt, kBlock, 0, s>>>(D.stiles, t0, map, D.patches, D.ps, D.active,
                                             D.ctype, u, nullptr, D.z3, b, F, D.nl);
    else
        k_stencil_flat<0><<<nt, kBlock, 0, s>>>(D.tiles, t0, map, D.patches, D.ps, D.active,
                                                D.ctype, u, nullptr, D.z3, b, F, D.nl);
}
static void jvp_launch(const Dev& D, hipStream_t s, int t0, int nt, const int32_t* map,
                       const double* u, const double* v, double* Jv) {
    if (nt <= 0) return;
    if (D.bricks == 3)
        k_stencil_s<1><<<nt, kBlock, 0, s>>>(D.stiles, t0, map, D.patches, D.ps, D.active,
                                             D.ctype, u, v, D.z3, nullptr, Jv, D.nl);
    else if (D.bricks == 1)
        k_stencil_z<1><<<nt, kBlock, 0, s>>>(D.stiles, t0, map, D.patches, D.ps, D.active,
                                             D.ctype, u, v, D.z3, nullptr, Jv, D.nl);
    else if (D.bricks == 2)
        k_stencil_w<1><<<nt, kBlock, 0, s>>>(D.stiles, t0, map, D.patches, D.ps, D.active,
                                             D.ctype, u, v, D.z3, nullptr, Jv, D.nl);
    else
        k_stencil_flat<1><<<nt, kBlock, 0, s>>>(D.tiles, t0, map, D.patches, D.ps, D.active,
                                                D.ctype, u, v, D.z3, nullptr, Jv, D.nl);
}
static int stencil_tiles(const Dev& D) {
    return D.bricks ? D.level_stile0[D.nlev] : D.level_tile0[D.nlev];
}

void residual(const Dev& D, hipStream_t s, int t0, int nt, const double* u, const double* b,
              double* F) {
    residual_launch(D, s, t0, nt, nullptr, u, b, F);
}
void residual_all(const Dev& D, hipStream_t s, const double* u, const double* b, double* F) {
    if (D.active && D.amap)
        residual_launch(D, s, 0, D.namap, D.amap, u, b, F);
    else
        residual_launch(D, s, 0, stencil_tiles(D), nullptr, u, b, F);
}
void residual_reflux(const Dev& D, hipStream_t s, const double* u, double* F) {
    if (D.nrcells == 0) return;
    k_reflux<0><<<nblocks(4 * (int64_t)D.nrcells), kBlock, 0, s>>>(D.rcells, D.nrcells, D.rfaces,
                                                      D.patches, D.ps, D.active, u,
                                                      nullptr, D.z3, F, D.nl);
}
void jvp(const Dev& D, hipStream_t s, int t0, int nt, const double* u, const double* v,
         double* Jv) {
    jvp_launch(D, s, t0, nt, nullptr, u, v, Jv);
}
void jvp_all(const Dev& D, hipStream_t s, const double* u, const double* v, double* Jv) {
    if (D.active && D.amap)
        jvp_launch(D, s, 0, D.namap, D.amap, u, v, Jv);
    else
        jvp_launch(D, s, 0, stencil_tiles(D), nullptr, u, v, Jv);
}
void jvp_reflux(const Dev& D, hipStream_t s, const double* u, const double* v, double* Jv) {
    if (D.nrcells == 0) return;
    k_reflux<1><<<nblocks(4 * (int64_t)D.nrcells), kBlock, 0, s>>>(D.rcells, D.nrcells, D.rfaces,
                                                      D.patches, D.ps, D.active, u, v,
                                                      D.z3, Jv, D.nl);
}

}  // namespace nrd
