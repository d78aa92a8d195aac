// Transposed Jacobian action of the NRD residual and its z-derivative on
// hierarchies of any depth (the residual of paper Sec. 3.1-3.3 and the
// synchronisation of Sec. 3.2.1 differentiated and run backwards).  The
// face formulas are the residual's (stencil.hip); their partial derivatives
// are written out here.
#include <hip/hip_runtime.h>

#include "device_util.h"
#include "kernels.h"

namespace nrd {

static inline int nblocks(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

// ---------------------------------------------------------------------------
// transpose (gather form): each cell collects the transposed contributions of
// its faces and of its own cell terms, so no atomics are needed.  lam's
// ghosts must hold the adjoint fill: sibling copies, and at a coarse-fine
// ghost 1/8 of the multiplier of the coarse cell it lies in (that cell's
// residual takes the mean of the four fine fluxes through the face, over the
// coarse width).  Covered cells have no residual and gather nothing here;
// faces whose flux flux matching supplies are skipped (the fine side carries
// them).  At a coarse-fine face the cell also takes the sensitivity of its
// ghost's values: 1/3 of it here (the ghost blends in the cell itself), all
// of it written to the ghost slot for the coarse sources to gather.  gz is
// per native cell and w.r.t. z (ghost z interpolates z, not z^3).
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void k_vjp(
    const Tile* __restrict__ tiles, int t0, const PatchInfo* __restrict__ P,
    const ProbScalars* __restrict__ ps, const int32_t* __restrict__ active,
    const uint8_t* __restrict__ ctype, const double* __restrict__ u,
    const double* __restrict__ lam, const double* __restrict__ z3,
    const double* __restrict__ zv, double* __restrict__ gout,
    double* __restrict__ gz, int64_t nl) {
    const Tile t = tiles[t0 + xcd_tile(blockIdx.x, gridDim.x)];
    if (active && !active[t.prob]) return;
    if ((int)threadIdx.x >= t.count) return;
    const PatchInfo& p = P[t.patch];
    const ProbScalars& q = ps[t.prob];
    int id[3];
    cell_coords(p, t.start + threadIdx.x, id[0], id[1], id[2]);
    const int c = native_index(p, id[0], id[1], id[2]);
    const bool amr = (p.flags & PF_CTYPE) != 0;
    const uint32_t ct = amr ? ctype[c] : 0u;
    if (ct & CT_COVERED) {
        gout[c] = 0.0;
        gout[c + nl] = 0.0;
        gz[c] = 0.0;
        return;
    }
    const int st[3] = {1, p.sy, p.sz};
    const double E = u[c], T = u[c + nl], z = z3[c];
    const double lE = lam[c], lT = lam[c + nl];
    const double dt = q.dt, kappa = q.kappa, lm = q.lam;
    double gE = q.c0 * lE, gT = q.c0 * lT, gZ = 0.0, gZlin = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double h = p.h[d], ih = p.ih[d];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const bool edge = id[d] == (s ? p.n[d] - 1 : 0);
            const bool phys = edge && ((p.phys >> (2 * d + s)) & 1);
            if (phys) {
                if ((p.robin >> (2 * d + s)) & 1) {
                    // F_c gets -dt q / h
                    const double R = q.R[2 * d + s];
                    const double T2 = T * T, T3 = T2 * T;
                    const double iD = rcp_nr(4.0 * T3 + 3.0 * z * h);
                    const double qq = 2.0 * T3 * (4.0 * R - E) * iD;
                    const double w = -dt * lE * ih;
                    gE += w * (-2.0 * T3) * iD;
                    gT += w * (6.0 * T2 * (4.0 * R - E) - qq * 12.0 * T2) * iD;
                    gZ += w * (-qq * 3.0 * h) * iD;
                }
                continue;
            }
            if ((ct >> (2 * d + s + 1)) & 1u) continue;    // flux matching
            const int nb = s ? c + st[d] : c - st[d];
            const bool cf = amr && edge && ctype[nb] == GK_CF;
            // face between lower a and upper b; c is a when s = 1
            const int a = s ? c : nb;
            const int bb = s ? nb : c;
            const double Ea = u[a], Eb = u[bb], Ta = u[a + nl], Tb = u[bb + nl];
            const double za = z3[a], zb = z3[bb];
            const double muE = dt * (lam[bb] - lam[a]) * ih;
            const double muT = dt * (lam[bb + nl] - lam[a + nl]) * ih;
            const double Tf = 0.5 * (Ta + Tb);
            const double Tf2 = Tf * Tf, Tf3 = Tf2 * Tf;
            const double S = Ea + Eb;
            const double dEv = Eb - Ea;
            const double adE = fabs(dEv);
            const double sg = (dEv > 0.0) ? 1.0 : ((dEv < 0.0) ? -1.0 : 0.0);
            const double Zh = 3.0 * (za + zb) * h;
            const double iD = rcp_nr(Zh * S + 4.0 * lm * Tf3 * adE);
            const double phi = 2.0 * Tf3 * S * dEv * iD;
            // partials of Phi_E w.r.t. c's own E, T, z^3
            const double sE = s ? -1.0 : 1.0;              // d(dE)/dE_c
            const double dN_E = 2.0 * Tf3 * (S * sE + dEv);
            const double dD_E = Zh + 4.0 * lm * Tf3 * sg * sE;
            const double dN_T = 3.0 * Tf2 * S * dEv;
            const double dD_T = 6.0 * lm * Tf2 * adE;
            const double dD_z = 3.0 * h * S;
            const double pT = muE * (dN_T - phi * dD_T) * iD;
            const double pZ = muE * (-phi * dD_z) * iD;
            gE += muE * (dN_E - phi * dD_E) * iD;
            gT += pT;
            gZ += pZ;
            const double sq = Tf * rsqrt_nr(Tf);
            const double DT = kappa * Tf2 * sq;
            const double base = 1.25 * kappa * Tf * sq * (Tb - Ta);
            gT += muT * (base + (s ? -DT : DT)) * ih;
            if (cf) {
                // the same partials w.r.t. the ghost's E, T, z
                const double gEn = muE * (2.0 * Tf3 * (dEv - S * sE) -
                                          phi * (Zh - 4.0 * lm * Tf3 * sg * sE)) * iD;
                const double gTn = pT + muT * (base + (s ? DT : -DT)) * ih;
                const double zg = zv[nb];
                const double gZn = 3.0 * zg * zg * pZ;
                gE += (1.0 / 3.0) * gEn;
                gT += (1.0 / 3.0) * gTn;
                gZlin += (1.0 / 3.0) * gZn;
                gout[nb] = gEn;
                gout[nb + nl] = gTn;
                gz[nb] = gZn;
            }
        }
    }
    const double T2 = T * T, T3 = T2 * T;
    const double r3 = rcp_nr(T3);
    const double x = lT - lE;
    gE += dt * x * (-z * r3);
    gT += dt * x * z * (1.0 + 3.0 * E * r3 * rcp_nr(T));
    gZ += dt * x * (T - E * r3);
    const double zc = zv[c];
    gout[c] = gE;
    gout[c + nl] = gT;
    gz[c] = 3.0 * zc * zc * gZ + gZlin;
}

// Coarse cells gather 2/3 x w/16 of the sensitivities left in the ghost
// slots they feed (E, T and z).
__global__ __launch_bounds__(kBlock) void k_cf_gather(
    const CFRow* __restrict__ rows, int n, const CFSrc* __restrict__ src,
    const int32_t* __restrict__ active, double* __restrict__ g, double* __restrict__ gz,
    int64_t nl) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const CFRow row = rows[r];
    if (active && !active[row.prob]) return;
    double aE = 0.0, aT = 0.0, aZ = 0.0;
    for (int k = row.first; k < row.first + row.count; ++k) {
        const CFSrc e = src[k];
        const double w = (2.0 / 3.0) * (e.w * 0.0625);
        aE += w * g[e.ghost];
        aT += w * g[e.ghost + nl];
        aZ += w * gz[e.ghost];
    }
    g[row.c] += aE;
    g[row.c + nl] += aT;
    gz[row.c] += aZ;
}

void vjp_full(const Dev& D, hipStream_t s, const double* u, double* lam, double* JTl,
              double* gz) {
    adjoint_ghost_fill(D, s, lam);
    const int nt = D.level_tile0[D.nlev];
    if (nt > 0)
        k_vjp<<<nt, kBlock, 0, s>>>(D.tiles, 0, D.patches, D.ps, D.active, D.ctype, u, lam,
                                    D.z3, D.z, JTl, gz, D.nl);
    if (D.ncfrows > 0)
        k_cf_gather<<<nblocks(D.ncfrows), kBlock, 0, s>>>(D.cfrows, D.ncfrows, D.cfsrc,
                                                          D.active, JTl, gz, D.nl);
    restrict_transpose(D, s, JTl, 2);
}

}  // namespace nrd
