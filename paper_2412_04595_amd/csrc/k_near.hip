// Near field (eq. phiNDR): Phi^N_i = sum'_{j, n: |r_ij + n o L| < r_c} q_j N(|r_ij + n o L|),
// N(r) = 1/r - F(r) (eq. SOGDEcomp), over xy images only (z is free), with a cell list
// of cells at least r_c wide (the paper's cell list, Sec. 2.2).
//
// F(r) and F'(r)/r are evaluated as Chebyshev series in x = 2 r^2/r_c^2 - 1 (Clenshaw),
// so the cost per pair does not depend on the number of Gaussians M (Remark rmk::sum
// asks for that; a polynomial in r^2 is this library's way of getting it).
//
// Coordinates enter the pair kernel as offsets from the particle's cell corner, formed
// in float64, so the float32 form does not lose the ~1e-5 absolute precision that raw
// float32 coordinates of a 100-wide box would.
#include "device_common.hpp"

namespace sog {

namespace {

struct NearGeom {
    double L[3];
    double ch[3];
    int nc[3];
};

__device__ __forceinline__ void cell_of(const NearGeom& g, double xw, double yw, double z, int c[3]) {
    double v[3] = {xw, yw, z};
    for (int d = 0; d < 3; ++d) {
        int k = (int)floor(v[d] / g.ch[d]);
        c[d] = min(max(k, 0), g.nc[d] - 1);
    }
}

__global__ void k_near_key(const double* __restrict__ x, int n, NearGeom g, int* __restrict__ key) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double xw = wrap_periodic(x[3 * i], g.L[0]), yw = wrap_periodic(x[3 * i + 1], g.L[1]);
        double z = x[3 * i + 2];
        if (!isfinite(xw)) xw = 0;
        if (!isfinite(yw)) yw = 0;
        if (!isfinite(z)) z = 0;
        int c[3];
        cell_of(g, xw, yw, z, c);
        key[i] = (c[0] * g.nc[1] + c[1]) * g.nc[2] + c[2];
    }
}

template <typename real>
__global__ void k_near_pack(const double* __restrict__ x, const double* __restrict__ q, int n, NearGeom g,
                            const int* __restrict__ perm, vec4<real>* __restrict__ pos, int* __restrict__ cell,
                            int* __restrict__ orig) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
        int i = perm[p];
        double xw = wrap_periodic(x[3 * i], g.L[0]), yw = wrap_periodic(x[3 * i + 1], g.L[1]);
        double z = x[3 * i + 2];
        double qq = q[i];
        if (!isfinite(xw)) xw = 0;
        if (!isfinite(yw)) yw = 0;
        if (!isfinite(z)) z = 0;
        if (!isfinite(qq)) qq = 0;
        int c[3];
        cell_of(g, xw, yw, z, c);
        vec4<real> v;
        v.x = (real)(xw - c[0] * g.ch[0]);
        v.y = (real)(yw - c[1] * g.ch[1]);
        v.z = (real)(z - c[2] * g.ch[2]);
        v.w = (real)qq;
        pos[p] = v;
        cell[p] = (c[0] * g.nc[1] + c[1]) * g.nc[2] + c[2];
        orig[p] = i;
    }
}

template <typename real>
struct NearArgs {
    const vec4<real>* pos;
    const int* cell;
    const int* orig;
    const int* cell_start;
    real* pphi;   // part 0 potentials (n)
    real* pgrad;  // part 0 gradients (n x 3)
    int n;
    int nc[3];
    real ch[3];
    real rc2, inv_rc2;
    int deg;
    real cF[kMaxNearDeg + 1];
    real cG[kMaxNearDeg + 1];
};

// One thread per target, targets in cell order so a wave walks the same neighbour cells.
template <typename real>
__global__ __launch_bounds__(256) void k_near(NearArgs<real> a) {
    const int nblk = (a.n + blockDim.x - 1) / blockDim.x;
    const int lb = xcd_logical_block(nblk);
    if (lb < 0) return;
    const int p = lb * blockDim.x + threadIdx.x;
    if (p >= a.n) return;
    const vec4<real> me = a.pos[p];
    const int cid = a.cell[p];
    const int cz = cid % a.nc[2], cy = (cid / a.nc[2]) % a.nc[1], cx = cid / (a.nc[2] * a.nc[1]);
    real phi = 0, gx = 0, gy = 0, gz = 0;
    for (int dz = -1; dz <= 1; ++dz) {
        const int zz = cz + dz;
        if (zz < 0 || zz >= a.nc[2]) continue;
        for (int dy = -1; dy <= 1; ++dy) {
            const int yy = imod(cy + dy, a.nc[1]);
            for (int dx = -1; dx <= 1; ++dx) {
                const int xx = imod(cx + dx, a.nc[0]);
                const int nb = (xx * a.nc[1] + yy) * a.nc[2] + zz;
                // geometric position of the neighbour cell's corner relative to ours
                const real ox = dx * a.ch[0], oy = dy * a.ch[1], oz = dz * a.ch[2];
                const bool same = (dx == 0 && dy == 0 && dz == 0);
                const int b = a.cell_start[nb], e = a.cell_start[nb + 1];
                for (int j = b; j < e; ++j) {
                    const vec4<real> o = a.pos[j];
                    const real rx = me.x - (o.x + ox), ry = me.y - (o.y + oy), rz = me.z - (o.z + oz);
                    const real r2 = rx * rx + ry * ry + rz * rz;
                    if (r2 < a.rc2 && !(same && j == p)) {
                        const real xs = (real)2 * r2 * a.inv_rc2 - (real)1;
                        // Clenshaw for both series
                        real bF1 = 0, bF2 = 0, bG1 = 0, bG2 = 0;
                        for (int k = a.deg; k >= 1; --k) {
                            const real tF = a.cF[k] + (real)2 * xs * bF1 - bF2;
                            const real tG = a.cG[k] + (real)2 * xs * bG1 - bG2;
                            bF2 = bF1; bF1 = tF;
                            bG2 = bG1; bG1 = tG;
                        }
                        const real F = a.cF[0] + xs * bF1 - bF2;
                        const real G = a.cG[0] + xs * bG1 - bG2;  // F'(r)/r
                        const real ri = drsqrt(r2);
                        const real N = ri - F;
                        const real dNr = -ri * ri * ri - G;  // N'(r)/r
                        phi += o.w * N;
                        const real c = o.w * dNr;
                        gx += c * rx;
                        gy += c * ry;
                        gz += c * rz;
                    }
                }
            }
        }
    }
    const int i = a.orig[p];
    a.pphi[i] = phi;
    a.pgrad[3 * i] = gx;
    a.pgrad[3 * i + 1] = gy;
    a.pgrad[3 * i + 2] = gz;
}

template <typename real>
hipError_t run_near(Plan& p, const double* x, const double* q) {
    const Resolved& r = p.r;
    Workspace& ws = p.ws;
    const int n = (int)r.n;
    NearGeom g;
    for (int d = 0; d < 3; ++d) {
        g.L[d] = r.L[d];
        g.ch[d] = r.ch[d];
        g.nc[d] = r.nc[d];
    }
    const int ncells = r.nc[0] * r.nc[1] * r.nc[2];
    int t = timer_id(p, "near_sort");
    timer_begin(p, t);
    const int blocks = std::min((n + 255) / 256, 8192);
    k_near_key<<<blocks, 256, 0, p.stream>>>(x, n, g, ws.key);
    hipError_t e = launch_counting_sort(p, ws.key, n, ncells, ws.cell_start, ws.cell_cursor, ws.perm);
    if (e != hipSuccess) return e;
    k_near_pack<real><<<blocks, 256, 0, p.stream>>>(x, q, n, g, ws.perm, (vec4<real>*)ws.near_pos, ws.near_cell,
                                                     ws.near_orig);
    timer_end(p, t);
    NearArgs<real> a;
    a.pos = (const vec4<real>*)ws.near_pos;
    a.cell = ws.near_cell;
    a.orig = ws.near_orig;
    a.cell_start = ws.cell_start;
    a.pphi = (real*)ws.parts_phi;
    a.pgrad = (real*)ws.parts_grad;
    a.n = n;
    for (int d = 0; d < 3; ++d) {
        a.nc[d] = r.nc[d];
        a.ch[d] = (real)r.ch[d];
    }
    a.rc2 = (real)(r.rc * r.rc);
    a.inv_rc2 = (real)(1.0 / (r.rc * r.rc));
    a.deg = r.near_deg;
    for (int k = 0; k <= kMaxNearDeg; ++k) {
        a.cF[k] = (real)r.near_cF[k];
        a.cG[k] = (real)r.near_cG[k];
    }
    t = timer_id(p, "near");
    timer_begin(p, t);
    k_near<real><<<xcd_grid((n + 255) / 256), 256, 0, p.stream>>>(a);
    timer_end(p, t);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_near(Plan& p, const double* x, const double* q) {
    if (p.r.prec == SOG_PREC_FP64) return run_near<double>(p, x, q);
    return run_near<float>(p, x, q);
}

}  // namespace sog
