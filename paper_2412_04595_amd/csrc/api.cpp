// The C ABI (include/sog.h): plans, device workspace, the call pipeline and timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"
#include "launch.hpp"

namespace sog {

namespace {
thread_local std::string g_last_error;
const double kPi = 3.14159265358979323846;

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

size_t real_size(const Resolved& r) { return r.prec == SOG_PREC_FP64 ? 8 : 4; }

sog_status hip_status(hipError_t e, const char* what) {
    if (e == hipSuccess) return SOG_OK;
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    if (e == hipErrorOutOfMemory) return SOG_ERR_OUT_OF_MEMORY;
    return SOG_ERR_DEVICE;
}

// Allocation with an optional cap (SOG_MAX_DEVICE_BYTES) so that the out-of-memory
// path can be exercised from the host.
struct Allocator {
    std::vector<void*> ptrs;
    size_t total = 0;
    size_t cap = SIZE_MAX;
    hipError_t err = hipSuccess;
    bool capped = false;
    Allocator() {
        const char* c = std::getenv("SOG_MAX_DEVICE_BYTES");
        if (c && *c) cap = (size_t)std::strtoull(c, nullptr, 10);
    }
    template <typename T>
    void get(T*& out, size_t bytes) {
        out = nullptr;
        if (err != hipSuccess || capped) return;
        bytes = std::max<size_t>(bytes, 16);
        bytes = (bytes + 255) & ~(size_t)255;
        if (total + bytes > cap) { capped = true; return; }
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) { err = e; return; }
        ptrs.push_back(p);
        total += bytes;
        out = (T*)p;
    }
};

template <typename T>
std::vector<T> to_real(const std::vector<double>& v) {
    std::vector<T> o(v.size());
    for (size_t i = 0; i < v.size(); ++i) o[i] = (T)v[i];
    return o;
}

// e^{-2 pi i t / n}, t < n, as interleaved (re, im)
std::vector<double> twiddles(int n, int count) {
    std::vector<double> t(2 * (size_t)count);
    for (int k = 0; k < count; ++k) {
        double a = -2.0 * kPi * (double)k / (double)n;
        t[2 * k] = std::cos(a);
        t[2 * k + 1] = std::sin(a);
    }
    return t;
}

hipError_t upload(void* dst, const std::vector<double>& v, bool f64) {
    if (v.empty()) return hipSuccess;
    if (f64) return hipMemcpy(dst, v.data(), v.size() * 8, hipMemcpyHostToDevice);
    std::vector<float> f = to_real<float>(v);
    return hipMemcpy(dst, f.data(), f.size() * 4, hipMemcpyHostToDevice);
}

// 1 / What(k)^2 for the Gaussian window (eq. GS), exponent returned separately
double inv_what2_log(double k, double H, double S, double* pref) {
    *pref = S / (kPi * H * H);
    return k * k * H * H / (2.0 * S);
}

// The static scratch of sog_energy_potential_force_static: device memory the library holds
// on every device it runs on from the load of its code object to the end of the process,
// for callers that cannot allocate.  Host code never uses the array's name as an address:
// static_scratch(dev) looks up its device address once per device.
constexpr size_t kStaticScratchBytes = (size_t)128 << 20;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of the scratch on device dev (current device set by the caller);
// looked up on the first use per device.
sog_status static_scratch(int dev, void** out) {
    *out = nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device ordinal out of range for the static scratch");
        return SOG_ERR_INVALID_ARG;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_status(e != hipSuccess ? e : hipErrorInvalidSymbol, "static scratch address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SOG_OK;
}

// Point the plan's per-call buffers into a region of at least p.region_bytes bytes (or
// clear them for nullptr).
void bind_region(Plan& p, void* base) {
    for (auto& sl : p.region_slots) *sl.first = base ? (void*)((char*)base + sl.second) : nullptr;
}

// Offsets of the per-call buffers (everything a call overwrites before it reads it) inside
// one region, 256-byte aligned: the plan's own allocation, or any other region of at least
// `total` bytes (bind_region).
struct Layout {
    std::vector<std::pair<void**, size_t>> slots;
    size_t total = 0;
    template <typename T>
    void get(T*& field, size_t bytes) {
        field = nullptr;
        bytes = (std::max<size_t>(bytes, 16) + 255) & ~(size_t)255;
        slots.push_back({reinterpret_cast<void**>(&field), total});
        total += bytes;
    }
};

sog_status build_plan(Plan& p) {
    Resolved& r = p.r;
    Workspace& ws = p.ws;
    const bool f64 = r.prec == SOG_PREC_FP64;
    const size_t rs = real_size(r), cs = 2 * rs;
    const int64_t n = r.n;
    Allocator A;  // tables, written once here
    Layout W;     // per-call buffers
    if (!p.on_device || p.graphable) {  // host staging, or the graph's fixed inputs and outputs
        W.get(ws.x, 3 * n * 8);
        W.get(ws.q, n * 8);
        W.get(ws.phi, n * 8);
        W.get(ws.force, 3 * n * 8);
        W.get(ws.energy, 8);
    }
    W.get(ws.qsum, kQsumSlots * 2 * 8);
    W.get(ws.status, 4);
    W.get(ws.parts, 12 * n * rs);
    W.get(ws.key, n * 8);  // near-field (cell, rank) pairs; the long-range FFT form's keys
    W.get(ws.perm, n * 4);
    const int ncells = r.nc[0] * r.nc[1] * r.nc[2];
    int64_t maxbins = ncells;
    W.get(ws.cell_start, (ncells + 1) * 4);
    W.get(ws.near_orig, n * 4);
    W.get(ws.near_pos, n * 4 * rs);
    if (f64) W.get(ws.near_pos32, n * 16);  // the float32 candidate test's copy
    W.get(ws.near_units, ((size_t)near_unit_slots(r) * 16 + 127) / 128 * 128 + 8 * 128);  // units, then 8 work counters
    if (r.has_mid) {
        const int ntiles = r.ntile[0] * r.ntile[1] * r.ntile[2];
        maxbins = std::max<int64_t>(maxbins, (int64_t)ntiles * kMidSub);
        const int Kz = r.Izs / 2 + 1;
        W.get(ws.tile_start, ((int64_t)ntiles * kMidSub + 1) * 4);
        A.get(ws.spread_nodes, 2 * 4 * 64);
        W.get(ws.mid_g, n * 16);
        W.get(ws.mid_u, n * 4 * rs);
        W.get(ws.grid, (size_t)r.I[0] * r.I[1] * r.Izs * rs);
        W.get(ws.cgrid, (size_t)r.I[0] * r.I[1] * cgrid_stride(r.Izs) * cs);
        A.get(ws.tw_x, r.I[0] * cs);
        A.get(ws.tw_y, r.I[1] * cs);
        A.get(ws.tw_z, (r.Izs / 2) * cs);
        A.get(ws.tw_zpost, Kz * cs);
        A.get(ws.mult_ax, (size_t)(r.m + 1) * r.I[0] * rs);
        A.get(ws.mult_ay, (size_t)(r.m + 1) * r.I[1] * rs);
        A.get(ws.mult_az, (size_t)(r.m + 1) * Kz * rs);
        A.get(ws.mult_c, (size_t)(r.m + 1) * rs);
        if (r.window == SOG_WINDOW_KB) A.get(ws.wpoly, (size_t)r.Pw * window_poly_row(r.nu) * rs);
    }
    if (r.has_long) {
        if (r.form == SOG_LONG_DIRECT) {
            ws.long_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + 1023) / 1024));
            A.get(ws.long_kt, (size_t)r.nh * r.P * r.P * 8);
            W.get(ws.long_mu, (size_t)ws.long_blocks * r.nh * r.P * 16);
            W.get(ws.long_a, (size_t)r.nh * r.P * cs);
        } else {
            const int nt2 = r.ntile2[0] * r.ntile2[1];
            const int planes = std::max(r.P, r.Ps);
            const int Ky = r.I2[1] / 2 + 1;
            maxbins = std::max<int64_t>(maxbins, nt2 + 1);
            W.get(ws.l2_tile_start, (nt2 + 1) * 4);
            W.get(ws.l2_tile_cursor, nt2 * 4);
            W.get(ws.l2_g, n * 16);
            W.get(ws.l2_u, n * 4 * rs);
            W.get(ws.l2_grid, (size_t)planes * r.I2[0] * r.I2[1] * rs);
            W.get(ws.l2_cgrid, (size_t)planes * r.I2[0] * cgrid_stride(r.I2[1]) * cs);
            A.get(ws.l2_tw_x, r.I2[0] * cs);
            A.get(ws.l2_tw_y, (r.I2[1] / 2) * cs);
            A.get(ws.l2_tw_ypost, Ky * cs);
            if (r.Q > 0) {
                A.get(ws.l2_el, (size_t)(r.M - r.m) * rs);
                A.get(ws.l2_coef, (size_t)(r.M - r.m) * r.Q * rs);
                A.get(ws.l2_bp, (size_t)r.Q * r.P * r.Ps * rs);
                A.get(ws.l2_winv_x, r.I2[0] * rs);
                A.get(ws.l2_winv_y, Ky * rs);
            } else {
                A.get(ws.l2_kt_r, (size_t)(r.I2[0] / 2 + 1) * Ky * r.P * r.Ps * rs);
            }
        }
    }
    W.get(ws.scan_tmp, ((maxbins + 1) / 1024 + 2) * 4);
    if (r.has_mid) {
        W.get(ws.key2, n * 8);  // mid-range (tile, rank) pairs
        W.get(ws.scan_tmp2, ((maxbins + 1) / 1024 + 2) * 4);
    }
    if (r.deterministic) {
        // bin member lists of the canonical order: the near-field and long-range sorts run
        // one after the other, the mid range's beside them
        W.get(ws.det_idx, n * 4);
        if (r.has_mid) W.get(ws.det_idx2, n * 4);
        if (r.has_long && r.form == SOG_LONG_FFT) W.get(ws.det_rank, n * 4);
    }
    ws.red_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(1024, (n + 255) / 256));
    W.get(ws.red, ws.red_blocks * 8);
    p.region_slots = W.slots;
    p.region_bytes = W.total;
    if (!p.static_region) A.get(p.region, W.total);
    ws.bytes = A.total;
    auto release = [&]() {
        for (void* q : A.ptrs) (void)hipFree(q);
        ws = Workspace();
        p.region = nullptr;
    };
    if (A.capped) {
        release();
        set_error("device workspace exceeds SOG_MAX_DEVICE_BYTES");
        return SOG_ERR_OUT_OF_MEMORY;
    }
    if (A.err != hipSuccess) {
        sog_status s = hip_status(A.err, "hipMalloc");
        release();
        return s;
    }
    bind_region(p, p.region);
    // tables (float64 on the host)
    hipError_t e = hipSuccess;
    if (r.has_mid) {
        if (!factor_fft(r.I[0], p.fx) || !factor_fft(r.I[1], p.fy) || !factor_fft(r.Izs / 2, p.fz)) {
            release();
            set_error("mid FFT length is not 2,3,5,7-smooth");
            return SOG_ERR_INVALID_ARG;
        }
        const int Kz = r.Izs / 2 + 1;
        if (e == hipSuccess) e = upload(ws.tw_x, twiddles(r.I[0], r.I[0]), f64);
        if (e == hipSuccess) e = upload(ws.tw_y, twiddles(r.I[1], r.I[1]), f64);
        if (e == hipSuccess) e = upload(ws.tw_z, twiddles(r.Izs / 2, r.Izs / 2), f64);
        if (e == hipSuccess) e = upload(ws.tw_zpost, twiddles(r.Izs, Kz), f64);
        // separable factors of Ghat_mid(k) / What(k)^2 per Gaussian
        const int nl = r.m + 1;
        std::vector<double> ax((size_t)nl * r.I[0]), ay((size_t)nl * r.I[1]), az((size_t)nl * Kz), cl(nl);
        const double Ng = (double)r.I[0] * r.I[1] * r.Izs;
        auto fill = [&](std::vector<double>& t, int cnt, int N, double Ld, double H, double hd) {
            // 1 / What(k)^2 of the ES and KB windows: h What_g(k h), What_g by quadrature (ES)
            // or in closed form (KB)
            const bool shaped = r.window == SOG_WINDOW_ES || r.window == SOG_WINDOW_KB;
            std::vector<double> inv_es2;
            if (shaped) {
                inv_es2.resize(cnt);
                for (int i = 0; i < cnt; ++i) {
                    const int f = (cnt == N && i >= (N + 1) / 2) ? i - N : i;
                    const double kap = 2.0 * kPi * f / Ld * hd;
                    const double w = hd * (r.window == SOG_WINDOW_ES ? es_hat_grid(kap, r.Pw, r.beta)
                                                                     : kb_hat_grid(kap, r.Pw, r.beta));
                    inv_es2[i] = 1.0 / (w * w);
                }
            }
            for (int l = 0; l < nl; ++l)
                for (int i = 0; i < cnt; ++i) {
                    // FFT frequency index: 0, 1, .., -1 over a full line (x, y); 0 .. N/2
                    // over the half spectrum (z)
                    const int f = (cnt == N && i >= (N + 1) / 2) ? i - N : i;
                    double k = 2.0 * kPi * f / Ld;
                    if (shaped) {
                        t[(size_t)l * cnt + i] = inv_es2[i] * std::exp(-r.s[l] * r.s[l] * k * k / 4.0);
                        continue;
                    }
                    double pref;
                    double ex = -r.s[l] * r.s[l] * k * k / 4.0 + inv_what2_log(k, H, r.S, &pref);
                    t[(size_t)l * cnt + i] = pref * std::exp(std::min(ex, 80.0));
                }
        };
        fill(ax, r.I[0], r.I[0], r.L[0], r.H[0], r.h[0]);
        fill(ay, r.I[1], r.I[1], r.L[1], r.H[1], r.h[1]);
        fill(az, Kz, r.Izs, r.Lzs, r.H[2], r.h[2]);
        for (int l = 0; l < nl; ++l) cl[l] = std::pow(kPi, 1.5) * r.w[l] * r.s[l] * r.s[l] * r.s[l] / Ng;
        if (e == hipSuccess) e = upload(ws.mult_ax, ax, f64);
        if (e == hipSuccess) e = upload(ws.mult_ay, ay, f64);
        if (e == hipSuccess) e = upload(ws.mult_az, az, f64);
        if (e == hipSuccess) e = upload(ws.mult_c, cl, f64);
        if (e == hipSuccess && r.window == SOG_WINDOW_KB) {
            std::vector<double> coef, padded;
            window_poly_fit(r.Pw, r.beta, r.nu, coef);
            // rows of window_poly_row(nu) coefficients, highest degree first: leading zeros
            const int row = window_poly_row(r.nu), pad = row - (r.nu + 1);
            padded.assign((size_t)r.Pw * row, 0.0);
            for (int o = 0; o < r.Pw; ++o)
                for (int j = 0; j <= r.nu; ++j) padded[(size_t)o * row + pad + j] = coef[(size_t)o * (r.nu + 1) + j];
            e = upload(ws.wpoly, padded, f64);
        }
        if (e == hipSuccess) e = hipMemcpy(ws.spread_nodes, r.node_oy, 4 * 64, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(ws.spread_nodes + 4 * 64, r.node_oz, 4 * 64, hipMemcpyHostToDevice);
    }
    if (r.has_long) {
        if (r.form == SOG_LONG_DIRECT) {
            std::vector<double> k2(r.nh);
            int kk = 0;
            for (int ny = 0; ny <= r.nk[1]; ++ny)
                for (int nx = (ny == 0 ? 0 : -r.nk[0]); nx <= r.nk[0]; ++nx, ++kk) {
                    double kx = 2.0 * kPi * nx / r.L[0], ky = 2.0 * kPi * ny / r.L[1];
                    k2[kk] = kx * kx + ky * ky;
                }
            std::vector<double> kt((size_t)r.nh * r.P * r.P);
            long_kernel_cheb_basis(r, k2.data(), r.nh, kt.data());
            if (e == hipSuccess) e = hipMemcpy(ws.long_kt, kt.data(), kt.size() * 8, hipMemcpyHostToDevice);
        } else {
            if (!factor_fft(r.I2[0], p.f2x) || !factor_fft(r.I2[1] / 2, p.f2y)) {
                release();
                set_error("long-range FFT length is not 2,3,5,7-smooth");
                return SOG_ERR_INVALID_ARG;
            }
            const int Ky = r.I2[1] / 2 + 1;
            if (e == hipSuccess) e = upload(ws.l2_tw_x, twiddles(r.I2[0], r.I2[0]), f64);
            if (e == hipSuccess) e = upload(ws.l2_tw_y, twiddles(r.I2[1] / 2, r.I2[1] / 2), f64);
            if (e == hipSuccess) e = upload(ws.l2_tw_ypost, twiddles(r.I2[1], Ky), f64);
            const double norm = 1.0 / ((double)r.I2[0] * r.I2[1]);
            // 1 / What2(k)^2 per direction (Gaussian window, eq. GS)
            auto winv = [&](int d, int cnt) {
                std::vector<double> v(cnt);
                for (int i = 0; i < cnt; ++i) {
                    const int N = r.I2[d];
                    const int f = (cnt == N && i >= (N + 1) / 2) ? i - N : i;
                    const double k = 2.0 * kPi * f / r.L[d];
                    double pref;
                    const double ex = inv_what2_log(k, r.H2[d], r.S2, &pref);
                    v[i] = pref * std::exp(std::min(ex, 80.0));
                }
                return v;
            };
            const std::vector<double> wx = winv(0, r.I2[0]), wy = winv(1, Ky);
            if (r.Q > 0) {
                // App. C: A_p(k) = sum_l coef[l][p] e^{-el[l] |k|^2}, with pi, the signs,
                // factorials, L_z^{2p} s_l^{2-2p} and the unnormalised inverse folded in
                const int nl = r.M - r.m;
                std::vector<double> el(nl), coef((size_t)nl * r.Q);
                for (int l = 0; l < nl; ++l) {
                    const double sl = r.s[r.m + 1 + l], s2 = sl * sl;
                    el[l] = s2 / 4.0;
                    double c = kPi * r.w[r.m + 1 + l] * s2 * norm;  // p = 0
                    for (int q = 0; q < r.Q; ++q) {
                        coef[(size_t)l * r.Q + q] = c;
                        c *= -(r.L[2] * r.L[2]) / (s2 * (q + 1));
                    }
                }
                // B_p[n][a]: ((z - z')/L_z)^{2p} = ((t - t')/2)^{2p}, interpolated at the P
                // Chebyshev nodes in the target t and expanded exactly in T_a(t'), a < P_s
                // (P_s = 2Q - 1 nodes reproduce every polynomial of degree 2Q - 2)
                std::vector<double> bp((size_t)r.Q * r.P * r.Ps, 0.0);
                std::vector<double> tc(r.P), te(r.Ps);
                for (int c = 0; c < r.P; ++c) tc[c] = std::cos((c + 0.5) * kPi / r.P);
                for (int c = 0; c < r.Ps; ++c) te[c] = std::cos((c + 0.5) * kPi / r.Ps);
                for (int q = 0; q < r.Q; ++q)
                    for (int nn = 0; nn < r.P; ++nn)
                        for (int a = 0; a < r.Ps; ++a) {
                            double acc = 0;
                            for (int c = 0; c < r.P; ++c)
                                for (int g = 0; g < r.Ps; ++g) {
                                    const double d = 0.5 * (tc[c] - te[g]);
                                    acc += std::cos(nn * (c + 0.5) * kPi / r.P) * std::cos(a * (g + 0.5) * kPi / r.Ps) *
                                           std::pow(d, 2 * q);
                                }
                            bp[((size_t)q * r.P + nn) * r.Ps + a] =
                                acc * (nn ? 2.0 : 1.0) / r.P * (a ? 2.0 : 1.0) / r.Ps;
                        }
                if (e == hipSuccess) e = upload(ws.l2_el, el, f64);
                if (e == hipSuccess) e = upload(ws.l2_coef, coef, f64);
                if (e == hipSuccess) e = upload(ws.l2_bp, bp, f64);
                if (e == hipSuccess) e = upload(ws.l2_winv_x, wx, f64);
                if (e == hipSuccess) e = upload(ws.l2_winv_y, wy, f64);
            } else {
                const int jx = r.I2[0] / 2 + 1;
                std::vector<double> k2((size_t)jx * Ky);
                for (int a = 0; a < jx; ++a)
                    for (int b = 0; b < Ky; ++b) {
                        const double kx = 2.0 * kPi * a / r.L[0], ky = 2.0 * kPi * b / r.L[1];
                        k2[(size_t)a * Ky + b] = kx * kx + ky * ky;
                    }
                std::vector<double> kt((size_t)jx * Ky * r.P * r.P);
                long_kernel_cheb_basis(r, k2.data(), jx * Ky, kt.data());
                // as P^2 planes over the modes (consecutive k_y adjacent: coalesced reads),
                // scaled by 1/What2^2 and the unnormalised inverse
                std::vector<double> ktp(kt.size());
                const size_t nm = (size_t)jx * Ky, pp = (size_t)r.P * r.P;
                for (int a = 0; a < jx; ++a)
                    for (int b = 0; b < Ky; ++b) {
                        const size_t md = (size_t)a * Ky + b;
                        const double sc = wx[a] * wy[b] * norm;
                        for (size_t i = 0; i < pp; ++i) ktp[i * nm + md] = kt[md * pp + i] * sc;
                    }
                if (e == hipSuccess) e = upload(ws.l2_kt_r, ktp, f64);
            }
        }
    }
    if (e != hipSuccess) {
        sog_status s = hip_status(e, "table upload");
        release();
        return s;
    }
    return SOG_OK;
}

void free_plan(Plan& p) {
    Workspace& ws = p.ws;
    // the tables (the per-call buffers live in p.region)
    void* ptrs[] = {ws.spread_nodes, ws.tw_x, ws.tw_y, ws.tw_z, ws.tw_zpost, ws.mult_ax, ws.mult_ay,
                    ws.mult_az, ws.mult_c, ws.long_modes, ws.long_kt, ws.l2_tw_x, ws.l2_tw_y, ws.l2_tw_ypost,
                    ws.l2_kt_r, ws.l2_el, ws.l2_coef, ws.l2_bp, ws.l2_winv_x, ws.l2_winv_y,
                    ws.wpoly, p.region};
    for (void* q : ptrs)
        if (q) (void)hipFree(q);
    if (p.gexec) (void)hipGraphExecDestroy(p.gexec);
    if (p.graph) (void)hipGraphDestroy(p.graph);
    if (p.cap) (void)hipStreamDestroy(p.cap);
    p.gexec = nullptr;
    p.graph = nullptr;
    p.cap = nullptr;
    p.region = nullptr;
    ws = Workspace();
    for (hipEvent_t ev : p.ev_pool) (void)hipEventDestroy(ev);
    if (p.ev_fork) (void)hipEventDestroy(p.ev_fork);
    if (p.ev_join) (void)hipEventDestroy(p.ev_join);
    if (p.ev_grid) (void)hipEventDestroy(p.ev_grid);
    if (p.side) (void)hipStreamDestroy(p.side);
    p.ev_fork = p.ev_join = p.ev_grid = nullptr;
    p.side = nullptr;
    for (auto& pe : p.pending) {
        (void)hipEventDestroy(pe.second.first);
        (void)hipEventDestroy(pe.second.second);
    }
    p.ev_pool.clear();
    p.pending.clear();
}

hipEvent_t take_event(Plan& p) {
    if (!p.ev_pool.empty()) {
        hipEvent_t e = p.ev_pool.back();
        p.ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

hipError_t collect_timers(Plan& p) {
    if (!p.timing) return hipSuccess;
    hipError_t e = hipStreamSynchronize(p.stream);
    for (auto& pe : p.pending) {
        float ms = 0;
        if (pe.second.first && pe.second.second && hipEventElapsedTime(&ms, pe.second.first, pe.second.second) == hipSuccess) {
            p.timers[pe.first].total_ms += ms;
            p.timers[pe.first].launches += 1;
        }
        if (pe.second.first) p.ev_pool.push_back(pe.second.first);
        if (pe.second.second) p.ev_pool.push_back(pe.second.second);
    }
    p.pending.clear();
    return e;
}

static sog_status launch_call(Plan& p, const double* x, const double* q, double* dphi, double* dforce, double* dgrad,
                              double* denergy, double* phi_parts, double* grad_parts);

sog_status run(Plan& p, const double* x_in, const double* q_in, double* energy, double* phi, double* force,
               double* grad, double* phi_parts, double* grad_parts) {
    if (!x_in || !q_in) {
        set_error("x and q must not be NULL");
        return SOG_ERR_INVALID_ARG;
    }
    DeviceGuard dg(p.device);
    Workspace& ws = p.ws;
    const int64_t n = p.r.n;
    const double* x = x_in;
    const double* q = q_in;
    hipError_t e = hipSuccess;
    if (!p.on_device) {
        e = hipMemcpyAsync(ws.x, x_in, 3 * n * 8, hipMemcpyHostToDevice, p.stream);
        if (e == hipSuccess) e = hipMemcpyAsync(ws.q, q_in, n * 8, hipMemcpyHostToDevice, p.stream);
        if (e != hipSuccess) return hip_status(e, "input copy");
        x = ws.x;
        q = ws.q;
    }
    const bool graph = p.graphable && !grad && !phi_parts && !grad_parts;
    if (graph) {
        // the graph reads its inputs from and writes its outputs to the plan's buffers
        if (p.on_device) {
            e = hipMemcpyAsync(ws.x, x_in, 3 * n * 8, hipMemcpyDeviceToDevice, p.stream);
            if (e == hipSuccess) e = hipMemcpyAsync(ws.q, q_in, n * 8, hipMemcpyDeviceToDevice, p.stream);
            if (e != hipSuccess) return hip_status(e, "input copy");
        }
        if (!p.gexec) {
            if (!p.cap && (e = hipStreamCreateWithFlags(&p.cap, hipStreamNonBlocking)) != hipSuccess)
                return hip_status(e, "capture stream");
            const hipStream_t caller = p.stream;
            p.stream = p.cap;
            e = hipStreamBeginCapture(p.cap, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) {
                p.stream = caller;
                return hip_status(e, "graph capture");
            }
            const sog_status ls = launch_call(p, ws.x, ws.q, ws.phi, ws.force, nullptr, ws.energy, nullptr, nullptr);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(p.cap, &g);
            p.stream = caller;
            if (ls != SOG_OK) {
                if (g) (void)hipGraphDestroy(g);
                return ls;
            }
            if (e != hipSuccess) return hip_status(e, "graph capture");
            p.graph = g;
            if ((e = hipGraphInstantiate(&p.gexec, p.graph, nullptr, nullptr, 0)) != hipSuccess) {
                p.gexec = nullptr;
                return hip_status(e, "graph instantiation");
            }
        }
        if ((e = hipGraphLaunch(p.gexec, p.stream)) != hipSuccess) return hip_status(e, "graph launch");
        if (p.on_device) {
            if (phi && e == hipSuccess) e = hipMemcpyAsync(phi, ws.phi, n * 8, hipMemcpyDeviceToDevice, p.stream);
            if (force && e == hipSuccess) e = hipMemcpyAsync(force, ws.force, 3 * n * 8, hipMemcpyDeviceToDevice, p.stream);
            if (energy && e == hipSuccess) e = hipMemcpyAsync(energy, ws.energy, 8, hipMemcpyDeviceToDevice, p.stream);
            if (e != hipSuccess) return hip_status(e, "output copy");
        }
    } else {
        double* dphi = p.on_device ? phi : (phi ? ws.phi : nullptr);
        double* dforce = p.on_device ? force : (force ? ws.force : nullptr);
        // host mode stages the gradient in the force buffer (the entry points ask for one of them)
        double* dgrad = p.on_device ? grad : (grad ? ws.force : nullptr);
        double* denergy = p.on_device ? energy : (energy ? ws.energy : nullptr);
        if (sog_status ls = launch_call(p, x, q, dphi, dforce, dgrad, denergy, phi_parts, grad_parts)) return ls;
    }
    if (!p.on_device && !phi_parts && !grad_parts) {
        if (phi && e == hipSuccess) e = hipMemcpyAsync(phi, ws.phi, n * 8, hipMemcpyDeviceToHost, p.stream);
        if (force && e == hipSuccess) e = hipMemcpyAsync(force, ws.force, 3 * n * 8, hipMemcpyDeviceToHost, p.stream);
        if (grad && e == hipSuccess) e = hipMemcpyAsync(grad, ws.force, 3 * n * 8, hipMemcpyDeviceToHost, p.stream);
        if (energy && e == hipSuccess) e = hipMemcpyAsync(energy, ws.energy, 8, hipMemcpyDeviceToHost, p.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
        if (e != hipSuccess) return hip_status(e, "output copy");
    }
    if ((e = collect_timers(p)) != hipSuccess) return hip_status(e, "timing");
    if (p.check) {
        double qslots[2 * kQsumSlots], qs[2] = {0.0, 0.0};
        int st = 0;
        e = hipMemcpyAsync(qslots, ws.qsum, sizeof(qslots), hipMemcpyDeviceToHost, p.stream);
        if (e == hipSuccess) e = hipMemcpyAsync(&st, ws.status, 4, hipMemcpyDeviceToHost, p.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
        if (e != hipSuccess) return hip_status(e, "status copy");
        for (int k = 0; k < kQsumSlots; ++k) {
            qs[0] += qslots[2 * k];
            qs[1] += qslots[2 * k + 1];
        }
        if (st & 1) {
            set_error("non-finite position or charge");
            return SOG_ERR_INVALID_ARG;
        }
        if (st & 2) {
            set_error("some z is outside [0, Lz]");
            return SOG_ERR_OUT_OF_BOX;
        }
        if (std::fabs(qs[0]) > 1e-10 * qs[1]) {
            set_error("charges are not neutral (|sum q| > 1e-10 sum |q|)");
            return SOG_ERR_NOT_NEUTRAL;
        }
    }
    return SOG_OK;
}

// The kernels of one call on the plan's stream (and its side stream), from the sorts to
// the combination: x, q on the device; outputs (device) as requested, or the parts.
static sog_status launch_call(Plan& p, const double* x, const double* q, double* dphi, double* dforce, double* dgrad,
                              double* denergy, double* phi_parts, double* grad_parts) {
    Workspace& ws = p.ws;
    const int64_t n = p.r.n;
    hipError_t e = hipSuccess;
    // Two streams: the near field and the long range on the plan's side stream, the mid
    // range on the caller's stream (they share no buffers: separate sort keys, scan space
    // and part records).  The ALU-bound near-field kernel waits for the gridding so that it
    // runs next to the memory-bound FFT passes and the gathering rather than next to the
    // gridding; the caller's stream waits for the side stream before the combination.
    const hipStream_t main_stream = p.stream;
    {
        struct Restore {
            Plan& p;
            hipStream_t s;
            ~Restore() { p.stream = s; }
        } restore{p, main_stream};
        if ((e = hipEventRecord(p.ev_fork, main_stream)) != hipSuccess) return hip_status(e, "fork");
        if ((e = hipStreamWaitEvent(p.side, p.ev_fork, 0)) != hipSuccess) return hip_status(e, "fork");
        p.stream = p.side;
        if ((e = launch_near(p, x, q, 1)) != hipSuccess) return hip_status(e, "near field");
        if (p.r.has_long) {
            if ((e = launch_long(p, x, q)) != hipSuccess) return hip_status(e, "long range");
        } else if ((e = launch_zero_parts(p, 2)) != hipSuccess) {
            return hip_status(e, "long range");
        }
        p.stream = main_stream;
        if (p.r.has_mid) {
            if ((e = launch_mid(p, x, q, 1)) != hipSuccess) return hip_status(e, "mid range");
        } else if ((e = launch_zero_parts(p, 1)) != hipSuccess) {
            return hip_status(e, "mid range");
        }
        if ((e = hipEventRecord(p.ev_grid, main_stream)) != hipSuccess) return hip_status(e, "fork");
        if ((e = hipStreamWaitEvent(p.side, p.ev_grid, 0)) != hipSuccess) return hip_status(e, "fork");
        p.stream = p.side;
        if ((e = launch_near(p, x, q, 2)) != hipSuccess) return hip_status(e, "near field");
        if ((e = hipEventRecord(p.ev_join, p.side)) != hipSuccess) return hip_status(e, "join");
    }
    if (p.r.has_mid && (e = launch_mid(p, x, q, 2)) != hipSuccess) return hip_status(e, "mid range");
    if ((e = hipStreamWaitEvent(main_stream, p.ev_join, 0)) != hipSuccess) return hip_status(e, "join");
    if (phi_parts || grad_parts) {
        double *dpp = nullptr, *dgp = nullptr;
        if (p.on_device) {
            if ((e = launch_parts_out(p, phi_parts, grad_parts)) != hipSuccess) return hip_status(e, "parts");
        } else {
            // temporary device buffers for the parts (diagnostic entry point only)
            if (phi_parts && (e = hipMalloc((void**)&dpp, 3 * n * 8)) != hipSuccess) return hip_status(e, "parts alloc");
            if (grad_parts && (e = hipMalloc((void**)&dgp, 9 * n * 8)) != hipSuccess) {
                if (dpp) (void)hipFree(dpp);
                return hip_status(e, "parts alloc");
            }
            e = launch_parts_out(p, dpp, dgp);
            if (e == hipSuccess && phi_parts) e = hipMemcpyAsync(phi_parts, dpp, 3 * n * 8, hipMemcpyDeviceToHost, p.stream);
            if (e == hipSuccess && grad_parts) e = hipMemcpyAsync(grad_parts, dgp, 9 * n * 8, hipMemcpyDeviceToHost, p.stream);
            if (e == hipSuccess) e = hipStreamSynchronize(p.stream);
            if (dpp) (void)hipFree(dpp);
            if (dgp) (void)hipFree(dgp);
            if (e != hipSuccess) return hip_status(e, "parts");
        }
    } else {
        if ((e = launch_combine(p, q, dphi, dforce, dgrad, denergy)) != hipSuccess) return hip_status(e, "combine");
    }
    return SOG_OK;
}

// A batch of independent systems.  Each system has its own plan (its cutoff, grids,
// windows and long-range form come from the planner), holding only its tables: its
// per-call buffers are bound into one region of the batch, and it owns no stream.  At
// batch-plan time every system's sequence of kernel launches is recorded (launch.hpp);
// systems whose sequences use the same kernels in the same order form a group, and the
// k-th launch of a group runs as one batched launch over all its systems, whose blocks
// are dealt to the systems by a block-offset table and read their system's recorded
// arguments from a table in device memory.  The batched launches of all groups are
// captured once into a graph (a few dozen kernel nodes on one capture stream) that every
// call launches on the caller's stream.  The graph reads and writes the batch's staging
// buffers, so it stays valid for any caller pointers.
struct BatchStage {
    hipError_t (*batched)(const void*, const int*, int, unsigned, size_t, hipStream_t) = nullptr;
    const void* dtab = nullptr;  // the group's argument records (device)
    const int* dboff = nullptr;  // the group's block offsets (device), nsys + 1
    int nsys = 0;
    unsigned blocks = 0;
    size_t lds = 0;
};

struct Batch {
    int device = 0;
    hipStream_t stream = nullptr;   // the caller's stream: copies, check and graph launch
    hipStream_t cap = nullptr;      // capture stream (graph creation only)
    std::vector<Plan*> plans;
    std::vector<int> group_of;      // group of each system
    int ngroups = 0;
    std::vector<int64_t> off;       // nsys + 1 particle offsets
    std::vector<double> lz;
    bool on_device = false, check = true;
    std::vector<void*> bufs;        // staging, tables and the systems' per-call region
    double *x = nullptr, *q = nullptr, *phi = nullptr, *force = nullptr, *energy = nullptr;
    double *qsum = nullptr, *dlz = nullptr;
    int64_t* doff = nullptr;
    int* status = nullptr;
    std::vector<BatchStage> stages;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

void free_batch(Batch& b) {
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    b.exec = nullptr;
    b.graph = nullptr;
    for (Plan* p : b.plans) {
        free_plan(*p);
        delete p;
    }
    b.plans.clear();
    for (void* v : b.bufs) (void)hipFree(v);
    b.bufs.clear();
    if (b.cap) (void)hipStreamDestroy(b.cap);
    b.cap = nullptr;
}

// One system of a batch: resolved, tables on the device, per-call buffers not yet bound.
sog_status make_member_plan(const double box[3], int64_t n, double tol, const sog_options& opt, int num_cus,
                            Plan*& out) {
    out = nullptr;
    Plan* p = new (std::nothrow) Plan();
    if (!p) {
        set_error("host allocation failed");
        return SOG_ERR_OUT_OF_MEMORY;
    }
    std::string err;
    sog_status s = resolve(box, n, tol, opt, p->r, err);
    if (s != SOG_OK) {
        set_error(err);
        delete p;
        return s;
    }
    p->device = opt.device;
    p->on_device = true;
    p->check = false;
    p->timing = false;
    p->static_region = true;
    p->num_cus = num_cus;
    if ((s = build_plan(*p)) != SOG_OK) {
        delete p;
        return s;
    }
    out = p;
    return SOG_OK;
}

// The launches of one system's call, in the order of one stream: the near field's sort,
// the long range, the mid range's sort and gridding, the pair kernel, the transforms and
// gathering, the combination.
hipError_t record_system(Plan& p, const double* x, const double* q, double* energy, double* phi, double* force) {
    hipError_t e = launch_near(p, x, q, 1);
    if (e == hipSuccess) e = p.r.has_long ? launch_long(p, x, q) : launch_zero_parts(p, 2);
    if (e == hipSuccess) e = p.r.has_mid ? launch_mid(p, x, q, 1) : launch_zero_parts(p, 1);
    if (e == hipSuccess) e = launch_near(p, x, q, 2);
    if (e == hipSuccess && p.r.has_mid) e = launch_mid(p, x, q, 2);
    if (e == hipSuccess) e = launch_combine(p, q, phi, force, nullptr, energy);
    return e;
}

// Record every system, group the systems by kernel sequence, upload the argument and
// block-offset tables, and capture the batched launches into the graph.
sog_status build_batch_stages(Batch& b, Allocator& A) {
    const int nsys = (int)b.plans.size();
    std::vector<std::vector<RecLaunch>> recs(nsys);
    for (int s = 0; s < nsys; ++s) {
        Plan& p = *b.plans[s];
        p.rec = &recs[s];
        const int64_t o = b.off[s];
        const hipError_t e = record_system(p, b.x + 3 * o, b.q + o, b.energy + s, b.phi + o, b.force + 3 * o);
        p.rec = nullptr;
        if (e != hipSuccess) return hip_status(e, ("recording system " + std::to_string(s)).c_str());
    }
    // groups: identical kernel sequences
    std::vector<int> rep;  // first system of each group
    b.group_of.assign(nsys, -1);
    for (int s = 0; s < nsys; ++s) {
        for (int g = 0; g < (int)rep.size(); ++g) {
            const auto& a = recs[rep[g]];
            const auto& c = recs[s];
            bool same = a.size() == c.size();
            for (size_t k = 0; same && k < a.size(); ++k)
                same = a[k].id == c[k].id && a[k].args.size() == c[k].args.size() && a[k].block == c[k].block;
            if (same) {
                b.group_of[s] = g;
                break;
            }
        }
        if (b.group_of[s] < 0) {
            b.group_of[s] = (int)rep.size();
            rep.push_back(s);
        }
    }
    b.ngroups = (int)rep.size();
    // host images of the tables: per group and launch, the records of its systems (an
    // array of the launch's argument pack, 256-byte aligned) and the block offsets
    struct Tab {
        size_t at, boff_at, stride;
        int g, k, cnt;
        unsigned blocks;
        size_t lds;
    };
    std::vector<Tab> tabs;
    size_t total = 0;
    for (int g = 0; g < b.ngroups; ++g) {
        std::vector<int> mem;
        for (int s = 0; s < nsys; ++s)
            if (b.group_of[s] == g) mem.push_back(s);
        const auto& seq = recs[rep[g]];
        for (size_t k = 0; k < seq.size(); ++k) {
            Tab t;
            t.g = g;
            t.k = (int)k;
            t.cnt = (int)mem.size();
            t.stride = seq[k].args.size();  // the records form an array of the launch's argument pack
            t.at = total;
            total += (t.stride * mem.size() + 255) / 256 * 256;
            t.boff_at = total;
            total += ((mem.size() + 1) * sizeof(int) + 255) / 256 * 256;
            t.blocks = 0;
            t.lds = 0;
            for (int s : mem) {
                t.blocks += recs[s][k].grid;
                t.lds = std::max(t.lds, recs[s][k].lds);
            }
            tabs.push_back(t);
        }
    }
    std::vector<unsigned char> host(total, 0);
    for (const Tab& t : tabs) {
        int i = 0;
        int acc = 0;
        int* boff = reinterpret_cast<int*>(host.data() + t.boff_at);
        for (int s = 0; s < nsys; ++s) {
            if (b.group_of[s] != t.g) continue;
            const RecLaunch& r = recs[s][t.k];
            std::memcpy(host.data() + t.at + (size_t)i * t.stride, r.args.data(), r.args.size());
            boff[i] = acc;
            acc += (int)r.grid;
            ++i;
        }
        boff[i] = acc;
    }
    unsigned char* dev = nullptr;
    A.get(dev, total);
    if (A.err != hipSuccess || A.capped) return A.capped ? SOG_ERR_OUT_OF_MEMORY : hip_status(A.err, "batch tables");
    hipError_t e = hipMemcpy(dev, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_status(e, "batch tables");
    for (const Tab& t : tabs) {
        const RecLaunch& r = recs[rep[t.g]][t.k];
        BatchStage st;
        st.batched = r.batched;
        st.dtab = dev + t.at;
        st.dboff = reinterpret_cast<const int*>(dev + t.boff_at);
        st.nsys = t.cnt;
        st.blocks = t.blocks;
        st.lds = t.lds;
        b.stages.push_back(st);
    }
    return SOG_OK;
}

// The batched launches of all groups, in order, captured into the batch's graph.
sog_status capture_batch(Batch& b) {
    hipError_t e = hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_status(e, "graph capture");
    hipError_t le = hipSuccess;
    for (const BatchStage& st : b.stages) {
        le = st.batched(st.dtab, st.dboff, st.nsys, st.blocks, st.lds, b.cap);
        if (le != hipSuccess) break;
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b.cap, &g);
    if (le != hipSuccess || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_status(le != hipSuccess ? le : e, "graph capture");
    }
    b.graph = g;
    e = hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        b.exec = nullptr;
        return hip_status(e, "graph instantiation");
    }
    return SOG_OK;
}

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

int timer_id(Plan& p, const char* name) {
    if (!p.timing) return -1;
    for (size_t i = 0; i < p.timers.size(); ++i)
        if (p.timers[i].name == name || std::strcmp(p.timers[i].name, name) == 0) return (int)i;
    p.timers.push_back(KernelTimer{name, 0.0, 0});
    return (int)p.timers.size() - 1;
}

void timer_begin(Plan& p, int id) {
    if (!p.timing || id < 0) return;
    hipEvent_t a = take_event(p), b = take_event(p);
    if (a) (void)hipEventRecord(a, p.stream);
    p.pending.push_back({id, {a, b}});
}

void timer_end(Plan& p, int id) {
    if (!p.timing || id < 0) return;
    for (auto it = p.pending.rbegin(); it != p.pending.rend(); ++it)
        if (it->first == id) {
            if (it->second.second) (void)hipEventRecord(it->second.second, p.stream);
            return;
        }
}

}  // namespace sog

using namespace sog;

extern "C" {

void sog_options_default(sog_options* opt) {
    if (!opt) return;
    std::memset(opt, 0, sizeof(*opt));
    opt->precision = SOG_PREC_FP64;
    opt->check_inputs = 1;
}

sog_status sog_plan(const double box[3], int64_t n, double tol, sog_plan_t* out) {
    return sog_plan_ex(box, n, tol, nullptr, out);
}

static sog_status create_plan(const double box[3], int64_t n, double tol, const sog_options& opt, Plan** out);
static sog_status autotune_plan(const double box[3], int64_t n, double tol, const sog_options& opt, Plan** out);

sog_status sog_plan_ex(const double box[3], int64_t n, double tol, const sog_options* opt_in, sog_plan_t* out) {
    if (!out || !box) {
        set_error("box and out must not be NULL");
        return SOG_ERR_INVALID_ARG;
    }
    *out = nullptr;
    sog_options opt;
    sog_options_default(&opt);
    if (opt_in) opt = *opt_in;
    if (opt.autotune != 0 && opt.autotune != 1) {
        set_error("autotune must be 0 or 1");
        return SOG_ERR_INVALID_ARG;
    }
    if (opt.autotune && opt.static_workspace) {
        set_error("autotune is not available with static_workspace");
        return SOG_ERR_INVALID_ARG;
    }
    Plan* p = nullptr;
    sog_status s = opt.autotune ? autotune_plan(box, n, tol, opt, &p) : create_plan(box, n, tol, opt, &p);
    if (s == SOG_OK) *out = reinterpret_cast<sog_plan_t>(p);
    return s;
}

// One plan from resolved options (the body of sog_plan_ex).
static sog_status create_plan(const double box[3], int64_t n, double tol, const sog_options& opt, Plan** out) {
    *out = nullptr;
    Plan* p = new (std::nothrow) Plan();
    if (!p) {
        set_error("host allocation failed");
        return SOG_ERR_OUT_OF_MEMORY;
    }
    std::string err;
    sog_status s = resolve(box, n, tol, opt, p->r, err);
    if (s != SOG_OK) {
        set_error(err);
        delete p;
        return s;
    }
    p->device = opt.device;
    p->stream = (hipStream_t)opt.stream;
    p->on_device = opt.pointers_on_device != 0;
    p->check = opt.check_inputs != 0;
    p->timing = opt.timing != 0;
    p->static_region = opt.static_workspace != 0;
    p->graphable = !opt.eager && !opt.timing && !opt.static_workspace;
    if (p->static_region && p->timing) {
        set_error("timing is not available with static_workspace (it creates events during calls)");
        delete p;
        return SOG_ERR_INVALID_ARG;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        set_error("no HIP device available");
        delete p;
        return SOG_ERR_DEVICE;
    }
    if (opt.device < 0 || opt.device >= ndev) {
        set_error("device ordinal out of range");
        delete p;
        return SOG_ERR_INVALID_ARG;
    }
    DeviceGuard dg(p->device);
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) == hipSuccess && cus > 0)
            p->num_cus = cus;
    }
    s = build_plan(*p);
    if (s != SOG_OK) {
        delete p;
        return s;
    }
    if (p->static_region) {
        // set-up of sog_energy_potential_force_static: the per-call buffers must fit the
        // static scratch, whose device address is looked up here
        void* base = nullptr;
        if (p->region_bytes > kStaticScratchBytes) {
            set_error("static_workspace: the plan's per-call buffers need " + std::to_string(p->region_bytes) +
                      " bytes, above the static scratch of " + std::to_string(kStaticScratchBytes) + " bytes");
            free_plan(*p);
            delete p;
            return SOG_ERR_OUT_OF_MEMORY;
        }
        if ((s = static_scratch(p->device, &base)) != SOG_OK) {
            free_plan(*p);
            delete p;
            return s;
        }
    }
    hipError_t he = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming);
    if (he == hipSuccess) he = hipEventCreateWithFlags(&p->ev_grid, hipEventDisableTiming);
    if (he != hipSuccess) {
        s = hip_status(he, "stream creation");
        free_plan(*p);
        delete p;
        return s;
    }
    *out = p;
    return SOG_OK;
}

// Autotuning: the planner's cheapest discretisations by its cost model, one per distinct
// r_c up to kTuneCandidates, each built as a plan (device pointers, no checks, no
// timing), given one warm-up call (which captures its graph), then timed on the plan's
// stream with HIP events over kTuneCalls calls back to back (as calls follow one another
// in use) after kTuneWarm untimed ones (so that the caches hold this candidate's data,
// not the previous one's), the candidates in turn for kTuneRounds rounds (so that no
// candidate alone meets a cold or still clocking-up device), each keeping its fastest
// round; inputs:
// uniformly random positions in the box with charges +1, -1
// alternating (the last one 0 for odd n: neutral).  The fastest (r_c, m) is then planned
// with the caller's options.  Inputs other than uniform ones may rank the candidates
// differently.
constexpr int kTuneCandidates = 3;
constexpr int kTuneRounds = 4;
constexpr int kTuneCalls = 3;
constexpr int kTuneWarm = 2;

static sog_status autotune_plan(const double box[3], int64_t n, double tol, const sog_options& opt, Plan** out) {
    *out = nullptr;
    std::string err;
    Resolved r0;
    std::vector<PlanCandidate> cands;
    sog_status s = resolve(box, n, tol, opt, r0, err, &cands);
    if (s != SOG_OK) {
        set_error(err);
        return s;
    }
    std::stable_sort(cands.begin(), cands.end(),
                     [](const PlanCandidate& a, const PlanCandidate& b) { return a.cost < b.cost; });
    // the cheapest candidate of each r_c (the split follows r_c closely), cheapest first
    std::vector<PlanCandidate> pick;
    for (const PlanCandidate& c : cands) {
        bool seen = false;
        for (const PlanCandidate& q : pick) seen = seen || q.rc == c.rc;
        if (!seen) pick.push_back(c);
        if ((int)pick.size() == kTuneCandidates) break;
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        set_error("no HIP device available");
        return SOG_ERR_DEVICE;
    }
    if (opt.device < 0 || opt.device >= ndev) {
        set_error("device ordinal out of range");
        return SOG_ERR_INVALID_ARG;
    }
    DeviceGuard dg(opt.device);
    // the synthetic sample, on the device
    std::vector<double> hx((size_t)n * 3), hq((size_t)n);
    {
        uint64_t st = 0x9e3779b97f4a7c15ull;
        auto next = [&]() {  // splitmix64
            st += 0x9e3779b97f4a7c15ull;
            uint64_t z = st;
            z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
            z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
            return (double)((z ^ (z >> 31)) >> 11) * (1.0 / 9007199254740992.0);
        };
        for (int64_t i = 0; i < n; ++i) {
            for (int d = 0; d < 3; ++d) hx[3 * i + d] = next() * box[d];
            hq[i] = (i % 2 == 0) ? 1.0 : -1.0;
        }
        if (n % 2) hq[n - 1] = 0.0;
    }
    double *dx = nullptr, *dq = nullptr, *dphi = nullptr, *dF = nullptr, *dU = nullptr;
    hipError_t he = hipMalloc(&dx, hx.size() * 8);
    if (he == hipSuccess) he = hipMalloc(&dq, hq.size() * 8);
    if (he == hipSuccess) he = hipMalloc(&dphi, (size_t)n * 8);
    if (he == hipSuccess) he = hipMalloc(&dF, (size_t)n * 24);
    if (he == hipSuccess) he = hipMalloc(&dU, 8);
    if (he == hipSuccess) he = hipMemcpy(dx, hx.data(), hx.size() * 8, hipMemcpyHostToDevice);
    if (he == hipSuccess) he = hipMemcpy(dq, hq.data(), hq.size() * 8, hipMemcpyHostToDevice);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (he == hipSuccess) he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    auto release = [&]() {
        (void)hipFree(dx);
        (void)hipFree(dq);
        (void)hipFree(dphi);
        (void)hipFree(dF);
        (void)hipFree(dU);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    if (he != hipSuccess) {
        release();
        return hip_status(he, "autotune sample");
    }
    std::vector<TunedCandidate> tuned;
    std::vector<Plan*> plans;
    auto free_plans = [&]() {
        for (Plan* q : plans) {
            free_plan(*q);
            delete q;
        }
        plans.clear();
    };
    for (const PlanCandidate& c : pick) {
        sog_options o = opt;
        o.autotune = 0;
        o.timing = 0;
        o.check_inputs = 0;
        o.pointers_on_device = 1;
        o.params.rc = c.rc;
        o.params.set_m = 1;
        o.params.m = c.m;
        o.params.eta = 0;
        Plan* p = nullptr;
        if (create_plan(box, n, tol, o, &p) != SOG_OK) continue;  // not buildable: not a candidate
        plans.push_back(p);
        tuned.push_back(TunedCandidate{c.rc, c.m, 0.0});
    }
    sog_status rs = SOG_OK;
    for (size_t i = 0; i < plans.size() && rs == SOG_OK; ++i) {
        rs = run(*plans[i], dx, dq, dU, dphi, dF, nullptr, nullptr, nullptr);
        if (rs == SOG_OK && (he = hipStreamSynchronize(plans[i]->stream)) != hipSuccess) break;
    }
    for (int round = 0; round < kTuneRounds && rs == SOG_OK && he == hipSuccess; ++round)
        for (size_t i = 0; i < plans.size() && rs == SOG_OK && he == hipSuccess; ++i) {
            float ms = 0;
            for (int k = 0; k < kTuneWarm && rs == SOG_OK; ++k)
                rs = run(*plans[i], dx, dq, dU, dphi, dF, nullptr, nullptr, nullptr);
            if (rs == SOG_OK) he = hipEventRecord(e0, plans[i]->stream);
            for (int k = 0; k < kTuneCalls && rs == SOG_OK && he == hipSuccess; ++k)
                rs = run(*plans[i], dx, dq, dU, dphi, dF, nullptr, nullptr, nullptr);
            if (rs == SOG_OK && he == hipSuccess) he = hipEventRecord(e1, plans[i]->stream);
            if (rs == SOG_OK && he == hipSuccess) he = hipEventSynchronize(e1);
            if (rs == SOG_OK && he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
            ms /= kTuneCalls;
            if (rs == SOG_OK && he == hipSuccess && (round == 0 || ms < tuned[i].ms)) tuned[i].ms = ms;
        }
    free_plans();
    if (rs != SOG_OK || he != hipSuccess) {
        release();
        return rs != SOG_OK ? rs : hip_status(he, "autotune timing");
    }
    release();
    if (tuned.empty()) {
        set_error("autotune: no candidate plan could be built");
        return SOG_ERR_DEVICE;
    }
    size_t best = 0;
    for (size_t i = 1; i < tuned.size(); ++i)
        if (tuned[i].ms < tuned[best].ms) best = i;
    sog_options o = opt;
    o.autotune = 0;
    o.params.rc = tuned[best].rc;
    o.params.set_m = 1;
    o.params.m = tuned[best].m;
    o.params.eta = 0;
    Plan* p = nullptr;
    s = create_plan(box, n, tol, o, &p);
    if (s != SOG_OK) return s;
    p->tuning = tuned;
    *out = p;
    return SOG_OK;
}

sog_status sog_plan_tuning(sog_plan_t plan, int32_t max, int32_t* count, double* rc, int32_t* m, double* ms) {
    if (!plan || !count || max < 0) {
        set_error("plan and count must not be NULL, max >= 0");
        return SOG_ERR_INVALID_ARG;
    }
    const Plan& p = *reinterpret_cast<const Plan*>(plan);
    *count = (int32_t)p.tuning.size();
    for (int32_t i = 0; i < std::min<int32_t>(max, *count); ++i) {
        if (rc) rc[i] = p.tuning[i].rc;
        if (m) m[i] = p.tuning[i].m;
        if (ms) ms[i] = p.tuning[i].ms;
    }
    return SOG_OK;
}

// A plan made with static_workspace holds no per-call buffers of its own: only
// sog_energy_potential_force_static runs it.
static sog_status own_region_plan(sog_plan_t plan) {
    if (!plan) {
        set_error("plan is NULL");
        return SOG_ERR_INVALID_ARG;
    }
    if (reinterpret_cast<Plan*>(plan)->static_region) {
        set_error("the plan was made with static_workspace: call sog_energy_potential_force_static");
        return SOG_ERR_INVALID_ARG;
    }
    return SOG_OK;
}

sog_status sog_energy_potential_force(sog_plan_t plan, const double* x, const double* q, double* energy,
                                      double* phi, double* force) {
    if (sog_status st = own_region_plan(plan)) return st;
    return run(*reinterpret_cast<Plan*>(plan), x, q, energy, phi, force, nullptr, nullptr, nullptr);
}

sog_status sog_energy_potential_gradient(sog_plan_t plan, const double* x, const double* q, double* energy,
                                         double* phi, double* grad) {
    if (sog_status st = own_region_plan(plan)) return st;
    return run(*reinterpret_cast<Plan*>(plan), x, q, energy, phi, nullptr, grad, nullptr, nullptr);
}

sog_status sog_potential_parts(sog_plan_t plan, const double* x, const double* q, double* phi_parts,
                               double* grad_parts) {
    if (sog_status st = own_region_plan(plan)) return st;
    if (!phi_parts && !grad_parts) {
        set_error("phi_parts and grad_parts are both NULL");
        return SOG_ERR_INVALID_ARG;
    }
    return run(*reinterpret_cast<Plan*>(plan), x, q, nullptr, nullptr, nullptr, nullptr, phi_parts, grad_parts);
}

sog_status sog_energy_potential_force_static(sog_plan_t plan, const double* x, const double* q, double* energy,
                                             double* phi, double* force) {
    if (!plan) {
        set_error("plan is NULL");
        return SOG_ERR_INVALID_ARG;
    }
    Plan& p = *reinterpret_cast<Plan*>(plan);
    if (p.timing) {
        set_error("sog_energy_potential_force_static does not take a plan with timing on");
        return SOG_ERR_INVALID_ARG;
    }
    if (p.region_bytes > kStaticScratchBytes) {
        set_error("the plan's per-call buffers need " + std::to_string(p.region_bytes) +
                  " bytes, above the static scratch of " + std::to_string(kStaticScratchBytes) + " bytes");
        return SOG_ERR_OUT_OF_MEMORY;
    }
    void* base = nullptr;
    {
        DeviceGuard dg(p.device);
        if (sog_status st = static_scratch(p.device, &base)) return st;
    }
    // launched kernel by kernel: a graph would bake in the static scratch's addresses
    // (and instantiating one allocates)
    const bool graphable = p.graphable;
    p.graphable = false;
    bind_region(p, base);
    const sog_status st = run(p, x, q, energy, phi, force, nullptr, nullptr, nullptr);
    bind_region(p, p.region);
    p.graphable = graphable;
    return st;
}

static void fill_params(const Resolved& r, sog_params* o);

sog_status sog_plan_resolve(const double box[3], int64_t n, double tol, const sog_options* opt_in, sog_params* out) {
    if (!box || !out) {
        set_error("box and out must not be NULL");
        return SOG_ERR_INVALID_ARG;
    }
    sog_options opt;
    sog_options_default(&opt);
    if (opt_in) opt = *opt_in;
    Resolved r;
    std::string err;
    sog_status s = resolve(box, n, tol, opt, r, err);
    if (s != SOG_OK) {
        set_error(err);
        return s;
    }
    fill_params(r, out);
    return SOG_OK;
}

sog_status sog_plan_info(sog_plan_t plan, sog_params* o) {
    if (!plan || !o) {
        set_error("plan and out must not be NULL");
        return SOG_ERR_INVALID_ARG;
    }
    fill_params(reinterpret_cast<Plan*>(plan)->r, o);
    return SOG_OK;
}

static void fill_params(const Resolved& r, sog_params* o) {
    std::memset(o, 0, sizeof(*o));
    o->b = r.b;
    o->r0 = r.r0;
    o->omega = r.omega;
    o->rc = r.rc;
    o->M = r.M;
    o->m = r.m;
    o->set_m = 1;
    o->eta = r.eta > 0 ? r.eta : (r.m >= 0 ? r.s[r.m] / r.L[2] : 0.0);
    if (r.has_mid) {
        for (int d = 0; d < 3; ++d) {
            o->mid_I[d] = r.I[d];
            o->mid_Pw[d] = r.Pw;
        }
        o->mid_Izs = r.Izs;
        o->mid_window = r.window;
        if (r.window == SOG_WINDOW_ES || r.window == SOG_WINDOW_KB)
            o->mid_beta = r.beta;
        else
            o->mid_S = r.S;
        if (r.window == SOG_WINDOW_KB) o->mid_nu = r.nu;
    }
    if (r.has_long) {
        o->long_form = r.form;
        o->long_P = r.P;
        if (r.form == SOG_LONG_DIRECT) {
            o->long_nk[0] = r.nk[0];
            o->long_nk[1] = r.nk[1];
        } else {
            o->long_I[0] = r.I2[0];
            o->long_I[1] = r.I2[1];
            o->long_Pw[0] = o->long_Pw[1] = r.Pw2;
            o->long_S = r.S2;
            o->long_Q = r.Q > 0 ? r.Q : -1;
        }
    }
}

sog_status sog_plan_sizes_get(sog_plan_t plan, sog_plan_sizes* o) {
    if (!plan || !o) {
        set_error("plan and out must not be NULL");
        return SOG_ERR_INVALID_ARG;
    }
    const Plan& p = *reinterpret_cast<Plan*>(plan);
    const Resolved& r = p.r;
    std::memset(o, 0, sizeof(*o));
    o->mid_grid_points = r.has_mid ? (int64_t)r.I[0] * r.I[1] * r.Izs : 0;
    if (r.has_long)
        o->long_points = (r.form == SOG_LONG_DIRECT) ? (int64_t)(2 * r.nk[0] + 1) * (2 * r.nk[1] + 1)
                                                     : (int64_t)r.I2[0] * r.I2[1];
    o->device_bytes = (int64_t)p.ws.bytes;
    for (int d = 0; d < 3; ++d) {
        o->near_cells[d] = r.nc[d];
        o->tile[d] = r.B[d];
    }
    o->near_degree = r.near_deg;
    o->mid_zband[0] = r.zband[0];
    o->mid_zband[1] = r.zband[1];
    return SOG_OK;
}

sog_status sog_kernel_times(sog_plan_t plan, sog_kernel_time* out, int32_t max, int32_t* count) {
    if (!plan || !count) {
        set_error("plan and count must not be NULL");
        return SOG_ERR_INVALID_ARG;
    }
    const Plan& p = *reinterpret_cast<Plan*>(plan);
    *count = (int32_t)p.timers.size();
    for (int32_t i = 0; i < max && i < (int32_t)p.timers.size() && out; ++i) {
        out[i].name = p.timers[i].name;
        out[i].total_ms = p.timers[i].total_ms;
        out[i].launches = p.timers[i].launches;
    }
    return SOG_OK;
}

sog_status sog_kernel_times_reset(sog_plan_t plan) {
    if (!plan) {
        set_error("plan is NULL");
        return SOG_ERR_INVALID_ARG;
    }
    Plan& p = *reinterpret_cast<Plan*>(plan);
    for (auto& t : p.timers) {
        t.total_ms = 0;
        t.launches = 0;
    }
    return SOG_OK;
}

void sog_destroy(sog_plan_t plan) {
    if (!plan) return;
    Plan* p = reinterpret_cast<Plan*>(plan);
    {
        DeviceGuard dg(p->device);
        (void)hipStreamSynchronize(p->stream);
        if (p->side) (void)hipStreamSynchronize(p->side);
        free_plan(*p);
    }
    delete p;
}

const char* sog_status_string(sog_status s) {
    switch (s) {
        case SOG_OK: return "SOG_OK";
        case SOG_ERR_INVALID_ARG: return "SOG_ERR_INVALID_ARG";
        case SOG_ERR_NOT_NEUTRAL: return "SOG_ERR_NOT_NEUTRAL";
        case SOG_ERR_OUT_OF_BOX: return "SOG_ERR_OUT_OF_BOX";
        case SOG_ERR_TOL_UNREACHABLE: return "SOG_ERR_TOL_UNREACHABLE";
        case SOG_ERR_OUT_OF_MEMORY: return "SOG_ERR_OUT_OF_MEMORY";
        case SOG_ERR_DEVICE: return "SOG_ERR_DEVICE";
    }
    return "SOG_ERR_UNKNOWN";
}

const char* sog_last_error(void) { return g_last_error.c_str(); }

sog_status sog_batch_plan(int32_t nsys, const double* boxes, const int64_t* n, double tol, const sog_options* opt_in,
                          sog_batch_t* out) {
    if (!out || !boxes || !n || nsys < 1) {
        set_error("nsys must be >= 1 and boxes, n, out must not be NULL");
        if (out) *out = nullptr;
        return SOG_ERR_INVALID_ARG;
    }
    *out = nullptr;
    sog_options opt;
    sog_options_default(&opt);
    if (opt_in) opt = *opt_in;
    if (opt.timing) {
        set_error("timing is not available for a batch");
        return SOG_ERR_INVALID_ARG;
    }
    Batch* b = new (std::nothrow) Batch();
    if (!b) {
        set_error("host allocation failed");
        return SOG_ERR_OUT_OF_MEMORY;
    }
    b->off.assign(1, 0);
    for (int s = 0; s < nsys; ++s) {
        if (n[s] < 2 || b->off.back() + n[s] > ((int64_t)1 << 31)) {
            set_error("system " + std::to_string(s) + ": n must be >= 2 and the total at most 2^31");
            delete b;
            return SOG_ERR_INVALID_ARG;
        }
        b->off.push_back(b->off.back() + n[s]);
        b->lz.push_back(boxes[3 * s + 2]);
    }
    // every system's parameters first, so that a bad system fails before any allocation
    for (int s = 0; s < nsys; ++s) {
        sog_params prm;
        sog_status st = sog_plan_resolve(boxes + 3 * s, n[s], tol, &opt, &prm);
        if (st != SOG_OK) {
            set_error("system " + std::to_string(s) + ": " + g_last_error);
            delete b;
            return st;
        }
    }
    b->device = opt.device;
    b->stream = (hipStream_t)opt.stream;
    b->on_device = opt.pointers_on_device != 0;
    b->check = opt.check_inputs != 0;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) {
        set_error("no HIP device available");
        delete b;
        return SOG_ERR_DEVICE;
    }
    if (opt.device < 0 || opt.device >= ndev) {
        set_error("device ordinal out of range");
        delete b;
        return SOG_ERR_INVALID_ARG;
    }
    DeviceGuard dg(b->device);
    int num_cus = 256;
    {
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) == hipSuccess && cus > 0)
            num_cus = cus;
    }
    Allocator A;
    auto fail = [&](sog_status st) {
        b->bufs = A.ptrs;
        free_batch(*b);
        delete b;
        return st;
    };
    const int64_t nt = b->off.back();
    A.get(b->x, 3 * nt * 8);
    A.get(b->q, nt * 8);
    A.get(b->phi, nt * 8);
    A.get(b->force, 3 * nt * 8);
    A.get(b->energy, nsys * 8);
    A.get(b->qsum, 2 * nsys * 8);
    A.get(b->dlz, nsys * 8);
    A.get(b->doff, (nsys + 1) * 8);
    A.get(b->status, nsys * 4);
    if (A.err != hipSuccess || A.capped) {
        set_error(A.capped ? "device memory cap (SOG_MAX_DEVICE_BYTES) reached" : "hipMalloc failed");
        return fail(SOG_ERR_OUT_OF_MEMORY);
    }
    hipError_t e = hipMemcpy(b->dlz, b->lz.data(), nsys * 8, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(b->doff, b->off.data(), (nsys + 1) * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(hip_status(e, "batch tables"));
    // the systems' plans (tables only), then their per-call buffers in one region
    size_t region = 0;
    std::vector<size_t> at(nsys);
    for (int s = 0; s < nsys; ++s) {
        Plan* p = nullptr;
        sog_status st = make_member_plan(boxes + 3 * s, n[s], tol, opt, num_cus, p);
        if (st != SOG_OK) {
            set_error("system " + std::to_string(s) + ": " + g_last_error);
            return fail(st);
        }
        b->plans.push_back(p);
        if (p->r.has_long && p->r.form == SOG_LONG_FFT) {
            set_error("system " + std::to_string(s) +
                      ": its plan takes the long range's FFT form, which batches do not run (a flat system with too "
                      "many long-range modes for the direct form); solve it with its own plan");
            return fail(SOG_ERR_INVALID_ARG);
        }
        at[s] = region;
        region += (p->region_bytes + 255) / 256 * 256;
    }
    unsigned char* reg = nullptr;
    A.get(reg, region);
    if (A.err != hipSuccess || A.capped) {
        set_error(A.capped ? "device memory cap (SOG_MAX_DEVICE_BYTES) reached" : "hipMalloc failed");
        return fail(SOG_ERR_OUT_OF_MEMORY);
    }
    for (int s = 0; s < nsys; ++s) bind_region(*b->plans[s], reg + at[s]);
    sog_status st = build_batch_stages(*b, A);
    if (st != SOG_OK) return fail(st);
    e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(hip_status(e, "stream creation"));
    st = capture_batch(*b);
    if (st != SOG_OK) return fail(st);
    b->bufs = A.ptrs;
    *out = reinterpret_cast<sog_batch_t>(b);
    return SOG_OK;
}

sog_status sog_batch_energy_potential_force(sog_batch_t batch, const double* x, const double* q, double* energy,
                                            double* phi, double* force) {
    if (!batch || !x || !q) {
        set_error("batch, x and q must not be NULL");
        return SOG_ERR_INVALID_ARG;
    }
    Batch& b = *reinterpret_cast<Batch*>(batch);
    DeviceGuard dg(b.device);
    const int nsys = (int)b.plans.size();
    const int64_t nt = b.off.back();
    const hipMemcpyKind in = b.on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const hipMemcpyKind outk = b.on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    hipError_t e = hipMemcpyAsync(b.x, x, 3 * nt * 8, in, b.stream);
    if (e == hipSuccess) e = hipMemcpyAsync(b.q, q, nt * 8, in, b.stream);
    if (e != hipSuccess) return hip_status(e, "input copy");
    if (b.check) {
        e = launch_batch_check(b.x, b.q, b.doff, nsys, b.dlz, nt, b.qsum, b.status, b.stream);
        std::vector<double> qs(2 * (size_t)nsys);
        std::vector<int> fl(nsys);
        if (e == hipSuccess) e = hipMemcpyAsync(qs.data(), b.qsum, 2 * nsys * 8, hipMemcpyDeviceToHost, b.stream);
        if (e == hipSuccess) e = hipMemcpyAsync(fl.data(), b.status, nsys * 4, hipMemcpyDeviceToHost, b.stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b.stream);
        if (e != hipSuccess) return hip_status(e, "input check");
        for (int s = 0; s < nsys; ++s) {
            const std::string sys = "system " + std::to_string(s) + ": ";
            if (fl[s] & 1) {
                set_error(sys + "non-finite position or charge");
                return SOG_ERR_INVALID_ARG;
            }
            if (fl[s] & 2) {
                set_error(sys + "some z is outside [0, Lz]");
                return SOG_ERR_OUT_OF_BOX;
            }
            if (std::fabs(qs[2 * s]) > 1e-10 * qs[2 * s + 1]) {
                set_error(sys + "charges are not neutral (|sum q| > 1e-10 sum |q|)");
                return SOG_ERR_NOT_NEUTRAL;
            }
        }
    }
    e = hipGraphLaunch(b.exec, b.stream);
    if (e != hipSuccess) return hip_status(e, "graph launch");
    if (energy) e = hipMemcpyAsync(energy, b.energy, nsys * 8, outk, b.stream);
    if (phi && e == hipSuccess) e = hipMemcpyAsync(phi, b.phi, nt * 8, outk, b.stream);
    if (force && e == hipSuccess) e = hipMemcpyAsync(force, b.force, 3 * nt * 8, outk, b.stream);
    if (e == hipSuccess && !b.on_device) e = hipStreamSynchronize(b.stream);
    if (e != hipSuccess) return hip_status(e, "output copy");
    return SOG_OK;
}

sog_status sog_batch_graph_info(sog_batch_t batch, int32_t* groups, int32_t* launches) {
    if (!batch || !groups || !launches) {
        set_error("batch, groups and launches must not be NULL");
        return SOG_ERR_INVALID_ARG;
    }
    const Batch& b = *reinterpret_cast<Batch*>(batch);
    *groups = b.ngroups;
    *launches = (int32_t)b.stages.size();
    return SOG_OK;
}

sog_status sog_batch_plan_info(sog_batch_t batch, int32_t s, sog_params* o) {
    if (!batch || !o) {
        set_error("batch and out must not be NULL");
        return SOG_ERR_INVALID_ARG;
    }
    Batch& b = *reinterpret_cast<Batch*>(batch);
    if (s < 0 || s >= (int)b.plans.size()) {
        set_error("system index out of range");
        return SOG_ERR_INVALID_ARG;
    }
    fill_params(b.plans[s]->r, o);
    return SOG_OK;
}

void sog_batch_destroy(sog_batch_t batch) {
    if (!batch) return;
    Batch* b = reinterpret_cast<Batch*>(batch);
    {
        DeviceGuard dg(b->device);
        (void)hipStreamSynchronize(b->stream);
        free_batch(*b);
    }
    delete b;
}

}  // extern "C"
