// libhbl C ABI: argument validation, error capture, the host-side "lattice
// compiler" (element -> first-order map coefficients), reference-particle
// bookkeeping and kernel launches.  No C++ exception crosses the ABI.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/hbl.h"
#include "hbl_internal.hpp"

namespace hbl {

// ------------------------------------------------------------------ errors
static thread_local char g_err[512] = "";

void set_error(int code, const char* fmt, ...) {
    char buf[448];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    snprintf(g_err, sizeof g_err, "[%d] %s", code, buf);
}

void clear_error() { g_err[0] = 0; }

// ----------------------------------------------------- per-device memory
namespace {
constexpr int kMaxDev = 64;
std::mutex g_mu;
double* g_ws[kMaxDev] = {};
size_t g_ws_bytes[kMaxDev] = {};

struct StageKey {
    double g_in, gp, h;
    int32_t nsub;
    bool operator<(const StageKey& o) const {
        return std::tie(g_in, gp, h, nsub) < std::tie(o.g_in, o.gp, o.h, o.nsub);
    }
};
std::map<StageKey, double*> g_stage_tables[kMaxDev];

int current_device() {
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess) return -1;
    return d;
}
}  // namespace

double* workspace(size_t bytes) {
    const int d = current_device();
    if (d < 0 || d >= kMaxDev) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_ws_bytes[d] < bytes) {
        if (g_ws[d]) (void)hipFree(g_ws[d]);
        g_ws[d] = nullptr;
        g_ws_bytes[d] = 0;
        size_t want = bytes < (1u << 20) ? (1u << 20) : bytes;
        void* p = nullptr;
        if (hipMalloc(&p, want) != hipSuccess) return nullptr;
        g_ws[d] = static_cast<double*>(p);
        g_ws_bytes[d] = want;
    }
    return g_ws[d];
}

// gamma_ref at the middle of each substep of a stage, cached per device.
static const double* stage_table(double g_in, double gp, double h, int32_t nsub, hbl_status* st) {
    const int d = current_device();
    if (d < 0 || d >= kMaxDev) {
        *st = HBL_EHIP;
        set_error(HBL_EHIP, "no current HIP device");
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    const StageKey key{g_in, gp, h, nsub};
    auto it = g_stage_tables[d].find(key);
    if (it != g_stage_tables[d].end()) return it->second;
    std::vector<double> tab(nsub);
    for (int32_t s = 0; s < nsub; ++s) tab[s] = g_in + gp * ((s + 0.5) * h);
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, sizeof(double) * nsub);
    if (e != hipSuccess) {
        *st = HBL_ENOMEM;
        set_error(HBL_ENOMEM, "stage table allocation failed: %s", hipGetErrorString(e));
        return nullptr;
    }
    e = hipMemcpy(p, tab.data(), sizeof(double) * nsub, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p);
        *st = HBL_EHIP;
        set_error(HBL_EHIP, "stage table upload failed: %s", hipGetErrorString(e));
        return nullptr;
    }
    if (g_stage_tables[d].size() > 256) {  // bounded cache: drop everything
        (void)hipDeviceSynchronize();
        for (auto& kv : g_stage_tables[d]) (void)hipFree(kv.second);
        g_stage_tables[d].clear();
    }
    g_stage_tables[d][key] = static_cast<double*>(p);
    return static_cast<double*>(p);
}

}  // namespace hbl

using namespace hbl;

// ------------------------------------------------------------- validation
namespace {

constexpr double kCLight = 299792458.0;
constexpr double kQe = 1.602176634e-19;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kMeKg = 9.1093837015e-31;

#define HBL_REQUIRE(cond, ...)                      \
    do {                                            \
        if (!(cond)) {                              \
            set_error(HBL_EINVAL, __VA_ARGS__);     \
            return HBL_EINVAL;                      \
        }                                           \
    } while (0)

#define HBL_HIP(call)                                                            \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess) {                                                  \
            set_error(HBL_EHIP, "%s: %s", #call, hipGetErrorString(e_));         \
            return HBL_EHIP;                                                     \
        }                                                                        \
    } while (0)

hbl_status check_bunch(const void* z, int64_t n, int64_t ld, const char* what) {
    if (n < 0) { set_error(HBL_EINVAL, "%s: n = %lld < 0", what, (long long)n); return HBL_EINVAL; }
    if (ld < n || ld < 0) { set_error(HBL_EINVAL, "%s: ld = %lld < n = %lld", what, (long long)ld, (long long)n); return HBL_EINVAL; }
    if (ld % 2 != 0) { set_error(HBL_EINVAL, "%s: ld = %lld must be even", what, (long long)ld); return HBL_EINVAL; }
    if (n > 0 && z == nullptr) { set_error(HBL_EINVAL, "%s: NULL bunch pointer", what); return HBL_EINVAL; }
    if (((uintptr_t)z & 15u) != 0) { set_error(HBL_EINVAL, "%s: bunch pointer not 16-byte aligned", what); return HBL_EINVAL; }
    if (ld > (INT64_MAX / 8) / 6) { set_error(HBL_EINVAL, "%s: ld too large", what); return HBL_EINVAL; }
    return HBL_OK;
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

hbl_status check_ref(const hbl_ref* ref) {
    if (!ref) { set_error(HBL_EINVAL, "NULL reference particle"); return HBL_EINVAL; }
    if (!finite_pos(ref->mass_MeV)) { set_error(HBL_EINVAL, "reference mass must be finite and > 0"); return HBL_EINVAL; }
    if (!(isfinite(ref->gamma) && ref->gamma > 1.0)) { set_error(HBL_EINVAL, "reference gamma must be finite and > 1 (got %g)", ref->gamma); return HBL_EINVAL; }
    if (!isfinite(ref->s)) { set_error(HBL_EINVAL, "reference s must be finite"); return HBL_EINVAL; }
    return HBL_OK;
}

// theta - sin(theta) without cancellation for small angles (Taylor series
// below 0.05 rad, terms decreasing by > 1e3 each).
double th_minus_sin(double th) {
    if (fabs(th) >= 0.05) return th - sin(th);
    const double t2 = th * th;
    double term = th * t2 / 6.0, acc = 0.0;
    for (int k = 1; k <= 8; ++k) {
        acc += term;
        term *= -t2 / ((2.0 * k + 2.0) * (2.0 * k + 3.0));
    }
    return acc;
}

// Element -> coefficients (first-order map of the linearised equations of
// motion over the element, for a reference of Lorentz factor gamma).
hbl_status compile_element(const hbl_element& e, double gamma, int32_t* kind, ElemCoef* c) {
    memset(c, 0, sizeof *c);
    const double bg = sqrt(gamma * gamma - 1.0), beta = bg / gamma;
    const double r56d = e.L / (bg * bg);
    switch (e.kind) {
        case HBL_DRIFT:
            HBL_REQUIRE(isfinite(e.L), "drift: L must be finite");
            *kind = kDrift;
            c->c[0] = e.L;
            c->c[1] = r56d;
            return HBL_OK;
        case HBL_QUAD: {
            HBL_REQUIRE(isfinite(e.L) && isfinite(e.k), "quad: L and k must be finite");
            if (e.k == 0.0) {  // zero gradient: a drift
                *kind = kDrift;
                c->c[0] = e.L;
                c->c[1] = r56d;
                return HBL_OK;
            }
            const double w = sqrt(fabs(e.k)), ph = w * e.L;
            const double fc = cos(ph), fs = sin(ph) / w, fm = -w * sin(ph);
            const double dc = cosh(ph), ds = sinh(ph) / w, dm = w * sinh(ph);
            const bool xf = e.k > 0.0;
            *kind = kQuad;
            c->c[0] = xf ? fc : dc; c->c[1] = xf ? fs : ds; c->c[2] = xf ? fm : dm; c->c[3] = xf ? fc : dc;
            c->c[4] = xf ? dc : fc; c->c[5] = xf ? ds : fs; c->c[6] = xf ? dm : fm; c->c[7] = xf ? dc : fc;
            c->c[8] = r56d;
            return HBL_OK;
        }
        case HBL_SBEND: {
            HBL_REQUIRE(isfinite(e.L) && isfinite(e.angle), "sbend: L and angle must be finite");
            if (e.angle == 0.0) {
                *kind = kDrift;
                c->c[0] = e.L;
                c->c[1] = r56d;
                return HBL_OK;
            }
            HBL_REQUIRE(e.L != 0.0, "sbend: nonzero angle needs nonzero length");
            const double th = e.angle, rho = e.L / th;
            const double C = cos(th), S = sin(th);
            const double omc = 2.0 * sin(0.5 * th) * sin(0.5 * th);  // 1 - cos
            *kind = kSbend;
            c->c[0] = C;
            c->c[1] = rho * S;
            c->c[2] = -rho * omc / beta;
            c->c[3] = -S / rho;
            c->c[4] = C;
            c->c[5] = -S / beta;
            c->c[6] = S / beta;
            c->c[7] = rho * omc / beta;
            c->c[8] = r56d - rho * th_minus_sin(th) / (beta * beta);
            c->c[9] = e.L;
            return HBL_OK;
        }
        case HBL_THIN_LENS:
            HBL_REQUIRE(isfinite(e.f) && e.f != 0.0, "thin lens: f must be finite and nonzero");
            *kind = kLens;
            c->c[0] = -1.0 / e.f;
            return HBL_OK;
        case HBL_STAGE:
            set_error(HBL_EINVAL, "a lattice holds linear elements only; apply stages with hbl_apply_stage");
            return HBL_EINVAL;
        default:
            set_error(HBL_EINVAL, "unknown element kind %d", (int)e.kind);
            return HBL_EINVAL;
    }
}

}  // namespace

struct hbl_lattice {
    int device;
    int32_t n_elem;
    double gamma;
    double length;
    int32_t* d_kinds;
    double* d_coef;
    std::vector<int32_t> kinds;
    std::vector<ElemCoef> coef;
};

extern "C" {

const char* hbl_last_error(void) { return g_err; }

const char* hbl_version(void) { return "hbl 0.1 (gfx950)"; }

hbl_status hbl_bunch_fill_gaussian(double* z, int64_t n, int64_t ld, uint64_t seed,
                                   const double mean[6], const double sigma[6], int64_t i0,
                                   hbl_stream stream) {
    clear_error();
    if (hbl_status st = check_bunch(z, n, ld, "fill_gaussian")) return st;
    HBL_REQUIRE(mean && sigma, "fill_gaussian: NULL mean or sigma");
    for (int j = 0; j < 6; ++j)
        HBL_REQUIRE(isfinite(mean[j]) && isfinite(sigma[j]) && sigma[j] >= 0.0,
                    "fill_gaussian: mean/sigma[%d] must be finite, sigma >= 0", j);
    HBL_REQUIRE(i0 >= 0 && i0 <= INT64_MAX - n, "fill_gaussian: bad first index");
    if (n == 0) return HBL_OK;
    HBL_HIP(launch_fill_gaussian(z, n, ld, seed, mean, sigma, i0, (hipStream_t)stream));
    return HBL_OK;
}

hbl_status hbl_lattice_create(const hbl_element* elems, int32_t n_elem, const hbl_ref* ref,
                              hbl_lattice** out) {
    clear_error();
    HBL_REQUIRE(out, "lattice_create: NULL output handle");
    *out = nullptr;
    HBL_REQUIRE(n_elem >= 0 && n_elem <= (1 << 20), "lattice_create: bad element count %d", (int)n_elem);
    HBL_REQUIRE(n_elem == 0 || elems, "lattice_create: NULL element array");
    if (hbl_status st = check_ref(ref)) return st;
    std::vector<int32_t> kinds(n_elem);
    std::vector<ElemCoef> coef(n_elem);
    double length = 0.0;
    for (int32_t i = 0; i < n_elem; ++i) {
        if (hbl_status st = compile_element(elems[i], ref->gamma, &kinds[i], &coef[i])) {
            char msg[512];
            snprintf(msg, sizeof msg, "%s", g_err);
            set_error(st, "element %d: %s", (int)i, msg);
            return st;
        }
        if (elems[i].kind != HBL_THIN_LENS) length += elems[i].L;
    }
    hbl_lattice* lat = new (std::nothrow) hbl_lattice();
    if (!lat) { set_error(HBL_ENOMEM, "lattice_create: out of host memory"); return HBL_ENOMEM; }
    lat->n_elem = n_elem;
    lat->gamma = ref->gamma;
    lat->length = length;
    lat->kinds = kinds;
    lat->coef = coef;
    lat->d_kinds = nullptr;
    lat->d_coef = nullptr;
    if (hipGetDevice(&lat->device) != hipSuccess) {
        delete lat;
        set_error(HBL_EHIP, "lattice_create: no HIP device");
        return HBL_EHIP;
    }
    if (n_elem > 0) {
        void *pk = nullptr, *pc = nullptr;
        if (hipMalloc(&pk, sizeof(int32_t) * n_elem) != hipSuccess ||
            hipMalloc(&pc, sizeof(ElemCoef) * n_elem) != hipSuccess) {
            if (pk) (void)hipFree(pk);
            delete lat;
            set_error(HBL_ENOMEM, "lattice_create: device allocation failed");
            return HBL_ENOMEM;
        }
        lat->d_kinds = static_cast<int32_t*>(pk);
        lat->d_coef = static_cast<double*>(pc);
        if (hipMemcpy(pk, kinds.data(), sizeof(int32_t) * n_elem, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(pc, coef.data(), sizeof(ElemCoef) * n_elem, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(pk);
            (void)hipFree(pc);
            delete lat;
            set_error(HBL_EHIP, "lattice_create: upload failed");
            return HBL_EHIP;
        }
    }
    *out = lat;
    return HBL_OK;
}

hbl_status hbl_lattice_destroy(hbl_lattice* lat) {
    clear_error();
    if (!lat) return HBL_OK;
    if (lat->d_kinds) (void)hipFree(lat->d_kinds);
    if (lat->d_coef) (void)hipFree(lat->d_coef);
    delete lat;
    return HBL_OK;
}

hbl_status hbl_lattice_info(const hbl_lattice* lat, double* length, int32_t* n_elem) {
    clear_error();
    HBL_REQUIRE(lat, "lattice_info: NULL handle");
    if (length) *length = lat->length;
    if (n_elem) *n_elem = lat->n_elem;
    return HBL_OK;
}

hbl_status hbl_push_lattice(double* z, int64_t n, int64_t ld, const hbl_lattice* lat, hbl_ref* ref,
                            uint32_t flags, hbl_stream stream) {
    clear_error();
    if (hbl_status st = check_bunch(z, n, ld, "push_lattice")) return st;
    HBL_REQUIRE(lat, "push_lattice: NULL lattice");
    if (hbl_status st = check_ref(ref)) return st;
    HBL_REQUIRE(ref->gamma == lat->gamma,
                "push_lattice: lattice compiled for gamma %.17g, reference has %.17g", lat->gamma,
                ref->gamma);
    HBL_REQUIRE(flags == HBL_FUSED || flags == HBL_UNFUSED, "push_lattice: unknown flags 0x%x", flags);
    if (n > 0 && lat->n_elem > 0) {
        hipStream_t s = (hipStream_t)stream;
        if (flags == HBL_FUSED) {
            HBL_HIP(launch_lattice_fused(z, n, ld, lat->d_kinds, lat->d_coef, lat->n_elem, s));
        } else {
            for (int32_t i = 0; i < lat->n_elem; ++i)
                HBL_HIP(launch_lattice_element(z, n, ld, lat->kinds[i], lat->coef[i], s));
        }
    }
    ref->s += lat->length;
    return HBL_OK;
}

hbl_status hbl_apply_stage(double* z, int64_t n, int64_t ld, const hbl_element* stage, hbl_ref* ref,
                           double* record, int64_t record_ld, hbl_stream stream) {
    clear_error();
    if (hbl_status st = check_bunch(z, n, ld, "apply_stage")) return st;
    HBL_REQUIRE(stage, "apply_stage: NULL stage");
    HBL_REQUIRE(stage->kind == HBL_STAGE, "apply_stage: element kind %d is not a stage", (int)stage->kind);
    HBL_REQUIRE(stage->nsub >= 1 && stage->nsub <= (1 << 24), "apply_stage: nsub = %d out of [1, 2^24]", (int)stage->nsub);
    HBL_REQUIRE(finite_pos(stage->L), "apply_stage: L must be finite and > 0");
    HBL_REQUIRE(isfinite(stage->n0_m3) && stage->n0_m3 >= 0.0, "apply_stage: n0 must be finite and >= 0");
    HBL_REQUIRE(isfinite(stage->dE_MeV), "apply_stage: dE must be finite");
    if (hbl_status st = check_ref(ref)) return st;
    const double g_in = ref->gamma;
    const double g_out = g_in + stage->dE_MeV / ref->mass_MeV;
    HBL_REQUIRE(g_out > 1.0 + 1e-6, "apply_stage: exit gamma %g must exceed 1", g_out);
    if (record) {
        if (hbl_status st = check_bunch(record, n, record_ld, "apply_stage record")) return st;
        const uintptr_t a0 = (uintptr_t)z, a1 = a0 + (uintptr_t)(5 * ld + n) * 8;
        const uintptr_t b0 = (uintptr_t)record, b1 = b0 + (uintptr_t)(5 * record_ld + n) * 8;
        HBL_REQUIRE(n == 0 || a1 <= b0 || b1 <= a0, "apply_stage: record buffer overlaps the bunch");
    }
    const double bg_in = sqrt(g_in * g_in - 1.0), bg_out = sqrt(g_out * g_out - 1.0);
    const int32_t N = stage->nsub;
    const double L = stage->L, h = L / N;
    const double gp = (g_out - g_in) / L;
    const double kp2 = stage->n0_m3 * kQe * kQe / (kEps0 * kMeKg * kCLight * kCLight);
    const double kappa = 0.5 * kp2;
    StageParams p;
    p.bg_in = bg_in;
    p.h = h;
    p.hk2 = h * h * kappa;
    p.half_hk2 = 0.5 * p.hk2;
    p.inv_h_bgout = 1.0 / (h * bg_out);
    p.pt_scale = bg_in / bg_out;
    p.r56 = (gp == 0.0) ? bg_in * L / (g_in * g_in * g_in)
                        : bg_in * (1.0 / (g_in * g_in) - 1.0 / (g_out * g_out)) / (2.0 * gp);
    p.nsub = N;
    // Newton steps for 1/gamma_i from the previous substep: the relative
    // change per substep is at most d = |gp h| / gamma_min, with particle
    // energy offsets |dgamma_i| up to 10% of the reference (a linear-optics
    // beam stays far inside); k steps reduce it to d^(2^k); require < 1e-17,
    // else divide every substep.
    const double gmin = fmin(g_in, g_out) * 0.9;
    const double d = fabs(gp * h) / gmin;
    int newton = 0;
    if (d < 0.25) {
        double err = d;
        newton = 1;
        while (newton < 4) {
            err = err * err;
            if (err < 1e-17) break;
            ++newton;
        }
        if (err >= 1e-17) newton = 0;
    }
    p.newton = newton;
    hbl_status st = HBL_OK;
    if (n > 0) {
        const double* tab = stage_table(g_in, gp, h, N, &st);
        if (!tab) return st;
        HBL_HIP(launch_stage(z, n, ld, record, record_ld, p, tab, (hipStream_t)stream));
    }
    ref->gamma = g_out;
    ref->s += L;
    return HBL_OK;
}

hbl_status hbl_moments_async(const double* z, int64_t n, int64_t ld, double* out27, hbl_stream stream) {
    clear_error();
    if (hbl_status st = check_bunch(z, n, ld, "moments")) return st;
    HBL_REQUIRE(n >= 1, "moments: need n >= 1");
    HBL_REQUIRE(out27 && ((uintptr_t)out27 & 7u) == 0, "moments: bad output pointer");
    double* ws = workspace(reduce_ws_bytes(n));
    if (!ws) { set_error(HBL_ENOMEM, "moments: workspace allocation failed"); return HBL_ENOMEM; }
    HBL_HIP(launch_moments(z, n, ld, ws, out27, (hipStream_t)stream));
    return HBL_OK;
}

hbl_status hbl_moments(const double* z, int64_t n, int64_t ld, double mean6[6], double cov21[21],
                       hbl_stream stream) {
    clear_error();
    if (hbl_status st = check_bunch(z, n, ld, "moments")) return st;
    HBL_REQUIRE(n >= 1, "moments: need n >= 1");
    HBL_REQUIRE(mean6 && cov21, "moments: NULL output");
    const size_t wsb = reduce_ws_bytes(n) + 64 * sizeof(double);
    double* ws = workspace(wsb);
    if (!ws) { set_error(HBL_ENOMEM, "moments: workspace allocation failed"); return HBL_ENOMEM; }
    double* dout = ws + (wsb / sizeof(double) - 64);
    hipStream_t s = (hipStream_t)stream;
    HBL_HIP(launch_moments(z, n, ld, ws, dout, s));
    double host[27];
    HBL_HIP(hipMemcpyAsync(host, dout, sizeof host, hipMemcpyDeviceToHost, s));
    HBL_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < 6; ++j) mean6[j] = host[j];
    for (int q = 0; q < 21; ++q) cov21[q] = host[6 + q];
    for (int q = 0; q < 27; ++q)
        if (!isfinite(host[q])) {
            set_error(HBL_ENONFINITE, "moments: bunch holds non-finite values");
            return HBL_ENONFINITE;
        }
    return HBL_OK;
}

hbl_status hbl_emittances(const double cov21[21], double eps3[3]) {
    clear_error();
    HBL_REQUIRE(cov21 && eps3, "emittances: NULL argument");
    static const int pos[3] = {0, 1, 2}, mom[3] = {3, 4, 5};
    for (int p = 0; p < 3; ++p) {
        const int j = pos[p], k = mom[p];
        const double a = cov21[j * 6 - j * (j - 1) / 2];
        const double b = cov21[j * 6 - j * (j - 1) / 2 + (k - j)];
        const double d = cov21[k * 6 - k * (k - 1) / 2];
        // Kahan's FMA product difference a*d - b*b
        const double w = b * b;
        const double e = fma(-b, b, w);
        const double f = fma(a, d, -w);
        const double det = f + e;
        eps3[p] = det > 0.0 ? sqrt(det) : 0.0;
        if (!isfinite(a) || !isfinite(b) || !isfinite(d)) {
            set_error(HBL_ENONFINITE, "emittances: non-finite covariance");
            return HBL_ENONFINITE;
        }
    }
    return HBL_OK;
}

hbl_status hbl_compare(const double* zs, const double* zf, int64_t n, int64_t ld, double rms6[6],
                       double centroid6[6], double eps_rel3[3], hbl_stream stream) {
    clear_error();
    if (hbl_status st = check_bunch(zs, n, ld, "compare(test)")) return st;
    if (hbl_status st = check_bunch(zf, n, ld, "compare(ref)")) return st;
    HBL_REQUIRE(n >= 1, "compare: need n >= 1");
    HBL_REQUIRE(rms6 && centroid6 && eps_rel3, "compare: NULL output");
    double ms[6], cs[21], mf[6], cf[21], es[3], ef[3];
    if (hbl_status st = hbl_moments(zs, n, ld, ms, cs, stream)) return st;
    if (hbl_status st = hbl_moments(zf, n, ld, mf, cf, stream)) return st;
    const size_t wsb = reduce_ws_bytes(n) + 64 * sizeof(double);
    double* ws = workspace(wsb);
    if (!ws) { set_error(HBL_ENOMEM, "compare: workspace allocation failed"); return HBL_ENOMEM; }
    double* dout = ws + (wsb / sizeof(double) - 64);
    hipStream_t s = (hipStream_t)stream;
    HBL_HIP(launch_diff2(zs, zf, n, ld, ws, dout, s));
    double d2[6];
    HBL_HIP(hipMemcpyAsync(d2, dout, sizeof d2, hipMemcpyDeviceToHost, s));
    HBL_HIP(hipStreamSynchronize(s));
    hbl_emittances(cs, es);
    if (hbl_status st = hbl_emittances(cf, ef)) return st;
    for (int j = 0; j < 6; ++j) {
        const double sig = sqrt(cf[j * 6 - j * (j - 1) / 2]);
        rms6[j] = sqrt(d2[j] / (double)n) / sig;
        centroid6[j] = (ms[j] - mf[j]) / sig;
    }
    for (int p = 0; p < 3; ++p) eps_rel3[p] = es[p] / ef[p] - 1.0;
    return HBL_OK;
}

}  // extern "C"
