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
#include "hbl_elements.hpp"

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
// reduction workspaces, one per (device, stream): {buffer, bytes}
std::map<std::pair<int, uintptr_t>, std::pair<double*, size_t>> g_ws;
constexpr size_t kMaxWorkspaces = 256;

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

// The reduction workspace of stream s on the current device, grown on demand
// and kept until the process ends.  Work on one stream runs in order, so the
// stream's reductions reuse its buffer; reductions on different streams get
// different buffers and never race.  Growing waits for the stream's earlier
// work (which may still read the old buffer) before freeing it; past
// kMaxWorkspaces buffers the device is synchronised and all are released.
double* workspace(size_t bytes, hipStream_t s) {
    const int d = current_device();
    if (d < 0 || d >= kMaxDev) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    const auto key = std::make_pair(d, (uintptr_t)s);
    auto it = g_ws.find(key);
    if (it == g_ws.end() && g_ws.size() >= kMaxWorkspaces) {
        if (hipDeviceSynchronize() != hipSuccess) return nullptr;
        for (auto& kv : g_ws) (void)hipFree(kv.second.first);
        g_ws.clear();
    }
    auto& e = g_ws[key];
    if (e.second < bytes) {
        if (e.first) {
            if (hipStreamSynchronize(s) != hipSuccess) return nullptr;
            (void)hipFree(e.first);
        }
        e = {nullptr, 0};
        const size_t want = bytes < (1u << 20) ? (1u << 20) : bytes;
        void* p = nullptr;
        if (hipMalloc(&p, want) != hipSuccess) return nullptr;
        e = {static_cast<double*>(p), want};
    }
    return e.first;
}

// gamma_ref at the middle of each substep of a stage, then the ramp increment
// gp * s_mid of each substep (used by energy-correlated gain), cached per
// device.
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
    std::vector<double> tab(2 * (size_t)nsub);
    for (int32_t s = 0; s < nsub; ++s) {
        tab[s] = g_in + gp * ((s + 0.5) * h);
        tab[nsub + s] = gp * ((s + 0.5) * h);
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, sizeof(double) * 2 * nsub);
    if (e != hipSuccess) {
        *st = HBL_ENOMEM;
        set_error(HBL_ENOMEM, "stage table allocation failed: %s", hipGetErrorString(e));
        return nullptr;
    }
    e = hipMemcpy(p, tab.data(), sizeof(double) * 2 * nsub, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p);
        *st = HBL_EHIP;
        set_error(HBL_EHIP, "stage table upload failed: %s", hipGetErrorString(e));
        return nullptr;
    }
    // kept until the process ends (2 nsub doubles per distinct stage): a table
    // handed to one thread may still be in use by work it has enqueued
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

// `bytes` bytes from p must lie in one HIP allocation of the current device:
// a host pointer, memory of another device or a range past the allocation
// would fault the kernel or corrupt a neighbour.  Called after the other
// checks, just before work is enqueued (a failed query's HIP error is
// cleared, so it cannot surface at a later launch).
hbl_status check_device(const void* p, size_t bytes, const char* what) {
    if (bytes == 0) return HBL_OK;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        set_error(HBL_EHIP, "%s: no current HIP device", what);
        return HBL_EHIP;
    }
    hipPointerAttribute_t a;
    memset(&a, 0, sizeof a);
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        set_error(HBL_EINVAL, "%s: %p is not HIP device memory", what, p);
        return HBL_EINVAL;
    }
    if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged) {
        set_error(HBL_EINVAL, "%s: %p is host memory, not device memory", what, p);
        return HBL_EINVAL;
    }
    if (a.device != dev) {
        set_error(HBL_EINVAL, "%s: memory of device %d used with device %d current", what, a.device, dev);
        return HBL_EINVAL;
    }
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p) != hipSuccess) {
        (void)hipGetLastError();
        set_error(HBL_EINVAL, "%s: no allocation holds %p", what, p);
        return HBL_EINVAL;
    }
    if ((uintptr_t)p + bytes > (uintptr_t)base + size) {
        set_error(HBL_EINVAL, "%s: %zu bytes from %p run past the end of their allocation", what, bytes, p);
        return HBL_EINVAL;
    }
    return HBL_OK;
}

// Bytes spanned by the six rows of a bunch of n particles, leading dimension ld.
size_t bunch_bytes(int64_t n, int64_t ld) { return n > 0 ? (size_t)(5 * ld + n) * sizeof(double) : 0; }

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
}  // namespace

GenCoef hbl::unify(int32_t kind, const ElemCoef& e, const double* chrom8) {
    GenCoef u;
    memset(&u, 0, sizeof u);
    double* g = u.g;
    const double* c = e.c;
    switch (kind) {
        case kDrift:  // x + L px, y + L py, t + r56 pt
            g[0] = 1.0; g[1] = c[0]; g[4] = 1.0; g[6] = 1.0; g[7] = c[0]; g[9] = 1.0; g[12] = c[1];
            break;
        case kQuad:
            g[0] = c[0]; g[1] = c[1]; g[3] = c[2]; g[4] = c[3];
            g[6] = c[4]; g[7] = c[5]; g[8] = c[6]; g[9] = c[7]; g[12] = c[8];
            break;
        case kSbend:
            g[0] = c[0]; g[1] = c[1]; g[2] = c[2]; g[3] = c[3]; g[4] = c[4]; g[5] = c[5];
            g[6] = 1.0; g[7] = c[9]; g[9] = 1.0; g[10] = c[6]; g[11] = c[7]; g[12] = c[8];
            break;
        default:      // thin lens: px + c0 x, py + c0 y
            g[0] = 1.0; g[3] = c[0]; g[4] = 1.0; g[6] = 1.0; g[8] = c[0]; g[9] = 1.0;
            break;
    }
    if (chrom8)
        for (int q = 0; q < 8; ++q) g[16 + q] = chrom8[q];
    return u;
}

namespace {

// First-order chromatic terms of a focusing plane [[a, b], [c, a]] of strength
// k: the particle sees k (1 - delta) to first order, so with w = sqrt|k| the
// entries change by delta times their derivative along dw/d(delta) = -w/2.
void plane_derivative(bool focusing, double w, double L, double* da, double* db, double* dc) {
    const double ph = w * L;
    if (focusing) {
        const double sn = sin(ph), cs = cos(ph);
        *da = 0.5 * ph * sn;
        *db = 0.5 * (sn / w - L * cs);
        *dc = 0.5 * w * (sn + ph * cs);
    } else {
        const double sh = sinh(ph), ch = cosh(ph);
        *da = -0.5 * ph * sh;
        *db = 0.5 * (sh / w - L * ch);
        *dc = -0.5 * w * (sh + ph * ch);
    }
}

// chrom8 receives the chromatic coefficients (the factors of pt, with
// delta = -pt/beta) when the element is chromatic; *chromatic says so.
hbl_status compile_element(const hbl_element& e, double gamma, int32_t* kind, ElemCoef* c, double chrom8[8],
                           bool* chromatic) {
    memset(c, 0, sizeof *c);
    for (int q = 0; q < 8; ++q) chrom8[q] = 0.0;
    *chromatic = false;
    const double bg = sqrt(gamma * gamma - 1.0), beta = bg / gamma;
    const double r56d = e.L / (bg * bg);
    HBL_REQUIRE(e.reserved == 0, "reserved field must be 0");
    HBL_REQUIRE(e.chirp == 0.0, "chirp applies to stages only");
    HBL_REQUIRE(e.chromatic == 0 || e.chromatic == 1, "chromatic must be 0 or 1");
    HBL_REQUIRE(e.chromatic == 0 || e.kind == HBL_QUAD || e.kind == HBL_THIN_LENS,
                "chromatic applies to quads and thin lenses only");
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
            if (e.chromatic) {
                double ax, bx, cx, ay, by, cy;
                plane_derivative(xf, w, e.L, &ax, &bx, &cx);
                plane_derivative(!xf, w, e.L, &ay, &by, &cy);
                const double m = -1.0 / beta;       // d(delta)/d(pt)
                chrom8[0] = m * ax; chrom8[1] = m * bx; chrom8[2] = m * cx; chrom8[3] = m * ax;
                chrom8[4] = m * ay; chrom8[5] = m * by; chrom8[6] = m * cy; chrom8[7] = m * ay;
                *chromatic = true;
            }
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
            if (e.chromatic) {      // kick c0 x (1 - delta) = c0 x + (c0 / beta) x pt
                chrom8[2] = c->c[0] / beta;
                chrom8[6] = c->c[0] / beta;
                *chromatic = true;
            }
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
    double* d_coef;   // one allocation: n GenCoef records, then n ElemCoef records
    double* d_gen;
    bool chromatic;   // any chromatic element
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
    if (hbl_status st = check_device(z, bunch_bytes(n, ld), "fill_gaussian")) return st;
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
    std::vector<double> chrom(8 * (size_t)n_elem);
    std::vector<char> is_chrom(n_elem);
    bool any_chrom = false;
    double length = 0.0;
    for (int32_t i = 0; i < n_elem; ++i) {
        bool ch = false;
        hbl_status st = compile_element(elems[i], ref->gamma, &kinds[i], &coef[i], &chrom[8 * (size_t)i], &ch);
        is_chrom[i] = ch;
        any_chrom = any_chrom || ch;
        if (st) {
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
    lat->d_gen = nullptr;
    lat->chromatic = any_chrom;
    if (hipGetDevice(&lat->device) != hipSuccess) {
        delete lat;
        set_error(HBL_EHIP, "lattice_create: no HIP device");
        return HBL_EHIP;
    }
    if (n_elem > 0) {
        void *pk = nullptr, *pc = nullptr;
        std::vector<GenCoef> gen((size_t)n_elem);
        for (int32_t i = 0; i < n_elem; ++i)
            gen[i] = unify(kinds[i], coef[i], is_chrom[i] ? &chrom[8 * (size_t)i] : nullptr);
        const size_t gen_bytes = sizeof(GenCoef) * n_elem;
        if (hipMalloc(&pk, sizeof(int32_t) * n_elem) != hipSuccess ||
            hipMalloc(&pc, gen_bytes + sizeof(ElemCoef) * n_elem) != hipSuccess) {
            if (pk) (void)hipFree(pk);
            delete lat;
            set_error(HBL_ENOMEM, "lattice_create: device allocation failed");
            return HBL_ENOMEM;
        }
        lat->d_kinds = static_cast<int32_t*>(pk);
        lat->d_gen = static_cast<double*>(pc);
        lat->d_coef = lat->d_gen + (size_t)kGen * n_elem;
        if (hipMemcpy(pk, kinds.data(), sizeof(int32_t) * n_elem, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(lat->d_gen, gen.data(), gen_bytes, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(lat->d_coef, coef.data(), sizeof(ElemCoef) * n_elem, hipMemcpyHostToDevice) != hipSuccess) {
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
    if (lat->d_gen) (void)hipFree(lat->d_gen);   // holds the ElemCoef records too
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
        if (hbl_status st = check_device(z, bunch_bytes(n, ld), "push_lattice")) return st;
        hipStream_t s = (hipStream_t)stream;
        if (flags == HBL_FUSED) {
            HBL_HIP(launch_lattice_fused(z, n, ld, lat->d_gen, lat->d_kinds, lat->n_elem, lat->chromatic, s));
        } else if (lat->chromatic) {   // one launch per element, through its unified record
            for (int32_t i = 0; i < lat->n_elem; ++i)
                HBL_HIP(launch_lattice_gen(z, n, ld, lat->d_gen + (size_t)kGen * i, true, s));
        } else {
            for (int32_t i = 0; i < lat->n_elem; ++i)
                HBL_HIP(launch_lattice_element(z, n, ld, lat->kinds[i], lat->coef[i], s));
        }
    }
    ref->s += lat->length;
    return HBL_OK;
}

}  // extern "C"

namespace {

LatticeView view_of(const hbl_lattice* lat) {
    LatticeView v{nullptr, nullptr, nullptr, 0, 0};
    if (lat) {
        v.kinds = lat->d_kinds;
        v.coef = lat->d_coef;
        v.gen = lat->d_gen;
        v.n = lat->n_elem;
        v.chromatic = lat->chromatic ? 1 : 0;
    }
    return v;
}

// A gap lattice must be compiled for the reference energy it is applied at.
hbl_status check_gap(const hbl_lattice* lat, double gamma, const char* what) {
    if (!lat) return HBL_OK;
    HBL_REQUIRE(lat->gamma == gamma, "%s lattice compiled for gamma %.17g, applied at gamma %.17g", what,
                lat->gamma, gamma);
    return HBL_OK;
}

// Largest relative change of a particle's gamma over one substep: the ramp
// gp h over the smallest gamma, particle energy offsets allowed down to 90 % of
// the reference (a linear-optics beam stays far inside); doubled for a chirped
// stage, whose particle ramp rate gp (1 + chirp t) is sized for |chirp t| <= 1.
double reciprocal_drift(double g_in, double g_out, double gp, double h, double chirp) {
    const double gmin = fmin(g_in, g_out) * 0.9;
    return fabs(gp * h) * (chirp != 0.0 ? 2.0 : 1.0) / gmin;
}

// Newton steps r <- r (2 - a r) that take the previous substep's reciprocal,
// relative error at most d, to 1/gamma_i: k steps leave d^(2^k); the fewest k
// in 1..4 with d^(2^k) < 1e-17, else 0 (divide every substep).
int32_t newton_steps(double d) {
    if (!(d < 0.25)) return 0;
    double err = d;
    for (int32_t k = 1; k <= 4; ++k) {
        err *= err;
        if (err < 1e-17) return k;
    }
    return 0;
}

hbl_status apply_stage_impl(double* z, int64_t n, int64_t ld, const hbl_lattice* pre, const hbl_element* stage,
                            const hbl_lattice* post, hbl_ref* ref, double* record, int64_t record_ld,
                            hbl_stream stream) {
    clear_error();
    if (hbl_status st = check_bunch(z, n, ld, "apply_stage")) return st;
    HBL_REQUIRE(stage, "apply_stage: NULL stage");
    HBL_REQUIRE(stage->kind == HBL_STAGE, "apply_stage: element kind %d is not a stage", (int)stage->kind);
    HBL_REQUIRE(stage->nsub >= 1 && stage->nsub <= (1 << 24), "apply_stage: nsub = %d out of [1, 2^24]", (int)stage->nsub);
    HBL_REQUIRE(finite_pos(stage->L), "apply_stage: L must be finite and > 0");
    HBL_REQUIRE(isfinite(stage->n0_m3) && stage->n0_m3 >= 0.0, "apply_stage: n0 must be finite and >= 0");
    HBL_REQUIRE(isfinite(stage->dE_MeV), "apply_stage: dE must be finite");
    HBL_REQUIRE(isfinite(stage->chirp), "apply_stage: chirp must be finite");
    HBL_REQUIRE(stage->chromatic == 0 && stage->reserved == 0, "apply_stage: chromatic/reserved must be 0 for a stage");
    if (hbl_status st = check_ref(ref)) return st;
    const double g_in = ref->gamma;
    const double g_out = g_in + stage->dE_MeV / ref->mass_MeV;
    HBL_REQUIRE(g_out > 1.0 + 1e-6, "apply_stage: exit gamma %g must exceed 1", g_out);
    if (hbl_status st = check_gap(pre, g_in, "apply_stage: entrance")) return st;
    if (hbl_status st = check_gap(post, g_out, "apply_stage: exit")) return st;
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
    p.chirp = stage->chirp;
    p.chirp_gain = stage->chirp * (g_out - g_in);
    p.chirp_t = stage->chirp * (gp * L * L / (2.0 * g_in * g_out * g_out));
    p.inv_bgout = 1.0 / bg_out;
    p.nsub = N;
    // 1/gamma_i by Newton steps from the previous substep's reciprocal (a
    // chirped particle beyond |chirp t| <= 1 divides in the kernel)
    p.newton = newton_steps(reciprocal_drift(g_in, g_out, gp, h, stage->chirp));
    hbl_status st = HBL_OK;
    if (n > 0) {
        if (hbl_status s2 = check_device(z, bunch_bytes(n, ld), "apply_stage")) return s2;
        if (record)
            if (hbl_status s2 = check_device(record, bunch_bytes(n, record_ld), "apply_stage record")) return s2;
        const double* tab = stage_table(g_in, gp, h, N, &st);
        if (!tab) return st;
        HBL_HIP(launch_stage(z, n, ld, record, record_ld, p, tab, view_of(pre), view_of(post),
                             (hipStream_t)stream));
    }
    ref->gamma = g_out;
    ref->s += (pre ? pre->length : 0.0) + L + (post ? post->length : 0.0);
    return HBL_OK;
}

}  // namespace

extern "C" {

hbl_status hbl_apply_stage(double* z, int64_t n, int64_t ld, const hbl_element* stage, hbl_ref* ref,
                           double* record, int64_t record_ld, hbl_stream stream) {
    return apply_stage_impl(z, n, ld, nullptr, stage, nullptr, ref, record, record_ld, stream);
}

hbl_status hbl_stage_newton_steps(const hbl_element* stage, const hbl_ref* ref, int32_t* steps) {
    clear_error();
    HBL_REQUIRE(stage && steps, "stage_newton_steps: NULL argument");
    HBL_REQUIRE(stage->kind == HBL_STAGE, "stage_newton_steps: element kind %d is not a stage", (int)stage->kind);
    HBL_REQUIRE(stage->nsub >= 1 && stage->nsub <= (1 << 24), "stage_newton_steps: nsub = %d out of [1, 2^24]",
                (int)stage->nsub);
    HBL_REQUIRE(finite_pos(stage->L), "stage_newton_steps: L must be finite and > 0");
    HBL_REQUIRE(isfinite(stage->dE_MeV) && isfinite(stage->chirp), "stage_newton_steps: dE and chirp must be finite");
    if (hbl_status st = check_ref(ref)) return st;
    const double g_in = ref->gamma, g_out = g_in + stage->dE_MeV / ref->mass_MeV;
    HBL_REQUIRE(g_out > 1.0 + 1e-6, "stage_newton_steps: exit gamma %g must exceed 1", g_out);
    const double h = stage->L / stage->nsub, gp = (g_out - g_in) / stage->L;
    *steps = newton_steps(reciprocal_drift(g_in, g_out, gp, h, stage->chirp));
    return HBL_OK;
}

hbl_status hbl_apply_stage_gaps(double* z, int64_t n, int64_t ld, const hbl_lattice* pre,
                                const hbl_element* stage, const hbl_lattice* post, hbl_ref* ref,
                                double* record, int64_t record_ld, hbl_stream stream) {
    return apply_stage_impl(z, n, ld, pre, stage, post, ref, record, record_ld, stream);
}

hbl_status hbl_moments_async(const double* z, int64_t n, int64_t ld, double* out27, hbl_stream stream) {
    clear_error();
    if (hbl_status st = check_bunch(z, n, ld, "moments")) return st;
    HBL_REQUIRE(n >= 1, "moments: need n >= 1");
    HBL_REQUIRE(out27 && ((uintptr_t)out27 & 7u) == 0, "moments: bad output pointer");
    if (hbl_status st = check_device(z, bunch_bytes(n, ld), "moments")) return st;
    if (hbl_status st = check_device(out27, 27 * sizeof(double), "moments output")) return st;
    double* ws = workspace(reduce_ws_bytes(n), (hipStream_t)stream);
    if (!ws) { set_error(HBL_ENOMEM, "moments: workspace allocation failed"); return HBL_ENOMEM; }
    HBL_HIP(launch_moments(z, n, ld, ws, out27, (hipStream_t)stream));
    return HBL_OK;
}

hbl_status hbl_moments_async_noalloc(const double* z, int64_t n, int64_t ld, double* out27, hbl_stream stream) {
    clear_error();
    if (hbl_status st = check_bunch(z, n, ld, "moments_async_noalloc")) return st;
    HBL_REQUIRE(n >= 1, "moments_async_noalloc: need n >= 1");
    HBL_REQUIRE(out27 && ((uintptr_t)out27 & 7u) == 0, "moments_async_noalloc: bad output pointer");
    const size_t need = reduce_ws_bytes(n), have = reduce_scratch_bytes();
    HBL_REQUIRE(need <= have, "moments_async_noalloc: n = %lld needs %zu bytes of scratch, more than the %zu reserved",
                (long long)n, need, have);
    if (hbl_status st = check_device(z, bunch_bytes(n, ld), "moments_async_noalloc")) return st;
    if (hbl_status st = check_device(out27, 27 * sizeof(double), "moments_async_noalloc output")) return st;
    double* ws = nullptr;
    HBL_HIP(reduce_scratch(&ws));
    HBL_HIP(launch_moments(z, n, ld, ws, out27, (hipStream_t)stream));
    return HBL_OK;
}

hbl_status hbl_moments(const double* z, int64_t n, int64_t ld, double mean6[6], double cov21[21],
                       hbl_stream stream) {
    clear_error();
    if (hbl_status st = check_bunch(z, n, ld, "moments")) return st;
    HBL_REQUIRE(n >= 1, "moments: need n >= 1");
    HBL_REQUIRE(mean6 && cov21, "moments: NULL output");
    if (hbl_status st = check_device(z, bunch_bytes(n, ld), "moments")) return st;
    const size_t wsb = reduce_ws_bytes(n) + 64 * sizeof(double);
    hipStream_t s = (hipStream_t)stream;
    double* ws = workspace(wsb, s);
    if (!ws) { set_error(HBL_ENOMEM, "moments: workspace allocation failed"); return HBL_ENOMEM; }
    double* dout = ws + (wsb / sizeof(double) - 64);
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
    hipStream_t s = (hipStream_t)stream;
    double* ws = workspace(wsb, s);
    if (!ws) { set_error(HBL_ENOMEM, "compare: workspace allocation failed"); return HBL_ENOMEM; }
    double* dout = ws + (wsb / sizeof(double) - 64);
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

// =================================================================== surrogate
namespace {

// Philox4x32-10 (Salmon et al., SC'11) on the host: parameter initialisation
// and the per-epoch Fisher-Yates orders.
void philox_host(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[1] = (uint32_t)p1;
        c[3] = (uint32_t)p0;
        c[0] = n0;
        c[2] = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Fisher-Yates from the identity: for i = n-1..1 swap i and
// j = floor(r (i+1) / 2^32), r = word i%4 of block (i/4, epoch, 'SHUF').
void epoch_order(int32_t* perm, int64_t n, uint64_t seed, int64_t epoch) {
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    uint32_t w[4] = {0, 0, 0, 0};
    int64_t blk = -1;
    for (int64_t i = n - 1; i >= 1; --i) {
        if ((i >> 2) != blk) {
            blk = i >> 2;
            w[0] = (uint32_t)blk;
            w[1] = (uint32_t)((uint64_t)blk >> 32);
            w[2] = (uint32_t)epoch;
            w[3] = 0x53485546u;
            philox_host(w, k0, k1);
        }
        const uint64_t j = ((uint64_t)w[i & 3] * (uint64_t)(i + 1)) >> 32;
        const int32_t t = perm[i];
        perm[i] = perm[j];
        perm[j] = t;
    }
}

constexpr int kMlpParams = 9158;
// keep_best = 2: candidates are the window epochs whose test loss is within
// this fraction of the window's lowest
constexpr double kEpsSelectLossTol = 0.10;
constexpr uint64_t kFileMagic = 0x31534C42484C4248ull;  // "HBLHBLS1"

}  // namespace

struct hbl_surrogate {
    int device;
    hbl_mlp_shape shape;
    float* d_params;
    float* d_m;
    float* d_v;
    uint32_t* d_img;
    double norm[24];
    bool has_norm;
    int64_t step;
    bool has_stage;
    double dE_MeV, L, gamma_in;
    // training scratch, allocated on first use
    float* d_part;
    float* d_loss_part;
    double* d_eval_part;
    double* d_loss_acc;
    float* d_best;          // parameters of the lowest test loss (keep_best)
    double* d_best_info;    // {lowest test loss, its epoch}
    int32_t part_blocks;
    int32_t loss_slots;
};

namespace {

void sur_free(hbl_surrogate* m) {
    if (!m) return;
    void* ptrs[] = {m->d_params, m->d_m,         m->d_v,          m->d_img,   m->d_part,
                    m->d_loss_part, m->d_eval_part, m->d_loss_acc, m->d_best, m->d_best_info};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete m;
}

hbl_status sur_alloc(hbl_surrogate** out, const hbl_mlp_shape* shape) {
    hbl_surrogate* m = new (std::nothrow) hbl_surrogate();
    if (!m) { set_error(HBL_ENOMEM, "surrogate: out of host memory"); return HBL_ENOMEM; }
    memset(m, 0, sizeof *m);
    m->shape = *shape;
    if (hipGetDevice(&m->device) != hipSuccess) {
        delete m;
        set_error(HBL_EHIP, "surrogate: no HIP device");
        return HBL_EHIP;
    }
    const size_t pb = sizeof(float) * kMlpParams;
    if (hipMalloc((void**)&m->d_params, pb) != hipSuccess || hipMalloc((void**)&m->d_m, pb) != hipSuccess ||
        hipMalloc((void**)&m->d_v, pb) != hipSuccess ||
        hipMalloc((void**)&m->d_img, sizeof(uint32_t) * mlp_image_words()) != hipSuccess) {
        sur_free(m);
        set_error(HBL_ENOMEM, "surrogate: device allocation failed");
        return HBL_ENOMEM;
    }
    if (hipMemset(m->d_m, 0, pb) != hipSuccess || hipMemset(m->d_v, 0, pb) != hipSuccess) {
        sur_free(m);
        set_error(HBL_EHIP, "surrogate: device init failed");
        return HBL_EHIP;
    }
    *out = m;
    return HBL_OK;
}

hbl_status check_shape(const hbl_mlp_shape* sh) {
    HBL_REQUIRE(sh, "surrogate: NULL shape");
    HBL_REQUIRE(sh->n_in == 6 && sh->width == 64 && sh->hidden == 3 && sh->n_out == 6,
                "surrogate: shape {%d,%d,%d,%d} not supported (kernels implement {6,64,3,6})", sh->n_in,
                sh->width, sh->hidden, sh->n_out);
    return HBL_OK;
}

hbl_status check_norm(const double* n) {
    for (int j = 0; j < 24; ++j) HBL_REQUIRE(isfinite(n[j]), "surrogate: non-finite normalisation entry %d", j);
    for (int j = 0; j < 6; ++j)
        HBL_REQUIRE(n[6 + j] > 0.0 && n[18 + j] > 0.0, "surrogate: normalisation sd[%d] must be > 0", j);
    return HBL_OK;
}

hbl_status repack(hbl_surrogate* m, hipStream_t s) {
    HBL_HIP(launch_mlp_pack(m->d_params, m->d_img, s));
    return HBL_OK;
}

hbl_status ensure_train_scratch(hbl_surrogate* m, int32_t blocks, int32_t loss_slots) {
    if (m->part_blocks < blocks) {
        if (m->d_part) (void)hipFree(m->d_part);
        if (m->d_loss_part) (void)hipFree(m->d_loss_part);
        m->d_part = nullptr;
        m->d_loss_part = nullptr;
        m->part_blocks = 0;
        if (hipMalloc((void**)&m->d_part, sizeof(float) * (size_t)blocks * kMlpParams) != hipSuccess ||
            hipMalloc((void**)&m->d_loss_part, sizeof(float) * blocks) != hipSuccess) {
            set_error(HBL_ENOMEM, "surrogate: training scratch allocation failed");
            return HBL_ENOMEM;
        }
        m->part_blocks = blocks;
    }
    if (!m->d_eval_part) {
        if (hipMalloc((void**)&m->d_eval_part, sizeof(double) * 512) != hipSuccess) {
            set_error(HBL_ENOMEM, "surrogate: scratch allocation failed");
            return HBL_ENOMEM;
        }
    }
    if (m->loss_slots < loss_slots) {
        if (m->d_loss_acc) (void)hipFree(m->d_loss_acc);
        m->d_loss_acc = nullptr;
        m->loss_slots = 0;
        if (hipMalloc((void**)&m->d_loss_acc, sizeof(double) * loss_slots) != hipSuccess) {
            set_error(HBL_ENOMEM, "surrogate: loss log allocation failed");
            return HBL_ENOMEM;
        }
        m->loss_slots = loss_slots;
    }
    return HBL_OK;
}

}  // namespace

extern "C" {

hbl_status hbl_surrogate_create(const hbl_mlp_shape* shape, uint64_t init_seed, hbl_surrogate** out) {
    clear_error();
    HBL_REQUIRE(out, "surrogate_create: NULL output handle");
    *out = nullptr;
    if (hbl_status st = check_shape(shape)) return st;
    // U(-1/sqrt(fan_in), 1/sqrt(fan_in)) for weights and biases
    std::vector<float> p(kMlpParams);
    const int fan[4] = {6, 64, 64, 64}, outs[4] = {64, 64, 64, 6};
    int64_t off = 0;
    for (int layer = 0; layer < 4; ++layer) {
        const double bound = 1.0 / sqrt((double)fan[layer]);
        const int64_t cnt = (int64_t)outs[layer] * (fan[layer] + 1);
        for (int64_t q = 0; q < cnt; ++q, ++off) {
            uint32_t c[4] = {(uint32_t)off, (uint32_t)((uint64_t)off >> 32), 0u, 0x4D4C5049u};
            philox_host(c, (uint32_t)init_seed, (uint32_t)(init_seed >> 32));
            const double u = (double)(c[0] >> 8) * (1.0 / 16777216.0);
            p[off] = (float)((2.0 * u - 1.0) * bound);
        }
    }
    hbl_surrogate* m = nullptr;
    if (hbl_status st = sur_alloc(&m, shape)) return st;
    if (hipMemcpy(m->d_params, p.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice) != hipSuccess) {
        sur_free(m);
        set_error(HBL_EHIP, "surrogate_create: upload failed");
        return HBL_EHIP;
    }
    if (hbl_status st = repack(m, nullptr)) { sur_free(m); return st; }
    if (hipDeviceSynchronize() != hipSuccess) { sur_free(m); set_error(HBL_EHIP, "surrogate_create: pack failed"); return HBL_EHIP; }
    *out = m;
    return HBL_OK;
}

hbl_status hbl_surrogate_destroy(hbl_surrogate* m) {
    clear_error();
    sur_free(m);
    return HBL_OK;
}

hbl_status hbl_surrogate_num_params(const hbl_surrogate* m, int64_t* n) {
    clear_error();
    HBL_REQUIRE(m && n, "surrogate_num_params: NULL argument");
    *n = kMlpParams;
    return HBL_OK;
}

hbl_status hbl_surrogate_get_params(const hbl_surrogate* m, float* host, int64_t n) {
    clear_error();
    HBL_REQUIRE(m && host, "surrogate_get_params: NULL argument");
    HBL_REQUIRE(n == kMlpParams, "surrogate_get_params: n = %lld, need %d", (long long)n, kMlpParams);
    HBL_HIP(hipDeviceSynchronize());
    HBL_HIP(hipMemcpy(host, m->d_params, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
    return HBL_OK;
}

hbl_status hbl_surrogate_set_params(hbl_surrogate* m, const float* host, int64_t n) {
    clear_error();
    HBL_REQUIRE(m && host, "surrogate_set_params: NULL argument");
    HBL_REQUIRE(n == kMlpParams, "surrogate_set_params: n = %lld, need %d", (long long)n, kMlpParams);
    for (int64_t q = 0; q < n; ++q) HBL_REQUIRE(isfinite(host[q]), "surrogate_set_params: non-finite parameter %lld", (long long)q);
    HBL_HIP(hipDeviceSynchronize());
    HBL_HIP(hipMemcpy(m->d_params, host, sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    if (hbl_status st = repack(m, nullptr)) return st;
    HBL_HIP(hipDeviceSynchronize());
    return HBL_OK;
}

hbl_status hbl_surrogate_get_norm(const hbl_surrogate* m, double norm24[24]) {
    clear_error();
    HBL_REQUIRE(m && norm24, "surrogate_get_norm: NULL argument");
    if (!m->has_norm) { set_error(HBL_ESTATE, "surrogate_get_norm: no normalisation set or trained"); return HBL_ESTATE; }
    memcpy(norm24, m->norm, sizeof m->norm);
    return HBL_OK;
}

hbl_status hbl_surrogate_set_norm(hbl_surrogate* m, const double norm24[24]) {
    clear_error();
    HBL_REQUIRE(m && norm24, "surrogate_set_norm: NULL argument");
    if (hbl_status st = check_norm(norm24)) return st;
    memcpy(m->norm, norm24, sizeof m->norm);
    m->has_norm = true;
    return HBL_OK;
}

hbl_status hbl_surrogate_set_stage(hbl_surrogate* m, const hbl_element* stage, const hbl_ref* at_entry) {
    clear_error();
    HBL_REQUIRE(m && stage, "surrogate_set_stage: NULL argument");
    HBL_REQUIRE(stage->kind == HBL_STAGE, "surrogate_set_stage: element is not a stage");
    HBL_REQUIRE(finite_pos(stage->L) && isfinite(stage->dE_MeV), "surrogate_set_stage: bad L or dE");
    if (hbl_status st = check_ref(at_entry)) return st;
    HBL_REQUIRE(at_entry->gamma + stage->dE_MeV / at_entry->mass_MeV > 1.0, "surrogate_set_stage: exit gamma must exceed 1");
    m->has_stage = true;
    m->dE_MeV = stage->dE_MeV;
    m->L = stage->L;
    m->gamma_in = at_entry->gamma;
    return HBL_OK;
}

}  // extern "C"

namespace {

hbl_status surrogate_apply_impl(double* z, int64_t n, int64_t ld, const hbl_lattice* pre,
                                const hbl_surrogate* m, const hbl_lattice* post, hbl_ref* ref,
                                hbl_stream stream) {
    clear_error();
    if (hbl_status st = check_bunch(z, n, ld, "surrogate_apply")) return st;
    HBL_REQUIRE(m, "surrogate_apply: NULL surrogate");
    if (!m->has_norm) { set_error(HBL_ESTATE, "surrogate_apply: no normalisation set or trained"); return HBL_ESTATE; }
    HBL_REQUIRE(!(pre || post) || m->has_stage, "surrogate_apply: gap lattices need a declared stage");
    if (m->has_stage) {
        if (hbl_status st = check_ref(ref)) return st;
        HBL_REQUIRE(fabs(ref->gamma / m->gamma_in - 1.0) < 1e-12,
                    "surrogate_apply: reference gamma %.17g differs from the trained entry gamma %.17g",
                    ref->gamma, m->gamma_in);
        if (hbl_status st = check_gap(pre, ref->gamma, "surrogate_apply: entrance")) return st;
        if (hbl_status st = check_gap(post, ref->gamma + m->dE_MeV / ref->mass_MeV, "surrogate_apply: exit"))
            return st;
    }
    if (n > 0)
        if (hbl_status st = check_device(z, bunch_bytes(n, ld), "surrogate_apply")) return st;
    if (n > 0) HBL_HIP(launch_mlp_infer(z, n, ld, m->d_img, m->norm, view_of(pre), view_of(post), (hipStream_t)stream));
    if (m->has_stage) {
        ref->gamma += m->dE_MeV / ref->mass_MeV;
        ref->s += (pre ? pre->length : 0.0) + m->L + (post ? post->length : 0.0);
    }
    return HBL_OK;
}

}  // namespace

extern "C" {

hbl_status hbl_surrogate_apply(double* z, int64_t n, int64_t ld, const hbl_surrogate* m, hbl_ref* ref,
                               hbl_stream stream) {
    return surrogate_apply_impl(z, n, ld, nullptr, m, nullptr, ref, stream);
}

hbl_status hbl_surrogate_apply_gaps(double* z, int64_t n, int64_t ld, const hbl_lattice* pre,
                                    const hbl_surrogate* m, const hbl_lattice* post, hbl_ref* ref,
                                    hbl_stream stream) {
    return surrogate_apply_impl(z, n, ld, pre, m, post, ref, stream);
}

hbl_status hbl_surrogate_loss_grad(hbl_surrogate* m, const double* zin, const double* zout, int64_t ld,
                                   const int32_t* idx, int32_t batch, float* grad, double* loss,
                                   hbl_stream stream) {
    clear_error();
    HBL_REQUIRE(m && idx && grad && loss, "surrogate_loss_grad: NULL argument");
    HBL_REQUIRE(batch >= 64 && batch % 64 == 0 && batch <= (1 << 20), "surrogate_loss_grad: batch %d must be a positive multiple of 64", batch);
    if (hbl_status st = check_bunch(zin, 1, ld, "surrogate_loss_grad(in)")) return st;
    if (hbl_status st = check_bunch(zout, 1, ld, "surrogate_loss_grad(out)")) return st;
    HBL_REQUIRE(zin && zout, "surrogate_loss_grad: NULL pairs");
    int32_t imax = 0;
    for (int32_t q = 0; q < batch; ++q) {
        HBL_REQUIRE(idx[q] >= 0 && idx[q] < ld, "surrogate_loss_grad: index %d out of range", idx[q]);
        imax = idx[q] > imax ? idx[q] : imax;
    }
    if (!m->has_norm) { set_error(HBL_ESTATE, "surrogate_loss_grad: no normalisation set"); return HBL_ESTATE; }
    if (hbl_status st = check_device(zin, bunch_bytes(imax + 1, ld), "surrogate_loss_grad(in)")) return st;
    if (hbl_status st = check_device(zout, bunch_bytes(imax + 1, ld), "surrogate_loss_grad(out)")) return st;
    const int32_t nb = batch / 64;
    if (hbl_status st = ensure_train_scratch(m, nb, 2)) return st;
    hipStream_t s = (hipStream_t)stream;
    int32_t* d_idx = nullptr;
    float* d_grad = nullptr;
    HBL_HIP(hipMalloc((void**)&d_idx, sizeof(int32_t) * batch));
    if (hipMalloc((void**)&d_grad, sizeof(float) * kMlpParams) != hipSuccess) {
        (void)hipFree(d_idx);
        set_error(HBL_ENOMEM, "surrogate_loss_grad: allocation failed");
        return HBL_ENOMEM;
    }
    hbl_status st = HBL_OK;
    std::vector<float> lp(nb);
    hipError_t e = hipMemcpyAsync(d_idx, idx, sizeof(int32_t) * batch, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_train_step(zin, zout, ld, d_idx, batch, m->d_img, m->d_part, m->d_loss_part, m->norm, s);
    if (e == hipSuccess) e = launch_grad_sum(m->d_part, nb, d_grad, s);
    if (e == hipSuccess) e = hipMemcpyAsync(grad, d_grad, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(lp.data(), m->d_loss_part, sizeof(float) * nb, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_error(HBL_EHIP, "surrogate_loss_grad: %s", hipGetErrorString(e));
        st = HBL_EHIP;
    } else {
        double sum = 0.0;
        for (int32_t b = 0; b < nb; ++b) sum += lp[b];
        *loss = sum / ((double)batch * 6.0);
    }
    (void)hipFree(d_idx);
    (void)hipFree(d_grad);
    return st;
}

hbl_status hbl_surrogate_train(hbl_surrogate* m, const double* zin, const double* zout, int64_t n_pairs,
                               int64_t ld, const hbl_train_cfg* cfg, float* loss_log, hbl_stream stream) {
    clear_error();
    HBL_REQUIRE(m && cfg, "surrogate_train: NULL argument");
    if (hbl_status st = check_bunch(zin, n_pairs, ld, "surrogate_train(in)")) return st;
    if (hbl_status st = check_bunch(zout, n_pairs, ld, "surrogate_train(out)")) return st;
    HBL_REQUIRE(cfg->batch >= 64 && cfg->batch % 64 == 0 && cfg->batch <= (1 << 20),
                "surrogate_train: batch %d must be a positive multiple of 64", cfg->batch);
    HBL_REQUIRE(cfg->epochs >= 0 && cfg->epochs <= 1000000, "surrogate_train: bad epoch count");
    HBL_REQUIRE(isfinite(cfg->lr) && cfg->lr > 0, "surrogate_train: lr must be > 0");
    HBL_REQUIRE(isfinite(cfg->lr_final) && cfg->lr_final > 0, "surrogate_train: lr_final must be > 0");
    HBL_REQUIRE(cfg->beta1 >= 0 && cfg->beta1 < 1 && cfg->beta2 >= 0 && cfg->beta2 < 1, "surrogate_train: betas must be in [0,1)");
    HBL_REQUIRE(isfinite(cfg->eps) && cfg->eps > 0, "surrogate_train: eps must be > 0");
    HBL_REQUIRE(cfg->train_frac > 0.0 && cfg->train_frac <= 1.0, "surrogate_train: train_frac must be in (0, 1]");
    HBL_REQUIRE(n_pairs <= INT32_MAX, "surrogate_train: at most 2^31-1 pairs");
    HBL_REQUIRE(cfg->keep_best >= 0 && cfg->keep_best <= 2, "surrogate_train: keep_best must be 0, 1 or 2");
    HBL_REQUIRE(cfg->resume == 0 || cfg->resume == 1, "surrogate_train: resume must be 0 or 1");
    HBL_REQUIRE(!cfg->resume || m->has_norm, "surrogate_train: resume needs a trained or loaded model");
    const int64_t n_train = llround(cfg->train_frac * (double)n_pairs);
    const int64_t n_test = n_pairs - n_train;
    HBL_REQUIRE(n_train >= cfg->batch, "surrogate_train: %lld training pairs < batch %d", (long long)n_train, cfg->batch);
    const int32_t nb = cfg->batch / 64;
    const int64_t steps_per_epoch = n_train / cfg->batch;
    HBL_REQUIRE(!cfg->resume || m->step % steps_per_epoch == 0,
                "surrogate_train: resume needs the step count (%lld) to be a whole number of epochs of %lld steps",
                (long long)m->step, (long long)steps_per_epoch);
    const int64_t epoch0 = cfg->resume ? m->step / steps_per_epoch : 0;
    if (hbl_status st = check_device(zin, bunch_bytes(n_pairs, ld), "surrogate_train(in)")) return st;
    if (hbl_status st = check_device(zout, bunch_bytes(n_pairs, ld), "surrogate_train(out)")) return st;
    hipStream_t s = (hipStream_t)stream;
    if (!cfg->resume) {
        // normalisation from the training split (§3), FP64 compensated moments
        double mi[6], ci[21], mo[6], co[21];
        if (hbl_status st = hbl_moments(zin, n_train, ld, mi, ci, stream)) return st;
        if (hbl_status st = hbl_moments(zout, n_train, ld, mo, co, stream)) return st;
        double norm[24];
        for (int j = 0; j < 6; ++j) {
            const int d = j * 6 - j * (j - 1) / 2;
            norm[j] = mi[j];
            norm[6 + j] = sqrt(ci[d]);
            norm[12 + j] = mo[j];
            norm[18 + j] = sqrt(co[d]);
        }
        if (hbl_status st = check_norm(norm)) {
            set_error(HBL_EINVAL, "surrogate_train: a coordinate has zero spread in the training split");
            return st;
        }
        memcpy(m->norm, norm, sizeof norm);
        m->has_norm = true;
    }
    if (hbl_status st = ensure_train_scratch(m, nb, 2 * (cfg->epochs > 0 ? cfg->epochs : 1))) return st;
    const bool keep_best = cfg->keep_best && n_test > 0 && cfg->epochs > 0;
    const bool by_eps = keep_best && cfg->keep_best == 2;
    if (keep_best && !m->d_best) {
        if (hipMalloc((void**)&m->d_best, sizeof(float) * kMlpParams) != hipSuccess ||
            hipMalloc((void**)&m->d_best_info, 2 * sizeof(double)) != hipSuccess) {
            set_error(HBL_ENOMEM, "surrogate_train: best-parameter buffer allocation failed");
            return HBL_ENOMEM;
        }
    }
    if (keep_best) HBL_HIP(launch_best_init(m->d_best_info, s));
    // fresh Adam state (kept when resuming)
    if (!cfg->resume) {
        HBL_HIP(hipMemsetAsync(m->d_m, 0, sizeof(float) * kMlpParams, s));
        HBL_HIP(hipMemsetAsync(m->d_v, 0, sizeof(float) * kMlpParams, s));
        m->step = 0;
    }
    HBL_HIP(hipMemsetAsync(m->d_loss_acc, 0, sizeof(double) * 2 * (cfg->epochs > 0 ? cfg->epochs : 1), s));
    if (hbl_status st = repack(m, s)) return st;
    const int64_t step0 = m->step;
    // double-buffered epoch orders: host pinned -> device
    int32_t* h_perm[2] = {nullptr, nullptr};
    int32_t* d_perm[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    hbl_status st = HBL_OK;
    auto fail = [&](hbl_status code, const char* what, hipError_t e) {
        set_error(code, "surrogate_train: %s: %s", what, hipGetErrorString(e));
        st = code;
    };
    for (int k = 0; k < 2 && st == HBL_OK; ++k) {
        hipError_t e = hipHostMalloc((void**)&h_perm[k], sizeof(int32_t) * n_train, 0);
        if (e == hipSuccess) e = hipMalloc((void**)&d_perm[k], sizeof(int32_t) * n_train);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev[k], hipEventDisableTiming);
        if (e != hipSuccess) fail(HBL_ENOMEM, "order buffers", e);
    }
    // emittance criterion: predictions of the test split in a bunch of their
    // own; the true test outputs' moments once; after each epoch of the
    // window (the last quarter of the epochs, at least the last) the
    // predictions' moments, a parameter snapshot and its {score, test loss}
    double* d_pred = nullptr;
    double* d_mom = nullptr;   // [0, 27): true test outputs, [32, 59): predictions
    double* d_ws = nullptr;
    float* d_snap = nullptr;
    double* d_rec = nullptr;
    const int64_t ld_pred = n_test + (n_test & 1);
    const int64_t n_win = cfg->epochs / 4 > 0 ? cfg->epochs / 4 : 1;
    const int64_t eps_from = cfg->epochs - n_win;
    if (by_eps && st == HBL_OK) {
        hipError_t e = hipMalloc((void**)&d_pred, sizeof(double) * 6 * (size_t)ld_pred);
        if (e == hipSuccess) e = hipMalloc((void**)&d_mom, sizeof(double) * 64);
        if (e == hipSuccess) e = hipMalloc((void**)&d_ws, reduce_ws_bytes(n_test));
        if (e == hipSuccess) e = hipMalloc((void**)&d_snap, sizeof(float) * kMlpParams * (size_t)n_win);
        if (e == hipSuccess) e = hipMalloc((void**)&d_rec, sizeof(double) * 2 * (size_t)n_win);
        if (e != hipSuccess) {
            fail(HBL_ENOMEM, "test-prediction buffers", e);
        } else {
            e = launch_moments(zout + n_train, n_test, ld, d_ws, d_mom, s);
            if (e != hipSuccess) fail(HBL_EHIP, "test-split moments", e);
        }
    }
    std::vector<int64_t> steps_done(cfg->epochs > 0 ? cfg->epochs : 1, 0);
    int64_t planned = (int64_t)cfg->epochs * steps_per_epoch;
    if (cfg->max_steps >= 0 && cfg->max_steps < planned) planned = cfg->max_steps;
    auto lr_at = [&](int64_t t) {  // t = 1..planned (this call's steps), half-cosine anneal
        if (planned <= 1 || cfg->lr_final == cfg->lr) return (double)cfg->lr;
        const double ph = 3.14159265358979323846 * (double)(t - 1) / (double)(planned - 1);
        return (double)cfg->lr_final + 0.5 * ((double)cfg->lr - (double)cfg->lr_final) * (1.0 + cos(ph));
    };
    for (int64_t ep = 0; ep < cfg->epochs && st == HBL_OK; ++ep) {
        const int k = (int)(ep & 1);
        hipError_t e = hipEventSynchronize(ev[k]);   // the copy two epochs ago has finished
        if (e != hipSuccess) { fail(HBL_EHIP, "event wait", e); break; }
        epoch_order(h_perm[k], n_train, cfg->shuffle_seed, epoch0 + ep);
        e = hipMemcpyAsync(d_perm[k], h_perm[k], sizeof(int32_t) * n_train, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipEventRecord(ev[k], s);
        if (e != hipSuccess) { fail(HBL_EHIP, "order upload", e); break; }
        for (int64_t step = 0; step < steps_per_epoch; ++step) {
            if (cfg->max_steps >= 0 && m->step - step0 >= cfg->max_steps) break;
            m->step += 1;
            e = launch_train_step(zin, zout, ld, d_perm[k] + step * cfg->batch, cfg->batch, m->d_img,
                                  m->d_part, m->d_loss_part, m->norm, s);
            if (e == hipSuccess)
                e = launch_train_adam(m->d_params, m->d_m, m->d_v, m->d_part, nb, m->d_loss_part,
                                      m->d_loss_acc + 2 * ep, 1.0 / ((double)cfg->batch * 6.0), m->step,
                                      (float)lr_at(m->step - step0), cfg->beta1, cfg->beta2, cfg->eps, s);
            if (e == hipSuccess) e = launch_mlp_pack(m->d_params, m->d_img, s);
            if (e != hipSuccess) { fail(HBL_EHIP, "step launch", e); break; }
            steps_done[ep] += 1;
        }
        if (st != HBL_OK) break;
        if (n_test > 0) {
            e = launch_eval_loss(zin, zout, ld, n_train, n_test, m->d_img, m->norm, m->d_eval_part,
                                 m->d_loss_acc + 2 * ep + 1, s);
            if (e == hipSuccess && keep_best && !by_eps)
                e = launch_keep_best(m->d_loss_acc + 2 * ep + 1, m->d_best_info, m->d_params, m->d_best, ep, s);
            if (e == hipSuccess && by_eps && ep >= eps_from) {
                e = hipMemcpy2DAsync(d_pred, sizeof(double) * ld_pred, zin + n_train, sizeof(double) * ld,
                                     sizeof(double) * n_test, 6, hipMemcpyDeviceToDevice, s);
                if (e == hipSuccess)
                    e = launch_mlp_infer(d_pred, n_test, ld_pred, m->d_img, m->norm, view_of(nullptr),
                                         view_of(nullptr), s);
                if (e == hipSuccess) e = launch_moments(d_pred, n_test, ld_pred, d_ws, d_mom + 32, s);
                if (e == hipSuccess)
                    e = launch_snapshot(d_mom + 32, d_mom, m->d_loss_acc + 2 * ep + 1, m->d_params,
                                        d_snap + (ep - eps_from) * kMlpParams, d_rec + 2 * (ep - eps_from), s);
            }
            if (e != hipSuccess) { fail(HBL_EHIP, "test loss launch", e); break; }
        }
    }
    if (st == HBL_OK && keep_best) {
        hipError_t e2 = by_eps ? launch_select_snapshot(d_rec, (int)n_win, kEpsSelectLossTol, d_snap, m->d_params,
                                                        m->d_best_info, s)
                               : launch_restore_best(m->d_best_info, m->d_best, m->d_params, s);
        if (e2 == hipSuccess) e2 = launch_mlp_pack(m->d_params, m->d_img, s);
        if (e2 != hipSuccess) fail(HBL_EHIP, "best-parameter restore", e2);
    }
    hipError_t e = hipStreamSynchronize(s);
    if (st == HBL_OK && e != hipSuccess) fail(HBL_EHIP, "training", e);
    if (st == HBL_OK && loss_log && cfg->epochs > 0) {
        std::vector<double> acc(2 * cfg->epochs);
        e = hipMemcpy(acc.data(), m->d_loss_acc, sizeof(double) * acc.size(), hipMemcpyDeviceToHost);
        if (e != hipSuccess) fail(HBL_EHIP, "loss readback", e);
        for (int64_t ep = 0; ep < cfg->epochs && st == HBL_OK; ++ep) {
            loss_log[2 * ep] = steps_done[ep] ? (float)(acc[2 * ep] / (double)steps_done[ep]) : 0.0f;
            loss_log[2 * ep + 1] = (float)acc[2 * ep + 1];
        }
    }
    for (int k = 0; k < 2; ++k) {
        if (ev[k]) (void)hipEventDestroy(ev[k]);
        if (d_perm[k]) (void)hipFree(d_perm[k]);
        if (h_perm[k]) (void)hipHostFree(h_perm[k]);
    }
    void* scratch_bufs[] = {d_pred, d_mom, d_ws, d_snap, d_rec};
    for (void* q : scratch_bufs)
        if (q) (void)hipFree(q);
    return st;
}

hbl_status hbl_surrogate_save(const hbl_surrogate* m, const char* path) {
    clear_error();
    HBL_REQUIRE(m && path, "surrogate_save: NULL argument");
    std::vector<float> blob(3 * (size_t)kMlpParams);
    HBL_HIP(hipDeviceSynchronize());
    HBL_HIP(hipMemcpy(blob.data(), m->d_params, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
    HBL_HIP(hipMemcpy(blob.data() + kMlpParams, m->d_m, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
    HBL_HIP(hipMemcpy(blob.data() + 2 * kMlpParams, m->d_v, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
    struct {
        uint64_t magic;
        int32_t shape[4];
        int32_t has_norm, has_stage;
        int64_t step;
        double norm[24];
        double dE_MeV, L, gamma_in;
    } hdr;
    memset(&hdr, 0, sizeof hdr);
    hdr.magic = kFileMagic;
    hdr.shape[0] = m->shape.n_in; hdr.shape[1] = m->shape.width; hdr.shape[2] = m->shape.hidden; hdr.shape[3] = m->shape.n_out;
    hdr.has_norm = m->has_norm;
    hdr.has_stage = m->has_stage;
    hdr.step = m->step;
    memcpy(hdr.norm, m->norm, sizeof hdr.norm);
    hdr.dE_MeV = m->dE_MeV; hdr.L = m->L; hdr.gamma_in = m->gamma_in;
    // FNV-1a 64 over header and payload
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void* p, size_t nbytes) {
        const unsigned char* c = (const unsigned char*)p;
        for (size_t q = 0; q < nbytes; ++q) { h ^= c[q]; h *= 1099511628211ull; }
    };
    mix(&hdr, sizeof hdr);
    mix(blob.data(), blob.size() * sizeof(float));
    FILE* f = fopen(path, "wb");
    if (!f) { set_error(HBL_EIO, "surrogate_save: cannot open %s", path); return HBL_EIO; }
    bool ok = fwrite(&hdr, sizeof hdr, 1, f) == 1 && fwrite(blob.data(), sizeof(float), blob.size(), f) == blob.size() &&
              fwrite(&h, sizeof h, 1, f) == 1;
    ok = (fclose(f) == 0) && ok;
    if (!ok) { set_error(HBL_EIO, "surrogate_save: write failed for %s", path); return HBL_EIO; }
    return HBL_OK;
}

hbl_status hbl_surrogate_load(const char* path, hbl_surrogate** out) {
    clear_error();
    HBL_REQUIRE(path && out, "surrogate_load: NULL argument");
    *out = nullptr;
    struct {
        uint64_t magic;
        int32_t shape[4];
        int32_t has_norm, has_stage;
        int64_t step;
        double norm[24];
        double dE_MeV, L, gamma_in;
    } hdr;
    std::vector<float> blob(3 * (size_t)kMlpParams);
    uint64_t stored = 0;
    FILE* f = fopen(path, "rb");
    if (!f) { set_error(HBL_EIO, "surrogate_load: cannot open %s", path); return HBL_EIO; }
    bool ok = fread(&hdr, sizeof hdr, 1, f) == 1 && fread(blob.data(), sizeof(float), blob.size(), f) == blob.size() &&
              fread(&stored, sizeof stored, 1, f) == 1;
    fclose(f);
    if (!ok) { set_error(HBL_EIO, "surrogate_load: %s is truncated", path); return HBL_EIO; }
    if (hdr.magic != kFileMagic) { set_error(HBL_EIO, "surrogate_load: %s is not a surrogate file", path); return HBL_EIO; }
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void* p, size_t nbytes) {
        const unsigned char* c = (const unsigned char*)p;
        for (size_t q = 0; q < nbytes; ++q) { h ^= c[q]; h *= 1099511628211ull; }
    };
    mix(&hdr, sizeof hdr);
    mix(blob.data(), blob.size() * sizeof(float));
    if (h != stored) { set_error(HBL_EIO, "surrogate_load: checksum mismatch in %s", path); return HBL_EIO; }
    hbl_mlp_shape sh = {hdr.shape[0], hdr.shape[1], hdr.shape[2], hdr.shape[3]};
    if (hbl_status st = check_shape(&sh)) return st;
    hbl_surrogate* m = nullptr;
    if (hbl_status st = sur_alloc(&m, &sh)) return st;
    hipError_t e = hipMemcpy(m->d_params, blob.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->d_m, blob.data() + kMlpParams, sizeof(float) * kMlpParams, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(m->d_v, blob.data() + 2 * kMlpParams, sizeof(float) * kMlpParams, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_mlp_pack(m->d_params, m->d_img, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) { sur_free(m); set_error(HBL_EHIP, "surrogate_load: upload failed: %s", hipGetErrorString(e)); return HBL_EHIP; }
    m->has_norm = hdr.has_norm != 0;
    memcpy(m->norm, hdr.norm, sizeof m->norm);
    m->has_stage = hdr.has_stage != 0;
    m->dE_MeV = hdr.dE_MeV; m->L = hdr.L; m->gamma_in = hdr.gamma_in;
    m->step = hdr.step;
    *out = m;
    return HBL_OK;
}

}  // extern "C"

// ====================================================== wide PReLU surrogate
struct hbl_prelu_net {
    int device;
    hbl_mlp_shape shape;
    int64_t nparams;
    int64_t chunk;            // particles per inference chunk (multiple of the tile)
    float* d_params;          // FP32 master parameters
    char* d_image;            // one allocation: the DenseImage arrays
    uint16_t* d_buf[2];       // activation ping-pong buffers, chunk x wp bf16 each
    DenseImage im;
    double norm[24];
    bool has_norm;
    bool has_stage;
    double dE_MeV, L, gamma_in;
    // training state, allocated on first use
    float* d_m;               // Adam moments
    float* d_v;
    float* d_grad;
    uint16_t* d_wt;           // transposed bf16 weights of layers 1..H-1, [wp][wp] each
    char* d_train;            // DenseTrainBufs arrays (one allocation)
    int32_t* d_idx;           // batch indices for loss_grad
    double* d_loss;           // loss accumulators
    int32_t train_bp, train_B;
    int64_t loss_slots;
    DenseTrainBufs tb;
    int64_t step;
};

namespace {

constexpr int64_t kPreluChunk = 65536;
// Default chunk: at 512 <= W' <= 832 the hidden layers run as persistent workgroups, and
// 98,304 particles (6 items per CU instead of 4) measured 4 % faster for 3 x 700 (27.7 vs
// 28.9 ms per 1e7); elsewhere 65,536 was the fastest measured (5 x 900: 75.5 ms against
// 76.7-79.2 at 49,152-262,144).
int64_t prelu_default_chunk(int64_t wp) { return wp >= 512 && wp <= 832 ? 98304 : kPreluChunk; }

int64_t prelu_nparams_of(const hbl_mlp_shape* sh) {
    const int64_t W = sh->width, H = sh->hidden;
    return 6 * W + W + 1 + (H - 1) * (W * W + W + 1) + 6 * W + 6;
}

hbl_status check_prelu_shape(const hbl_mlp_shape* sh) {
    HBL_REQUIRE(sh, "prelu: NULL shape");
    HBL_REQUIRE(sh->n_in == 6 && sh->n_out == 6, "prelu: n_in and n_out must be 6");
    HBL_REQUIRE(sh->width >= 8 && sh->width <= kDenseMaxWidth, "prelu: width %d outside [8, %d]", sh->width,
                kDenseMaxWidth);
    HBL_REQUIRE(sh->hidden >= 1 && sh->hidden <= kDenseMaxHidden, "prelu: hidden %d outside [1, %d]", sh->hidden,
                kDenseMaxHidden);
    return HBL_OK;
}

void prelu_free(hbl_prelu_net* m) {
    if (!m) return;
    void* ptrs[] = {m->d_params, m->d_image, m->d_buf[0], m->d_buf[1], m->d_m,   m->d_v,
                    m->d_grad,   m->d_wt,    m->d_train,  m->d_idx,    m->d_loss};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete m;
}

// Lay the DenseImage arrays out in one allocation (256-byte aligned pieces).
size_t prelu_image_layout(const hbl_mlp_shape* sh, DenseImage* im, char* base) {
    const int64_t wp = (sh->width + 63) / 64 * 64;
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off += (bytes + 255) / 256 * 256;
        return p;
    };
    im->wp = (int32_t)wp;
    im->w0 = (float*)take(sizeof(float) * wp * 6);
    im->b0 = (float*)take(sizeof(float) * wp);
    im->slope = (float*)take(sizeof(float) * kDenseMaxHidden);
    for (int l = 0; l <= kDenseMaxHidden; ++l) { im->w[l] = nullptr; im->b[l] = nullptr; im->wb[l] = nullptr; }
    for (int l = 1; l <= sh->hidden; ++l) {
        const int64_t rows = l == sh->hidden ? 16 : wp;
        im->w[l] = (uint16_t*)take(sizeof(uint16_t) * rows * wp);
        im->b[l] = (float*)take(sizeof(float) * rows);
        if (l < sh->hidden && dense_blocked((int)wp)) im->wb[l] = (uint16_t*)take(sizeof(uint16_t) * wp * wp);
    }
    return off;
}

hbl_status prelu_repack(hbl_prelu_net* m, hipStream_t s) {
    const DenseShape sh{m->shape.width, m->shape.hidden};
    HBL_HIP(launch_dense_pack(m->d_params, sh, m->im, s));
    return HBL_OK;
}

}  // namespace

extern "C" {

hbl_status hbl_prelu_create(const hbl_mlp_shape* shape, uint64_t init_seed, hbl_prelu_net** out) {
    clear_error();
    HBL_REQUIRE(out, "prelu_create: NULL output handle");
    *out = nullptr;
    if (hbl_status st = check_prelu_shape(shape)) return st;
    const int64_t np = prelu_nparams_of(shape);
    std::vector<float> p(np);
    const int W = shape->width, H = shape->hidden;
    int64_t off = 0;
    for (int l = 0; l <= H; ++l) {
        const int ni = l == 0 ? 6 : W, no = l == H ? 6 : W;
        const double bound = 1.0 / sqrt((double)ni);
        const int64_t cnt = (int64_t)no * (ni + 1);
        for (int64_t q = 0; q < cnt; ++q, ++off) {
            uint32_t c[4] = {(uint32_t)off, (uint32_t)((uint64_t)off >> 32), 0u, 0x4D4C5049u};
            philox_host(c, (uint32_t)init_seed, (uint32_t)(init_seed >> 32));
            const double u = (double)(c[0] >> 8) * (1.0 / 16777216.0);
            p[off] = (float)((2.0 * u - 1.0) * bound);
        }
        if (l < H) p[off++] = 0.25f;
    }
    hbl_prelu_net* m = new (std::nothrow) hbl_prelu_net();
    if (!m) { set_error(HBL_ENOMEM, "prelu_create: out of host memory"); return HBL_ENOMEM; }
    m->shape = *shape;
    m->nparams = np;
    if (hipGetDevice(&m->device) != hipSuccess) { delete m; set_error(HBL_EHIP, "prelu_create: no HIP device"); return HBL_EHIP; }
    const size_t img_bytes = prelu_image_layout(shape, &m->im, nullptr);
    m->chunk = prelu_default_chunk((shape->width + 63) / 64 * 64);
    const size_t buf_bytes = sizeof(uint16_t) * (size_t)m->chunk * m->im.wp;
    hipError_t e = hipMalloc((void**)&m->d_params, sizeof(float) * np);
    if (e == hipSuccess) e = hipMalloc((void**)&m->d_image, img_bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&m->d_buf[0], buf_bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&m->d_buf[1], buf_bytes);
    if (e != hipSuccess) { prelu_free(m); set_error(HBL_ENOMEM, "prelu_create: device allocation failed"); return HBL_ENOMEM; }
    prelu_image_layout(shape, &m->im, m->d_image);
    e = hipMemset(m->d_image, 0, img_bytes);
    if (e == hipSuccess) e = hipMemcpy(m->d_params, p.data(), sizeof(float) * np, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_dense_pack(m->d_params, DenseShape{W, H}, m->im, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) { prelu_free(m); set_error(HBL_EHIP, "prelu_create: %s", hipGetErrorString(e)); return HBL_EHIP; }
    *out = m;
    return HBL_OK;
}

hbl_status hbl_prelu_destroy(hbl_prelu_net* m) {
    clear_error();
    if (m) (void)hipDeviceSynchronize();
    prelu_free(m);
    return HBL_OK;
}

hbl_status hbl_prelu_num_params(const hbl_prelu_net* m, int64_t* n) {
    clear_error();
    HBL_REQUIRE(m && n, "prelu_num_params: NULL argument");
    *n = m->nparams;
    return HBL_OK;
}

hbl_status hbl_prelu_get_params(const hbl_prelu_net* m, float* host, int64_t n) {
    clear_error();
    HBL_REQUIRE(m && host, "prelu_get_params: NULL argument");
    HBL_REQUIRE(n == m->nparams, "prelu_get_params: n = %lld, the network has %lld", (long long)n, (long long)m->nparams);
    HBL_HIP(hipDeviceSynchronize());
    HBL_HIP(hipMemcpy(host, m->d_params, sizeof(float) * n, hipMemcpyDeviceToHost));
    return HBL_OK;
}

hbl_status hbl_prelu_set_params(hbl_prelu_net* m, const float* host, int64_t n) {
    clear_error();
    HBL_REQUIRE(m && host, "prelu_set_params: NULL argument");
    HBL_REQUIRE(n == m->nparams, "prelu_set_params: n = %lld, the network has %lld", (long long)n, (long long)m->nparams);
    for (int64_t q = 0; q < n; ++q) HBL_REQUIRE(isfinite(host[q]), "prelu_set_params: parameter %lld not finite", (long long)q);
    HBL_HIP(hipDeviceSynchronize());
    HBL_HIP(hipMemcpy(m->d_params, host, sizeof(float) * n, hipMemcpyHostToDevice));
    if (hbl_status st = prelu_repack(m, nullptr)) return st;
    HBL_HIP(hipDeviceSynchronize());
    return HBL_OK;
}

hbl_status hbl_prelu_set_chunk(hbl_prelu_net* m, int64_t particles) {
    clear_error();
    HBL_REQUIRE(m, "prelu_set_chunk: NULL network");
    const int64_t tile = dense_tile_rows();
    HBL_REQUIRE(particles >= tile && particles <= (int64_t)1 << 22 && particles % tile == 0,
                "prelu_set_chunk: %lld particles must be a multiple of %lld in [%lld, 2^22]", (long long)particles,
                (long long)tile, (long long)tile);
    if (particles == m->chunk) return HBL_OK;
    HBL_HIP(hipDeviceSynchronize());
    const size_t bytes = sizeof(uint16_t) * (size_t)particles * m->im.wp;
    uint16_t* b[2] = {nullptr, nullptr};
    hipError_t e = hipMalloc((void**)&b[0], bytes);
    if (e == hipSuccess) e = hipMalloc((void**)&b[1], bytes);
    if (e != hipSuccess) {
        if (b[0]) (void)hipFree(b[0]);
        set_error(HBL_ENOMEM, "prelu_set_chunk: device allocation failed");
        return HBL_ENOMEM;
    }
    (void)hipFree(m->d_buf[0]);
    (void)hipFree(m->d_buf[1]);
    m->d_buf[0] = b[0];
    m->d_buf[1] = b[1];
    m->chunk = particles;
    return HBL_OK;
}

hbl_status hbl_prelu_set_norm(hbl_prelu_net* m, const double norm24[24]) {
    clear_error();
    HBL_REQUIRE(m && norm24, "prelu_set_norm: NULL argument");
    if (hbl_status st = check_norm(norm24)) return st;
    memcpy(m->norm, norm24, sizeof m->norm);
    m->has_norm = true;
    return HBL_OK;
}

hbl_status hbl_prelu_get_norm(const hbl_prelu_net* m, double norm24[24]) {
    clear_error();
    HBL_REQUIRE(m && norm24, "prelu_get_norm: NULL argument");
    if (!m->has_norm) { set_error(HBL_ESTATE, "prelu_get_norm: no normalisation set"); return HBL_ESTATE; }
    memcpy(norm24, m->norm, sizeof m->norm);
    return HBL_OK;
}

hbl_status hbl_prelu_set_stage(hbl_prelu_net* m, const hbl_element* stage, const hbl_ref* at_entry) {
    clear_error();
    HBL_REQUIRE(m && stage, "prelu_set_stage: NULL argument");
    HBL_REQUIRE(stage->kind == HBL_STAGE, "prelu_set_stage: element is not a stage");
    HBL_REQUIRE(finite_pos(stage->L) && isfinite(stage->dE_MeV), "prelu_set_stage: bad L or dE");
    if (hbl_status st = check_ref(at_entry)) return st;
    HBL_REQUIRE(at_entry->gamma + stage->dE_MeV / at_entry->mass_MeV > 1.0, "prelu_set_stage: exit gamma must exceed 1");
    m->has_stage = true;
    m->dE_MeV = stage->dE_MeV;
    m->L = stage->L;
    m->gamma_in = at_entry->gamma;
    return HBL_OK;
}

}  // extern "C"

namespace {

hbl_status prelu_apply_impl(double* z, int64_t n, int64_t ld, const hbl_lattice* pre, const hbl_prelu_net* m,
                            const hbl_lattice* post, hbl_ref* ref, hbl_stream stream) {
    clear_error();
    if (hbl_status st = check_bunch(z, n, ld, "prelu_apply")) return st;
    HBL_REQUIRE(m, "prelu_apply: NULL network");
    if (!m->has_norm) { set_error(HBL_ESTATE, "prelu_apply: no normalisation set"); return HBL_ESTATE; }
    HBL_REQUIRE(!(pre || post) || m->has_stage, "prelu_apply: gap lattices need a declared stage");
    if (m->has_stage) {
        if (hbl_status st = check_ref(ref)) return st;
        HBL_REQUIRE(fabs(ref->gamma / m->gamma_in - 1.0) < 1e-12,
                    "prelu_apply: reference gamma %.17g differs from the declared entry gamma %.17g", ref->gamma,
                    m->gamma_in);
        if (hbl_status st = check_gap(pre, ref->gamma, "prelu_apply: entrance")) return st;
        if (hbl_status st = check_gap(post, ref->gamma + m->dE_MeV / ref->mass_MeV, "prelu_apply: exit")) return st;
    }
    if (n > 0) {
        if (hbl_status st = check_device(z, bunch_bytes(n, ld), "prelu_apply")) return st;
        DenseNorm nm;
        for (int j = 0; j < 6; ++j) {
            nm.mu_in[j] = m->norm[j];
            nm.sd_in[j] = m->norm[6 + j];
            nm.mu_out[j] = m->norm[12 + j];
            nm.sd_out[j] = m->norm[18 + j];
        }
        HBL_HIP(launch_dense_infer(z, n, ld, DenseShape{m->shape.width, m->shape.hidden}, m->im, nm, view_of(pre),
                                   view_of(post), m->d_buf[0], m->d_buf[1], m->chunk, (hipStream_t)stream));
    }
    if (m->has_stage) {
        ref->gamma += m->dE_MeV / ref->mass_MeV;
        ref->s += (pre ? pre->length : 0.0) + m->L + (post ? post->length : 0.0);
    }
    return HBL_OK;
}

}  // namespace

extern "C" {

hbl_status hbl_prelu_apply(double* z, int64_t n, int64_t ld, const hbl_prelu_net* m, hbl_ref* ref,
                           hbl_stream stream) {
    return prelu_apply_impl(z, n, ld, nullptr, m, nullptr, ref, stream);
}

hbl_status hbl_prelu_apply_gaps(double* z, int64_t n, int64_t ld, const hbl_lattice* pre, const hbl_prelu_net* m,
                                const hbl_lattice* post, hbl_ref* ref, hbl_stream stream) {
    return prelu_apply_impl(z, n, ld, pre, m, post, ref, stream);
}

}  // extern "C"

// ------------------------------------------------------- wide PReLU training
namespace {

uint16_t* const* prelu_wt(const hbl_prelu_net* m, uint16_t** wt) {
    const int64_t wp = m->im.wp;
    for (int l = 0; l <= kDenseMaxHidden; ++l) wt[l] = nullptr;
    for (int l = 1; l < m->shape.hidden; ++l) wt[l] = m->d_wt + (int64_t)(l - 1) * wp * wp;
    return wt;
}

// Adam moments, gradient and the transposed weight images (zeroed once).
hbl_status prelu_opt_state(hbl_prelu_net* m) {
    if (m->d_m) return HBL_OK;
    const int64_t wp = m->im.wp, H = m->shape.hidden;
    const size_t pb = sizeof(float) * (size_t)m->nparams, wtb = sizeof(uint16_t) * (size_t)(H - 1) * wp * wp;
    float *dm = nullptr, *dv = nullptr, *dg = nullptr;
    uint16_t* wt = nullptr;
    hipError_t e = hipMalloc((void**)&dm, pb);
    if (e == hipSuccess) e = hipMalloc((void**)&dv, pb);
    if (e == hipSuccess) e = hipMalloc((void**)&dg, pb);
    if (e == hipSuccess && H > 1) e = hipMalloc((void**)&wt, wtb);
    if (e == hipSuccess) e = hipMemset(dm, 0, pb);
    if (e == hipSuccess) e = hipMemset(dv, 0, pb);
    if (e == hipSuccess && wt) e = hipMemset(wt, 0, wtb);
    if (e != hipSuccess) {                 // all or nothing: the handle stays as it was
        void* ptrs[] = {dm, dv, dg, wt};
        for (void* q : ptrs)
            if (q) (void)hipFree(q);
        set_error(HBL_ENOMEM, "prelu: optimiser state allocation failed: %s", hipGetErrorString(e));
        return HBL_ENOMEM;
    }
    m->d_m = dm;
    m->d_v = dv;
    m->d_grad = dg;
    m->d_wt = wt;
    return HBL_OK;
}

// Training buffers for batches of B samples (grow-only in the padded size).
hbl_status prelu_train_buffers(hbl_prelu_net* m, int32_t B, int64_t loss_slots, hipStream_t s) {
    const int tile = dense_tile_rows();
    const int32_t bp = (B + tile - 1) / tile * tile;
    const int64_t wp = m->im.wp, H = m->shape.hidden;
    const int32_t np = (int32_t)((wp + 1 + tile - 1) / tile * tile);
    if (hbl_status st = prelu_opt_state(m)) return st;
    if (loss_slots > m->loss_slots) {
        if (m->d_loss) { HBL_HIP(hipStreamSynchronize(s)); (void)hipFree(m->d_loss); m->d_loss = nullptr; }
        HBL_HIP(hipMalloc((void**)&m->d_loss, sizeof(double) * loss_slots));
        m->loss_slots = loss_slots;
    }
    if (bp > m->train_bp) {
        // the old buffers go first; until the new ones are in place the
        // handle has none (train_bp = 0), so a failure here cannot leave
        // stale pointers behind
        if (m->d_train) { HBL_HIP(hipStreamSynchronize(s)); (void)hipFree(m->d_train); m->d_train = nullptr; }
        if (m->d_idx) { (void)hipFree(m->d_idx); m->d_idx = nullptr; }
        m->train_bp = 0;
        m->train_B = -1;
        size_t off = 0;
        auto take = [&](size_t bytes) { const size_t o = off; off += (bytes + 255) / 256 * 256; return o; };
        DenseTrainBufs t{};
        size_t o_x0t = take(2ull * 256 * bp), o_h[kDenseMaxHidden], o_v[kDenseMaxHidden], o_ht[kDenseMaxHidden];
        for (int l = 0; l < H; ++l) {
            o_h[l] = take(2ull * bp * wp);
            o_v[l] = take(2ull * bp * wp);
            o_ht[l] = take(2ull * np * bp);
        }
        size_t o_dv0 = take(2ull * bp * wp), o_dv1 = take(2ull * bp * wp), o_dvt = take(2ull * wp * bp);
        size_t o_dyt = take(2ull * 16 * bp), o_dy = take(4ull * 8 * bp), o_lossp = take(4ull * bp);
        size_t o_part = take(4ull * kDensePartMax * kDenseMaxHidden);
        HBL_HIP(hipMalloc((void**)&m->d_train, off));
        HBL_HIP(hipMemset(m->d_train, 0, off));
        HBL_HIP(hipMalloc((void**)&m->d_idx, sizeof(int32_t) * bp));
        char* b = m->d_train;
        t.x0t = (uint16_t*)(b + o_x0t);
        for (int l = 0; l < H; ++l) {
            t.h[l] = (uint16_t*)(b + o_h[l]);
            t.v[l] = (uint16_t*)(b + o_v[l]);
            t.ht[l] = (uint16_t*)(b + o_ht[l]);
        }
        t.dv[0] = (uint16_t*)(b + o_dv0);
        t.dv[1] = (uint16_t*)(b + o_dv1);
        t.dvt = (uint16_t*)(b + o_dvt);
        t.dyt = (uint16_t*)(b + o_dyt);
        t.dy = (float*)(b + o_dy);
        t.lossp = (float*)(b + o_lossp);
        t.part = (float*)(b + o_part);
        t.np = np;
        m->tb = t;
        m->train_bp = bp;
        m->train_B = -1;
    }
    m->tb.bp = bp;
    if (B != m->train_B) {
        m->tb.B = B;
        HBL_HIP(launch_dense_fill_ones(m->tb, (int32_t)wp, (int32_t)H, s));
        m->train_B = B;
    }
    return HBL_OK;
}

DenseNorm prelu_norm(const hbl_prelu_net* m) {
    DenseNorm nm;
    for (int j = 0; j < 6; ++j) {
        nm.mu_in[j] = m->norm[j];
        nm.sd_in[j] = m->norm[6 + j];
        nm.mu_out[j] = m->norm[12 + j];
        nm.sd_out[j] = m->norm[18 + j];
    }
    return nm;
}

hbl_status prelu_repack_all(hbl_prelu_net* m, hipStream_t s) {
    const DenseShape sh{m->shape.width, m->shape.hidden};
    uint16_t* wt[kDenseMaxHidden + 1];
    HBL_HIP(launch_dense_pack(m->d_params, sh, m->im, s));
    if (m->d_wt) HBL_HIP(launch_dense_pack_t(m->d_params, sh, m->im.wp, prelu_wt(m, wt), s));
    return HBL_OK;
}

}  // namespace

extern "C" {

hbl_status hbl_prelu_loss_grad(hbl_prelu_net* m, const double* zin, const double* zout, int64_t ld,
                               const int32_t* idx, int32_t batch, float* grad, double* loss, hbl_stream stream) {
    clear_error();
    HBL_REQUIRE(m && idx && grad && loss, "prelu_loss_grad: NULL argument");
    HBL_REQUIRE(batch >= 1 && batch <= 16384, "prelu_loss_grad: batch %d outside [1, 16384]", batch);
    if (hbl_status st = check_bunch(zin, 1, ld, "prelu_loss_grad(in)")) return st;
    if (hbl_status st = check_bunch(zout, 1, ld, "prelu_loss_grad(out)")) return st;
    HBL_REQUIRE(zin && zout, "prelu_loss_grad: NULL pairs");
    int32_t imax = 0;
    for (int32_t q = 0; q < batch; ++q) {
        HBL_REQUIRE(idx[q] >= 0 && idx[q] < ld, "prelu_loss_grad: index %d out of range", idx[q]);
        imax = idx[q] > imax ? idx[q] : imax;
    }
    if (!m->has_norm) { set_error(HBL_ESTATE, "prelu_loss_grad: no normalisation set"); return HBL_ESTATE; }
    if (hbl_status st = check_device(zin, bunch_bytes(imax + 1, ld), "prelu_loss_grad(in)")) return st;
    if (hbl_status st = check_device(zout, bunch_bytes(imax + 1, ld), "prelu_loss_grad(out)")) return st;
    hipStream_t s = (hipStream_t)stream;
    if (hbl_status st = prelu_train_buffers(m, batch, 1, s)) return st;
    if (hbl_status st = prelu_repack_all(m, s)) return st;
    DenseTrainBufs tb = m->tb;
    tb.idx = m->d_idx;
    uint16_t* wt[kDenseMaxHidden + 1];
    HBL_HIP(hipMemcpyAsync(m->d_idx, idx, sizeof(int32_t) * batch, hipMemcpyHostToDevice, s));
    HBL_HIP(hipMemsetAsync(m->d_loss, 0, sizeof(double), s));
    HBL_HIP(launch_dense_train_step(zin, zout, ld, DenseShape{m->shape.width, m->shape.hidden}, m->im, prelu_wt(m, wt),
                                    prelu_norm(m), tb, m->d_params, m->d_grad, m->d_loss, 1.0 / (6.0 * batch), s));
    HBL_HIP(hipMemcpyAsync(grad, m->d_grad, sizeof(float) * m->nparams, hipMemcpyDeviceToHost, s));
    HBL_HIP(hipMemcpyAsync(loss, m->d_loss, sizeof(double), hipMemcpyDeviceToHost, s));
    HBL_HIP(hipStreamSynchronize(s));
    return HBL_OK;
}

hbl_status hbl_prelu_train(hbl_prelu_net* m, const double* zin, const double* zout, int64_t n_pairs, int64_t ld,
                           const hbl_train_cfg* cfg, float* loss_log, hbl_stream stream) {
    clear_error();
    HBL_REQUIRE(m && cfg, "prelu_train: NULL argument");
    if (hbl_status st = check_bunch(zin, n_pairs, ld, "prelu_train(in)")) return st;
    if (hbl_status st = check_bunch(zout, n_pairs, ld, "prelu_train(out)")) return st;
    HBL_REQUIRE(cfg->batch >= 1 && cfg->batch <= 16384, "prelu_train: batch %d outside [1, 16384]", cfg->batch);
    HBL_REQUIRE(cfg->epochs >= 0 && cfg->epochs <= 1000000, "prelu_train: bad epoch count");
    HBL_REQUIRE(isfinite(cfg->lr) && cfg->lr > 0, "prelu_train: lr must be > 0");
    HBL_REQUIRE(isfinite(cfg->lr_final) && cfg->lr_final > 0, "prelu_train: lr_final must be > 0");
    HBL_REQUIRE(cfg->beta1 >= 0 && cfg->beta1 < 1 && cfg->beta2 >= 0 && cfg->beta2 < 1, "prelu_train: betas must be in [0,1)");
    HBL_REQUIRE(isfinite(cfg->eps) && cfg->eps > 0, "prelu_train: eps must be > 0");
    HBL_REQUIRE(cfg->train_frac > 0.0 && cfg->train_frac <= 1.0, "prelu_train: train_frac must be in (0, 1]");
    HBL_REQUIRE(n_pairs <= INT32_MAX, "prelu_train: at most 2^31-1 pairs");
    HBL_REQUIRE(cfg->keep_best == 0 && cfg->resume == 0,
                "prelu_train: keep_best and resume are not supported by the paper-shaped network (must be 0)");
    const int64_t n_train = llround(cfg->train_frac * (double)n_pairs);
    const int64_t n_test = n_pairs - n_train;
    HBL_REQUIRE(n_train >= cfg->batch, "prelu_train: %lld training pairs < batch %d", (long long)n_train, cfg->batch);
    if (hbl_status st = check_device(zin, bunch_bytes(n_pairs, ld), "prelu_train(in)")) return st;
    if (hbl_status st = check_device(zout, bunch_bytes(n_pairs, ld), "prelu_train(out)")) return st;
    hipStream_t s = (hipStream_t)stream;
    double mi[6], ci[21], mo[6], co[21];
    if (hbl_status st = hbl_moments(zin, n_train, ld, mi, ci, stream)) return st;
    if (hbl_status st = hbl_moments(zout, n_train, ld, mo, co, stream)) return st;
    double norm[24];
    for (int j = 0; j < 6; ++j) {
        const int d = j * 6 - j * (j - 1) / 2;
        norm[j] = mi[j];
        norm[6 + j] = sqrt(ci[d]);
        norm[12 + j] = mo[j];
        norm[18 + j] = sqrt(co[d]);
    }
    if (hbl_status st = check_norm(norm)) {
        set_error(HBL_EINVAL, "prelu_train: a coordinate has zero spread in the training split");
        return st;
    }
    memcpy(m->norm, norm, sizeof norm);
    m->has_norm = true;
    const int64_t epochs = cfg->epochs;
    if (hbl_status st = prelu_train_buffers(m, cfg->batch, 2 * (epochs > 0 ? epochs : 1), s)) return st;
    HBL_HIP(hipMemsetAsync(m->d_m, 0, sizeof(float) * m->nparams, s));
    HBL_HIP(hipMemsetAsync(m->d_v, 0, sizeof(float) * m->nparams, s));
    HBL_HIP(hipMemsetAsync(m->d_loss, 0, sizeof(double) * 2 * (epochs > 0 ? epochs : 1), s));
    if (hbl_status st = prelu_repack_all(m, s)) return st;
    m->step = 0;
    const DenseShape sh{m->shape.width, m->shape.hidden};
    const DenseNorm nm = prelu_norm(m);
    uint16_t* wt[kDenseMaxHidden + 1];
    prelu_wt(m, wt);
    const int64_t steps_per_epoch = n_train / cfg->batch;
    int64_t planned = epochs * steps_per_epoch;
    if (cfg->max_steps >= 0 && cfg->max_steps < planned) planned = cfg->max_steps;
    auto lr_at = [&](int64_t t) {
        if (planned <= 1 || cfg->lr_final == cfg->lr) return (double)cfg->lr;
        const double ph = 3.14159265358979323846 * (double)(t - 1) / (double)(planned - 1);
        return (double)cfg->lr_final + 0.5 * ((double)cfg->lr - (double)cfg->lr_final) * (1.0 + cos(ph));
    };
    int32_t* h_perm[2] = {nullptr, nullptr};
    int32_t* d_perm[2] = {nullptr, nullptr};
    int32_t* d_test = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hbl_status st = HBL_OK;
    auto fail = [&](hbl_status code, const char* what, hipError_t e) {
        set_error(code, "prelu_train: %s: %s", what, hipGetErrorString(e));
        st = code;
    };
    for (int k = 0; k < 2 && st == HBL_OK; ++k) {
        hipError_t e = hipHostMalloc((void**)&h_perm[k], sizeof(int32_t) * n_train, 0);
        if (e == hipSuccess) e = hipMalloc((void**)&d_perm[k], sizeof(int32_t) * n_train);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev[k], hipEventDisableTiming);
        if (e != hipSuccess) fail(HBL_ENOMEM, "order buffers", e);
    }
    if (st == HBL_OK && n_test > 0) {
        std::vector<int32_t> ti(n_test);
        for (int64_t i = 0; i < n_test; ++i) ti[i] = (int32_t)(n_train + i);
        hipError_t e = hipMalloc((void**)&d_test, sizeof(int32_t) * n_test);
        if (e == hipSuccess) e = hipMemcpy(d_test, ti.data(), sizeof(int32_t) * n_test, hipMemcpyHostToDevice);
        if (e != hipSuccess) fail(HBL_ENOMEM, "test indices", e);
    }
    std::vector<int64_t> steps_done(epochs > 0 ? epochs : 1, 0);
    for (int64_t ep = 0; ep < epochs && st == HBL_OK; ++ep) {
        const int k = (int)(ep & 1);
        hipError_t e = hipEventSynchronize(ev[k]);
        if (e != hipSuccess) { fail(HBL_EHIP, "event wait", e); break; }
        epoch_order(h_perm[k], n_train, cfg->shuffle_seed, ep);
        e = hipMemcpyAsync(d_perm[k], h_perm[k], sizeof(int32_t) * n_train, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipEventRecord(ev[k], s);
        if (e != hipSuccess) { fail(HBL_EHIP, "order upload", e); break; }
        DenseTrainBufs tb = m->tb;
        for (int64_t step = 0; step < steps_per_epoch; ++step) {
            if (cfg->max_steps >= 0 && m->step >= cfg->max_steps) break;
            m->step += 1;
            tb.idx = d_perm[k] + step * cfg->batch;
            e = launch_dense_train_step(zin, zout, ld, sh, m->im, wt, nm, tb, m->d_params, m->d_grad,
                                        m->d_loss + 2 * ep, 1.0 / (6.0 * cfg->batch), s);
            if (e == hipSuccess)
                e = launch_dense_adam_pack(m->d_params, m->d_m, m->d_v, m->d_grad, m->nparams, m->step,
                                           (float)lr_at(m->step), cfg->beta1, cfg->beta2, cfg->eps, sh, m->im,
                                           m->d_wt ? wt : nullptr, s);
            if (e != hipSuccess) { fail(HBL_EHIP, "step launch", e); break; }
            steps_done[ep] += 1;
        }
        if (st != HBL_OK) break;
        // test loss over the held-out pairs, in batches of the training size
        for (int64_t t0 = 0; t0 < n_test; t0 += cfg->batch) {
            const int32_t nb = (int32_t)std::min<int64_t>(cfg->batch, n_test - t0);
            DenseTrainBufs te = m->tb;
            te.idx = d_test + t0;
            te.B = nb;
            e = launch_dense_train_step(zin, zout, ld, sh, m->im, wt, nm, te, m->d_params, nullptr,
                                        m->d_loss + 2 * ep + 1, 1.0 / (6.0 * (double)n_test), s);
            if (e != hipSuccess) { fail(HBL_EHIP, "test loss launch", e); break; }
        }
    }
    hipError_t e = hipStreamSynchronize(s);
    if (st == HBL_OK && e != hipSuccess) fail(HBL_EHIP, "training", e);
    if (st == HBL_OK && loss_log && epochs > 0) {
        std::vector<double> acc(2 * epochs);
        e = hipMemcpy(acc.data(), m->d_loss, sizeof(double) * acc.size(), hipMemcpyDeviceToHost);
        if (e != hipSuccess) fail(HBL_EHIP, "loss readback", e);
        for (int64_t ep = 0; ep < epochs && st == HBL_OK; ++ep) {
            loss_log[2 * ep] = steps_done[ep] ? (float)(acc[2 * ep] / (double)steps_done[ep]) : 0.0f;
            loss_log[2 * ep + 1] = (float)acc[2 * ep + 1];
        }
    }
    for (int k = 0; k < 2; ++k) {
        if (ev[k]) (void)hipEventDestroy(ev[k]);
        if (d_perm[k]) (void)hipFree(d_perm[k]);
        if (h_perm[k]) (void)hipHostFree(h_perm[k]);
    }
    if (d_test) (void)hipFree(d_test);
    return st;
}

}  // extern "C"

// ------------------------------------------------------- wide PReLU model file
namespace {

constexpr uint64_t kPreluMagic = 0x31504C42484C4248ull;  // "HBLHBLP1"

struct PreluFileHeader {
    uint64_t magic;
    int32_t shape[4];
    int32_t has_norm, has_stage, has_moments, pad;
    int64_t step, nparams;
    double norm[24];
    double dE_MeV, L, gamma_in;
};

uint64_t fnv1a(uint64_t h, const void* p, size_t nbytes) {
    const unsigned char* c = (const unsigned char*)p;
    for (size_t q = 0; q < nbytes; ++q) { h ^= c[q]; h *= 1099511628211ull; }
    return h;
}

}  // namespace

extern "C" {

hbl_status hbl_prelu_save(const hbl_prelu_net* m, const char* path) {
    clear_error();
    HBL_REQUIRE(m && path, "prelu_save: NULL argument");
    const size_t np = (size_t)m->nparams;
    const bool mom = m->d_m != nullptr;
    std::vector<float> blob((mom ? 3 : 1) * np);
    HBL_HIP(hipDeviceSynchronize());
    HBL_HIP(hipMemcpy(blob.data(), m->d_params, sizeof(float) * np, hipMemcpyDeviceToHost));
    if (mom) {
        HBL_HIP(hipMemcpy(blob.data() + np, m->d_m, sizeof(float) * np, hipMemcpyDeviceToHost));
        HBL_HIP(hipMemcpy(blob.data() + 2 * np, m->d_v, sizeof(float) * np, hipMemcpyDeviceToHost));
    }
    PreluFileHeader hdr;
    memset(&hdr, 0, sizeof hdr);
    hdr.magic = kPreluMagic;
    hdr.shape[0] = m->shape.n_in; hdr.shape[1] = m->shape.width; hdr.shape[2] = m->shape.hidden; hdr.shape[3] = m->shape.n_out;
    hdr.has_norm = m->has_norm;
    hdr.has_stage = m->has_stage;
    hdr.has_moments = mom;
    hdr.step = m->step;
    hdr.nparams = m->nparams;
    memcpy(hdr.norm, m->norm, sizeof hdr.norm);
    hdr.dE_MeV = m->dE_MeV; hdr.L = m->L; hdr.gamma_in = m->gamma_in;
    uint64_t h = fnv1a(1469598103934665603ull, &hdr, sizeof hdr);
    h = fnv1a(h, blob.data(), blob.size() * sizeof(float));
    FILE* f = fopen(path, "wb");
    if (!f) { set_error(HBL_EIO, "prelu_save: cannot open %s", path); return HBL_EIO; }
    bool ok = fwrite(&hdr, sizeof hdr, 1, f) == 1 && fwrite(blob.data(), sizeof(float), blob.size(), f) == blob.size() &&
              fwrite(&h, sizeof h, 1, f) == 1;
    ok = (fclose(f) == 0) && ok;
    if (!ok) { set_error(HBL_EIO, "prelu_save: write failed for %s", path); return HBL_EIO; }
    return HBL_OK;
}

hbl_status hbl_prelu_load(const char* path, hbl_prelu_net** out) {
    clear_error();
    HBL_REQUIRE(path && out, "prelu_load: NULL argument");
    *out = nullptr;
    FILE* f = fopen(path, "rb");
    if (!f) { set_error(HBL_EIO, "prelu_load: cannot open %s", path); return HBL_EIO; }
    PreluFileHeader hdr;
    bool ok = fread(&hdr, sizeof hdr, 1, f) == 1;
    if (!ok || hdr.magic != kPreluMagic) {
        fclose(f);
        set_error(HBL_EIO, "prelu_load: %s is not a PReLU network file", path);
        return HBL_EIO;
    }
    hbl_mlp_shape sh = {hdr.shape[0], hdr.shape[1], hdr.shape[2], hdr.shape[3]};
    if (check_prelu_shape(&sh) != HBL_OK || hdr.nparams != prelu_nparams_of(&sh) || hdr.has_moments < 0 ||
        hdr.has_moments > 1) {
        fclose(f);
        set_error(HBL_EIO, "prelu_load: %s has an inconsistent header", path);
        return HBL_EIO;
    }
    const size_t np = (size_t)hdr.nparams;
    std::vector<float> blob((hdr.has_moments ? 3 : 1) * np);
    uint64_t stored = 0;
    ok = fread(blob.data(), sizeof(float), blob.size(), f) == blob.size() && fread(&stored, sizeof stored, 1, f) == 1;
    fclose(f);
    if (!ok) { set_error(HBL_EIO, "prelu_load: %s is truncated", path); return HBL_EIO; }
    uint64_t h = fnv1a(1469598103934665603ull, &hdr, sizeof hdr);
    h = fnv1a(h, blob.data(), blob.size() * sizeof(float));
    if (h != stored) { set_error(HBL_EIO, "prelu_load: checksum mismatch in %s", path); return HBL_EIO; }
    hbl_prelu_net* m = nullptr;
    if (hbl_status st = hbl_prelu_create(&sh, 0, &m)) return st;
    hipError_t e = hipMemcpy(m->d_params, blob.data(), sizeof(float) * np, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_dense_pack(m->d_params, DenseShape{sh.width, sh.hidden}, m->im, nullptr);
    if (e == hipSuccess && hdr.has_moments) {
        if (prelu_opt_state(m) != HBL_OK) e = hipErrorOutOfMemory;
        if (e == hipSuccess) e = hipMemcpy(m->d_m, blob.data() + np, sizeof(float) * np, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(m->d_v, blob.data() + 2 * np, sizeof(float) * np, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        prelu_free(m);
        set_error(HBL_EHIP, "prelu_load: upload failed: %s", hipGetErrorString(e));
        return HBL_EHIP;
    }
    m->has_norm = hdr.has_norm != 0;
    memcpy(m->norm, hdr.norm, sizeof m->norm);
    m->has_stage = hdr.has_stage != 0;
    m->dE_MeV = hdr.dE_MeV; m->L = hdr.L; m->gamma_in = hdr.gamma_in;
    m->step = hdr.step;
    *out = m;
    return HBL_OK;
}

}  // extern "C"
