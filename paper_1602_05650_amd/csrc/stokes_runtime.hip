// Runtime support of libstokes.so: status and error strings, the per-(device,
// stream) scratch workspace, and the local slender-body operator.
#include <math.h>

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "stokes_internal.hpp"

namespace stokes {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return STOKES_E_DEVICE;
}

// ---- workspace --------------------------------------------------------------
static std::mutex g_ws_mu;
static std::map<std::pair<int, hipStream_t>, Workspace*> g_ws;

int workspace_get(hipStream_t stream, size_t bytes, Workspace** out) {
    int dev = 0;
    STOKES_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace*& ws = g_ws[{dev, stream}];
    if (!ws) {
        ws = new Workspace();
        hipError_t e = hipHostMalloc(&ws->host, 256, hipHostMallocDefault);
        if (e != hipSuccess) {
            delete ws;
            ws = nullptr;
            return hip_fail(e, "hipHostMalloc(workspace status buffer)");
        }
    }
    if (ws->bytes < bytes) {
        // the old buffer may still be read by work queued on this stream
        if (ws->dev) {
            STOKES_HIP(hipStreamSynchronize(stream));
            STOKES_HIP(hipFree(ws->dev));
            ws->dev = nullptr;
            ws->bytes = 0;
        }
        size_t nb = bytes + bytes / 4 + (1 << 20);
        hipError_t e = hipMalloc(&ws->dev, nb);
        if (e != hipSuccess) {
            ws->dev = nullptr;
            (void)hipGetLastError();
            return fail(STOKES_E_NOMEM, std::string("workspace of ") + std::to_string(nb) +
                                            " bytes: " + hipGetErrorString(e));
        }
        ws->bytes = nb;
    }
    *out = ws;
    return STOKES_OK;
}

// ---- kernel timing -------------------------------------------------------------
static std::atomic<bool> g_prof_on{false};
static std::mutex g_prof_mu;
static std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_done;   // recorded pairs
static thread_local hipEvent_t t_prof_start = nullptr;

void prof_begin(hipStream_t st) {
    if (!g_prof_on.load(std::memory_order_relaxed)) return;
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return;
    if (hipEventRecord(e, st) != hipSuccess) {
        (void)hipEventDestroy(e);
        return;
    }
    t_prof_start = e;
}

void prof_end(hipStream_t st) {
    if (!t_prof_start) return;
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess || hipEventRecord(e, st) != hipSuccess) {
        if (e) (void)hipEventDestroy(e);
        (void)hipEventDestroy(t_prof_start);
        t_prof_start = nullptr;
        return;
    }
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_done.emplace_back(t_prof_start, e);
    t_prof_start = nullptr;
}

// ---- local slender-body operator (eq. main-sb-local) -------------------------
//   M f     = (1/(8 pi mu)) [ (kappa + 2) f + (kappa - 2) t (t.f) ],  kappa = -ln(eps^2 e)
//   M^-1 v  = 8 pi mu [ t (t.v) / (2 kappa) + (v - t (t.v)) / (kappa + 2) ]
__global__ void local_sbt_kernel(int64_t n, const double* __restrict__ t, const double* f,
                                 double kap, double mu, int inverse, double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double tx = t[i], ty = t[n + i], tz = t[2 * n + i];
    const double fx = f[i], fy = f[n + i], fz = f[2 * n + i];
    const double tf = tx * fx + ty * fy + tz * fz;
    const double pi8mu = 8.0 * 3.14159265358979323846 * mu;
    double a, b;   // out = a f + b t (t.f)
    if (!inverse) {
        a = (kap + 2.0) / pi8mu;
        b = (kap - 2.0) / pi8mu;
    } else {
        a = pi8mu / (kap + 2.0);
        b = pi8mu / (2.0 * kap) - a;
    }
    out[i] = a * fx + b * tf * tx;
    out[n + i] = a * fy + b * tf * ty;
    out[2 * n + i] = a * fz + b * tf * tz;
}

}  // namespace stokes

using namespace stokes;

extern "C" int stokes_local_sbt(int64_t n, const double* tangent, const double* f, double eps,
                                double mu, int inverse, double* out, void* stream) {
    if (n < 0) return fail(STOKES_E_INVAL, "stokes_local_sbt: n < 0");
    if (n > 0 && (!tangent || !f || !out)) return fail(STOKES_E_INVAL, "stokes_local_sbt: null pointer");
    if (!(mu > 0.0)) return fail(STOKES_E_INVAL, "stokes_local_sbt: mu must be > 0");
    if (!(eps > 0.0 && eps < 0.5)) return fail(STOKES_E_INVAL, "stokes_local_sbt: eps must be in (0, 0.5)");
    if (n == 0) return STOKES_OK;
    const double kap = -log(eps * eps * M_E);
    hipLaunchKernelGGL(local_sbt_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), n, tangent, f, kap, mu, inverse ? 1 : 0, out);
    STOKES_HIP(hipGetLastError());
    return STOKES_OK;
}

extern "C" int stokes_profile_enable(int on) {
    g_prof_on.store(on != 0);
    return STOKES_OK;
}

extern "C" int stokes_profile_read(double* ms, int64_t* launches) {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        ev.swap(g_prof_done);
    }
    double total = 0.0;
    int rc = STOKES_OK;
    for (auto& p : ev) {
        float t = 0.0f;
        hipError_t e = hipEventSynchronize(p.second);
        if (e == hipSuccess) e = hipEventElapsedTime(&t, p.first, p.second);
        if (e != hipSuccess && rc == STOKES_OK) rc = hip_fail(e, "stokes_profile_read");
        total += t;
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    if (ms) *ms = total;
    if (launches) *launches = (int64_t)ev.size();
    return rc;
}

extern "C" const char* stokes_status_string(int status) {
    switch (status) {
        case STOKES_OK: return "STOKES_OK";
        case STOKES_E_INVAL: return "STOKES_E_INVAL";
        case STOKES_E_NOMEM: return "STOKES_E_NOMEM";
        case STOKES_E_DEVICE: return "STOKES_E_DEVICE";
        case STOKES_E_NONFINITE: return "STOKES_E_NONFINITE";
        case STOKES_E_BUSY: return "STOKES_E_BUSY";
        case STOKES_E_CANCELED: return "STOKES_E_CANCELED";
        case STOKES_E_TIMEOUT: return "STOKES_E_TIMEOUT";
        case STOKES_E_NOTFOUND: return "STOKES_E_NOTFOUND";
        default: return "STOKES_E_UNKNOWN";
    }
}

extern "C" const char* stokes_last_error(void) { return g_last_error.c_str(); }

extern "C" int stokes_version(void) { return 10000; }

extern "C" int stokes_release_workspace(void) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    int rc = STOKES_OK;
    for (auto& kv : g_ws) {
        Workspace* ws = kv.second;
        if (!ws) continue;
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(kv.first.first);
        if (hipDeviceSynchronize() != hipSuccess) rc = STOKES_E_DEVICE;
        if (ws->dev) (void)hipFree(ws->dev);
        if (ws->host) (void)hipHostFree(ws->host);
        (void)hipSetDevice(cur);
        delete ws;
    }
    g_ws.clear();
    fiberstep_release();
    batch_res_drain();
    if (rc) set_error("stokes_release_workspace: device synchronisation failed");
    return rc;
}
