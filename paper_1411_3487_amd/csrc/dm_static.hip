// dm_static.hip -- the FP64 plain-form mode step without allocation
// (dm_step_modes_f64_static in dnamodes.h).
//
// Callers that may not allocate device memory pass their own mode
// amplitudes; the transform tables, the one-step coefficients, the chain
// indices and the two work buffers of the step (positions, reused for the
// coupling, and forces) live in one file-scope device array, `scratch`,
// which every GPU the library runs on holds until the process ends.  Its
// device address is taken once per device with hipGetSymbolAddress (the
// array's name is only a host-side stand-in) and used wherever host code
// needs it.  The tables are rebuilt on the device at every call, and every
// byte the step reads is written earlier in the same call, so nothing needs
// clearing.  Calls that overlap on one GPU share the array and race.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "../../include/dnamodes.h"
#include "dm_internal.h"

namespace dm {
namespace {

__device__ __align__(256) unsigned char scratch[DM_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];  // device address of `scratch` per device (null until taken)

// Errors go where dm_last_error(NULL) reads them.
int fail(int code, const char *fmt, ...)
{
    char buf[256];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    set_ctxless_error(buf);
    return code;
}

// Bytes of the array used for M beads and n chains (each part 256-aligned):
// inverse and forward tables (M x M each), E, C, W (M each), chain indices,
// and two work buffers of 3 M n doubles.
size_t part(size_t bytes) { return (bytes + 255) & ~(size_t)255; }
size_t static_bytes(int M, int n)
{
    const size_t mm = (size_t)M * M, w = (size_t)3 * M * n;
    return 2 * part(8 * mm) + 3 * part(8 * (size_t)M) + part(4 * (size_t)n) + 2 * part(8 * w);
}

// phi_{n,p} of Eq. (c8) as the inverse table A[n][p] (column p = 0 zeroed:
// the internal coordinates) and the forward table A[p][n]; the angle
// p (n + 1/2) pi / M is reduced exactly as the integer p (2n + 1) mod 4M.
__global__ __launch_bounds__(256) void static_phi_kernel(double *__restrict__ Ainv,
                                                         double *__restrict__ Afwd, int M)
{
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (size_t)M * M) return;
    const int n = (int)(idx / M), p = (int)(idx % M);
    double v;
    if (p == 0) {
        v = sqrt(1.0 / M);
    } else {
        const long m = ((long)p * (2 * n + 1)) % (4L * M);
        v = sqrt(2.0 / M) * cospi((double)m / (2.0 * M));
    }
    Ainv[(size_t)n * M + p] = p == 0 ? 0.0 : v;
    Afwd[(size_t)p * M + n] = v;
}

// Rates and one-step coefficients (Eqs. c9, e9, d3, f2, d6) in their
// cancellation-free forms, s_p = sin(p pi / 2M):
//   zeta_p = 16 nu s^4, zeta^l_p - zeta_p = (1 - 2 nu) 4 s^2,
//   E = exp(-zeta dtau), C = -E expm1(-(zeta^l - zeta) dtau) / (zeta^l - zeta),
//   W = sqrt(-T* expm1(-2 zeta dtau) / zeta), limits C = dtau E, W = sqrt(2 T* dtau).
// Also the chain indices chain0 + j.
__global__ __launch_bounds__(256) void static_coef_kernel(double *__restrict__ E,
                                                          double *__restrict__ C,
                                                          double *__restrict__ W,
                                                          int32_t *__restrict__ ids, int M,
                                                          int nch, double nu, double T_star,
                                                          double dtau, uint32_t chain0)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nch) ids[i] = (int32_t)(chain0 + (uint32_t)i);
    if (i >= M) return;
    if (i == 0) {
        E[0] = 1.0;
        C[0] = dtau;
        W[0] = sqrt(2.0 * T_star * dtau);
        return;
    }
    const double s = sinpi((double)i / (2.0 * M)), s2 = s * s;
    const double z = 16.0 * nu * s2 * s2, dz = (1.0 - 2.0 * nu) * 4.0 * s2;
    const double e = exp(-z * dtau);
    E[i] = e;
    C[i] = dz > 0.0 ? -e * expm1(-dz * dtau) / dz : dtau * e;
    W[i] = z > 0.0 ? sqrt(-T_star * expm1(-2.0 * z * dtau) / z) : sqrt(2.0 * T_star * dtau);
}

int scratch_ptr(unsigned char **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(DM_EHIP, "hipGetDevice failed: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(DM_EHIP, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(DM_EHIP, "hipGetSymbolAddress(scratch) failed: %s",
                        hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = static_cast<unsigned char *>(g_ptr[dev]);
    return DM_OK;
}

}  // namespace
}  // namespace dm

extern "C" int dm_step_modes_f64_static(double *R_dev, int32_t n_chains, int32_t M,
                                        double T_star, double nu, double dtau,
                                        double gamma_dot, int32_t nonlinear, uint64_t seed,
                                        uint32_t chain0, int64_t step0, int64_t n_steps,
                                        void *hip_stream)
{
    using namespace dm;
    set_ctxless_error("");
    if (!R_dev) return fail(DM_EINVAL, "R_dev is NULL");
    if ((uintptr_t)R_dev % 16 != 0) return fail(DM_EINVAL, "R_dev must be 16-byte aligned");
    if (n_chains < 1 || M < 2 || M > 2048)
        return fail(DM_EINVAL, "need n_chains >= 1 and 2 <= M <= 2048 (got %d, %d)", n_chains, M);
    if (!(nu >= 0.0 && nu < 0.5)) return fail(DM_EINVAL, "nu = %g outside [0, 1/2)", nu);
    if (!(T_star > 0.0) || !std::isfinite(T_star) || !(dtau > 0.0) || !std::isfinite(dtau) ||
        !std::isfinite(gamma_dot))
        return fail(DM_EINVAL, "T* and dtau must be positive and finite, gamma_dot finite");
    if (n_steps < 0 || step0 < 0) return fail(DM_EINVAL, "n_steps and step0 must be >= 0");
    if ((uint64_t)chain0 + (uint64_t)n_chains > (1ull << 31))
        return fail(DM_EINVAL, "chain indices chain0 + j must stay below 2^31");
    const size_t need = static_bytes(M, n_chains);
    if (need > (size_t)DM_STATIC_SCRATCH_BYTES)
        return fail(DM_EINVAL,
                    "%d chains of %d beads need %zu bytes of work space; the fixed array holds "
                    "%zu (DM_STATIC_SCRATCH_BYTES)",
                    n_chains, M, need, (size_t)DM_STATIC_SCRATCH_BYTES);
    unsigned char *base = nullptr;
    int rc = scratch_ptr(&base);
    if (rc) return rc;
    const size_t mm = (size_t)M * M, w = (size_t)3 * M * n_chains;
    unsigned char *q = base;
    auto take = [&](size_t bytes) {
        unsigned char *p = q;
        q += part(bytes);
        return p;
    };
    double *Ainv = (double *)take(8 * mm), *Afwd = (double *)take(8 * mm);
    double *E = (double *)take(8 * (size_t)M), *C = (double *)take(8 * (size_t)M),
           *W = (double *)take(8 * (size_t)M);
    int32_t *ids = (int32_t *)take(4 * (size_t)n_chains);
    double *rwork = (double *)take(8 * w), *Fwork = (double *)take(8 * w);
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(static_phi_kernel, dim3((unsigned)((mm + 255) / 256)), dim3(256), 0, st,
                       Ainv, Afwd, M);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) {
        const int nt = M > n_chains ? M : n_chains;
        hipLaunchKernelGGL(static_coef_kernel, dim3((nt + 255) / 256), dim3(256), 0, st, E, C, W,
                           ids, M, n_chains, nu, T_star, dtau, chain0);
        e = hipGetLastError();
    }
    const double lin = 1.0 - 2.0 * nu, gdt = gamma_dot * dtau;
    for (int64_t s = 0; s < n_steps && e == hipSuccess; ++s) {
        if (nonlinear) {
            e = launch_gemm_f64(Ainv, R_dev, rwork, M, 3 * n_chains, st);
            if (e == hipSuccess) e = launch_stencil_f64(rwork, Fwork, M, n_chains, lin, st);
            if (e == hipSuccess) e = launch_gemm_f64(Afwd, Fwork, rwork, M, 3 * n_chains, st);
        }
        if (e == hipSuccess)
            e = launch_mode_update_f64(R_dev, rwork, E, C, W, ids, M, n_chains, seed, nullptr,
                                       step0 + s, gdt, nonlinear ? 1 : 0, st);
    }
    if (e != hipSuccess) return fail(DM_EHIP, "kernel launch failed: %s", hipGetErrorString(e));
    return DM_OK;
}
