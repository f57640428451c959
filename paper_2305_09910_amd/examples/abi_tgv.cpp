// abi_tgv.cpp -- the C ABI used from plain host code, without Python or torch.
//
// A 32^3 periodic Taylor-Green vortex (D3Q19, TRT, nu = 0.01): the caller
// allocates the workspace and the fields with hipMalloc, creates a context,
// steps it and reads the FP64 totals and the velocity field back.  Prints
// one line "mass <M> amp_ratio <r> expected <e>" and exits 0 when the mass
// equals the cell count to 1e-7 relative and the velocity amplitude has
// decayed as exp(-2 nu k^2 t) to within 1%; non-zero otherwise.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <vector>

#include "../../include/lbm.h"

#define CHECK_HIP(x)                                                      \
    do {                                                                  \
        hipError_t e_ = (x);                                              \
        if (e_ != hipSuccess) {                                           \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_)); \
            return 2;                                                     \
        }                                                                 \
    } while (0)

#define CHECK_LBM(c, x)                                                        \
    do {                                                                       \
        int r_ = (x);                                                          \
        if (r_ != LBM_OK) {                                                    \
            std::fprintf(stderr, "%s: %d %s\n", #x, r_, lbm_last_error(c));   \
            return 3;                                                          \
        }                                                                      \
    } while (0)

int main()
{
    const int n = 32, steps = 1000;
    const double nu = 0.01, tau = 3 * nu + 0.5, u0 = 0.05, pi = std::acos(-1.0), k = 2 * pi / n;
    const size_t cells = (size_t)n * n * n;

    lbm_domain d;
    lbm_domain_defaults(&d);
    d.nx = d.ny = d.nz = n;
    size_t ws_bytes = 0;
    CHECK_LBM(nullptr, lbm_workspace_bytes(&d, LBM_D3Q19, &ws_bytes));
    void *ws = nullptr;
    CHECK_HIP(hipMalloc(&ws, ws_bytes));  // hipMalloc returns 256-byte aligned memory
    d.workspace = ws;
    d.workspace_bytes = ws_bytes;
    d.stream = nullptr;

    lbm_ctx *ctx = nullptr;
    const double force[3] = {0, 0, 0};
    CHECK_LBM(nullptr, lbm_create(&d, LBM_D3Q19, nullptr, tau, force, &ctx));

    // Taylor-Green fields: u = u0 cos kx sin ky, v = -u0 sin kx cos ky,
    // rho = 1 - (3 u0^2 / 4)(cos 2kx + cos 2ky)
    std::vector<double> rho(cells), u(3 * cells, 0.0);
    for (int z = 0; z < n; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                const size_t c = ((size_t)z * n + y) * n + x;
                rho[c] = 1.0 - 0.75 * u0 * u0 * (std::cos(2 * k * x) + std::cos(2 * k * y));
                u[c] = u0 * std::cos(k * x) * std::sin(k * y);
                u[cells + c] = -u0 * std::sin(k * x) * std::cos(k * y);
            }
    double *rho_d = nullptr, *u_d = nullptr;
    CHECK_HIP(hipMalloc((void **)&rho_d, cells * sizeof(double)));
    CHECK_HIP(hipMalloc((void **)&u_d, 3 * cells * sizeof(double)));
    CHECK_HIP(hipMemcpy(rho_d, rho.data(), cells * sizeof(double), hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(u_d, u.data(), 3 * cells * sizeof(double), hipMemcpyHostToDevice));
    CHECK_LBM(ctx, lbm_init_equilibrium(ctx, rho_d, u_d));
    CHECK_LBM(ctx, lbm_step(ctx, steps));

    double mass = 0, mom[3] = {0, 0, 0};
    CHECK_LBM(ctx, lbm_totals(ctx, &mass, mom));

    float *rf = nullptr, *uf = nullptr;
    CHECK_HIP(hipMalloc((void **)&rf, cells * sizeof(float)));
    CHECK_HIP(hipMalloc((void **)&uf, 3 * cells * sizeof(float)));
    CHECK_LBM(ctx, lbm_moments(ctx, rf, uf));
    std::vector<float> uh(3 * cells);
    CHECK_HIP(hipMemcpy(uh.data(), uf, 3 * cells * sizeof(float), hipMemcpyDeviceToHost));

    // projection of u_x on the initial mode
    double num = 0, den = 0;
    for (int z = 0; z < n; ++z)
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                const size_t c = ((size_t)z * n + y) * n + x;
                const double m = std::cos(k * x) * std::sin(k * y);
                num += uh[c] * m;
                den += m * m;
            }
    const double ratio = num / den / u0, expect = std::exp(-2 * nu * k * k * steps);
    std::printf("mass %.12f amp_ratio %.6f expected %.6f\n", mass, ratio, expect);

    lbm_destroy(ctx);
    hipFree(uf);
    hipFree(rf);
    hipFree(u_d);
    hipFree(rho_d);
    hipFree(ws);
    const bool ok = std::fabs(mass / (double)cells - 1.0) < 1e-7 && std::fabs(ratio / expect - 1.0) < 0.01;
    return ok ? 0 : 1;
}
