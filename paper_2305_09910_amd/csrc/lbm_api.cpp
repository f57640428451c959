// lbm_api.cpp -- the C ABI declared in include/lbm.h.
//
// Host-side validation, workspace carve-up and kernel launches on the
// caller's stream.  The library allocates no device memory: everything lives
// in the caller's workspace.  Layout of the workspace (each part 256-byte
// aligned):
//   populations  q * n storage elements, [z][y][q][x] (rows of q direction segments);
//                with the Esoteric Twist each non-periodic axis has one more
//                cell (the ghost layer beyond its + face); with sparse
//                addressing q * nf elements in chunks of 64 fluid cells
//   velocities   (HRR only) two velocity fields of 3 * n FP32, the input and
//                output of the finite-difference gradient; with the
//                populations they form the state that checkpoints copy
//   mask         n uint32 words, then one word per cell row and run of 64
//                cells along x (only with use_flags)
//   sparse       (sparse addressing only) fluid map (n int32), fluid cells'
//                linear indices (nf uint32) and neighbour table ((q-1) * nf uint32)
//   totals       partial sums (1024 blocks x 5 doubles) and the final 5
//   closure      MLP parameters (1313 + 24 FP32), their per-lane operand table
//                (63 x 64 words) and a fallback counter
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/lbm.h"
#include "internal.h"

using namespace lbm;

struct lbm_ctx {
    LatticeArgs a;
    SparseArgs sp;
    float *uvel[2];  // HRR velocity fields: step t reads uvel[t & 1], writes uvel[(t + 1) & 1]
    float hrr_sigma;
    int q, st, cl, coll;
    int sc_flags;                             // SC_SOLID_ODD | SC_MASK_RUNS for masked AA domains with sparse solids
    int bc_kind[6];                           // the domain's face kinds (LBM_BC_INTERFACE kept)
    double tau_d, force_d[3], magic_d, mrt_d[5];  // the parameters as given (refinement checks)
    int64_t time;
    hipStream_t stream;
    char *ws;
    size_t ws_bytes;
    double *partial, *final_out;
    float *mlp;
    uint32_t *mlp_tab;
    unsigned long long *fallbacks;
    uint32_t *mask;
    int64_t nfluid;
    int mlp_ready;
    size_t state_bytes;
    char err[512];
};

static thread_local char g_err[512] = "";

static int fail(lbm_ctx *c, int code, const char *fmt, ...)
{
    char *buf = c ? c->err : g_err;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, 512, fmt, ap);
    va_end(ap);
    return code;
}

static int hip_fail(lbm_ctx *c, hipError_t e, const char *what)
{
    return fail(c, LBM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHECK(c, call, what)                         \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_fail(c, e_, what); \
    } while (0)

static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Layout {
    size_t pdf, uvel, mask, fmap, fcell, nbt, partial, final_out, mlp, mlp_tab, fallback, total, pdf_bytes;
    size_t uvel_bytes, state_bytes;  // one velocity field; populations plus velocity fields
    int sx, sy, sz;  // cells of the population store per axis
};

// nf: fluid cells, which size the stores of sparse addressing (the cell
// count when the flags are not known: an upper bound)
static int make_layout(const lbm_domain *d, int q, Layout *L, lbm_ctx *c, int64_t nf = -1)
{
    if (!d) return fail(c, LBM_EINVAL, "domain is NULL");
    if (q != 19 && q != 27) return fail(c, LBM_EINVAL, "stencil must be 19 or 27, got %d", q);
    if (d->nx < 1 || d->ny < 1 || d->nz < 1)
        return fail(c, LBM_EINVAL, "domain sizes must be >= 1 (got %d x %d x %d)", d->nx, d->ny, d->nz);
    if (d->storage < LBM_STORE_F32 || d->storage > LBM_STORE_BF16DEV)
        return fail(c, LBM_EINVAL, "unknown storage %d", d->storage);
    if (d->closure < LBM_LES_NONE || d->closure > LBM_LES_MLP)
        return fail(c, LBM_EINVAL, "unknown closure %d", d->closure);
    if (d->streaming != LBM_STREAM_AA && d->streaming != LBM_STREAM_ET && d->streaming != LBM_STREAM_AA_SPARSE)
        return fail(c, LBM_EINVAL, "unknown streaming scheme %d", d->streaming);
    const uint64_t n = (uint64_t)d->nx * (uint64_t)d->ny * (uint64_t)d->nz;
    // Cell indices are 64-bit; rows (z, y) are counted in 32 bits, and the
    // launch grid spans ny and nz in its second and third dimension.
    if (d->ny > 65535 || d->nz > 65535)
        return fail(c, LBM_EINVAL, "ny and nz must be at most 65535 (got %d, %d)", d->ny, d->nz);
    const bool sp = d->streaming == LBM_STREAM_AA_SPARSE;
    if (sp && n >= (1ull << 32))
        return fail(c, LBM_ENOMEM, "sparse addressing: domain of %llu cells exceeds 2^32 cells", (unsigned long long)n);
    const bool et = d->streaming == LBM_STREAM_ET;
    const size_t elem = d->storage == LBM_STORE_F32 ? 4 : 2;
    // Row pitch: whole 128-byte lines, so that every direction segment
    // starts on a line (the ghost column of the Esoteric Twist would
    // otherwise shift all rows); the padding is never accessed.
    const int line = (int)(128 / elem);
    const int rx = d->nx + (et && d->bc[0] != LBM_BC_PERIODIC);
    L->sx = (rx + line - 1) / line * line;
    L->sy = d->ny + (et && d->bc[2] != LBM_BC_PERIODIC);
    L->sz = d->nz + (et && d->bc[4] != LBM_BC_PERIODIC);
    const uint64_t ns = (uint64_t)L->sx * (uint64_t)L->sy * (uint64_t)L->sz;
    if (nf < 0 || nf > (int64_t)n) nf = (int64_t)n;
    if (sp && nf >= (1ll << 31))
        return fail(c, LBM_ENOMEM, "sparse addressing: %lld fluid cells exceed 2^31", (long long)nf);
    const uint64_t chunks = ((uint64_t)nf + SP_CHUNK - 1) / SP_CHUNK;
    size_t off = 0;
    L->pdf = off;
    L->pdf_bytes = sp ? (size_t)q * chunks * SP_CHUNK * elem : (size_t)q * ns * elem;
    off += al256(L->pdf_bytes);
    L->uvel = off;
    L->uvel_bytes = d->collision == LBM_COLL_HRR ? al256((size_t)12 * n) : 0;
    off += 2 * L->uvel_bytes;
    L->state_bytes = d->collision == LBM_COLL_HRR ? off : L->pdf_bytes;
    L->mask = off;
    if (d->use_flags) off += al256(4 * (n + (uint64_t)d->ny * (uint64_t)d->nz * mask_runs(d->nx)));
    L->fmap = L->fcell = L->nbt = off;
    if (sp) {
        off += al256(4 * n);
        L->fcell = off;
        off += al256(4 * chunks * SP_CHUNK);
        L->nbt = off;
        off += al256((size_t)4 * (q - 1) * chunks * SP_CHUNK);
    }
    L->partial = off;
    off += al256((size_t)totals_blocks() * 5 * sizeof(double));
    L->final_out = off;
    off += al256(5 * sizeof(double));
    L->mlp = off;
    off += al256((MLP_NPARAM + MLP_NNORM) * sizeof(float));
    L->mlp_tab = off;
    off += al256(63 * 64 * sizeof(uint32_t));
    L->fallback = off;
    off += 256;
    L->total = off;
    return LBM_OK;
}

extern "C" {

void lbm_domain_defaults(lbm_domain *d)
{
    if (!d) return;
    memset(d, 0, sizeof *d);
    for (int f = 0; f < 6; ++f) {
        d->bc[f] = LBM_BC_PERIODIC;
        d->rho_bc[f] = 1.0;
    }
    d->storage = LBM_STORE_F32;
    d->closure = LBM_LES_NONE;
    d->magic = 3.0 / 16.0;
    d->cs_smag = 0.1;
    d->collision = LBM_COLL_TRT;
    const double r[5] = {1.19, 1.4, 1.2, 1.4, 1.98};
    for (int k = 0; k < 5; ++k) d->mrt_rates[k] = r[k];
    d->hrr_sigma = 0.995;
}

int lbm_workspace_bytes(const lbm_domain *d, int stencil, size_t *out)
{
    if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
    Layout L;
    int rc = make_layout(d, stencil, &L, nullptr);
    if (rc) return rc;
    *out = L.total;
    return LBM_OK;
}

static int64_t count_fluid(const lbm_domain *d, const uint8_t *flags)
{
    const int64_t n = (int64_t)d->nx * d->ny * d->nz;
    if (!flags) return n;
    int64_t nf = 0;
    for (int64_t k = 0; k < n; ++k) nf += flags[k] == 0;
    return nf;
}

int lbm_workspace_bytes_flags(const lbm_domain *d, int stencil, const uint8_t *flags, size_t *out)
{
    if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
    if (!d) return fail(nullptr, LBM_EINVAL, "domain is NULL");
    Layout L;
    int rc = make_layout(d, stencil, &L, nullptr, count_fluid(d, flags));
    if (rc) return rc;
    *out = L.total;
    return LBM_OK;
}

int lbm_create(const lbm_domain *d, int stencil, const uint8_t *flags, double tau, const double force[3],
               lbm_ctx **out)
{
    if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    Layout L;
    int rc = make_layout(d, stencil, &L, nullptr);
    if (rc) return rc;
    const bool sp = d->streaming == LBM_STREAM_AA_SPARSE;
    if (flags && !d->use_flags) return fail(nullptr, LBM_EINVAL, "flags given but domain.use_flags is 0");
    const int64_t nf = count_fluid(d, flags);
    if (sp && (rc = make_layout(d, stencil, &L, nullptr, nf))) return rc;  // stores sized by the fluid cells
    if (!(tau > 0.5) || !isfinite(tau)) return fail(nullptr, LBM_EINVAL, "tau must be > 1/2 (got %g)", tau);
    if (!(d->magic > 0.0) || !isfinite(d->magic)) return fail(nullptr, LBM_EINVAL, "magic must be > 0");
    if (d->closure != LBM_LES_NONE && !(d->cs_smag >= 0.0)) return fail(nullptr, LBM_EINVAL, "cs_smag must be >= 0");
    bool iface = false;
    for (int f = 0; f < 6; ++f) {
        if (d->bc[f] < LBM_BC_PERIODIC || d->bc[f] > LBM_BC_INTERFACE)
            return fail(nullptr, LBM_EINVAL, "unknown boundary kind %d on face %d", d->bc[f], f);
        if (d->bc[f] == LBM_BC_INTERFACE) {
            if (f != 2 && f != 3) return fail(nullptr, LBM_EINVAL, "refinement interfaces are -y or +y faces (face %d)", f);
            iface = true;
        }
    }
    if (iface) {
        if (d->streaming != LBM_STREAM_AA)
            return fail(nullptr, LBM_EINVAL, "refinement interfaces need the dense AA pattern");
        if (d->collision == LBM_COLL_HRR) return fail(nullptr, LBM_EINVAL, "refinement interfaces do not run with HRR");
        if (flags)
            for (int f = 2; f <= 3; ++f) {
                if (d->bc[f] != LBM_BC_INTERFACE) continue;
                const int64_t y = f == 2 ? 0 : d->ny - 1;
                for (int64_t z = 0; z < d->nz; ++z)
                    for (int64_t x = 0; x < d->nx; ++x)
                        if (flags[(z * d->ny + y) * d->nx + x])
                            return fail(nullptr, LBM_EINVAL, "solid cell in the interface row of face %d", f);
            }
    }
    for (int a = 0; a < 3; ++a)
        if ((d->bc[2 * a] == LBM_BC_PERIODIC) != (d->bc[2 * a + 1] == LBM_BC_PERIODIC))
            return fail(nullptr, LBM_EINVAL, "axis %d: a periodic face needs a periodic opposite face", a);
    if (d->collision != LBM_COLL_TRT && d->collision != LBM_COLL_MRT && d->collision != LBM_COLL_HRR)
        return fail(nullptr, LBM_EINVAL, "unknown collision %d", d->collision);
    if (d->collision == LBM_COLL_HRR) {
        if (stencil != LBM_D3Q19) return fail(nullptr, LBM_EINVAL, "the HRR collision is built for D3Q19");
        if (d->streaming != LBM_STREAM_AA)
            return fail(nullptr, LBM_EINVAL, "the HRR collision runs with the dense AA pattern only");
        if (d->closure != LBM_LES_NONE) return fail(nullptr, LBM_EINVAL, "the HRR collision runs without a closure");
        if (!(d->hrr_sigma >= 0.0 && d->hrr_sigma <= 1.0))
            return fail(nullptr, LBM_EINVAL, "hrr_sigma must lie in [0, 1]");
    }
    if (d->collision == LBM_COLL_MRT) {
        if (d->closure == LBM_LES_MLP) return fail(nullptr, LBM_EINVAL, "the MLP closure runs with TRT only");
        for (int k = 0; k < 5; ++k)
            if (!(d->mrt_rates[k] > 0.0 && d->mrt_rates[k] < 2.0))
                return fail(nullptr, LBM_EINVAL, "mrt_rates[%d] must lie in (0, 2)", k);
    }
    if (!d->workspace) return fail(nullptr, LBM_EINVAL, "workspace is NULL");
    if (((uintptr_t)d->workspace & 255) != 0) return fail(nullptr, LBM_EINVAL, "workspace must be 256-byte aligned");
    if (d->workspace_bytes < L.total)
        return fail(nullptr, LBM_EINVAL, "workspace too small: %zu < %zu bytes", d->workspace_bytes, L.total);
    if (force)
        for (int a = 0; a < 3; ++a)
            if (!isfinite(force[a])) return fail(nullptr, LBM_EINVAL, "force must be finite");

    lbm_ctx *c = new (std::nothrow) lbm_ctx;
    if (!c) return fail(nullptr, LBM_ENOMEM, "out of host memory");
    memset(c, 0, sizeof *c);
    c->q = stencil;
    c->st = d->storage;
    c->cl = d->closure;
    c->coll = d->collision;
    for (int f = 0; f < 6; ++f) c->bc_kind[f] = d->bc[f];
    c->tau_d = tau;
    for (int k = 0; k < 3; ++k) c->force_d[k] = force ? force[k] : 0.0;
    c->magic_d = d->magic;
    for (int k = 0; k < 5; ++k) c->mrt_d[k] = d->mrt_rates[k];
    c->stream = (hipStream_t)d->stream;
    c->ws = (char *)d->workspace;
    c->ws_bytes = d->workspace_bytes;
    c->partial = (double *)(c->ws + L.partial);
    c->final_out = (double *)(c->ws + L.final_out);
    c->mlp = (float *)(c->ws + L.mlp);
    c->fallbacks = (unsigned long long *)(c->ws + L.fallback);
    c->mask = d->use_flags ? (uint32_t *)(c->ws + L.mask) : nullptr;
    c->state_bytes = L.state_bytes;
    c->uvel[0] = L.uvel_bytes ? (float *)(c->ws + L.uvel) : nullptr;
    c->uvel[1] = L.uvel_bytes ? (float *)(c->ws + L.uvel + L.uvel_bytes) : nullptr;
    c->hrr_sigma = (float)d->hrr_sigma;

    LatticeArgs &a = c->a;
    memset(&a, 0, sizeof a);
    a.pdf = c->ws + L.pdf;
    a.mask = c->mask;
    a.nx = d->nx;
    a.ny = d->ny;
    a.nz = d->nz;
    const uint64_t ncell = (uint64_t)d->nx * d->ny * d->nz;
    a.nrows = (uint32_t)d->ny * (uint32_t)d->nz;
    a.sx = L.sx;
    a.sy = L.sy;
    a.et = d->streaming == LBM_STREAM_ET;
    c->sp.on = sp;
    c->sp.nf = (uint32_t)nf;
    c->sp.fmap = sp ? (const int32_t *)(c->ws + L.fmap) : nullptr;
    c->sp.nbt = sp ? (const uint32_t *)(c->ws + L.nbt) : nullptr;
    for (int k = 0; k < 3; ++k) a.per[k] = d->bc[2 * k] == LBM_BC_PERIODIC;
    a.any_vp = 0;
    for (int f = 0; f < 6; ++f) {
        // an interface face is a no-slip face for the lattice's own steps
        a.bc[f] = d->bc[f] == LBM_BC_INTERFACE ? LBM_BC_NOSLIP : d->bc[f];
        if (d->bc[f] == LBM_BC_VELOCITY || d->bc[f] == LBM_BC_PRESSURE) a.any_vp = 1;
        for (int k = 0; k < 3; ++k) a.ubc[f][k] = (float)d->u_bc[f][k];
        a.rhobc[f] = (float)d->rho_bc[f];
    }
    for (int k = 0; k < 3; ++k) a.F[k] = force ? (float)force[k] : 0.f;
    a.tau = (float)tau;
    a.magic = (float)d->magic;
    a.cs = (float)d->cs_smag;
    a.omp = (float)(1.0 / tau);
    a.omm = (float)(1.0 / (0.5 + d->magic / (tau - 0.5)));
    for (int k = 0; k < 5; ++k) a.mrt[k] = (float)d->mrt_rates[k];
    a.mlp = c->mlp;
    a.mlp_tab = (const uint32_t *)(c->ws + L.mlp_tab);
    c->mlp_tab = (uint32_t *)(c->ws + L.mlp_tab);
    a.fallbacks = c->fallbacks;

    c->nfluid = nf;
    // Solid lanes fill their own slots on odd steps where solids are sparse:
    // whole lines along solid surfaces for the solid cells' extra bytes
    // (measured: about -2% per step at 10% solid, +18% at 70%).
    c->sc_flags = (c->mask && !sp && !a.et && (double)(ncell - (uint64_t)nf) <= 0.2 * (double)ncell)
                      ? SC_SOLID_ODD | SC_MASK_RUNS
                      : 0;
    hipError_t e = hipMemsetAsync(c->fallbacks, 0, sizeof(unsigned long long), c->stream);
    if (e == hipSuccess && c->mask) {
        // stage the flags in a region that is still undefined and holds at
        // least n bytes: the population store, or the fluid map (sparse)
        uint8_t *stage = (uint8_t *)(sp ? c->ws + L.fmap : a.pdf);
        if (flags)
            e = hipMemcpyAsync(stage, flags, ncell, hipMemcpyHostToDevice, c->stream);
        else
            e = hipMemsetAsync(stage, 0, ncell, c->stream);
        if (e == hipSuccess) e = launch_build_mask(a, stencil, stage, c->mask, c->stream);
    }
    if (e == hipSuccess && sp) {
        // fluid index of every cell (row order) and the linear index of every
        // fluid cell; the neighbour table is built from them on the device
        int32_t *fmap = new (std::nothrow) int32_t[ncell];  // ncell < 2^32 with sparse addressing
        uint32_t *fcell = new (std::nothrow) uint32_t[nf > 0 ? nf : 1];
        if (!fmap || !fcell) {
            delete[] fmap;
            delete[] fcell;
            delete c;
            return fail(nullptr, LBM_ENOMEM, "out of host memory for the fluid map");
        }
        uint32_t k = 0;
        for (uint32_t cell = 0; cell < (uint32_t)ncell; ++cell) {
            if (flags && flags[cell]) {
                fmap[cell] = -1;
            } else {
                fmap[cell] = (int32_t)k;
                fcell[k++] = cell;
            }
        }
        e = hipMemcpyAsync(c->ws + L.fmap, fmap, (size_t)4 * ncell, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess && nf > 0)
            e = hipMemcpyAsync(c->ws + L.fcell, fcell, (size_t)4 * nf, hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess)
            e = launch_build_sparse_table(a, c->sp, stencil, (const uint32_t *)(c->ws + L.fcell), (uint32_t *)(c->ws + L.nbt),
                                          c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);  // before the host arrays go
        delete[] fmap;
        delete[] fcell;
    }
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        hip_fail(nullptr, e, "lbm_create");
        delete c;
        return LBM_EDEVICE;
    }
    *out = c;
    return LBM_OK;
}

int lbm_destroy(lbm_ctx *ctx)
{
    delete ctx;
    return LBM_OK;
}

const char *lbm_last_error(const lbm_ctx *ctx) { return ctx ? ctx->err : g_err; }

// HRR: the velocity field of the initial state (the finite-difference
// gradient's input on the first step) into uvel[0] and uvel[1]; the moments
// kernel's density output goes to uvel[1] first (it holds 3 n floats).
static int hrr_fill_velocity(lbm_ctx *c)
{
    if (c->coll != LBM_COLL_HRR) return LBM_OK;
    HIPCHECK(c, launch_moments(c->a, c->sp, c->q, c->st, 0, c->uvel[1], c->uvel[0], c->stream), "hrr velocity");
    HIPCHECK(c, hipMemcpyAsync(c->uvel[1], c->uvel[0], (size_t)12 * cells(c->a), hipMemcpyDeviceToDevice, c->stream),
             "hrr velocity copy");
    return LBM_OK;
}

int lbm_init_equilibrium(lbm_ctx *c, const double *rho_dev, const double *u_dev)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "context is NULL");
    if (!rho_dev || !u_dev) return fail(c, LBM_EINVAL, "rho/u is NULL");
    HIPCHECK(c, launch_init_eq(c->a, c->sp, c->q, c->st, rho_dev, u_dev, c->stream), "init_equilibrium");
    c->time = 0;
    return hrr_fill_velocity(c);
}

int lbm_set_pdfs(lbm_ctx *c, const double *f_dev)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "context is NULL");
    if (!f_dev) return fail(c, LBM_EINVAL, "f is NULL");
    HIPCHECK(c, launch_set_pdfs(c->a, c->sp, c->q, c->st, f_dev, c->stream), "set_pdfs");
    c->time = 0;
    return hrr_fill_velocity(c);
}

int lbm_get_pdfs(lbm_ctx *c, double *f_dev)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "context is NULL");
    if (!f_dev) return fail(c, LBM_EINVAL, "f is NULL");
    HIPCHECK(c, launch_get_pdfs(c->a, c->sp, c->q, c->st, (int)(c->time & 1), f_dev, c->stream), "get_pdfs");
    return LBM_OK;
}

int lbm_gather_pdfs(lbm_ctx *c, const int64_t *cells_dev, int64_t n, double *out_dev)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "context is NULL");
    if (n < 0) return fail(c, LBM_EINVAL, "n must be >= 0");
    if (n > 0 && (!cells_dev || !out_dev)) return fail(c, LBM_EINVAL, "cells/out is NULL");
    HIPCHECK(c, launch_gather(c->a, c->sp, c->q, c->st, (int)(c->time & 1), cells_dev, n, out_dev, c->stream), "gather");
    return LBM_OK;
}

static HrrArgs hrr_args(const lbm_ctx *c, int odd)
{
    HrrArgs h;
    h.uprev = c->uvel[odd];
    h.unext = c->uvel[odd ^ 1];
    h.sigma = c->hrr_sigma;
    return h;
}

static int step_once(lbm_ctx *c)
{
    const int odd = (int)(c->time & 1);
    hipError_t e = c->sp.on  ? launch_step_sparse(c->a, c->sp, c->q, c->st, c->cl, c->coll, odd, c->stream)
                   : c->a.et ? launch_step_et(c->a, c->q, c->st, c->cl, c->coll, odd, c->stream)
                             : launch_step(c->a, hrr_args(c, odd), c->q, c->st, c->cl, c->coll, odd | c->sc_flags,
                                           c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "stream_collide launch");
    ++c->time;
    return LBM_OK;
}

int lbm_step(lbm_ctx *c, int64_t n)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "context is NULL");
    if (n < 0) return fail(c, LBM_EINVAL, "step count must be >= 0 (got %lld)", (long long)n);
    if (c->cl == LBM_LES_MLP && !c->mlp_ready)
        return fail(c, LBM_ESTATE, "MLP closure selected but lbm_set_closure_weights was not called");
    for (int64_t k = 0; k < n; ++k) {
        const int rc = step_once(c);
        if (rc) return rc;
    }
    return LBM_OK;
}

int64_t lbm_time(const lbm_ctx *c) { return c ? c->time : -1; }

int lbm_moments(lbm_ctx *c, float *rho_dev, float *u_dev)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "context is NULL");
    if (!rho_dev || !u_dev) return fail(c, LBM_EINVAL, "rho/u is NULL");
    HIPCHECK(c, launch_moments(c->a, c->sp, c->q, c->st, (int)(c->time & 1), rho_dev, u_dev, c->stream), "moments");
    return LBM_OK;
}

int lbm_totals(lbm_ctx *c, double *mass, double mom[3])
{
    if (!c) return fail(nullptr, LBM_EINVAL, "context is NULL");
    if (!mass || !mom) return fail(c, LBM_EINVAL, "mass/mom is NULL");
    HIPCHECK(c, launch_totals(c->a, c->sp, c->q, c->st, (int)(c->time & 1), c->partial, c->final_out, c->stream),
             "totals");
    double h[5];
    HIPCHECK(c, hipMemcpyAsync(h, c->final_out, sizeof h, hipMemcpyDeviceToHost, c->stream), "totals copy");
    HIPCHECK(c, hipStreamSynchronize(c->stream), "totals sync");
    *mass = (double)c->nfluid + h[0];
    mom[0] = h[1];
    mom[1] = h[2];
    mom[2] = h[3];
    if (h[4] != 0.0 || !isfinite(h[0]) || !isfinite(h[1]) || !isfinite(h[2]) || !isfinite(h[3]))
        return fail(c, LBM_ENONFINITE, "non-finite populations in %.0f fluid cells", h[4]);
    return LBM_OK;
}

int lbm_state_bytes(const lbm_ctx *c, size_t *out)
{
    if (!c || !out) return fail(nullptr, LBM_EINVAL, "context/out is NULL");
    *out = c->state_bytes;
    return LBM_OK;
}

int lbm_save_state(lbm_ctx *c, void *dst_dev, int64_t *time)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "context is NULL");
    if (!dst_dev || !time) return fail(c, LBM_EINVAL, "dst/time is NULL");
    HIPCHECK(c, hipMemcpyAsync(dst_dev, c->a.pdf, c->state_bytes, hipMemcpyDeviceToDevice, c->stream), "save_state");
    *time = c->time;
    return LBM_OK;
}

int lbm_load_state(lbm_ctx *c, const void *src_dev, int64_t time)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "context is NULL");
    if (!src_dev || time < 0) return fail(c, LBM_EINVAL, "src is NULL or time < 0");
    HIPCHECK(c, hipMemcpyAsync(c->a.pdf, src_dev, c->state_bytes, hipMemcpyDeviceToDevice, c->stream), "load_state");
    c->time = time;
    return LBM_OK;
}

int lbm_set_closure_weights(lbm_ctx *c, const float *params, size_t n)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "context is NULL");
    if (!params || n != (size_t)(MLP_NPARAM + MLP_NNORM))
        return fail(c, LBM_EINVAL, "closure weights: expected %d floats", MLP_NPARAM + MLP_NNORM);
    for (size_t k = 0; k < n; ++k)
        if (!isfinite(params[k])) return fail(c, LBM_EINVAL, "closure weight %zu is not finite", k);
    for (int k = 0; k < 6; ++k)
        if (!(params[MLP_NPARAM + 6 + k] > 0.f)) return fail(c, LBM_EINVAL, "sigma[%d] must be > 0", k);
    HIPCHECK(c, hipMemcpyAsync(c->mlp, params, n * sizeof(float), hipMemcpyHostToDevice, c->stream), "weights");
    HIPCHECK(c, launch_build_mlp_table(c->mlp, c->mlp_tab, c->stream), "weights table");
    HIPCHECK(c, hipStreamSynchronize(c->stream), "weights sync");
    c->mlp_ready = 1;
    return LBM_OK;
}

int lbm_closure_features(lbm_ctx *c, float *x_dev)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "context is NULL");
    if (!x_dev) return fail(c, LBM_EINVAL, "closure_features: x is NULL");
    HIPCHECK(c, launch_closure_features(c->a, c->sp, c->q, c->st, (int)(c->time & 1), x_dev, c->stream),
             "closure_features");
    return LBM_OK;
}

int lbm_closure_fallbacks(lbm_ctx *c, int64_t *count)
{
    if (!c || !count) return fail(c, LBM_EINVAL, "context/count is NULL");
    unsigned long long h = 0;
    HIPCHECK(c, hipMemcpyAsync(&h, c->fallbacks, sizeof h, hipMemcpyDeviceToHost, c->stream), "fallbacks copy");
    HIPCHECK(c, hipStreamSynchronize(c->stream), "fallbacks sync");
    HIPCHECK(c, hipMemsetAsync(c->fallbacks, 0, sizeof h, c->stream), "fallbacks reset");
    *count = (int64_t)h;
    return LBM_OK;
}

int lbm_box_filter4(int32_t nx, int32_t ny, int32_t nz, const float *rho_dev, const float *u_dev, float *out_dev,
                    void *stream)
{
    if (nx < 4 || ny < 4 || nz < 4 || nx % 4 || ny % 4 || nz % 4)
        return fail(nullptr, LBM_EINVAL, "box filter: sizes must be positive multiples of 4");
    if ((uint64_t)nx * ny * nz >= (1ull << 31)) return fail(nullptr, LBM_ENOMEM, "box filter: too many cells");
    if (!rho_dev || !u_dev || !out_dev) return fail(nullptr, LBM_EINVAL, "box filter: NULL pointer");
    hipError_t e = launch_box_filter4(nx, ny, nz, rho_dev, u_dev, out_dev, (hipStream_t)stream);
    return e == hipSuccess ? LBM_OK : hip_fail(nullptr, e, "box_filter4");
}

int lbm_closure_dataset(int32_t cx, int32_t cy, int32_t cz, const int32_t periodic[3], const float *filt_dev,
                        double tau, double cs, float *x_dev, float *t_dev, void *stream)
{
    if (cx < 1 || cy < 1 || cz < 1) return fail(nullptr, LBM_EINVAL, "dataset: sizes must be >= 1");
    if ((uint64_t)cx * cy * cz >= (1ull << 31)) return fail(nullptr, LBM_ENOMEM, "dataset: too many cells");
    if (!periodic || !filt_dev || !x_dev || !t_dev) return fail(nullptr, LBM_EINVAL, "dataset: NULL pointer");
    if (!(tau > 0.5) || !(cs >= 0.0)) return fail(nullptr, LBM_EINVAL, "dataset: tau must be > 1/2, cs >= 0");
    int per[3] = {periodic[0] != 0, periodic[1] != 0, periodic[2] != 0};
    hipError_t e = launch_closure_dataset(cx, cy, cz, per, filt_dev, (float)tau, (float)cs, x_dev, t_dev,
                                          (hipStream_t)stream);
    return e == hipSuccess ? LBM_OK : hip_fail(nullptr, e, "closure_dataset");
}

int lbm_mlp_forward(const float *params_dev, const float *x_dev, int64_t n, float *y_dev, void *stream)
{
    if (n < 0) return fail(nullptr, LBM_EINVAL, "mlp_forward: n must be >= 0");
    if (n > 0 && (!params_dev || !x_dev || !y_dev)) return fail(nullptr, LBM_EINVAL, "mlp_forward: NULL pointer");
    hipError_t e = launch_mlp_forward(params_dev, x_dev, n, y_dev, (hipStream_t)stream);
    return e == hipSuccess ? LBM_OK : hip_fail(nullptr, e, "mlp_forward");
}

size_t lbm_mlp_work_bytes(int64_t n) { return mlp_work_bytes(n < 0 ? 0 : n); }

int lbm_mlp_loss_grad(const float *params_dev, const float *x_dev, const float *t_dev, int64_t n, float *grad_dev,
                      float *loss_dev, void *work_dev, void *stream)
{
    if (n < 1) return fail(nullptr, LBM_EINVAL, "mlp_loss_grad: n must be >= 1");
    if (!params_dev || !x_dev || !t_dev || !grad_dev || !loss_dev || !work_dev)
        return fail(nullptr, LBM_EINVAL, "mlp_loss_grad: NULL pointer");
    hipError_t e = launch_mlp_loss_grad(params_dev, x_dev, t_dev, n, grad_dev, loss_dev, work_dev, (hipStream_t)stream);
    return e == hipSuccess ? LBM_OK : hip_fail(nullptr, e, "mlp_loss_grad");
}

int lbm_mlp_loss_grad_noalloc(const float *params_dev, const float *x_dev, const float *t_dev, int64_t n,
                              float *grad_dev, float *loss_dev, void *stream)
{
    if (n < 1) return fail(nullptr, LBM_EINVAL, "mlp_loss_grad_noalloc: n must be >= 1");
    if (!params_dev || !x_dev || !t_dev || !grad_dev || !loss_dev)
        return fail(nullptr, LBM_EINVAL, "mlp_loss_grad_noalloc: NULL pointer");
    if (mlp_work_bytes(n) > mlp_noalloc_scratch_bytes())
        return fail(nullptr, LBM_EINVAL,
                    "mlp_loss_grad_noalloc: the partials of %lld samples need %zu bytes, more than the %zu-byte "
                    "static scratch",
                    (long long)n, mlp_work_bytes(n), mlp_noalloc_scratch_bytes());
    hipError_t e = launch_mlp_loss_grad_noalloc(params_dev, x_dev, t_dev, n, grad_dev, loss_dev, (hipStream_t)stream);
    return e == hipSuccess ? LBM_OK : hip_fail(nullptr, e, "mlp_loss_grad_noalloc");
}

int lbm_mlp_adam(float *params_dev, const float *grad_dev, float *m_dev, float *v_dev, int64_t step, double lr,
                 double beta1, double beta2, double eps, void *stream)
{
    if (!params_dev || !grad_dev || !m_dev || !v_dev) return fail(nullptr, LBM_EINVAL, "mlp_adam: NULL pointer");
    if (step < 1) return fail(nullptr, LBM_EINVAL, "mlp_adam: step is 1-based");
    hipError_t e = launch_mlp_adam(params_dev, grad_dev, m_dev, v_dev, step, (float)lr, (float)beta1, (float)beta2,
                                   (float)eps, (hipStream_t)stream);
    return e == hipSuccess ? LBM_OK : hip_fail(nullptr, e, "mlp_adam");
}

int lbm_stream_copy(const void *src_dev, void *dst_dev, size_t bytes, void *stream)
{
    if (!src_dev || !dst_dev) return fail(nullptr, LBM_EINVAL, "copy: NULL pointer");
    if (bytes % 16) return fail(nullptr, LBM_EINVAL, "copy: bytes must be a multiple of 16");
    if (((uintptr_t)src_dev | (uintptr_t)dst_dev) & 15)
        return fail(nullptr, LBM_EINVAL, "copy: src and dst must be 16-byte aligned");
    hipError_t e = launch_copy(src_dev, dst_dev, bytes, (hipStream_t)stream);
    return e == hipSuccess ? LBM_OK : hip_fail(nullptr, e, "stream_copy");
}

// ---------------------------------------------------------------------------
// 2:1 grid refinement
// ---------------------------------------------------------------------------
static size_t refine_plane_floats(int q, int64_t nx, int64_t nz) { return (size_t)q * (size_t)nx * (size_t)nz; }

int lbm_refine_work_bytes(const lbm_domain *d, int stencil, size_t *bytes)
{
    if (!d || !bytes) return fail(nullptr, LBM_EINVAL, "refine_work_bytes: NULL pointer");
    if (stencil != 19 && stencil != 27) return fail(nullptr, LBM_EINVAL, "stencil must be 19 or 27, got %d", stencil);
    if (d->nx < 1 || d->nz < 1) return fail(nullptr, LBM_EINVAL, "domain sizes must be >= 1");
    *bytes = 2 * refine_plane_floats(stencil, d->nx, d->nz) * sizeof(float);
    return LBM_OK;
}

static bool rel_close(double a, double b) { return fabs(a - b) <= 1e-9 * fmax(fabs(a), fabs(b)) + 1e-300; }

// Does node kf fit below (above = 0) or above (above = 1) node kc as its
// 2:1 finer level?  Failures are reported on the root context.
static int refine_check(lbm_ctx *root, int kc, const lbm_ctx *c, int kf, const lbm_ctx *f, int above)
{
    const char *side = above ? "above" : "below";
    if (f == c) return fail(root, LBM_EINVAL, "refine: node %d is its own child", kc);
    if (f->q != c->q) return fail(root, LBM_EINVAL, "refine: node %d (%s node %d) has another stencil", kf, side, kc);
    if (f->a.nx != 2 * c->a.nx || f->a.nz != 2 * c->a.nz)
        return fail(root, LBM_EINVAL, "refine: node %d (%s node %d) must have twice its nx and nz (%d x %d, coarse %d x %d)",
                    kf, side, kc, f->a.nx, f->a.nz, c->a.nx, c->a.nz);
    if (f->bc_kind[above ? 2 : 3] != LBM_BC_INTERFACE)
        return fail(root, LBM_EINVAL, "refine: the %s face of node %d facing node %d is not an interface",
                    above ? "-y" : "+y", kf, kc);
    if (f->coll != c->coll) return fail(root, LBM_EINVAL, "refine: node %d has another collision than node %d", kf, kc);
    if (f->magic_d != c->magic_d)
        return fail(root, LBM_EINVAL, "refine: node %d has another magic parameter than node %d", kf, kc);
    if (c->coll == LBM_COLL_MRT)
        for (int k = 0; k < 5; ++k)
            if (f->mrt_d[k] != c->mrt_d[k])
                return fail(root, LBM_EINVAL, "refine: node %d has other MRT ghost rates than node %d", kf, kc);
    if (!rel_close(f->tau_d, 0.5 + 2.0 * (c->tau_d - 0.5)))
        return fail(root, LBM_EINVAL, "refine: node %d needs tau = 1/2 + 2 (tau_c - 1/2) = %.17g (got %.17g)", kf,
                    0.5 + 2.0 * (c->tau_d - 0.5), f->tau_d);
    for (int k = 0; k < 3; ++k)
        if (!(rel_close(f->force_d[k], 0.5 * c->force_d[k]) || (f->force_d[k] == 0.0 && c->force_d[k] == 0.0)))
            return fail(root, LBM_EINVAL, "refine: node %d needs force = force of node %d / 2", kf, kc);
    if (f->stream != c->stream) return fail(root, LBM_EINVAL, "refine: node %d runs on another stream", kf);
    return LBM_OK;
}

// Advance node k one step: its own step, then per child two child steps
// (recursively), each followed by the exchange across their interface; the
// second exchange also fills node k's interface row toward that child.
static int refine_advance(const lbm_refine_node *nodes, int k)
{
    lbm_ctx *c = nodes[k].ctx;
    int rc = step_once(c);
    if (rc) return rc;
    const size_t plane = refine_plane_floats(c->q, c->a.nx, c->a.nz);
    const int child[2] = {nodes[k].fine_lo, nodes[k].fine_hi};
    for (int side = 0; side < 2; ++side) {
        if (child[side] < 0) continue;
        lbm_ctx *f = nodes[child[side]].ctx;
        const int dy = side ? 1 : -1, yc = side ? c->a.ny - 1 : 0, yf = side ? 0 : f->a.ny - 1;
        float *acc = (float *)nodes[k].work_dev + (size_t)side * plane;
        for (int sub = 0; sub < 2; ++sub) {
            if ((rc = refine_advance(nodes, child[side]))) return rc;
            HIPCHECK(c, launch_refine_exchange(c->a, c->st, yc, f->a, c->q, f->st, yf, dy, sub, acc, c->stream),
                     "refine exchange");
        }
    }
    return LBM_OK;
}

static int refine_tree_step(const lbm_refine_node *nodes, int32_t count, int64_t n)
{
    if (!nodes || count < 1 || count > 4096) return fail(nullptr, LBM_EINVAL, "refine: need 1 to 4096 nodes");
    for (int k = 0; k < count; ++k)
        if (!nodes[k].ctx) return fail(nullptr, LBM_EINVAL, "refine: node %d has no context", k);
    lbm_ctx *root = nodes[0].ctx;
    if (n < 0) return fail(root, LBM_EINVAL, "refine: step count must be >= 0");
    std::vector<int> parents(count, 0), up(count, 0);  // face toward the parent (2 or 3), 0 for none
    for (int k = 0; k < count; ++k) {
        lbm_ctx *c = nodes[k].ctx;
        if (!c->a.per[0] || !c->a.per[2]) return fail(root, LBM_EINVAL, "refine: x and z must be periodic on node %d", k);
        if (c->sp.on || c->a.et) return fail(root, LBM_EINVAL, "refine: node %d must use the dense AA pattern", k);
        if (c->cl != LBM_LES_NONE) return fail(root, LBM_EINVAL, "refine: node %d has a closure", k);
        if (c->coll == LBM_COLL_HRR) return fail(root, LBM_EINVAL, "refine: HRR is not supported");
        const int child[2] = {nodes[k].fine_lo, nodes[k].fine_hi};
        for (int side = 0; side < 2; ++side) {
            if (child[side] < 0) continue;
            if (child[side] <= k || child[side] >= count)
                return fail(root, LBM_EINVAL, "refine: child %d of node %d must come after it", child[side], k);
            ++parents[child[side]];
            up[child[side]] = side ? 2 : 3;  // a lower child meets its parent with its +y face
            const int rc = refine_check(root, k, c, child[side], nodes[child[side]].ctx, side);
            if (rc) return rc;
        }
        if (child[0] >= 0 || child[1] >= 0) {
            const size_t need = 2 * refine_plane_floats(c->q, c->a.nx, c->a.nz) * sizeof(float);
            if (!nodes[k].work_dev || ((uintptr_t)nodes[k].work_dev & 3) != 0)
                return fail(root, LBM_EINVAL, "refine: node %d needs a 4-byte aligned work buffer", k);
            if (nodes[k].work_bytes < need)
                return fail(root, LBM_EINVAL, "refine: node %d work buffer too small: %zu < %zu bytes", k,
                            nodes[k].work_bytes, need);
        }
    }
    for (int k = 1; k < count; ++k)
        if (parents[k] != 1) return fail(root, LBM_EINVAL, "refine: node %d has %d parents", k, parents[k]);
    // a parent's sums live from its child's first substep to the second, across
    // the child's own exchanges: the work buffers must not overlap
    std::vector<std::pair<uintptr_t, int>> ws;
    for (int k = 0; k < count; ++k)
        if (nodes[k].fine_lo >= 0 || nodes[k].fine_hi >= 0) ws.push_back({(uintptr_t)nodes[k].work_dev, k});
    std::sort(ws.begin(), ws.end());
    for (size_t j = 1; j < ws.size(); ++j) {
        const lbm_ctx *c = nodes[ws[j - 1].second].ctx;
        const uintptr_t end = ws[j - 1].first + 2 * refine_plane_floats(c->q, c->a.nx, c->a.nz) * sizeof(float);
        if (ws[j].first < end)
            return fail(root, LBM_EINVAL, "refine: the work buffers of nodes %d and %d overlap", ws[j - 1].second,
                        ws[j].second);
    }
    for (int k = 0; k < count; ++k) {
        const int child[2] = {nodes[k].fine_lo, nodes[k].fine_hi};
        for (int side = 0; side < 2; ++side) {
            const int face = side ? 3 : 2;
            const bool has = child[side] >= 0, toward = up[k] == face;
            if (has && toward) return fail(root, LBM_EINVAL, "refine: node %d has a child on its parent's side", k);
            if ((nodes[k].ctx->bc_kind[face] == LBM_BC_INTERFACE) != (has || toward))
                return fail(root, LBM_EINVAL, "refine: node %d: a y face is an interface exactly where it meets another level",
                            k);
        }
    }
    for (int64_t t = 0; t < n; ++t) {
        const int rc = refine_advance(nodes, 0);
        if (rc) return rc;
    }
    return LBM_OK;
}

int lbm_refine_tree_step(const lbm_refine_node *nodes, int32_t count, int64_t n)
{
    try {  // the validation's small host arrays
        return refine_tree_step(nodes, count, n);
    } catch (const std::bad_alloc &) {
        return fail(nodes && count > 0 ? nodes[0].ctx : nullptr, LBM_ENOMEM, "refine: out of host memory");
    }
}

int lbm_refine_step(lbm_ctx *c, lbm_ctx *lo, lbm_ctx *hi, void *work_dev, size_t work_bytes, int64_t n)
{
    if (!c) return fail(nullptr, LBM_EINVAL, "refine: coarse context is NULL");
    if (!lo && !hi) return fail(c, LBM_EINVAL, "refine: no fine lattice");
    if (lo && hi && lo == hi) return fail(c, LBM_EINVAL, "refine: fine_lo and fine_hi are the same lattice");
    if (!work_dev) return fail(c, LBM_EINVAL, "refine: work buffer is NULL");
    lbm_refine_node nodes[3];
    int count = 1;
    nodes[0] = {c, -1, -1, work_dev, work_bytes};
    if (lo) {
        nodes[count] = {lo, -1, -1, nullptr, 0};
        nodes[0].fine_lo = count++;
    }
    if (hi) {
        nodes[count] = {hi, -1, -1, nullptr, 0};
        nodes[0].fine_hi = count++;
    }
    return lbm_refine_tree_step(nodes, count, n);
}

}  // extern "C"
