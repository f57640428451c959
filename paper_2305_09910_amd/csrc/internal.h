// internal.h -- launch interface between the C ABI (lbm_api.cpp) and the
// HIP kernels (lbm_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

enum { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2 };
enum { CL_NONE = 0, CL_SMAG = 1, CL_MLP = 2 };
enum { COLL_TRT = 0, COLL_MRT = 1, COLL_HRR = 2 };

// launch_step's `odd` argument: bit 0 the step parity; SC_SOLID_ODD asks the
// masked AA kernel to fill solid cells' own slots on odd steps (whole
// cache lines along solid surfaces; worth it when solids are sparse)
constexpr int SC_SOLID_ODD = 2;
// SC_MASK_RUNS: the masked AA kernel reads a cell's mask word only where the
// run word of its 64 cells is nonzero (sparse solids; with dense solids
// nearly every run is nonzero and the extra dependent load costs time)
constexpr int SC_MASK_RUNS = 4;
enum { BC_PERIODIC = 0, BC_NOSLIP = 1, BC_VELOCITY = 2, BC_PRESSURE = 3 };

// Bit 31 of a cell's mask word marks the cell itself as solid; bit i
// (1 <= i < q) marks the neighbour x + c_i (reached through periodic faces
// only) as solid.
constexpr uint32_t SELF_SOLID = 0x80000000u;

// Sparse addressing: fluid cells k = 0 .. nf-1 in row order, stored in
// chunks of 64 (one wavefront): population i of cell k at
// ((k / 64) q + i) 64 + k % 64, neighbour-table entry j (1 <= j < q) at
// ((k / 64) (q - 1) + j - 1) 64 + k % 64.  A table entry is the fluid index
// of the neighbour x + c_j, or NB_SOLID when that neighbour is solid, or
// NB_FACE0 + f when the link leaves through non-periodic face f (the face
// that decides the link's boundary condition).
constexpr int SP_CHUNK = 64;
constexpr uint32_t NB_FACE0 = 0xFFFFFFF0u;
constexpr uint32_t NB_SOLID = 0xFFFFFFFFu;

// MLP closure parameter block in device memory (FP32), see lbm.h.
constexpr int MLP_NPARAM = 1313;
constexpr int MLP_NNORM = 24;

// Everything a lattice kernel needs, passed by value.
struct LatticeArgs {
    void *pdf;               // [z][y][q][x] storage elements (deviations f_i - w_i)
    const uint32_t *mask;    // [n] or nullptr
    int nx, ny, nz;
    uint32_t nrows;          // cell rows ny * nz (< 2^32; the cell count nrows * nx is 64-bit)
    int sx, sy;              // cells per stored row and rows per stored plane: nx, ny, or one more
                             // for the ghost layer of the Esoteric Twist on a non-periodic + face
    int et;                  // streaming scheme: 0 AA pattern, 1 Esoteric Twist
    int per[3];              // axis periodic?
    int bc[6];               // face kinds
    int any_vp;              // any velocity / pressure face
    float ubc[6][3];
    float rhobc[6];
    float F[3];
    float tau, magic, cs;    // molecular tau, TRT magic, Smagorinsky constant
    float omp, omm;          // omega+ and omega- of the molecular tau
    float mrt[5];            // MRT ghost rates: energy, energy square, heat flux, fourth order, third order
    const float *mlp;        // closure parameters (device) or nullptr
    const uint32_t *mlp_tab; // per-lane operand table of the closure network (device)
    unsigned long long *fallbacks;  // MLP fallback counter (device) or nullptr
};

// cell count of a lattice
__host__ __device__ inline uint64_t cells(const LatticeArgs &a) { return (uint64_t)a.nrows * (uint32_t)a.nx; }
// After the n mask words: per cell row, one word per run of 64 cells along x,
// nonzero when a cell of the run has a nonzero mask word (a solid cell or a
// link cut by one), so that wavefronts far from solids skip the mask words.
__host__ __device__ inline uint32_t mask_runs(int nx) { return ((uint32_t)nx + 63u) >> 6; }

// Sparse addressing (the AA pattern over the fluid cells only), passed as an
// argument of its own to the kernels that use it: the dense step kernels keep
// exactly their argument block (its layout moves their compiled code).
struct SparseArgs {
    int on;                  // sparse addressing in use
    uint32_t nf;             // fluid cells
    const int32_t *fmap;     // [n] fluid index of each cell, -1 for solid cells
    const uint32_t *nbt;     // neighbour table [chunk][q - 1][64]
};

// Hybrid recursive regularised collision (D3Q19): the velocity fields of its
// finite-difference gradient, passed as a kernel argument of its own (after
// the others, so that the dense kernels' argument block keeps its layout).
// Step t reads the field of step t - 1 and writes its own.
struct HrrArgs {
    const float *uprev;  // [3][n] velocities of the previous step
    float *unext;        // [3][n] velocities of this step
    float sigma;         // weight of the projected non-equilibrium flux
};

struct Launch {
    dim3 grid, block;
};
Launch lattice_launch(const LatticeArgs &a);

// Kernel launchers (return hipError_t of the launch).
hipError_t launch_build_mask(const LatticeArgs &a, int q, const uint8_t *flags, uint32_t *mask, hipStream_t s);
// odd: bit 0 the step parity, optionally | SC_SOLID_ODD | SC_MASK_RUNS
hipError_t launch_step(const LatticeArgs &a, const HrrArgs &h, int q, int st, int cl, int coll, int odd, hipStream_t s);
// Esoteric Twist step (lbm_et.hip)
hipError_t launch_step_et(const LatticeArgs &a, int q, int st, int cl, int coll, int odd, hipStream_t s);
// sparse addressing (lbm_sparse.hip): neighbour table from the fluid map and
// the fluid cells' linear indices, and the step
hipError_t launch_build_sparse_table(const LatticeArgs &a, const SparseArgs &sp, int q, const uint32_t *fcell,
                                     uint32_t *table, hipStream_t s);
hipError_t launch_step_sparse(const LatticeArgs &a, const SparseArgs &sp, int q, int st, int cl, int coll, int odd,
                              hipStream_t s);
// State kernels (any scheme).
hipError_t launch_init_eq(const LatticeArgs &a, const SparseArgs &sp, int q, int st, const double *rho,
                          const double *u, hipStream_t s);
hipError_t launch_set_pdfs(const LatticeArgs &a, const SparseArgs &sp, int q, int st, const double *f, hipStream_t s);
hipError_t launch_get_pdfs(const LatticeArgs &a, const SparseArgs &sp, int q, int st, int odd, double *f,
                           hipStream_t s);
hipError_t launch_gather(const LatticeArgs &a, const SparseArgs &sp, int q, int st, int odd, const int64_t *cells,
                         int64_t ncell, double *out, hipStream_t s);
hipError_t launch_moments(const LatticeArgs &a, const SparseArgs &sp, int q, int st, int odd, float *rho, float *u,
                          hipStream_t s);
// totals: partial[nblk][5] doubles then final[5] = {sum drho, jx, jy, jz, nonfinite-count}
int totals_blocks();
hipError_t launch_totals(const LatticeArgs &a, const SparseArgs &sp, int q, int st, int odd, double *partial,
                         double *final_out, hipStream_t s);
hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s);

// 2:1 refinement exchange after a fine step (lbm_refine.hip): coarse lattice c
// (storage sc, interface row yc), fine lattice f (storage sf, interface row
// yf), dy = +1 for f above c; acc [q][nz_c][nx_c] FP32
hipError_t launch_refine_exchange(const LatticeArgs &c, int sc, int yc, const LatticeArgs &f, int q, int sf, int yf,
                                  int dy, int last, float *acc, hipStream_t s);
// operand table of the closure network (63 x 64 words) from its parameters
hipError_t launch_build_mlp_table(const float *params, uint32_t *table, hipStream_t s);

// closure training path (lbm_closure.hip)
hipError_t launch_closure_features(const LatticeArgs &a, const SparseArgs &sp, int q, int st, int odd, float *x,
                                   hipStream_t s);
hipError_t launch_box_filter4(int nx, int ny, int nz, const float *rho, const float *u, float *out, hipStream_t s);
hipError_t launch_closure_dataset(int cx, int cy, int cz, const int *per, const float *filt, float tau, float cs,
                                  float *x, float *t, hipStream_t s);
hipError_t launch_mlp_forward(const float *params, const float *x, int64_t n, float *y, hipStream_t s);
size_t mlp_work_bytes(int64_t n);
hipError_t launch_mlp_loss_grad(const float *params, const float *x, const float *t, int64_t n, float *grad,
                                float *loss, void *work, hipStream_t s);
// the same with the partial gradients in the library's static scratch array
// instead of a caller workspace (hipErrorInvalidValue if they would not fit)
size_t mlp_noalloc_scratch_bytes();
hipError_t launch_mlp_loss_grad_noalloc(const float *params, const float *x, const float *t, int64_t n,
                                        float *grad, float *loss, hipStream_t s);
hipError_t launch_mlp_adam(float *p, const float *g, float *m, float *v, int64_t step, float lr, float b1, float b2,
                           float eps, hipStream_t s);

}  // namespace lbm
