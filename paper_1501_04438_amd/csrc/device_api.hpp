// device_api.hpp -- host-side entry points of the device code (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <vector>

namespace gsk {

struct DipoleArgs;

// Everything one evaluation needs.  Device pointers; X1 holds (n+1) n^(d-1)
// complex values, X2 (3D only) 2 n^2 (n+1).
struct EvalArgs {
    int d = 3, n = 0;
    const double* rho = nullptr;
    double* u = nullptr;
    double2* X1 = nullptr;
    double2* X2 = nullptr;
    const double* spec = nullptr;     // octant (n+1)^d, 1/M folded in
    const double2* tw = nullptr;      // exp(-i pi m / n), m < 2n
    int dipolar = 0;
    double dxi[3] = {0, 0, 0};        // pi / (2 L_j) of the x, y, z axes
    double cdiag[3] = {0, 0, 0};
    double ccross[3] = {0, 0, 0};
    double nm_over_M = 0.0;
    int max_blocks_fused = 0;         // persistent grid size of the 3D fused pass (0 = device fill)
    int kx0 = 0, kxn = 0;             // 3D passes 2-4: the kx slab [kx0, kx0 + kxn); X2 holds the slab
    // Launch variants (none changes a single bit of the result): bit p-1 clear selects
    // plain (cached) memory accesses for pass p instead of its cache-hint default;
    // fused_grid_mult = rounds of co-resident blocks in the persistent fused pass (3D; the 2D
    // fused pass runs one block per pencil group).
    int hint_bits = 27;
    int fused_grid_mult = 4;
    // Tile shapes of the cubic passes (bits 0-1 x passes, 2-3 y passes, 4-5 fused pass; 0 =
    // compiled defaults; see eval_instance.hip); the same bits for every value.
    int tile_bits = 0;
    // Energy (when energy != nullptr): E = escale * sum_i rho_i u_i, summed in the fused pass
    // by Parseval's identity, one partial per pencil in epart (epencils of them, then room for
    // energy_total_scratch() more), their fixed-order total written to *energy after pass 5.
    double* energy = nullptr;
    double* epart = nullptr;
    int epencils = 0;
    double escale = 0.0;
    double oscale = 1.0;              // with the energy: the outputs are stored times oscale
    // Grids whose axes have their own n (rectangular grids): the extents of the x, y, z axes
    // (n above is unused unless nx = ny (= nz) = n) and each axis' twiddle table.
    int nx = 0, ny = 0, nz = 0;
    const double2* twx = nullptr;
    const double2* twy = nullptr;
    const double2* twz = nullptr;
    // Padding 3 (host side only): the passes run on the transform grid's copy E (rho = u =
    // E); the caller's density pad_in (px, py, pz points) is copied into E before the first
    // step and the potential out to pad_out after the last.
    const double* pad_in = nullptr;
    double* pad_out = nullptr;
    int px = 0, py = 0, pz = 0;
    // Padding 3 on a cubic transform grid: no copies; the x-forward pass reads the density rho
    // (px, py, pz points) in place and the x-inverse pass writes the potential u at those
    // points only.
    int emb = 0;
};

// The density (nx, ny, nz points, x fastest) into the first points of each axis of a grid
// of (Nx, Ny, Nz) points, zeros at the others; and those points of such a grid back out.
hipError_t launch_pad_embed(const double* rho, double* E, int nx, int ny, int nz, int Nx, int Ny, int Nz,
                            hipStream_t s);
hipError_t launch_pad_crop(const double* E, double* u, int nx, int ny, int nz, int Nx, int Ny, int Nz,
                           hipStream_t s);

// Pencils of the fused pass (one energy partial sum each) of an (nx, ny, .) transform grid:
// 3D (nx + 1) 2 ny, 2D nx + 1.
int energy_pencils(int d, int nx, int ny);
// Doubles the energy total needs after the partials (its first-stage sums).
int energy_total_scratch();
// energy[0] = scale * (part[0] + ... + part[count-1]) in a fixed order (one block).
hipError_t launch_energy_finish(const double* part, int count, double scale, double* energy, hipStream_t s);
// The same total for any count: chunk sums into part[count ..] first when count is large.
hipError_t launch_energy_total(double* part, int count, double scale, double* energy, hipStream_t s);

// Passes: 1 x_r2c, 2 y_fwd, 3 fused, 4 y_inv, 5 x_c2r.  `which` < 0 runs all five on the
// slab given in the arguments (a whole evaluation when the slab covers kx = 0..n).  A grid
// whose extents nx, ny (, nz) differ runs each pass at the length of the axis it transforms.
hipError_t launch_eval(const EvalArgs& a, hipStream_t s, int which = -1);
bool eval_size_supported(int d, int n);
// Tile variants compiled for length n: bit 0 x double, 1 y half, 2 y double, 3 fused half,
// 4 fused double.
int tile_variants(int n);
int eval_sizes(int d, long long* out, int cap);

// Octant indices (k1, k2, k3) = (kx, ky, kz) in 3D and (k1, k3) = (kx, ky) in 2D.
struct AssemblyArgs {
    int d = 3, n1 = 0, Qp = 0, ldk = 0;
    int n1b = 0, n1c = 0;             // extents of k2, k3 (0: n1, a cubic octant)
    const double* AT = nullptr;       // [Qp][ldk]: w_q F_x[k][q]
    const double* FB = nullptr;       // [Qp][ldk]: F_y[k][q] (3D)
    const double* FC = nullptr;       // [Qp][ldk]: F_z[k][q] (3D), F_y[k][q] (2D)
    double* out = nullptr;
    double A0 = 0, c2 = 0, invM = 0;
    double dxi[3] = {0, 0, 0};        // pi / (2 L) of the axes of k1, k2, k3 (2D: k1, -, k3)
    int dxx = 0;                      // multiply by -xi_k1^2 (the d_xx symbol)
    int lapu = 0;                     // 0, or the padding factor: Laplacian on the density's own grid (assembly.hpp)
};
// Row blocks per wave chosen for n1; returns the padded k length the operands need.
int assembly_ldk(int n1);
hipError_t launch_assembly(const AssemblyArgs& a, hipStream_t s);
hipError_t load_assembly(const AssemblyArgs& a);   // loads the kernel's code object (no launch)

// Batched evaluation of independent problems (sizes up to 128, batch.hpp).
struct BatchMember {
    int d = 3, n = 0, dipolar = 0;
    const double* rho = nullptr;
    double* u = nullptr;
    double2* X1 = nullptr;
    double2* X2 = nullptr;
    const double* spec = nullptr;
    const double2* tw = nullptr;
    double dxi[3] = {0, 0, 0}, cdiag[3] = {0, 0, 0}, ccross[3] = {0, 0, 0}, nm_over_M = 0.0;
};
bool batch_size_supported(int d, int n);
// packed device descriptors of the members (copy to device memory as is)
void batch_problems(const std::vector<BatchMember>& m, std::vector<unsigned char>& out);
constexpr int BATCH_TASK_INTS = 6;
// Pass-major task list; mult = block-fulls of tiles per task; largest_first orders the
// members of each pass by size.  pass_off/pass_cnt: the tasks of pass p (index p).
void batch_tasks(const std::vector<BatchMember>& m, int mult, bool largest_first, std::vector<int>& tasks,
                 int pass_off[6], int pass_cnt[6]);
// unsigned counters of the queue schedule (start zeroed); the error flag is the word after them
int batch_counters(int nprob);
int batch_resident_blocks();              // co-resident blocks of the batch kernels on this device
// Queue schedule: nq task queues (tasks qoff[q] .. qoff[q+1]-1 of a concatenated list),
// qmap[hardware die id] = queue or -1; local = every problem's tasks in one queue
// served only by blocks on one die.
struct BatchQueueSpec {
    int nq = 1, local = 0;
    int qmap[16] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    std::vector<int> qoff = {0, 0};
};
// Per-queue pass-major task lists: members dealt to nq queues by decreasing work,
// each to the least loaded queue.
void batch_queue_tasks(const std::vector<BatchMember>& m, int mult, int nq, std::vector<int>& tasks,
                       std::vector<int>& qoff);
// Hardware ids of the dies (XCDs) blocks run on, sorted; probed once per device.
int batch_xcc_ids(int* ids, int cap);
// spin_limit: polls after which a dependency wait raises the error flag and goes on
hipError_t launch_batch_queue(const void* probs, const void* tasks, const BatchQueueSpec& spec, unsigned* ctr,
                              int nctr, int grid, unsigned spin_limit, hipStream_t s);
hipError_t launch_batch_phased(const void* probs, const void* tasks, const int pass_off[6], const int pass_cnt[6],
                               int grid, hipStream_t s);

// Phased-by-size schedule: (pass, n, first task, count) runs of a task list whose
// tasks of one pass are grouped by size (largest_first), one launch per run.
void batch_size_runs(const std::vector<BatchMember>& m, const std::vector<int>& tasks, std::vector<int>& runs);
hipError_t launch_batch_sized(const void* probs, const void* tasks, const std::vector<int>& runs, hipStream_t s);

}  // namespace gsk
