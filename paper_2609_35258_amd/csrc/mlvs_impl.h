// Internal declarations shared by the host code and the HIP kernels of libmlvs.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace mlvs {

// Per-cell parameter block (double).  Written by the cell stage of each step.
enum {
    P_RHO = 0, P_U, P_V, P_T, P_QX, P_QY, P_TAU,
    P_A0, P_A1, P_A2, P_A3,          // compatibility-correction coefficients
    P_ALPHA, P_BETA,                 // phi_bar+ = alpha phi~ + beta phi_S
    P_NEG,                           // 1 if the corrected target had g < 0
    NPARAM = 16
};

// Per-cell raw moments of the stored g~, h~ (double): the eleven sums read by
// the cell stage, taken about the velocity shift (M_U0, M_V0).
enum { M_U0 = 11, M_V0 = 12, NMOM = 16 };

// Per-face raw moments of phi_bar_f written by the reconstruction stage, per
// (velocity chunk, face): the eleven sums (interior faces; boundary faces: [0]
// the outgoing mass flux), then the velocity shift (u0, v0) they are taken
// about -- the layout of the cell moments, so NFMOM = NMOM.
enum { NFMOM = NMOM };

// Per-face record written by the face-target stage and read by the update
// (double).  KIND: 0 interior, else the boundary kind; C1, C2: the weights of
// phi_bar_f and of the target (area included); RN..B3, E4..CKRT: the target in
// the evaluation form of the kernels; CORR: 1 if the compatibility factor
// applies; C8: 1 if it has the eight-moment terms.
enum {
    FP_KIND = 0, FP_ROW, FP_NX, FP_NY, FP_C1, FP_C2,
    FP_RN, FP_UX, FP_UY, FP_I2RT, FP_RT, FP_IRT, FP_XQX, FP_XQY,
    FP_B0, FP_B1, FP_B2, FP_B3, FP_CORR,
    FP_E4, FP_E5, FP_E6, FP_E7, FP_CKRT, FP_C8,   // eight-moment terms (see Eq in kernels.hip)
    NFP = 26
};

// One velocity space (a representative level or an interface level).
struct LevelDesc {
    int N;             // points
    int stride;        // row stride in elements (multiple of 64)
    int n_rows_state;  // cells on this level
    int pad;
    const double* xi_x;
    const double* xi_y;
    const double* w;
    const float* xy32;      // (xi_x, xi_y) pairs rounded to float (FP32 storage reads these)
    void* g;   void* h;     // state g~, h~           [cells][stride]
    void* fg;  void* fh;    // phi_bar+ of the step: [cells][stride] followed by the ghost
                            // rows (neighbours on other levels mapped onto this level)
    void* Fg;  void* Fh;    // face rows (flux)        [rows][stride]
    double Minv[16];        // inverse of the state-independent 4x4 mapping matrix
    double G6inv[36];       // nine-moment mapping: inverse of the 6x6 g matrix,
    double B36[18];         //   coupling of the g correction into the h moments,
    double H3inv[9];        //   inverse of the 3x3 h matrix
};

struct Phys {
    int D, K;
    double R, Pr, omega, mu_ref, T_ref, dt;
    int compat, face_compat, map_moments;
    int positivity;                 // 1: exponential fallback of distribution maps
    int mesh_kind;                  // 0 structured (van Leer per index direction), 1 unstructured
};

// Encoded neighbour: >= 0 same-level cell id; -1 none (boundary);
// <= -2: ghost row (-2 - v) in the cell's level.
struct CellGeom {
    double vol;
    double G[4];       // inverse of [t_i; t_j] (row-major)
    double dist[4];    // |x_n - x_c| for W, E, S, N (1 when absent)
    double inv_dist[4];  // 1 / dist
    // unstructured meshes (slot k = the cell's k-th edge):
    double lx[4], ly[4];    // least-squares gradient = sum_k (lx, ly)[k] (phi_k - phi_c) (0: no neighbour)
    double fox[4], foy[4];  // x_f - x_c of each face (0: no face)
    double eps2;            // Venkatakrishnan's eps^2
};

struct FaceItem {      // same-level interior face (R >= 0) or boundary face (R = -1 - bc id)
    int L, R, lev, row;  // boundary: L is the interior cell, normal points out of the domain
    double nx, ny, area, dLx, dLy, dRx, dRy;
};

struct BCDev {
    int kind, pad;
    double rho, u, v, T;
};

// CSR projection table dst <- src: for each dst point, entries (src index, fraction).
struct PairTable {
    const int* off;
    const int* idx;
    const double* frac;
};

struct XFaceItem {     // cross-level interior face
    int L, R, levA, levB, levI, rowA, rowB, scratch;   // scratch: row in levI's face rows
    PairTable IfromA, IfromB, AfromI, BfromI;
    double nx, ny, area, dLx, dLy, dRx, dRy;
};

struct GhostItem {     // neighbour n (on level src) mapped onto level dst
    int n, dst, row, pad;
    PairTable tab;     // dst <- src
};

struct RemapItem {     // cell moved from an old level to a new one
    int c, src_lev, src_slot, dst_lev, dst_slot, pad;
    PairTable tab;     // dst <- src (null off => identical spaces: copy)
};

// The persistent step's arguments, in device memory so that a captured
// launch reads the current level set's work lists and counts.
struct StepArgs {
    const LevelDesc* lvs;
    const GhostItem* ghosts;
    const FaceItem* faces;       // same-level interior faces, then boundary faces
    const XFaceItem* xfaces;
    const int* order;            // cells in traversal order
    const int* cell_lev;
    const int* cell_slot;
    const int* cell_nbr;
    const int* cell_frow;
    const CellGeom* geom;
    const BCDev* bcs;
    double* params;
    double* cmom;
    double* fpar;
    unsigned long long* neg;
    unsigned int* sync;          // [0] barrier arrivals (cleared before each launch), [1] sticky error flag
    int n_ghosts, n_faces, n_xfaces, n_cells;
};

// Launch wrappers (kernels.hip).  `S` selects float (32) or double (64) storage.
int variant_count();
// order: the cells in traversal order (a permutation of 0..n_cells-1)
hipError_t launch_cell_prep(int prec, hipStream_t st, const LevelDesc* lv, const int* cell_lev,
                            const int* cell_slot, const int* order, int n_cells, Phys ph, double* params,
                            const double* cmom, int CH, int var = 1);
hipError_t launch_raw_moments(int prec, hipStream_t st, const LevelDesc* lv, const int* cell_lev,
                              const int* cell_slot, int n_cells, const double* params, double* cmom, int CH,
                              int nch);
hipError_t launch_ghost(int prec, hipStream_t st, const LevelDesc* lv, const GhostItem* items, int n,
                        const int* cell_lev, const int* cell_slot, const double* params, Phys ph,
                        unsigned long long* neg);
hipError_t launch_face_rec(int prec, hipStream_t st, const LevelDesc* lv, const FaceItem* items, int n,
                           const int* cell_slot, const int* cell_nbr, const CellGeom* geom,
                           const double* params, Phys ph, double* fmom, int CH, int nch, int var = 1);
hipError_t launch_face_target(int prec, hipStream_t st, const LevelDesc* lv, const FaceItem* items, int n,
                              const BCDev* bcs, Phys ph, const double* fmom, double* fpar, int CH, int var = 1);
hipError_t launch_xface(int prec, hipStream_t st, const LevelDesc* lv, const XFaceItem* items, int n,
                        const int* cell_slot, const int* cell_nbr, const CellGeom* geom,
                        const double* params, Phys ph, unsigned long long* neg, int var = 1);
// The persistent step (one launch per time step over the work lists in A,
// preceded by a one-thread kernel that clears the barrier counter in sync):
// `var` 0 or 1 (one or two velocity points per lane and load batch).  The
// grid is the kernel's occupancy times the number of compute units.
int persistent_variant_count();
hipError_t launch_step_persistent(int prec, hipStream_t st, const StepArgs* A, unsigned int* sync, Phys ph, int var,
                                  int* grid_used);
// Fused forms for level sets that fit one velocity chunk: reconstruction +
// target in one wave per face; update + the next step's cell stage in one
// wave per cell.
hipError_t launch_face_full(int prec, hipStream_t st, const LevelDesc* lv, const FaceItem* items, int n,
                            const int* cell_slot, const int* cell_nbr, const CellGeom* geom, const double* params,
                            const BCDev* bcs, Phys ph, double* fpar, int var = 1);
hipError_t launch_update_cell(int prec, hipStream_t st, const LevelDesc* lv, const int* cell_lev,
                              const int* cell_slot, const int* order, int n_cells, const CellGeom* geom,
                              const int* cell_frow, const FaceItem* items, const double* fpar, double* params,
                              Phys ph, double* cmom, int var = 1);
hipError_t launch_update(int prec, hipStream_t st, const LevelDesc* lv, const int* cell_lev,
                         const int* cell_slot, const int* order, int n_cells, const CellGeom* geom,
                         const int* cell_frow, const FaceItem* items, const double* fpar, const double* params,
                         Phys ph, double* cmom, int CH, int nch, int var = 1);
hipError_t launch_init_eq(int prec, hipStream_t st, const LevelDesc* lv, const int* cell_lev,
                          const int* cell_slot, int n_cells, const double* rho_u_v_T, Phys ph,
                          double* params);
hipError_t launch_cell_moments(int prec, hipStream_t st, const LevelDesc* lv, const int* cell_lev,
                               const int* cell_slot, int n_cells, const CellGeom* geom, Phys ph,
                               double* out6, double* out_tot4, double* out8 = nullptr, double* out3 = nullptr);
hipError_t launch_sum_rows(hipStream_t st, const double* in, int n, int width, double* out);
// Strict-mode state check (rec[0] count of bad cells, rec[1] smallest bad cell;
// the caller clears rec to {0, ~0}).
hipError_t launch_check_state(hipStream_t st, const LevelDesc* lv, const int* cell_lev, int n_cells, Phys ph,
                              const double* cmom, int CH, unsigned long long* rec);
hipError_t launch_remap(int prec, hipStream_t st, const LevelDesc* old_lv, const LevelDesc* new_lv,
                        const RemapItem* items, int n, Phys ph, unsigned long long* neg);
// Criterion (Sec. 3.2).  ptab_all: per level point [|xi_p|^2, sum w|x|, sum
// w|y|, sum w x^2, sum w|xy|, sum w y^2] over its base members, levels one
// after another (ptab_off: first point of each level); ctab: per aligned
// block of scales 1, 2, 3 of the base grid [W, Wx, Wy, P[2][2], Q[2][2][2]]
// (see kernels.hip); axes: x [nx], wx [nx], y [ny], wy [ny].
hipError_t launch_criterion(int prec, hipStream_t st, const LevelDesc* lv, const int* cell_lev,
                            const int* cell_slot, int n_cells, const int* pt_of_base_all,
                            const int* pt_off, const double* ptab_all, const int* ptab_off,
                            const uint8_t* kappa_all, const double* ctab, const double* axes, int nx, int ny,
                            double C_split, double C_merge, double eps_merge, int flux_test,
                            uint8_t* kappa_out, unsigned long long* hash_out, const int* cell_list = nullptr);
// dst row r (width16 units of 16 bytes) = src row rows[r], r < n
hipError_t launch_gather_rows_16(hipStream_t st, const void* src, int width16, const int* rows, int n, void* dst);
hipError_t launch_gather_rows_u8(hipStream_t st, const uint8_t* src, int width, const int* rows, int n,
                                 uint8_t* dst);
hipError_t launch_compare_rows_u8(hipStream_t st, const uint8_t* all, int width, const int* rep_of_cell,
                                  const uint8_t* reps, int n, unsigned long long* mismatch);

// learned selector (selector.hip)
int mlp_nparams(int K);
hipError_t launch_features(hipStream_t st, const double* f8, const int* nbr_cell, const CellGeom* geom, int n,
                           double R, double T_ref, double mu_ref, double omega, int unstructured, float* out);
// Device bytes of the partial-gradient buffer a batch of B samples needs.
size_t mlp_part_bytes(int B, int K);
// Forward and backward of a batch: probabilities (prob [B][K], may be null),
// the gradient (grad [mlp_nparams(K)], zero on the standardisation block) and
// the summed loss, through the caller's partial-gradient buffer `part`.
hipError_t launch_mlp_eval(hipStream_t st, const float* P, int K, const float* X, const int* y, int B, float* prob,
                           void* part, float* grad, double* loss_sum);
// One Adam step (step number t >= 1) on the batch idx[0..B) of (X, y).
hipError_t launch_mlp_train_step(hipStream_t st, float* P, int K, const float* X, const int* y, const int* idx, int B,
                                 void* part, double* loss_sum, float* M, float* V, float lr, float b1, float b2,
                                 float eps, int t);
// Forward/backward of a batch of at most NOALLOC_MAX_BATCH samples with the
// partial gradients in the library's fixed device array (no allocation; calls
// on one GPU share the array).  prob, grad, loss_sum may be null.
constexpr int NOALLOC_MAX_BATCH = 4096;
size_t noalloc_scratch_bytes();
hipError_t launch_mlp_eval_noalloc(hipStream_t st, const float* P, int K, const float* X, const int* y, int B,
                                   float* prob, float* grad, double* loss_sum);
hipError_t launch_mlp_predict(hipStream_t st, const float* P, int K, const float* X, int B, int bf16, int* cls,
                              float* prob);
// Tail-mass check of the proposed level pred[c] of every cell listed in
// groups [n_groups][TAIL_GROUP]: cells of one level per group, -1 padded.
constexpr int TAIL_GROUP = 4;
hipError_t launch_tail_check(int prec, hipStream_t st, const LevelDesc* lv, const int* cell_lev, const int* cell_slot,
                             const int* groups, int n_groups, const int* ptb_all, const int* ptb_off,
                             const uint8_t* kappa_all, const int* pred, const double* bw, int nx, int ny,
                             double C_split, int* accept);
hipError_t launch_labels(hipStream_t st, const uint8_t* kcell, int n, int Nb, const uint8_t* kappa_all,
                         const int* order, int K, int* out);

}  // namespace mlvs
