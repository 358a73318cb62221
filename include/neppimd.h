/*
 * neppimd.h - C ABI of the MI355X (gfx950) NEP path-integral MD hot path.
 *
 * What is computed (citations are to arXiv:2409.04430):
 *   - the NEP site-energy model of Sec. II.C: U = sum_i U_i, each U_i a
 *     one-hidden-layer tanh network of radial (Chebyshev x cutoff) and
 *     angular (Legendre / spherical-harmonic) descriptors, NEP4 style
 *     per-species networks;
 *   - bead forces F_j^(i) = -dU/dr_j^(i) and the virial of Sec. II.A;
 *   - the ring-polymer normal-mode transform (Eqs. (3)-(4), (7)-(8)), the
 *     Cayley free ring-polymer step (Eqs. (5)-(6)), the half kick (Eq. (9))
 *     and the Langevin thermostat on normal-mode momenta (Eqs. (10)-(12))
 *     in its PILE (all modes), TRPMD (k > 0) and RPMD (none) forms.
 *
 * Conventions
 *   Units: eV, Angstrom, amu, fs, K.  Velocities in A/fs.
 *   Every function returns int32_t status: NEP_OK (0) or an error code > 0;
 *   nep_last_error() then returns a message for the calling thread.  No C++
 *   exception and no abort crosses this ABI.
 *   Array arguments marked "dev" are device pointers owned by the caller;
 *   the library never frees them.  Arrays marked "host" are host pointers.
 *   Opaque handles are owned by the library and released by *_destroy.
 *   Functions that take a hipStream_t enqueue work on that stream and return
 *   before it finishes.  Argument errors are found on the host before any
 *   launch; conditions found on the device (neighbour-list overflow,
 *   non-finite forces, out-of-range species) set sticky flag bits that the
 *   *_poll functions read (those functions synchronise the stream).
 *   Enqueueing calls allocate nothing on the device, except neighbor_build
 *   when a larger cell grid than any before is needed.
 *
 * Layouts
 *   pos, vel:  [P][N][3] float64, bead-major (bead j of the paper is index
 *              j-1), positions unwrapped (any periodic image).
 *   F:         [P][N][3] float32, eV/A.
 *   E:         [P] float64, per-bead total potential energy U(r_j).
 *   W:         [P][9] float64, per-bead virial W_ab = -sum_i sum_j' r_ij'^a
 *              (dU_i/dr_ij')^b, row-major (a, b).
 *   types:     [N] int32, species index 0..n_species-1 (atoms grouped by
 *              species run fastest).
 *   box:       host double[9], the cell's edge vectors a, b, c as rows (a
 *              point is r = s H with fractional s); right-handed (det > 0).
 *              Orthorhombic cells (zero off-diagonal entries) take per-axis
 *              minimum images; general (triclinic) cells reduce the
 *              fractional difference s = d H^-1 by rint per axis and map it
 *              back, which is the nearest image for every pair closer than
 *              half the smallest distance between opposite faces.
 */
#ifndef NEPPIMD_H
#define NEPPIMD_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nep_model nep_model;
typedef struct nep_nlist nep_nlist;
typedef struct nep_ws nep_ws;
typedef struct pimd_ctx pimd_ctx;

enum nep_status {
    NEP_OK = 0,
    NEP_ERR_INVALID_ARG = 1,      /* null pointer, bad size, mismatched handle */
    NEP_ERR_PARAMS_FILE = 2,      /* model file missing or malformed */
    NEP_ERR_UNSUPPORTED = 3,      /* model shape, species count, bead count or cell not supported */
    NEP_ERR_BOX_TOO_SMALL = 4,    /* a box edge is shorter than twice the largest cutoff */
    NEP_ERR_NEIGHBOR_OVERFLOW = 5,/* reported by nep_nlist_poll when a list exceeded its capacity */
    NEP_ERR_NONFINITE = 6,        /* reported by nep_poll_flags for NaN/Inf forces */
    NEP_ERR_HIP = 7,              /* a HIP runtime call failed */
    NEP_ERR_NOMEM = 8             /* device or host allocation failed */
};

/* Sticky device flag bits. */
enum nep_flag_bits {
    NEP_FLAG_NEIGHBOR_OVERFLOW = 1u,  /* some list held more neighbours than its capacity */
    NEP_FLAG_NONFINITE = 2u,          /* a force or a position was NaN or Inf */
    NEP_FLAG_BAD_TYPE = 4u,           /* a species index was outside 0..n_species-1 */
    NEP_FLAG_CELL_TOO_SMALL = 8u      /* a general (triclinic) cell's smallest face distance is not above
                                         the candidate radius rc + 2 D + skin: the lists may miss pairs */
};

/* Thread-local message describing the last error of the calling thread. */
const char *nep_last_error(void);

/* ------------------------------------------------------------------ */
/* Model (Sec. II.C)                                                   */
/* ------------------------------------------------------------------ */

typedef struct nep_hparams {
    int32_t n_species;      /* 1..4 */
    int32_t n_max_radial;   /* radial descriptors n = 0..n_max_radial */
    int32_t n_max_angular;  /* angular descriptors n = 0..n_max_angular */
    int32_t basis_radial;   /* Chebyshev functions k = 0..basis_radial */
    int32_t basis_angular;
    int32_t l_max;          /* angular l = 1..l_max */
    int32_t four_body;      /* 1: one (2,2,2)-coupled invariant per angular n */
    int32_t hidden;         /* hidden-layer width */
    int32_t dim;            /* descriptor length */
    double rc_radial;       /* A */
    double rc_angular;      /* A */
} nep_hparams;

/* Parse the plain-text model file at `path` (host) and upload its weights
 * to the current device.  The file holds the hyperparameters, the radial
 * and angular Chebyshev coefficients c[ti][tj][n][k], one scale per
 * descriptor, per-species network weights W0[H][D], b0[H], w1[H] and the
 * shared output bias b1.  Supported shapes: l_max 1..4, basis sizes 1..8,
 * n_max_radial and n_max_angular 0..8, four_body (needs l_max >= 2),
 * 1..4 species, 1..512 hidden units, 0 < rc_angular <= rc_radial.  The
 * kernels are compiled for (n_max_radial, n_max_angular, four_body) in
 * {(4,4,0), (6,4,0), (4,4,1), (8,6,0), (8,8,1)} with basis sizes 8 and
 * l_max = 4; a model of another shape runs on the first of these that
 * contains it (listed by descriptor length), its parameters placed in that
 * layout with zeros elsewhere, so every extra term is an exact zero and the
 * results are those of the model itself, at the cost of the larger shape.
 * nep_model_info reports the file's shape; the parameters of such an
 * embedded model are not exposed (nep_model_params) or trainable
 * (nep_train_ws_create), both NEP_ERR_UNSUPPORTED.  Errors:
 * NEP_ERR_PARAMS_FILE, NEP_ERR_UNSUPPORTED, NEP_ERR_HIP, NEP_ERR_NOMEM.
 * *out is owned by the caller and released with nep_model_destroy. */
int32_t nep_load_params(const char *path, nep_model **out);

/* Copy the hyperparameters of a model into *out (host). */
int32_t nep_model_info(const nep_model *model, nep_hparams *out);

void nep_model_destroy(nep_model *model);

/* Arithmetic of the per-atom network (Sec. II.C) in nep_compute. */
enum nep_mlp_mode {
    NEP_MLP_FP32 = 0,       /* FP32 vector arithmetic (default) */
    NEP_MLP_BF16_MFMA = 1,  /* BF16 weights on the matrix cores, FP32 accumulate */
    NEP_MLP_FP32_MFMA = 2,  /* FP32 weights as three BF16 terms on the matrix cores, FP32 accumulate */
    NEP_MLP_FP32_AUTO = 3   /* FP32 accuracy, the faster of the two forms for this model's shape */
};

/* Select the network arithmetic used by nep_compute (Sec. II.C network,
 * batched over the (atom, bead) rows of a wavefront as [64 x D] x [D x H]
 * and [64 x H] x [H x D] products on the matrix cores, 16 x 16 x 32 BF16
 * tiles with FP32 accumulation; activations enter exactly, each as a sum
 * of three BF16 terms).  NEP_MLP_BF16_MFMA: W0 rounded to the nearest BF16
 * value (ties to even).  NEP_MLP_FP32_MFMA: W0 as three BF16 terms whose sum
 * is the FP32 weight exactly; of the nine term products the six largest are
 * kept (each dropped one is below 2^-22 of its full product), so the result
 * has FP32 accuracy.  Both need D <= 64 and H <= 128 (NEP_ERR_UNSUPPORTED
 * otherwise).  NEP_MLP_FP32_AUTO resolves, from the shape alone, to
 * NEP_MLP_FP32_MFMA for models with more than five angular radial functions
 * (n_max_angular >= 5) whose network fits the tiles, and to NEP_MLP_FP32
 * otherwise: with at most five, nep_compute keeps the angular sums A_nlm in
 * registers through a vector-unit network, which the matrix-core network
 * cannot afford.  The operand copy is taken now, on `stream`, from the
 * current device weights: call again after the weights change
 * (nep_adam_step).  Not for concurrent use with nep_compute on another
 * stream.  Errors: NEP_ERR_INVALID_ARG, NEP_ERR_UNSUPPORTED, NEP_ERR_HIP. */
int32_t nep_model_set_mlp(nep_model *model, int32_t mode, hipStream_t stream);

/* The arithmetic of the per-atom network (Sec. II.C) in use (*mode, host):
 * NEP_MLP_FP32, NEP_MLP_BF16_MFMA or NEP_MLP_FP32_MFMA, never
 * NEP_MLP_FP32_AUTO.  Errors: NEP_ERR_INVALID_ARG. */
int32_t nep_model_mlp(const nep_model *model, int32_t *mode);

/* ------------------------------------------------------------------ */
/* Neighbour lists (per bead, minimum image, cell list)                */
/* ------------------------------------------------------------------ */

/* Create neighbour sets for P <= 64 beads of N <= 2^28 atoms on the
 * current device.  cap_radial and cap_angular bound the candidate rows of
 * one atom (all species, radius rc + 2 D + skin; see neighbor_build), at
 * most 8192 each.  The handle also holds the angular pair buffer that
 * nep_compute fills (4 N cap_angular P floats).
 * Errors: NEP_ERR_INVALID_ARG, NEP_ERR_NOMEM. */
int32_t nep_nlist_create(const nep_model *model, int32_t P, int32_t N, int32_t cap_radial, int32_t cap_angular,
                         nep_nlist **out);
void nep_nlist_destroy(nep_nlist *nl);

/* Batches of independent periodic systems (uneven sizes) share one handle:
 * atoms [offsets[s], offsets[s+1]) form system s (offsets host [nsys+1],
 * starting at 0, non-decreasing, nsys <= 4096), all with the same P beads
 * and model.  Arrays are concatenated along the atom axis; boxes are host
 * [nsys][9].  Every kernel of a call covers all systems at once: the
 * neighbour kernels look up each atom's system, and the force kernels take
 * tiles (an atom range of one system) so that per-system sums need no
 * atomics.  The single-system calls are the case nsys = 1.  A box change
 * re-uploads the geometry with a synchronous copy (not capturable); a
 * changed general (triclinic) cell also rebuilds the candidate rows.
 * Errors as the single-system calls. */
int32_t nep_nlist_create_batched(const nep_model *model, int32_t P, int32_t nsys, const int32_t *offsets,
                                 int32_t cap_radial, int32_t cap_angular, nep_nlist **out);
int32_t neighbor_build_batched(const nep_model *model, nep_nlist *nl, const double *pos, const double *boxes,
                               const int32_t *types, int32_t P, int32_t N, hipStream_t stream);

/* Neighbour sets for every bead b and atom i: the atoms i' != i with
 * |mic(r_i' - r_i)|^2 < rc^2, for the radial and the angular cutoff (Sec.
 * II.A: periodic boundary conditions).  The minimum image of d = r_i' - r_i
 * is d - L rint(d / L) per axis (orthorhombic cells) or (f - rint(f)) H with
 * f_c = (d_x G_xc + d_y G_yc) + d_z G_zc, G = H^-1, H the cell's edge vectors
 * as rows (general cells), and the test is (dx*dx + dy*dy) + dz*dz < rc*rc
 * in IEEE FP64 without contraction, so the sets are exactly those of a
 * brute-force search; the force path takes the same decision on packed
 * FP32 pair vectors and falls back to the FP64 test near the cutoff.
 * This call builds what the sets are drawn from: per atom, candidate rows
 * shared by all beads from one cell-list search over the ring-polymer
 * centroids (radius rc + 2 D [+ skin], D the largest bead-to-centroid
 * distance measured on the device in the same call; every bead pair closer
 * than rc has centroids closer than rc + 2 D), sorted by (species, index),
 * and per call the "union" lists: the candidates inside the cutoff for at
 * least one bead.  Positions must keep the P beads of an atom in one
 * periodic image (unwrapped ring polymers).  pos [P][N][3] dev, types [N]
 * dev, box host[9].  Errors: NEP_ERR_INVALID_ARG (also a singular,
 * left-handed or non-finite cell), NEP_ERR_BOX_TOO_SMALL (two opposite faces
 * closer than 2 rc, rc the larger cutoff, or too close to it for the packed
 * positions: w/2 - rc must exceed 2 w/1023, w the face distance),
 * NEP_ERR_HIP, NEP_ERR_NOMEM.  A candidate row longer than its capacity
 * sets NEP_FLAG_NEIGHBOR_OVERFLOW (the row is then truncated and the
 * results of nep_compute are not valid).  In a general cell the centroid
 * search takes nearest-image distances from the fractional reduction and,
 * for vectors at least half the smallest face distance w_min long, from the
 * 26 neighbouring images as well, which is exact below w_min; when the
 * candidate radius rc + 2 D + skin (rc the larger cutoff) is not below w_min
 * the call sets NEP_FLAG_CELL_TOO_SMALL and the lists are not valid (a
 * larger cell, less spread beads or a smaller skin avoid it). */
int32_t neighbor_build(const nep_model *model, nep_nlist *nl, const double *pos, const double box[9],
                       const int32_t *types, int32_t P, int32_t N, hipStream_t stream);

/* Reuse of the candidate rows (a Verlet skin on the centroid search): with
 * skin > 0 the rows are built with radius rc + 2 D + skin and kept while
 * (rc + 2 max_i (D_i + |c_i - lambda c_i,build|)) / lambda_min - rc
 * - 2 D_build <= skin for both cutoffs, D_i the largest bead distance from
 * atom i's centroid, D = max_i D_i, lambda = L / L_build per axis of the box
 * (so 2 max_i (D_i + |c_i - c_i,build|) - 2 D_build <= skin for an
 * unchanged box),
 * which keeps them a superset of every bead pair within the cutoffs
 * (triangle inequality, any periodic image); the decision is taken on the
 * device, without a host round trip.  A box scaled by a barostat therefore
 * keeps the rows until the skin is used up.  The species of the atoms must
 * not change between calls on one handle unless nep_nlist_invalidate is
 * called.  skin = 0 (the default)
 * rebuilds on every call.  Errors: NEP_ERR_INVALID_ARG (skin outside
 * [0, 10] A). */
int32_t nep_nlist_set_skin(nep_nlist *nl, double skin);

/* Force a candidate-row rebuild on the next neighbor_build. */
int32_t nep_nlist_invalidate(nep_nlist *nl);

/* Device layout (pointers stay owned by the handle), per atom i:
 *   cand_radial [N][cap_radial] int32: candidates, entry (j << 2) |
 *       species(j), sorted by (species, j);
 *   cand_radial_off [N][5] int32: species block starts, [n_species] = length;
 *   cand_angular, cand_angular_off: the same for the angular radius;
 *   cand_angular_rev [N][cap_angular] int32: for slot k of atom i holding
 *       j, the slot of i in j's angular row (-1 only if j's row overflowed);
 *   union_radial [N][cap_radial] int32: the candidates j (row order) that
 *       are inside rc_radial for at least one bead of the last build;
 *   union_radial_end [N][4] int32: end of species block t in that list;
 *   union_angular, union_angular_end: the same for the angular cutoff,
 *       holding slots k of the angular row instead of atom indices;
 *   union_radial_mask [N][cap_radial] uint64: for entry e of atom i's radial
 *       union list, bit b set iff the pair is inside rc_radial in bead b
 *       (the exact per-bead decision the force kernels apply);
 *   union_angular_mask: the same for the angular union list.
 * The per-bead set of bead b and atom i is therefore {union entry e : bit b
 * of mask e}.  Entries past a row's length are not written. */
typedef struct nep_nlist_layout {
    int32_t P, N, n_species, cap_radial, cap_angular;
    const int32_t *cand_radial;
    const int32_t *cand_radial_off;
    const int32_t *cand_angular;
    const int32_t *cand_angular_off;
    const int32_t *cand_angular_rev;
    const int32_t *union_radial;
    const int32_t *union_radial_end;
    const int32_t *union_angular;
    const int32_t *union_angular_end;
    const uint64_t *union_radial_mask;
    const uint64_t *union_angular_mask;
} nep_nlist_layout;
int32_t nep_nlist_view(const nep_nlist *nl, nep_nlist_layout *out);

/* Write the per-bead neighbour lists of the positions of the last
 * neighbor_build (for tests and analysis; the force path does not need
 * them; boxes host [nsys][9] as given to that build): for bead b and atom
 * i the neighbours in (species, index) order at
 * nbr_radial[b][s][i] (s < min(count, cap_radial)) and their count at
 * cnt_radial[b][i] (the full count, which may exceed cap_radial); the same
 * for the angular cutoff.  pos [P][N][3] dev must be the positions of that
 * build.  All outputs dev int32.  Errors: NEP_ERR_INVALID_ARG. */
int32_t nep_nlist_materialize(const nep_model *model, const nep_nlist *nl, const double *pos, const double *boxes,
                              int32_t P, int32_t N, int32_t cap_radial, int32_t cap_angular, int32_t *nbr_radial,
                              int32_t *cnt_radial, int32_t *nbr_angular, int32_t *cnt_angular, hipStream_t stream);

typedef struct nep_nlist_status {
    uint32_t flags;            /* nep_flag_bits seen by neighbor_build */
    int32_t max_union_radial;  /* longest radial union list of an atom */
    int32_t max_union_angular; /* longest angular union list */
    int32_t max_cand_radial;   /* longest radial candidate row (rebuild calls) */
    int32_t max_cand_angular;  /* longest angular candidate row (rebuild calls) */
    float bead_spread;         /* largest distance of a bead from its centroid, A */
    int32_t rebuilds;          /* candidate-row rebuilds since the last clear */
} nep_nlist_status;

/* Synchronise `stream`, read the sticky status of the lists into *out and,
 * if clear != 0, reset it.  Returns NEP_ERR_NEIGHBOR_OVERFLOW if the
 * overflow bit is set (after filling *out). */
int32_t nep_nlist_poll(nep_nlist *nl, nep_nlist_status *out, int32_t clear, hipStream_t stream);

/* ------------------------------------------------------------------ */
/* Energy, forces, virial                                              */
/* ------------------------------------------------------------------ */

/* Workspace for P beads of N atoms (descriptor adjoints, partial sums,
 * flags) on the current device. */
int32_t nep_ws_create(const nep_model *model, int32_t P, int32_t N, nep_ws **out);
/* Workspace for a batch (see nep_nlist_create_batched); the partition must
 * equal the list's. */
int32_t nep_ws_create_batched(const nep_model *model, int32_t P, int32_t nsys, const int32_t *offsets, nep_ws **out);
void nep_ws_destroy(nep_ws *ws);

/* NEP energy, forces and virial of every bead (Sec. II.C site energies,
 * Sec. II.A bead forces and virial), from neighbour sets built by
 * neighbor_build on the same pos/box/types; the positions that call packed
 * are reused, so pos must not change between the two calls.  The angular
 * pair terms
 * dU_i/dr_ij are stored in the handle's pair buffer and gathered back by
 * the reverse slots, so no atomics are used.
 *   E      [P]      dev float64  per-bead sum of site energies
 *   F      [P][N][3] dev float32 forces, F_i = sum_j (dU_i/dr_ij - dU_j/dr_ji)
 *   W      [P][9]   dev float64  per-bead virial
 *   E_atom [P][N]   dev float32  site energies U_i, or NULL
 *   W_atom [P][N][9] dev float32 per-atom virial -1/2 sum_j r_ij (x)
 *                   (dU_i/dr_ij - dU_j/dr_ji), or NULL
 * Positions enter as FP64 and are packed per bead as fine-grid cell
 * indices plus FP32 offsets, from which pair vectors are formed (error
 * about 1e-6 A); the rest is FP32 arithmetic with FP64 accumulation of
 * forces, energies and virials.
 * The summation order is fixed, so repeated calls give identical bits.
 * Errors: NEP_ERR_INVALID_ARG (sizes differ from the handles', lists built
 * with other cutoffs than the model's), NEP_ERR_HIP.
 * Non-finite forces set NEP_FLAG_NONFINITE in the workspace. */
int32_t nep_compute(const nep_model *model, nep_nlist *nl, nep_ws *ws, const double *pos,
                    const double box[9], const int32_t *types, int32_t P, int32_t N, double *E, float *F,
                    double *W, float *E_atom, float *W_atom, hipStream_t stream);

/* nep_compute over a batch: boxes host [nsys][9], E [nsys][P] and W
 * [nsys][P][9] per system and bead, the other arrays concatenated along
 * the atom axis. */
int32_t nep_compute_batched(const nep_model *model, nep_nlist *nl, nep_ws *ws, const double *pos,
                            const double *boxes, const int32_t *types, int32_t P, int32_t N, double *E, float *F,
                            double *W, float *E_atom, float *W_atom, hipStream_t stream);

/* Tile shape of the force kernels: 1, 2 or 4 wavefronts per workgroup, each
 * wavefront holding 64 / G atoms with their G >= P beads (default 4).  The
 * tile table is re-uploaded synchronously.  Errors: NEP_ERR_INVALID_ARG. */
int32_t nep_ws_set_tile(nep_ws *ws, int32_t waves_per_group);
int32_t nep_ws_get_tile(const nep_ws *ws, int32_t *waves_per_group);

/* Where the weights of the FP32 per-atom network (Sec. II.C) are read from
 * in nep_compute (vector-unit network): staged in LDS once per workgroup
 * (default; used only where S H (D + 2) floats fit 60 KiB, else global) or
 * read from global memory.
 * Both evaluate the same products in the same order, so E, F and W are
 * bitwise the same; only the speed differs.  No effect on the matrix-core
 * networks.  Errors: NEP_ERR_INVALID_ARG. */
enum nep_weight_staging { NEP_WEIGHTS_LDS = 0, NEP_WEIGHTS_GLOBAL = 1 };
int32_t nep_ws_set_weight_staging(nep_ws *ws, int32_t staging);
int32_t nep_ws_get_weight_staging(const nep_ws *ws, int32_t *staging);

/* Autotuner: times nep_compute_batched (one warm-up plus `reps` calls, HIP
 * events on `stream`) for every tile shape (1, 2, 4 wavefronts per
 * workgroup) and weight staging (LDS, global; LDS only where the weights
 * fit, and one staging for the matrix-core networks), keeps the fastest in
 * the workspace and reports it in best[2] (host: wavefronts per workgroup,
 * staging), with the mean times in ms_out[6] (host, entry 2 c + st for tile
 * choice c and staging st, -1 where a staging does not apply; may be NULL).
 * Forces and virials do not depend on either knob (energies regroup per
 * tile).  E, F, W are overwritten.  Synchronises the stream.  Errors as
 * nep_compute_batched. */
int32_t nep_autotune(const nep_model *model, nep_nlist *nl, nep_ws *ws, const double *pos, const double *boxes,
                     const int32_t *types, int32_t P, int32_t N, double *E, float *F, double *W, int32_t reps,
                     float *ms_out, int32_t *best, hipStream_t stream);

/* Synchronise `stream`, read the workspace flags into *flags and, if
 * clear != 0, reset them.  Returns NEP_ERR_NONFINITE if that bit is set. */
int32_t nep_poll_flags(nep_ws *ws, uint32_t *flags, int32_t clear, hipStream_t stream);

/* Defer the per-bead energy and virial sums (Sec. II.A virial, Sec. II.C
 * total energy) of the next nep_compute / nep_compute_batched call on ws:
 * that call writes forces (and the per-atom arrays) as usual but leaves E
 * and W to the next trpmd_step_nep call given ws, which completes them
 * inside its integrator launch (one launch fewer per MD step).  Until then
 * E and W hold stale values.  Host state only: arms that one call, which
 * disarms it; a later nep_compute on ws without a deferral drops sums left
 * pending.  Errors: NEP_ERR_INVALID_ARG (null ws). */
int32_t nep_ws_defer_reduce(nep_ws *ws);

/* ------------------------------------------------------------------ */
/* Ring polymer (Sec. II.A, Eqs. (3)-(12))                             */
/* ------------------------------------------------------------------ */

enum pimd_mode { PIMD_MODE_PILE = 0, PIMD_MODE_TRPMD = 1, PIMD_MODE_RPMD = 2 };
enum pimd_stage { PIMD_STAGE_PRE = 0, PIMD_STAGE_POST = 1, PIMD_STAGE_FUSED = 2 };

typedef struct pimd_params {
    double dt_fs;      /* time step */
    double T_K;        /* physical temperature; beads run at P T */
    double tau_T_fs;   /* centroid friction time, gamma_0 = 1/tau (PILE only) */
    int32_t mode;      /* enum pimd_mode */
    uint64_t seed;     /* key of the counter-based normal generator */
} pimd_params;

/* Integrator context for P beads of N atoms: the orthogonal matrix C_jk
 * (j = 1..P as printed in Sec. II.A; odd P has no (-1)^j row), the
 * frequencies omega_k = 2 omega_P sin(k pi / P) with omega_P = P kB T / hbar,
 * the Cayley coefficients and c_1k = exp(-gamma_k dt / 2), c_2k =
 * sqrt(1 - c_1k^2), gamma_0 = 1/tau, gamma_k = omega_k.  mass [N] dev amu is
 * copied.  Supported P: 1..64.  Errors: NEP_ERR_INVALID_ARG,
 * NEP_ERR_UNSUPPORTED, NEP_ERR_HIP, NEP_ERR_NOMEM. */
int32_t pimd_create(int32_t P, int32_t N, const pimd_params *params, const double *mass, pimd_ctx **out);
void pimd_destroy(pimd_ctx *ctx);

/* dir = +1: out_k = sum_j C_jk in_j (beads -> normal modes, Eqs. (3)-(4));
 * dir = -1: out_j = sum_k C_jk in_k (modes -> beads, the transpose map).
 * in, out [P][N][3] dev float64 (mode index in place of the bead index);
 * in == out is not allowed. */
int32_t rp_normal_modes(const pimd_ctx *ctx, int32_t dir, const double *in, double *out, hipStream_t stream);

/* One integrator stage, in place on pos and vel, with forces F at the
 * current positions:
 *   PRE   = O, B, A: thermostat (Eqs. (10)-(12)) with noise stage 0 of
 *           `step`, half kick (Eq. (9)), transform + Cayley + back transform
 *           (Eqs. (3)-(8)); then the caller evaluates forces;
 *   POST  = B, O with noise stage 1 of `step`;
 *   FUSED = POST(step) followed by PRE(step + 1).
 * Thermostatted modes: all (PILE), k > 0 (TRPMD), none (RPMD).  Normals:
 * Philox-4x32-10 keyed by the seed with counter (atom, (component P + k)/4,
 * step mod 2^32, 2 (step >> 32) + stage), uniforms (x + 1) 2^-32 and
 * Box-Muller pairs.  pos, vel [P][N][3] dev float64; F [P][N][3] dev float32.
 * Errors: NEP_ERR_INVALID_ARG, NEP_ERR_HIP. */
int32_t trpmd_step(const pimd_ctx *ctx, double *pos, double *vel, const float *F, int64_t step, int32_t stage,
                   hipStream_t stream);

/* trpmd_step with the step number read from device memory (*step_in, int64)
 * by the launch itself; a POST or FUSED stage also writes step + 1 to
 * *step_out (dev int64, another word than step_in: the launch's workgroups
 * all read step_in), so consecutive steps alternate two counters and no
 * extra launch advances them.  For graph capture: captured steps replay with
 * fresh noise (an even number of captured steps returns the count to the
 * first counter).  step_out is ignored for PRE.  Errors as trpmd_step, and
 * NEP_ERR_INVALID_ARG for a null counter or step_out == step_in. */
int32_t trpmd_step_dev(const pimd_ctx *ctx, double *pos, double *vel, const float *F, const int64_t *step_in,
                       int64_t *step_out, int32_t stage, hipStream_t stream);

/* One integrator stage (Eqs. (3)-(12), as trpmd_step: step_in = NULL uses
 * the host step number `step`; otherwise as trpmd_step_dev with the device
 * counters step_in / step_out and `step` ignored) that also completes the
 * per-bead energy and virial sums left pending in ws by a deferred
 * nep_compute (nep_ws_defer_reduce), in the same launch: extra workgroups
 * of the stage, one wavefront per (system, bead, component), the same
 * fixed-order sums as nep_compute's own, so E and W are bitwise the same.
 * With nothing pending it is the plain stage.  Call it on the stream of
 * that nep_compute, before anything else overwrites ws.  ws must have the
 * context's P and N.  Errors as trpmd_step / trpmd_step_dev, and
 * NEP_ERR_INVALID_ARG for a null ws or mismatched sizes. */
int32_t trpmd_step_nep(const pimd_ctx *ctx, double *pos, double *vel, const float *F, int64_t step,
                       const int64_t *step_in, int64_t *step_out, int32_t stage, nep_ws *ws, hipStream_t stream);

/* ------------------------------------------------------------------ */
/* Observables and pressure control (Sec. II.A, Sec. II.D)             */
/* ------------------------------------------------------------------ */

/* Entries of the observables vector written by pimd_observables. */
enum pimd_obs_index {
    PIMD_OBS_EPOT = 0,      /* potential energy: mean of the per-bead energies (eV) */
    PIMD_OBS_KINETIC = 1,   /* centroid virial kinetic energy (eV) */
    PIMD_OBS_VIRIAL = 2,    /* virial tensor W [3][3], row = displacement axis (eV) */
    PIMD_OBS_PRESSURE = 11, /* pressure tensor [3][3] (GPa) */
    PIMD_OBS_PSCALAR = 20,  /* trace of the pressure tensor / 3 (GPa) */
    PIMD_OBS_COUNT = 21
};

/* Ring-polymer observables of one system (Sec. II.A): with the centroid
 * r_c of each atom and the bead displacements dr_j = r_j - r_c, taken through
 * the periodic boundaries (each bead at its image nearest the atom's first
 * bead),
 *   K = 3/2 N kB T - 1/2 sum_i (1/P) sum_j dr_j . F_j,
 *   W = -sum_i (1/P) sum_j dr_j (x) F_j + (1/P) sum_j W_bead[j],
 *   pressure tensor = (N kB T 1 + W) / V,
 * T the context's physical temperature.  pos, F [P][N][3] dev (float64,
 * float32), W_bead [P][9] and E_bead [P] dev float64 (the per-bead virial
 * and energy of nep_compute), box host [9] (V its determinant), out
 * [PIMD_OBS_COUNT] dev float64, written on the stream (pos and F may be
 * null when N = 0).  The partial sums
 * live in the context: calls on one context must not overlap.  The sum
 * order is fixed, so results are bitwise reproducible.  Errors:
 * NEP_ERR_INVALID_ARG (also a singular or left-handed cell),
 * NEP_ERR_HIP. */
int32_t pimd_observables(const pimd_ctx *ctx, const double *pos, const float *F, const double *W_bead,
                         const double *E_bead, const double box[9], double *out, hipStream_t stream);

typedef struct pimd_barostat {
    double p0_GPa[3];       /* target pressure per axis (isotropic: all three equal) */
    double beta_per_GPa;    /* compressibility, >= 0 */
    double tau_p_fs;        /* coupling time, > 0 */
    int32_t anisotropic;    /* 0: couple tr(P)/3 on every axis; 1: each axis to its own P_aa */
} pimd_barostat;

/* Berendsen-like pressure control of the workflow (Sec. II.D), applied after
 * the closing half of a step: per axis mu_a = 1 - beta dt / (3 tau_p) (p0_a -
 * p_a), with p_a = P_aa (anisotropic) or tr(P)/3 (isotropic) read from obs
 * (the vector of pimd_observables, dev), dt the context's time step; every
 * bead coordinate pos[j][i][a] (dev, in place) is multiplied by mu_a and the
 * factors are written to mu [3] (dev).  The caller scales its cell edges by
 * the same factors before the next neighbour build (a changed box rebuilds
 * the candidate rows).  Errors: NEP_ERR_INVALID_ARG (null argument, beta < 0,
 * tau_p <= 0, non-finite target), NEP_ERR_HIP. */
int32_t pimd_berendsen(const pimd_ctx *ctx, double *pos, const double *obs, const pimd_barostat *params,
                       double *mu, hipStream_t stream);

/* Bead mean of a ring-polymer array (positions of unwrapped ring polymers,
 * or velocities, e.g. for velocity dumps of the centroid dynamics):
 * out[i][a] = (sum_j x[j][i][a]) / P, beads summed in order.  x [P][N][3]
 * dev float64, out [N][3] dev float64, out != x.  Errors:
 * NEP_ERR_INVALID_ARG, NEP_ERR_HIP. */
int32_t pimd_centroid(const pimd_ctx *ctx, const double *x, double *out, hipStream_t stream);

/* Pair-distance histogram per species pair (the partial radial distribution
 * functions of the water analysis, Sec. III), read off the radial union lists
 * of the last neighbor_build on these positions: for every bead b and
 * ordered pair (i, j != i) of that bead with r = |mic(r_j - r_i)| (FP64,
 * the minimum image of the list test, no contraction) and k = floor(r nbins / rmax)
 * < nbins, hist[(type_i S + type_j) nbins + k] += 1.  hist [S][S][nbins] dev
 * uint64 is accumulated, not cleared (so frames add up).  rmax must lie in
 * (0, rc_radial (1 - 1e-9)] so that every counted pair is on the lists;
 * S^2 nbins <= 16384.  One system per list.  g_ab(r) follows as
 * hist / (frames P N_a rho_b shell volume), rho_b = (N_b - [a == b]) / V.
 * Lists that overflowed (NEP_FLAG_NEIGHBOR_OVERFLOW) give incomplete counts.
 * The first call on a list allocates a bead-minor copy of the positions
 * (24 P N bytes) kept by the list.
 * Errors: NEP_ERR_INVALID_ARG (sizes, rmax, nbins, box differing from the
 * last build, lists not built), NEP_ERR_UNSUPPORTED (batched list),
 * NEP_ERR_HIP. */
int32_t nep_rdf_accumulate(const nep_model *model, nep_nlist *nl, const double *pos, const double box[9],
                           const int32_t *types, int32_t P, int32_t N, double rmax, int32_t nbins, uint64_t *hist,
                           hipStream_t stream);

/* nep_rdf_accumulate for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments and the same histogram, but the bead-minor
 * copy of the positions lives in a 24 MiB array of the library's device
 * code object instead of a list-owned allocation, so the call allocates
 * nothing (no device memory, no timing events; its kernels are not timed by
 * nep_profile_*).  Limit: P N <= 1,048,576 (bead, atom) rows, else
 * NEP_ERR_INVALID_ARG with the sizes in the message.  Each device holds one
 * such array for the life of the process, shared by every call on that
 * device: calls that overlap on one device (different streams, or threads)
 * race and must be ordered by the caller.  Every call rewrites the part it
 * uses before reading it.  Errors as nep_rdf_accumulate, and NEP_ERR_HIP if
 * the array's device address cannot be obtained. */
int32_t nep_rdf_accumulate_noalloc(const nep_model *model, nep_nlist *nl, const double *pos, const double box[9],
                                   const int32_t *types, int32_t P, int32_t N, double rmax, int32_t nbins,
                                   uint64_t *hist, hipStream_t stream);

/* ------------------------------------------------------------------ */
/* D3 dispersion of NEP-D3 (Sec. II.C, the MOF model)                  */
/* ------------------------------------------------------------------ */

typedef struct nep_d3 nep_d3;
typedef struct nep_d3_ws nep_d3_ws;

/* Parse a D3 parameter file (host) and upload its tables to the current
 * device.  The paper adds D3 dispersion with Becke-Johnson damping to its
 * MOF model, with a 12 A dispersion cutoff and a 6 A coordination-number
 * cutoff; the form is the published D3 one, in eV and A:
 *   CN_i  = sum_{j, r < rc_cn} 1 / (1 + exp(-k1 (k2 (R_i + R_j) / r - 1)))
 *   C6_ij = sum_ab C6ref_ij(a,b) L_ab / sum_ab L_ab,
 *           L_ab = exp(-k3 [(CN_i - CNref_i,a)^2 + (CN_j - CNref_j,b)^2])
 *   C8_ij = 3 C6_ij q_i q_j,  f_ij = a1 sqrt(C8_ij / C6_ij) + a2
 *   E     = -1/2 sum_i sum_{j, r < rc} [s6 C6_ij / (r^6 + f^6) + s8 C8_ij / (r^8 + f^8)]
 * with hard cutoffs (strict r^2 < rc^2).  File layout: "nep_d3_params 1",
 * "species S" (1..4), "cutoff rc rc_cn" (rc_cn <= rc), "damping s6 s8 a1
 * a2", "constants k1 k2 k3", then "rcov", "q", "nref" (1..5 references)
 * per species, "cnref" (each species' references) and "c6ref" (for every
 * species pair, nref_i x nref_j values, eV A^6).  Errors:
 * NEP_ERR_PARAMS_FILE, NEP_ERR_UNSUPPORTED, NEP_ERR_HIP, NEP_ERR_NOMEM.
 * Released with nep_d3_destroy. */
int32_t nep_d3_load(const char *path, nep_d3 **out);
void nep_d3_destroy(nep_d3 *d3);

/* The cutoff descriptor of the D3 lists: a model handle (owned by d3, not
 * to be destroyed) whose radial cutoff is rc and angular cutoff rc_cn, for
 * nep_nlist_create / neighbor_build only (it has no network: the NEP
 * entry points reject it).  The D3 lists are a neighbour handle of their
 * own, built on the same positions as the NEP lists. */
int32_t nep_d3_list_model(const nep_d3 *d3, const nep_model **out);

/* Workspace for P beads of N atoms (coordination numbers, dE/dCN, direct
 * forces, partial sums).  Errors: NEP_ERR_INVALID_ARG, NEP_ERR_NOMEM. */
int32_t nep_d3_ws_create(const nep_d3 *d3, int32_t P, int32_t N, nep_d3_ws **out);
void nep_d3_ws_destroy(nep_d3_ws *ws);

/* D3 energy, forces and virial of every bead from lists built by
 * neighbor_build with the model of nep_d3_list_model on the same
 * positions (one system per list).  F_i = -dE/dr_i through the explicit
 * distances and through CN_i and CN_j; W_ab = -sum over ordered pairs of
 * r_ij^a (dE/dr_ij)^b (the convention of nep_compute).  With accumulate != 0
 * the results are added to E [P], F [P][N][3] and W [P][9] (dev; e.g. after
 * nep_compute, giving NEP-D3), else they overwrite them.  FP64 arithmetic
 * throughout (the pair terms of a near-perfect crystal nearly cancel, so
 * FP32 pair terms would cost their net force its relative accuracy); fixed
 * sum order.  Errors: NEP_ERR_INVALID_ARG (sizes, lists built with other
 * cutoffs, box differing from the last build), NEP_ERR_UNSUPPORTED (a
 * batched list), NEP_ERR_HIP. */
int32_t nep_d3_compute(const nep_d3 *d3, nep_nlist *nl, nep_d3_ws *ws, const double *pos, const double box[9],
                       const int32_t *types, int32_t P, int32_t N, double *E, float *F, double *W,
                       int32_t accumulate, hipStream_t stream);

/* ------------------------------------------------------------------ */
/* Training (gradient of an energy / force / virial loss, Adam)        */
/* ------------------------------------------------------------------ */

/* Offsets (in floats) of the parameter blocks inside a model's device
 * parameter array: c_radial [S][S][n_R+1][9], c_angular [S][S][n_A+1][9],
 * q_scale [D], W0 [S][H][D], b0 [S][H], w1 [S][H], b1 [1], then the 24
 * spherical-harmonic constants (not parameters). */
typedef struct nep_param_offsets {
    int32_t c_radial, c_angular, q_scale, W0, b0, w1, b1, sh;
} nep_param_offsets;

/* Device parameter array of a model (owned by the model; the NEP kernels
 * read it, so writing it changes the model), its length and block offsets.
 * Errors: NEP_ERR_INVALID_ARG, NEP_ERR_UNSUPPORTED (a model embedded in a
 * larger kernel shape, nep_load_params). */
int32_t nep_model_params(nep_model *model, float **params, int32_t *count, nep_param_offsets *offsets);

typedef struct nep_train_ws nep_train_ws;

/* Training workspace for P configurations of N atoms (the beads of a
 * neighbour handle of one system).  Models with the four-body term, and
 * models embedded in a larger kernel shape (nep_load_params), are not
 * trainable (NEP_ERR_UNSUPPORTED).  Errors: NEP_ERR_INVALID_ARG,
 * NEP_ERR_UNSUPPORTED, NEP_ERR_NOMEM. */
int32_t nep_train_ws_create(const nep_model *model, int32_t P, int32_t N, nep_train_ws **out);

/* Training workspace (the loss gradient above; the paper fits NEP models by
 * SNES, Sec. II.C) for a batch of nsys systems (atoms [off[s], off[s+1])
 * form system s, off host [nsys+1], as for nep_nlist_create_batched), P
 * configurations each: one nep_param_grad_batched call then covers nsys
 * independent labelled snapshots.  Errors as nep_train_ws_create. */
int32_t nep_train_ws_create_batched(const nep_model *model, int32_t P, int32_t nsys, const int32_t *off,
                                    nep_train_ws **out);
void nep_train_ws_destroy(nep_train_ws *tw);

/* Loss and parameter gradient for the P configurations pos [P][N][3] (the
 * lists nl must have been built at pos) with references E_ref [P] (eV),
 * F_ref [P][N][3] (eV/A), W_ref [P][9] (eV), all device:
 *   L = sum_b lE (dE_b/N)^2 + lF sum_i |dF_bi|^2 / (3N) + lW sum_ab (dW_b,ab/N)^2
 * with lambda = {lE, lF, lW} (host).  grad [count] (device, the model's
 * parameter layout) is accumulated: += dL/dtheta for W0, b0, w1, b1,
 * c_radial and c_angular (other entries untouched); loss [4] (device) is
 * accumulated: total, energy, force and virial parts.  The force and virial
 * parts enter as mixed derivatives through a forward-mode pass of the
 * descriptor along the residual field.  The model must use FP32 weights
 * (NEP_ERR_INVALID_ARG after nep_model_set_mlp(NEP_MLP_BF16_MFMA)).  Errors
 * as nep_compute. */
int32_t nep_param_grad(const nep_model *model, nep_nlist *nl, nep_ws *ws, nep_train_ws *tw, const double *pos,
                       const double box[9], const int32_t *types, int32_t P, int32_t N, const double *E_ref,
                       const float *F_ref, const double *W_ref, const double lambda[3], float *grad, double *loss,
                       hipStream_t stream);

/* nep_param_grad over a batch of systems: the list, the workspace and the
 * training workspace hold the same partition; boxes [nsys][9] (host),
 * E_ref [nsys][P], F_ref [P][N][3], W_ref [nsys][P][9] (device).  The loss
 * is the sum of each system's loss above, N its own atom count.  Errors as
 * nep_param_grad (NEP_ERR_INVALID_ARG when the partitions differ). */
int32_t nep_param_grad_batched(const nep_model *model, nep_nlist *nl, nep_ws *ws, nep_train_ws *tw,
                               const double *pos, const double *boxes, const int32_t *types, int32_t P, int32_t N,
                               const double *E_ref, const float *F_ref, const double *W_ref,
                               const double lambda[3], float *grad, double *loss, hipStream_t stream);

/* One Adam step (Kingma and Ba, with bias correction) on the model's
 * parameters: theta -= lr mhat / (sqrt(vhat) + eps), for the parameter
 * groups in mask (bits: 1 network W0, b0, w1, b1; 2 c_radial; 4 c_angular).  m1, m2
 * [count] device moment arrays (zero before step 1), step >= 1.  Errors:
 * NEP_ERR_INVALID_ARG. */
int32_t nep_adam_step(nep_model *model, nep_train_ws *tw, const float *grad, float *m1, float *m2, int64_t step,
                      float lr, float beta1, float beta2, float eps, int32_t mask, hipStream_t stream);

/* Force error of a model against another (the judge of a learned
 * student against its teacher): work[0] = sqrt(sum_e (Fa[e] - Fb[e])^2 / n)
 * over the n = 3 P N components of two force arrays Fa, Fb (device FP32,
 * same layout), in eV/A.  work (device, caller-owned, 1025 doubles) also
 * holds the partial sums; the sum order is fixed, so the result is bitwise
 * reproducible.  n = 0 gives 0.  Errors: NEP_ERR_INVALID_ARG. */
int32_t nep_force_rmse(const float *Fa, const float *Fb, int64_t n, double *work, hipStream_t stream);

/* ------------------------------------------------------------------ */
/* Kernel timing                                                       */
/* ------------------------------------------------------------------ */

/* Turn per-kernel timing on (on != 0) or off for the whole process.  While
 * on, every kernel the library launches is bracketed by two hipEvents
 * recorded on the caller's stream; events come from a library-owned pool. */
int32_t nep_profile_enable(int32_t on);

/* Restrict timing to the kernel kind `id` (-1: every kind, the default), so
 * that a timed region carries two events per launch of one kernel only.
 * Errors: NEP_ERR_INVALID_ARG for an unknown id. */
int32_t nep_profile_select(int32_t id);

/* Number of kernel kinds and the name of kind `id` ("descriptor", "force",
 * "nlist", "trpmd", ...); "" for an unknown id. */
int32_t nep_profile_num_kernels(void);
const char *nep_profile_kernel_name(int32_t id);

/* Wait for every recorded launch, then write per-kind totals:
 * total_ms[nep_profile_num_kernels()] (host) summed event-to-event
 * durations, launches[...] (host) launch counts.  reset != 0 starts new
 * totals.  Errors: NEP_ERR_INVALID_ARG, NEP_ERR_HIP. */
int32_t nep_profile_read(double *total_ms, int64_t *launches, int32_t reset);

#ifdef __cplusplus
}
#endif

#endif /* NEPPIMD_H */
