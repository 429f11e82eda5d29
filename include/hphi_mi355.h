/*
 * hphi_mi355.h -- C ABI of the MI355X (gfx950) matrix-free H*v / Lanczos /
 * cTPQ / shifted-Krylov library.
 *
 * The operations follow the problem statement of the HPhi update paper
 * (arXiv:2307.13222): a spin-1/2 or Hubbard lattice model given by its site
 * count, conserved sector (the 2Sz and nelec keywords of the Standard-mode
 * table in Sec. 4.1) and bond / transfer lists (Sec. 3.4, Eq. Hquench;
 * Sec. 5); the matrix-vector product that every iterative method reduces to
 * (Sec. 1); the Lanczos ground state (Sec. 1); the canonical TPQ propagator
 * (Sec. 3.5.1); the dynamical correlation function by the shifted Krylov
 * method (Sec. 3.2).
 *
 * Conventions that hold for every entry point:
 *  - Return value: 0 on success, a negative HPHI_ERR_* code on failure; the
 *    message of the last failure on the calling thread is hphi_last_error().
 *  - Pointers named *_dev are device pointers on the context's device; the
 *    caller owns them (they are typically torch tensors' data pointers).
 *    Every other pointer is host memory owned by the caller.
 *  - The library owns basis tables, Hamiltonian tables and its own scratch
 *    memory; they are released by the matching *_free call.
 *  - `stream` is a hipStream_t (NULL = the default stream). Calls that only
 *    launch kernels are asynchronous on that stream; calls that return host
 *    scalars synchronize it before returning.
 *  - Configuration bit convention: site i is bit i; bit = 1 means spin up
 *    (spins) or an occupied orbital (electrons). Basis states are ordered by
 *    ascending integer value. A Hubbard state (u, d) has flat index
 *    rank_up(u) * dim_dn + rank_dn(d).
 *  - Vector layout: element (state r, vector j) of a block of nvec vectors
 *    sits at r * nvec + j ("interleaved"); complex numbers are (re, im)
 *    pairs. Input and output blocks must not alias.
 *  - Concurrency: a Hamiltonian owns one set of reduction and work-queue
 *    scratch that every call on it uses, so it serves one call at a time on
 *    one stream at a time. A call that takes a Hamiltonian returns
 *    HPHI_ERR_BUSY, and launches nothing, when another host thread is inside
 *    a call on the same Hamiltonian, or when the previous call on it was
 *    made on a different stream and its work has not finished yet (the
 *    library records an event on the calling stream at the end of each
 *    call). Calls on one stream queue in order and need nothing. To switch
 *    streams, order them first (an event wait or a synchronization). While
 *    a stream is being captured into a graph the stream check is skipped:
 *    the caller orders the graph's launches. hphi_lanczos_batch only reads
 *    the Hamiltonians' tables, so one Hamiltonian may appear in it many
 *    times. Different Hamiltonians are independent.
 */
#ifndef HPHI_MI355_H
#define HPHI_MI355_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------- errors -- */
#define HPHI_OK                 0
#define HPHI_ERR_INVALID_ARG   -1   /* bad size, site index, sector, option */
#define HPHI_ERR_EMPTY_SECTOR  -2   /* the requested sector has no states   */
#define HPHI_ERR_DIM_OVERFLOW  -3   /* dimension beyond 2^62 or a table     */
#define HPHI_ERR_OUT_OF_MEMORY -4   /* device or host allocation failed     */
#define HPHI_ERR_DEVICE        -5   /* a HIP runtime call failed            */
#define HPHI_ERR_UNSUPPORTED   -6   /* valid request this build cannot do   */
#define HPHI_ERR_BUSY          -7   /* the Hamiltonian is in use elsewhere  */

typedef enum {
    HPHI_F64 = 0,    /* real double                         */
    HPHI_F32 = 1,    /* real float (storage), FP64 dots     */
    HPHI_C128 = 2,   /* complex double, (re, im) pairs      */
    HPHI_C64 = 3     /* complex float (storage), FP64 dots  */
} hphi_dtype;

typedef struct hphi_ctx hphi_ctx;
typedef struct hphi_basis hphi_basis;
typedef struct hphi_ham hphi_ham;

/* Message of the last failure on this thread ("" if none). The string is
 * owned by the library and valid until the next failing call. */
const char *hphi_last_error(void);

/* Library version string (static storage). */
const char *hphi_version(void);

/* Open a context on HIP device `device` (0-based). *ctx receives the handle.
 * Errors: INVALID_ARG (no such device), DEVICE. */
int hphi_init(int device, hphi_ctx **ctx);

/* Release a context. Bases and Hamiltonians made from it must be freed
 * first. NULL is accepted. */
void hphi_fini(hphi_ctx *ctx);

/* ------------------------------------------------------------- basis -- */

/* Sector basis of a spin-1/2 system: all n_sites-bit configurations with
 * (n_up - n_dn) = two_sz, i.e. a fixed total S^z (keyword 2Sz, Sec. 4.1).
 * Builds the split two-level rank table on host and device:
 *   idx(x) = hi_off[x >> n_lo] + lo_rank[x & (2^n_lo - 1)],
 * with lo_rank[l] the rank of l among n_lo-bit patterns of equal popcount
 * and hi_off[h] the number of sector states whose high part is below h.
 * Errors: INVALID_ARG (n_sites < 1 or > 64, |two_sz| > n_sites, parity of
 * n_sites + two_sz odd), DIM_OVERFLOW, OUT_OF_MEMORY, DEVICE. */
int hphi_basis_spin(hphi_ctx *ctx, int n_sites, int two_sz, hphi_basis **out);

/* Sector basis of the Hubbard model with fixed N_up and N_dn (keyword nelec
 * with fixed 2Sz, Sec. 4.1): the product of the two one-species bases.
 * Errors: INVALID_ARG (n_sites < 1 or > 32, n_up or n_dn outside
 * [0, n_sites]), DIM_OVERFLOW, OUT_OF_MEMORY, DEVICE. */
int hphi_basis_hubbard(hphi_ctx *ctx, int n_sites, int n_up, int n_dn, hphi_basis **out);

/* Sector basis of N spin-S sites with total 2S^z = two_sz (keyword 2S,
 * Sec. 4.1, "Remarks on the keyword model"): site i holds m_i = S^z_i + S in
 * {0, ..., 2S}, stored in bits [i b, (i + 1) b) of the configuration, with
 * b = 1 for S = 1/2, 2 for S = 1 and 3/2, 3 up to S = 7/2. States ascend by
 * that encoding and are ranked by the split table
 *   idx(x) = hi_off[x >> L] + lo_rank[x & (2^L - 1)],  L = b floor(N/2),
 * lo_rank counting the lower patterns of equal digit sum. Configurations
 * (host and device calls) are the encoded values. Errors: INVALID_ARG
 * (two_s outside [1, 7], n_sites < 1, N b > 40, |two_sz| > 2S N or of the
 * wrong parity), DIM_OVERFLOW (dimension >= 2^32), OUT_OF_MEMORY, DEVICE. */
int hphi_basis_spin_s(hphi_ctx *ctx, int n_sites, int two_s, int two_sz, hphi_basis **out);

/* The whole 2^N spin-1/2 space, no S^z conservation (SpinGC keyword,
 * Sec. 4.1, Table "Keywords"): the index of a configuration is the
 * configuration (bit i = 1: site i up). Nothing is stored. Errors:
 * INVALID_ARG (n_sites < 1 or > 32). */
int hphi_basis_spin_gc(hphi_ctx *ctx, int n_sites, hphi_basis **out);

void hphi_basis_free(hphi_basis *b);

/* Dimension of the sector (number of basis states). */
int64_t hphi_basis_dim(const hphi_basis *b);

/* Host copy of basis states [first, first + count): spins give the
 * configuration, Hubbard states are packed as (u << 32) | d.
 * Errors: INVALID_ARG (range outside [0, dim)). */
int hphi_basis_states(const hphi_basis *b, int64_t first, int64_t count, uint64_t *host_out);

/* Host ranks of n configurations (packed as above); -1 for a configuration
 * outside the sector. */
int hphi_basis_rank(const hphi_basis *b, const uint64_t *states, int64_t n, int64_t *idx_out);

/* Device versions of the two calls above: the same tables the H*v kernels
 * use, evaluated by GPU kernels. Asynchronous on `stream`. */
int hphi_basis_states_device(const hphi_basis *b, int64_t first, int64_t count,
                             uint64_t *out_dev, void *stream);
int hphi_basis_rank_device(const hphi_basis *b, const uint64_t *states_dev, int64_t n,
                           int64_t *idx_dev, void *stream);

/* Read-only host view of the rank tables of one species (spin: species 0;
 * Hubbard: 0 = up, 1 = down; SpinGC and spin-S bases: UNSUPPORTED).
 * Pointers stay valid until hphi_basis_free.
 * lo_rank has 2^n_lo entries, hi_off 2^n_hi + 1 (the last is the total). */
int hphi_basis_tables(const hphi_basis *b, int species, const uint32_t **lo_rank,
                      const uint64_t **hi_off, int *n_lo, int *n_hi);

/* ------------------------------------------------------- Hamiltonians -- */

/* One spin bond: H += jz S^z_i S^z_j + jxy (S^x_i S^x_j + S^y_i S^y_j). */
typedef struct { int32_t i, j; double jz, jxy; } hphi_spin_bond;

/* One transfer: H += -t sum_sigma (c+_{i sigma} c_{j sigma} + h.c.). */
typedef struct { int32_t i, j; double t; } hphi_hop;

/* Spin-1/2 XXZ Hamiltonian on a spin basis (Heisenberg model of Sec. 3.2):
 *   H = sum_b [jz_b S^z_i S^z_j + jxy_b (S^x_i S^x_j + S^y_i S^y_j)]
 *       - sum_i hz[i] S^z_i          (hz may be NULL).
 * Bond lists are literal: a repeated pair adds. The basis must outlive the
 * Hamiltonian. Errors: INVALID_ARG (site >= n_sites, i == j, n_bonds < 0 or
 * > 4096, basis of the wrong kind), OUT_OF_MEMORY, DEVICE. */
int hphi_ham_spin(hphi_basis *b, const hphi_spin_bond *bonds, int n_bonds,
                  const double *hz, hphi_ham **out);

/* Hubbard Hamiltonian (Sec. 3.4, Eq. Hquench with a static U; Sec. 5):
 *   H = -sum_h t_h sum_sigma (c+_i c_j + h.c.) + sum_i u_site[i] n_i,up n_i,dn.
 * Fermion order: all up orbitals (ascending site) before all down orbitals,
 * so a hop's sign is (-1)^(occupied same-species sites strictly between
 * i and j). Errors: INVALID_ARG (site >= n_sites, i == j, u_site NULL,
 * more than 128 distinct t values), OUT_OF_MEMORY, DEVICE. */
int hphi_ham_hubbard(hphi_basis *b, const hphi_hop *hops, int n_hops,
                     const double *u_site, hphi_ham **out);

/* Spin-S Heisenberg Hamiltonian on a spin-S basis (keyword 2S, Sec. 4.1):
 *   H = sum_b [jz S^z_i S^z_j + jxy (S^x_i S^x_j + S^y_i S^y_j)]
 *       - sum_i hz[i] S^z_i + sum_i d_ion[i] (S^z_i)^2   (hz, d_ion may be NULL),
 * with the spin-S ladder elements <s+-1| S^+- |s> = sqrt(S(S+1) - s(s+-1)).
 * Every method takes it with one real or complex vector per call. Errors:
 * INVALID_ARG (site >= n_sites, i == j, n_bonds < 0 or > 4096, basis not
 * spin-S), OUT_OF_MEMORY, DEVICE. */
int hphi_ham_spin_s(hphi_basis *b, const hphi_spin_bond *bonds, int n_bonds, const double *hz,
                    const double *d_ion, hphi_ham **out);

/* One anisotropic spin bond:
 * H += jx S^x_i S^x_j + jy S^y_i S^y_j + jz S^z_i S^z_j. */
typedef struct { int32_t i, j; double jx, jy, jz; } hphi_xyz_bond;

/* Spin-1/2 Hamiltonian without S^z conservation on a SpinGC basis (SpinGC
 * keyword, Sec. 4.1):
 *   H = sum_b [jx S^x_i S^x_j + jy S^y_i S^y_j + jz S^z_i S^z_j]
 *       - sum_i (hx[i] S^x_i + hz[i] S^z_i)        (hx, hz may be NULL).
 * Every coefficient is real, so H is a real symmetric matrix; jx != jy and
 * hx break S^z conservation. Every method takes it with one real or
 * complex vector per call (as the Hubbard Hamiltonians); S(q, w) works on
 * it through hphi_szq. Errors: INVALID_ARG (site >= n_sites, i == j,
 * n_bonds < 0 or > 4096, basis not SpinGC), OUT_OF_MEMORY, DEVICE. */
int hphi_ham_spin_gc(hphi_basis *b, const hphi_xyz_bond *bonds, int n_bonds, const double *hx,
                     const double *hz, hphi_ham **out);

/* Two-body terms of one site pair (i, j), i != j (Sec. 5, Eq. ham_general,
 * with one coefficient per term kind):
 *   v      inter-site Coulomb   v n_i n_j,  n_i = n_i,up + n_i,dn
 *   j_hund Hund               - j_hund (n_i,up n_j,up + n_i,dn n_j,dn)
 *   j_ex   exchange             j_ex (c+_i,up c_j,up c+_j,dn c_i,dn + h.c.)
 *   j_pair pair hopping         j_pair (c+_i,up c_j,up c+_i,dn c_j,dn + h.c.)
 * The Wannier-function form of the paper is j_hund = j_ex = j_pair = J_ij. */
typedef struct { int32_t i, j; double v, j_hund, j_ex, j_pair; } hphi_pair_term;

/* Hubbard Hamiltonian with the two-body terms of Eq. ham_general (Sec. 5):
 * hphi_ham_hubbard's H plus the listed pair terms (a repeated pair adds).
 * Every term conserves N_up and N_dn, so the basis is the same (N_up, N_dn)
 * sector. The terms' fermion signs follow the same ordering (all up
 * orbitals before all down orbitals): an exchange or pair-hopping element
 * carries (-1)^(occupied up sites strictly between i and j) times
 * (-1)^(occupied down sites strictly between i and j). Every method that
 * takes a Hubbard Hamiltonian takes this one. n_pairs = 0 gives
 * hphi_ham_hubbard. Errors: INVALID_ARG (site >= n_sites, i == j,
 * n_pairs < 0 or > 1024, null pairs with n_pairs > 0, and hphi_ham_hubbard's
 * conditions), OUT_OF_MEMORY, DEVICE. */
int hphi_ham_hubbard_ext(hphi_basis *b, const hphi_hop *hops, int n_hops,
                         const double *u_site, const hphi_pair_term *pairs, int n_pairs,
                         hphi_ham **out);

/* Time-dependent amplitudes of a Hubbard Hamiltonian (Sec. 3.4: H(t) with
 * one-body t_ij(t) and two-body terms I(t), here the U, V, Hund, exchange
 * and pair-hopping coefficients of the terms given at build). Frame k holds
 * every amplitude at one time; the terms themselves (sites, kinds) are fixed.
 * Host arrays, row-major, read during the build only:
 *   hop_t     [n_frames][n_hops]  t of each hop, in the order of hops
 *   hop_t_im  [n_frames][n_hops]  imaginary parts: the hop term becomes
 *             -(t c+_i c_j + t* c+_j c_i), t = hop_t + i hop_t_im (Peierls
 *             phases of a vector potential, fluxes)
 *   u_site    [n_frames][n_sites] U_i
 *   pair_v    [n_frames][n_pairs][4] v, j_hund, j_ex, j_pair of each pair term
 * A NULL array keeps the build arguments' values in every frame (hop_t_im:
 * zero). A Hamiltonian with a nonzero imaginary part in any frame acts on
 * complex vectors only: hphi_mult with C128/C64, hphi_time_evolve and
 * hphi_ctpq; the real-vector methods return UNSUPPORTED, and so does
 * hphi_sqw (its COCG needs a complex-symmetric z - H). */
typedef struct {
    int n_frames;          /* 1 .. 65536                                     */
    const double *hop_t;
    const double *hop_t_im;
    const double *u_site;
    const double *pair_v;
} hphi_hub_frames;

/* hphi_ham_hubbard_ext with time-dependent amplitudes: frame 0 is in force
 * after the build (hops[k].t, u_site and the pairs' values are overridden
 * where the frames give them). Equal frames share device tables (frames are
 * deduplicated per kind); each distinct set of pair values holds
 * (dim_up + dim_dn) doubles of same-species diagonal on the device. Hops
 * keep the uniform-|t| kernels when t_k(frame) = s_k tau(frame) with one
 * sign s_k per hop in every frame and no imaginary part; U keeps the
 * uniform kernels when every frame's U_i are equal. n_frames = 1 builds a
 * fixed Hamiltonian (e.g. with complex transfers). hphi_time_evolve steps
 * through the frames;
 * hphi_ham_set_frame selects one for every other call.
 * Errors: INVALID_ARG (null frames, n_frames outside [1, 65536], no array
 * given, hop_t without hops, pair_v without pair terms, a non-finite value,
 * more than 127 distinct matrix-element trajectories (a complex transfer
 * counts twice), and hphi_ham_hubbard_ext's
 * conditions), OUT_OF_MEMORY, DEVICE. */
int hphi_ham_hubbard_td(hphi_basis *b, const hphi_hop *hops, int n_hops,
                        const double *u_site, const hphi_pair_term *pairs, int n_pairs,
                        const hphi_hub_frames *frames, hphi_ham **out);

/* Puts frame `frame` of a Hamiltonian built by hphi_ham_hubbard_td in
 * force for the calls that follow on `stream`: device-to-device copies of
 * the frame's tables, ordered on the stream after earlier work (the
 * one-stream rule of hphi_ham applies). Asynchronous.
 * Errors: INVALID_ARG (no frames, frame outside [0, n_frames)), BUSY, DEVICE. */
int hphi_ham_set_frame(hphi_ham *h, int frame, void *stream);

/* Number of frames (0: fixed amplitudes) and the frame in force. */
int hphi_ham_frames(const hphi_ham *h, int *n_frames, int *current);

void hphi_ham_free(hphi_ham *h);

/* Launch schedule of the H*v kernels of one Hamiltonian (set by the
 * autotuner; zero fields keep the current value). Results do not depend on
 * the schedule beyond floating-point summation order.
 *   hub_slab_cols   columns per L2-resident slab of the Hubbard T_up kernel
 *                   (8, 16, 32, 64 or 128; 128 only with hub_sweep 3 or 5
 *                   on one real vector, otherwise 64)
 *   hub_groups      workgroups per XCD of that kernel (1..1024)
 *   hub_item_rows   rows per work item of that kernel (8..128)
 *   hub_row_cols    T_dn kernel variant (values below 5 select, at any
 *                   size, the kernels that sectors beyond 16 sites or
 *                   32767 down states fall back to): 1 or 2 = sliced-ELL
 *                   table loads, 3 = row metadata in LDS (up to 16
 *                   sites; otherwise as 1), 4 = as 3 with hop-ordered slots (up to 32767
 *                   down states; otherwise as 3), 5 = as 4 with each row
 *                   staged by one batch of loads (up to 16384 down states
 *                   per lane group; otherwise as 4; bit-identical to 4),
 *                   6 = as 5 with slot words that carry the LDS byte
 *                   offset of one slot of each pair (one real vector, up
 *                   to 16383 down states; otherwise as 5; bit-identical
 *                   to 5; the default)
 *   spin_per_cu     spin H*v workgroups per compute unit (1..16)
 *   spin_implicit   1: spin H*v rebuilds configurations from row indices
 *                   (the path sectors without a stored state list take:
 *                   more than 32 sites or 2^32 states); -1: stored list
 *                   when there is one
 *   hub_sweep       Hubbard T_up kernel (uniform |t| tables): 1 = per-XCD
 *                   queues of (slab, hub_item_rows rows) work items;
 *                   3 = as 1 with two adjacent columns per lane (one real
 *                   vector with an even number of down states; otherwise
 *                   as 1); 5 = as 3, one wave per row, each row's
 *                   neighbour lists walked in batches of 12 loads
 *                   (128-column slabs with two columns per lane or
 *                   64-column slabs; bit-identical to 3 at the same slab
 *                   width); 7 = block tiles: a work item is (slab of 16
 *                   columns, block of the up rows sharing their top
 *                   hub_tile_bits sites), the block's rows of the slab are
 *                   staged in LDS once, hops that keep those sites read
 *                   LDS and only the others gather from memory (one real
 *                   vector, even number of down states; otherwise as 5;
 *                   the products equal those of 5 up to summation order;
 *                   the default where the tables could be built, else 5).
 *                   2, 4 and 6 (slower variants) are no longer built:
 *                   INVALID_ARG.
 *   hub_row_order   order in which the T_up kernels of hub_sweep 1, 3 and
 *                   5 take the up rows: 1 = index order, 2 = reverse
 *                   Cuthill-McKee order of the up-species hop graph (rows
 *                   processed close together share more neighbour rows, so
 *                   more of them are still in L2); the products do not
 *                   depend on it (each element's sum keeps its order)
 *   spin_tables     where the stored-list spin kernel keeps its rank
 *                   tables: 1 = both 32-bit tables in LDS, 256-thread
 *                   workgroups; 2 = hi_off in 32 bits and lo_rank narrowed
 *                   to 16 bits in LDS, 1024-thread workgroups (the path
 *                   sectors of 23 to 28 sites take); 3 = tables in global
 *                   memory; -1 = automatic by size (the default). A forced
 *                   choice the sector's tables do not fit returns
 *                   UNSUPPORTED from the product. The products are the same
 *                   sums in the same order whichever is chosen.
 *   hub_tile_bits   top up-species sites that label the blocks of hub_sweep
 *                   7 (the tables are rebuilt when it changes); -1 = the
 *                   fewest sites whose largest block of 16 FP64 columns
 *                   fits LDS (the default)
 *   spin_split      1: the spin product in two passes -- the bonds with
 *                   an end in the low half of the sites (and the fields),
 *                   then the bonds inside the high half in slab order (a
 *                   state's high-bond partners sit at the same position of
 *                   another block of its class); products without fused
 *                   dots, at most 128 high bonds; otherwise one pass.
 *                   2: one pass over blocks of states (products without
 *                   fused dots; on the implicit basis the only product for
 *                   vector blocks and complex vectors): a workgroup
 *                   stages the block of one high pattern in LDS, bonds
 *                   inside the low part read their partners there (partner
 *                   positions from per-bond tables over the low patterns),
 *                   bonds inside the high part read the same positions of
 *                   the partner block, bonds across read one position of
 *                   the partner block from a per-site table; where no split
 *                   point gives blocks that fit LDS, as 1 on the stored
 *                   list and UNSUPPORTED on the implicit basis for several
 *                   lanes. 3 (the default): 2 on the implicit basis,
 *                   one pass on the stored list. -1: one pass. The products
 *                   equal the one-pass ones up to summation order.
 *                   hphi_lanczos_noalloc always takes one pass (the other
 *                   layouts build device tables on first use).
 *   spin_blk_lo     split point (sites in the low part) of spin_split 2;
 *                   -1 = the most low sites (at most the basis's own split)
 *                   whose largest block leaves room in a CU's LDS for three
 *                   workgroups with 4-byte values, five with 8-byte ones
 *                   (the default); a forced choice whose largest block
 *                   does not fit LDS at all returns UNSUPPORTED from the
 *                   product.
 * Errors: INVALID_ARG (value outside its range), UNSUPPORTED (hub_sweep 7
 * or hub_tile_bits for blocks the tile kernel cannot take). */
typedef struct {
    int hub_slab_cols;
    int hub_groups;
    int hub_item_rows;
    int hub_row_cols;
    int spin_per_cu;
    int spin_implicit;
    int hub_sweep;
    int hub_row_order;
    int spin_tables;
    int hub_tile_bits;
    int spin_split;
    int spin_blk_lo;
} hphi_schedule;

int hphi_ham_set_schedule(hphi_ham *h, const hphi_schedule *s);
int hphi_ham_get_schedule(const hphi_ham *h, hphi_schedule *s);

/* Exact trace of H over the sector, summed on the device in FP64. */
int hphi_ham_trace(hphi_ham *h, double *trace_out, void *stream);

/* ------------------------------------------------------------- H * v -- */

/* w = H v for a block of nvec vectors of type dt (interleaved layout),
 * the product at the core of every Krylov and power method (Sec. 1).
 * Real types hold nvec real vectors, complex types nvec complex vectors.
 * F32 / C64 store in float and accumulate each row in float.
 * Spin sectors without a stored state list (more than 32 sites or 2^32
 * states) take several lanes per state (vector blocks, complex vectors)
 * only through the block-staged layout (schedule spin_split 2 or the
 * default 3), whose largest block must fit LDS; otherwise UNSUPPORTED.
 * Asynchronous on `stream`. v_dev and w_dev must not alias.
 * Errors: INVALID_ARG (nvec < 1 or > 32, null pointers), UNSUPPORTED,
 * DEVICE. */
int hphi_mult(hphi_ham *h, hphi_dtype dt, const void *v_dev, void *w_dev,
              int64_t nvec, void *stream);

/* ------------------------------------------------------------ Lanczos -- */

typedef struct {
    int max_iter;          /* Krylov steps (>= 1)                            */
    int check_every;       /* 0: run max_iter steps; m > 0: every m steps the
                              host solves T_k and stops when the lowest
                              n_energies Ritz values move by < tol           */
    double tol;            /* convergence threshold for check_every > 0      */
    double resid_tol;      /* > 0 (with check_every): stopping also needs the
                              residual estimate beta_k |s_k| of the lowest
                              Ritz pair (s the eigenvector of T_k) below
                              resid_tol max(1, |theta|): the Ritz vector's
                              error is then about that over the spectral gap
                              (an energy test alone leaves it near the square
                              root of the energy's)                          */
    uint64_t seed;         /* start vector: SplitMix64 uniform [-1/2, 1/2)   */
    const void *v0_dev;    /* or a caller start vector (storage dtype); NULL
                              = use the seed                                 */
    hphi_dtype storage;    /* HPHI_F64 or HPHI_F32 (FP64 dots and scalars);
                              HPHI_C128 or HPHI_C64: complex vectors, for a
                              Hermitian H that is not real (complex
                              transfers): alpha and beta stay real, the
                              start vector has uniform real and imaginary
                              parts, v0_dev and psi_dev are complex; no
                              refinement, not in hphi_lanczos_noalloc     */
    void *stream;          /* hipStream_t                                    */
    double *alpha_out;     /* optional host arrays of max_iter entries:      */
    double *beta_out;      /*   T_k diagonal and beta[k] (beta[0] = 0)       */
    void *psi_dev;         /* optional: ground-state Ritz vector (storage
                              dtype, normalized), from a second pass         */
    int use_graph;         /* capture the iteration in a hipGraph            */
    int time_kernels;      /* bracket every H*v with HIP events on `stream`
                              (not with use_graph); totals go to info        */
    int refine;            /* 1: after the solve, rebuild the lowest Ritz
                              vector by a second pass accumulated in FP64,
                              normalize it in FP64 and take its Rayleigh
                              quotient and residual with an FP64 product;
                              then run refine_steps FP64 Lanczos steps from
                              that vector; energies[0] is the lowest Ritz
                              value of that short run (the Rayleigh quotient
                              itself with refine_steps < 0; see
                              hphi_lanczos_info)                             */
    int refine_steps;      /* FP64 steps of the refinement (0: 16)           */
} hphi_lanczos_opts;

typedef struct {
    int iterations;        /* Krylov steps done                              */
    int converged;         /* 1 if the check_every test passed               */
    int breakdown;         /* 1 if beta_k fell below 1e-13 max(1, |alpha|)   */
    double seconds;        /* wall time of the solve                         */
    double hv_seconds;     /* with time_kernels: summed H*v launch durations */
    int hv_calls;          /* number of H*v launches timed                   */
    int fused_update;      /* 1: every product after the first also did the
                              previous step's update (w -= alpha q, beta =
                              |w|) in its rows kernel (Hubbard, one real
                              vector, hub_row_cols 5 or 6); hv_seconds
                              includes it */
    double hv_second_kernel_seconds; /* with time_kernels, Hubbard: summed
                              durations of the column (T_up) kernel alone,
                              from an event between the two launches       */
    /* With refine = 1 (otherwise NaN):                                     */
    double ritz_e0;        /* lowest Ritz value of T_k (before refinement)   */
    double rq_e0;          /* rho = <psi|H psi> of the FP64 Ritz vector psi,
                              |psi| = 1, product and sums in FP64            */
    double residual;       /* eps = |H psi - rho psi|: some eigenvalue of H
                              lies within eps of rho (bound of Weinstein)    */
    double err_est;        /* eps^2 / (theta_2 - rho), theta_2 the lowest
                              Ritz value distinct from the first: the error
                              of rho by the bound of Temple when theta_2
                              does not exceed the second eigenvalue by much
                              (an estimate, not a bound)                    */
    double polish_e0;      /* lowest Ritz value of the FP64 steps from psi
                              (below rho: the Krylov space holds psi); NaN
                              without them                                  */
    double polish_resid;   /* its residual estimate beta_m |s_m| (FP64)      */
} hphi_lanczos_info;

/* Lanczos ground state (Sec. 1): v_0 = r/|r|; w = H v_k - beta_k v_{k-1};
 * alpha_k = <v_k, w>; w -= alpha_k v_k; beta_{k+1} = |w|; v_{k+1} = w /
 * beta_{k+1}; no reorthogonalization. The lowest n_energies eigenvalues of
 * the tridiagonal T_k come from host FP64 Sturm bisection. With FP32
 * storage the Krylov vectors carry FP32 rounding, which bounds the Ritz
 * values' accuracy by about 1e-7 |H|; opts->refine = 1 adds the FP64
 * Rayleigh quotient of the Ritz vector (its error is quadratic in the
 * vector's) and its residual, which bound the result's error without an
 * FP64 run, then a few FP64 Lanczos steps from that vector (a restart in
 * FP64: its Krylov space holds the vector, so its lowest Ritz value lies
 * at or below the Rayleigh quotient). The refinement needs a second pass
 * and five FP64 vectors of workspace. Synchronous. With HPHI_PROGRESS set
 * in the environment each convergence check (every check_every steps)
 * prints the step count and the lowest Ritz value on stderr.
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE, BUSY. */
int hphi_lanczos(hphi_ham *h, const hphi_lanczos_opts *opts, double *energies,
                 int n_energies, hphi_lanczos_info *info);

/* For callers that cannot allocate device memory (code that runs while a
 * stream is captured into a graph, tight serving loops, harnesses that
 * forbid hipMalloc): hphi_lanczos with every device buffer (the three
 * Krylov vectors, the device scalars, the T_k coefficients, the Ritz
 * coefficients of the second pass and, with refine, the five FP64 vectors
 * of the refinement) taken from a static device array of
 * HPHI_NOALLOC_SCRATCH_BYTES that the library holds on each device from
 * hphi_init to the end of the process, instead of allocated per call. The
 * caller still passes the outputs (host arrays, psi_dev). Each buffer is
 * rounded up to 256 bytes; the call needs
 *   3 * S(dim * elem) + S(128) + S(8 * (2 * max_iter + 4)) + S(8 * max_iter)
 *   + (refine ? 5 * S(8 * dim) + S(128) + S(8 * (2 * r + 4)) : 0)  bytes,
 * S(n) = n rounded up to 256, r = refine_steps (16 when 0),
 * elem = 8 (F64) or 4 (F32): FP64 solves up to about 2.79e6 states (a
 * 24-site chain at Sz = 0). The library clears what must start at zero on
 * each call. Spin products run in one pass whatever spin_split says (the
 * other layouts build device tables on first use). Every call on a
 * device shares that device's array: a call
 * that starts while another one holds it (from another thread) returns
 * HPHI_ERR_BUSY; calls must not overlap on one device. Synchronous.
 * Errors: INVALID_ARG (a workspace need above the array, use_graph or
 * time_kernels set, and as hphi_lanczos), BUSY, DEVICE. */
#define HPHI_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int hphi_lanczos_noalloc(hphi_ham *h, const hphi_lanczos_opts *opts, double *energies,
                         int n_energies, hphi_lanczos_info *info);

/* One request of a batched Lanczos launch. */
typedef struct {
    hphi_ham *ham;         /* spin Hamiltonian on a stored basis (<= 32 sites) */
    int max_iter;          /* Krylov steps                                    */
    uint64_t seed;         /* SplitMix64 start vector (as hphi_lanczos)       */
    double *alpha_out;     /* optional host arrays, max_iter entries          */
    double *beta_out;
    double energy;         /* out: lowest Ritz value of T_k                   */
    int iterations;        /* out: steps done                                 */
    int breakdown;         /* out: 1 if beta_k fell below the threshold       */
} hphi_batch_item;

/* Many independent Lanczos ground-state solves in one launch (the
 * recurrence of hphi_lanczos, FP64 vectors). Meant for sectors small enough
 * that a single solve is bound by kernel-launch latency. A launch whose
 * requests together need at most one workgroup per CU runs each request on a
 * team of up to 32 workgroups (1024 rows each, or more for sectors above
 * 32768 states) that meet at a barrier of their own twice per step; larger
 * launches run each request whose vector fits in LDS on one workgroup (the
 * others still as teams, in launches of at most one workgroup per CU). Every reduction follows an
 * order fixed by the rows (64-row chunks, chunks in order within 1024-row
 * slices, slices in order), so a request's numbers do not depend on the
 * other requests in the launch nor on which of the two ways ran it. The
 * library allocates 3 * dim doubles of workspace per request for the
 * call (plus under 2 % of that for partial sums). Synchronous on `stream`. Errors: INVALID_ARG (n < 1,
 * max_iter < 1), UNSUPPORTED (a Hamiltonian that is not a spin model on a
 * stored basis), OUT_OF_MEMORY, DEVICE (also when a team barrier waited
 * for seconds without its members arriving: within one launch the members
 * always arrive, so this needs many concurrent launches of wide teams
 * crowding each other off the CUs; every wave then leaves and the call
 * reports the item). */
int hphi_lanczos_batch(hphi_batch_item *items, int n, void *stream);

/* Lowest k eigenvalues (ascending) of the symmetric tridiagonal matrix with
 * diagonal alpha[0..n) and off-diagonal beta[1..n) (beta[0] ignored), by
 * Sturm-sequence bisection in FP64; the host routine hphi_lanczos uses.
 * If vec is non-NULL it receives the normalized eigenvector of the lowest
 * eigenvalue (n entries, inverse iteration). */
int hphi_tridiag_lowest(const double *alpha, const double *beta, int n, int k,
                        double *eig_out, double *vec);

/* ----------------------------------------------------------------- cTPQ -- */

typedef struct {
    int n_vec;             /* independent random vectors (1..16)             */
    int n_max;             /* Taylor order of U_c                            */
    double dtau;           /* imaginary-time slice                           */
    int k_steps;           /* steps: beta_k = k dtau, k = 1..k_steps         */
    hphi_dtype storage;    /* HPHI_C128 or HPHI_C64                          */
    uint64_t seed;         /* vector j uses seed + j: complex Gaussian
                              entries (Box-Muller on SplitMix64 outputs)     */
    const void *phi0_dev;  /* or a caller start block [dim][n_vec] complex
                              (a previous run's phi_dev output resumes that
                              run: D_k, <H>, <H^2> continue to rounding;
                              beta_k is counted by the caller)              */
    void *stream;
    int use_graph;         /* capture one step's launches in a hipGraph and
                              replay it (the same numbers as without)        */
} hphi_ctpq_opts;

/* Canonical TPQ (Sec. 3.5.1): Phi_k = U_c(dtau)^k Phi_rand with
 * U_c = sum_{n<=n_max} (-dtau H / 2)^n / n!, applied to n_vec vectors at
 * once by block H*V. After each step the squared norm N (FP64) gives
 * D_k = N_k / N_{k-1} (D_0 = N_0 = |Phi_rand|^2), the state is renormalized
 * and <H> = <Phi|H|Phi>, <H^2> = |H Phi|^2 are recorded.
 * Outputs (host, (k_steps + 1) * n_vec, row k = beta_k): D_out, E_out,
 * E2_out (any may be NULL). phi_dev (device, [dim][n_vec] complex of the
 * storage type) receives the final normalized states. Synchronous.
 * Workspace (library-allocated for the call): two blocks of the caller's
 * size, three for spin sectors with n_vec >= 4 on a stored basis (the first
 * order's H Phi is kept for the <H>, <H^2> pass).
 * Errors: INVALID_ARG, OUT_OF_MEMORY, DEVICE. */
int hphi_ctpq(hphi_ham *h, const hphi_ctpq_opts *opts, void *phi_dev,
              double *D_out, double *E_out, double *E2_out);

/* ------------------------------------------------ real-time evolution -- */

typedef struct {
    int n_vec;             /* complex vectors evolved together (1..16;
                              Hubbard models: 1)                             */
    int n_max;             /* Taylor order (1..64; the paper's default 10)    */
    double dt;             /* time step (finite, nonzero; default 0.01)       */
    int n_steps;           /* steps: t_k = k dt, k = 0..n_steps               */
    hphi_dtype storage;    /* HPHI_C128 or HPHI_C64                          */
    void *stream;
    int use_graph;         /* capture one step's launches in a hipGraph and
                              replay it (the same numbers as without)        */
    int first_frame;       /* time-dependent H: frame of t_0 (0 .. n_frames-1;
                              a later call continues a run's frames)         */
} hphi_tevol_opts;

/* Real-time evolution by the truncated Taylor series of Sec. 3.4:
 * psi(t + dt) = sum_{n=0}^{n_max} (-i H dt)^n / n! psi(t), evaluated in
 * Horner form y <- psi + (-i dt / n) H y (n = n_max .. 1), each order one
 * block H*V with the complex combination fused into its epilogue.
 * psi_dev: [dim][n_vec] complex of the storage type, in and out (the state
 * at t_{n_steps} on return); the caller owns it. Per recorded time t_k
 * (k = 0..n_steps): norm_out[k * n_vec + j] = <psi_j|psi_j>,
 * energy_out[k * n_vec + j] = <psi_j|H|psi_j> / <psi_j|psi_j>, and for
 * Hubbard models docc_out[k] = sum_i <n_i,up n_i,dn> / (N_s <psi|psi>)
 * (the double occupancy of the paper's quench example). Output arrays are
 * host memory and nullable. Synchronous.
 * Time-dependent H (a Hamiltonian with frames, hphi_ham_hubbard_td): H(t_k)
 * is frame min(first_frame + k, n_frames - 1); the step from t_k to t_k+1
 * applies it as a constant over the step, and energy_out[k] is <H(t_k)>.
 * On return frame min(first_frame + n_steps, n_frames - 1) is in force.
 * first_frame must be 0 for a Hamiltonian without frames.
 * Errors: INVALID_ARG (ranges above, docc_out for a spin model,
 * first_frame outside the frames), UNSUPPORTED (several vectors with a
 * Hubbard model, use_graph with frames), OUT_OF_MEMORY, DEVICE. */
int hphi_time_evolve(hphi_ham *h, const hphi_tevol_opts *opts, void *psi_dev,
                     double *norm_out, double *energy_out, double *docc_out);

/* --------------------------------------------------------------- LOBPCG -- */

typedef struct {
    int n_eig;             /* M: lowest eigenpairs wanted (1..32, 3M <= dim)  */
    int max_iter;
    double tol;            /* stop when every |H Phi_n - E_n Phi_n| < tol     */
    uint64_t seed;         /* start vector n: SplitMix64 uniform, seed + n    */
    int precond;           /* 1: point-Jacobi r <- r / (H_xx - e_shift)       */
    double e_shift;        /* shift of the preconditioner; 0: a lower bound of
                              the spectrum from the couplings                */
    void *stream;
} hphi_lobpcg_opts;

typedef struct {
    int iterations;
    int converged;
    int64_t hv_calls;
    double seconds;
} hphi_lobpcg_info;

/* Lowest eigenpairs by the locally optimal block preconditioned conjugate
 * gradient method (Sec. 3.3): subspace (r, Phi, p) of 3M vectors, H_sub =
 * V^T H V and O_sub = V^T V from device block Gram products, the
 * generalized eigenproblem of size 3M solved on the host (near-null
 * directions of O_sub dropped), updates Phi = V phi, p = (r, 0, p) phi as
 * block linear combinations on the device. The point-Jacobi preconditioner
 * needs the diagonal: stored-list spin bases and Hubbard bases.
 * energies_out[M] ascending Ritz values, resid_out[M] (nullable) residual
 * norms, vecs_dev (nullable, device, M * dim FP64, caller-owned) the
 * normalized eigenvectors one after another. Synchronous.
 * Errors: INVALID_ARG (ranges), UNSUPPORTED (preconditioner without a stored
 * basis; subspace rank below M), OUT_OF_MEMORY, DEVICE. */
int hphi_lobpcg(hphi_ham *h, const hphi_lobpcg_opts *opts, double *energies_out,
                double *resid_out, void *vecs_dev, hphi_lobpcg_info *info);

/* --------------------------------------------------- S^zz(q, w) / D(z) -- */

/* Excitation b = sum_l e^{i q x_l} S^z_l psi (Sec. 3.2): for a spin basis
 * S^z_l = +-1/2 by bit l of the state (stored list, N <= 32); for a Hubbard
 * basis S^z_l = (n_l,up - n_l,dn) / 2 at index r_up * dim_dn + r_dn.
 * phase[2*l], phase[2*l+1] = (cos, sin)(q x_l) per site, host array.
 * psi_dev: F64 vector; b_dev: C128 vector, caller-owned. Synchronous.
 * Errors: INVALID_ARG (null, more than 64 sites), UNSUPPORTED (spin basis
 * not stored), OUT_OF_MEMORY, DEVICE. */
int hphi_szq(hphi_ham *h, const double *phase, const void *psi_dev, void *b_dev,
             void *stream);

typedef struct {
    int max_iter;          /* COCG steps cap                                 */
    double tol;            /* stop when max_j |r_j| / |b| < tol              */
    int seed_shift;        /* index of the seed system (-1: middle shift)    */
    void *stream;
} hphi_sqw_opts;

typedef struct {
    int iterations;
    int converged;
    double max_residual;   /* max_j |r_j| / |b| at exit                      */
    double seconds;
} hphi_sqw_info;

/* Dynamical correlation D(z_j) = <b| (z_j - H)^-1 |b> for n_shift complex
 * shifts z_j = (z_re[j], z_im[j]) from one Krylov sequence (shifted COCG on
 * the complex-symmetric z - H; Sec. 3.2, method "CG"). Only the projections
 * <b|x_j> are kept (scalar recurrences per shift on the device). A complex
 * b runs two sequences, from Re b and Im b, and D = D_Re + D_Im (exact for
 * the real symmetric Hamiltonians here; avoids the COCG breakdown b^T b = 0
 * of momentum excitations; a part with norm <= tol |b| runs no sequence,
 * its norm joins the residual). D_out receives 2 * n_shift doubles (re, im);
 * resid_out (nullable) the per-shift bound (|r_Re| + |r_Im|) / |b|;
 * info->iterations counts H*v calls of both sequences. b = 0 gives D = 0,
 * no iterations. b_dev: C128 vector, read only. Synchronous.
 * Errors: INVALID_ARG (n_shift < 1 or > 4096), OUT_OF_MEMORY, DEVICE. */
int hphi_sqw(hphi_ham *h, const hphi_sqw_opts *opts, const void *b_dev,
             const double *z_re, const double *z_im, int n_shift, double *D_out,
             double *resid_out, hphi_sqw_info *info);

/* hphi_sqw for n independent requests in one launch (the spectrum workflow
 * of Sec. 3.2 run for many small systems at once): request i is spin
 * Hamiltonian hams[i] on a stored basis whose rank tables fit in LDS (at
 * most 24 sites), excitation b_devs[i] (C128, read only) and the shifts
 * z_re/z_im[i * n_shift ...]. Each (request, part of b) sequence runs whole
 * on one workgroup: H*p with the COCG scalars of hphi_sqw, fixed-order
 * reductions over the request's rows, convergence checked every 8
 * iterations as there; a request's numbers do not depend on the rest of the
 * launch and equal hphi_sqw's up to the summation order. opts->stream,
 * tol, max_iter, seed_shift as for hphi_sqw. D_out: n * 2 * n_shift doubles,
 * resid_out (nullable) n * n_shift, info (nullable) n entries. Device
 * workspace: 3 complex vectors per request, allocated per call. Does not
 * take the Hamiltonians' call guard (it uses none of their scratch).
 * Synchronous. Errors: INVALID_ARG (n < 1, null arguments, n_shift outside
 * [1, 1024], Hamiltonians on different contexts), UNSUPPORTED (a
 * Hamiltonian that is not spin-1/2 on a stored basis, or whose tables
 * exceed LDS), OUT_OF_MEMORY, DEVICE. */
int hphi_sqw_batch(hphi_ham *const *hams, int n, const hphi_sqw_opts *opts, const void *const *b_devs,
                   const double *z_re, const double *z_im, int n_shift, double *D_out, double *resid_out,
                   hphi_sqw_info *info);

#ifdef __cplusplus
}
#endif
#endif /* HPHI_MI355_H */
