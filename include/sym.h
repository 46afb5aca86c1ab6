/*
 * sym.h -- C ABI of libsym.so: the one-loop Symanzik improved gauge action, its
 * molecular-dynamics force and a leapfrog update, on AMD Instinct MI355X (gfx950).
 *
 * Source of the method: D. Li, "The Calculation of Force in Lattice Quantum
 * Chromodynamics", arXiv:1808.02281, Sec. II ("One-loop Symanzik improved action").
 *
 * Conventions
 *   L = {Lx, Ly, Lz, Lt}: lattice dimensions, each even and >= 4, periodic in all four
 *     directions; V = Lx*Ly*Lz*Lt sites, 4V links; V/2 <= 2^24.
 *   Directions mu = 0..3 are x, y, z, t; U_{n,mu} lives on the link (n, n+mu) and
 *     U_{n,-mu} = U^dagger_{n-mu,mu}.
 *   prec: SYM_F32 (links, forces and momenta stored as float; products in float; every
 *     global sum -- action, Hamiltonian -- and the exponential of the link update in
 *     double) or SYM_F64 (everything in double).
 *   Link-field layout ("SoA even-odd"): for site n = (x,y,z,t) let
 *     lex = ((t*Lz + z)*Ly + y)*Lx + x, parity p = (x+y+z+t) & 1, cb = lex >> 1.
 *     The matrix element (row r, col c) of link (n, mu) is the complex number
 *     (re, im) at complex index ((mu*2 + p)*9 + 3*r + c) * (V/2) + cb, i.e. the buffer
 *     is real[4][2][9][V/2][2] of float or double. Force and momentum fields use the
 *     same layout.
 *   Canonical layout (sym_pack / sym_unpack only): complex array-of-structures
 *     (Lt, Lz, Ly, Lx, 4, 3, 3), row-major, float or double pairs per prec.
 *
 * Memory, streams, errors
 *   Every pointer argument except c_out/alpha_s_out of sym_coeffs is device memory,
 *   16-byte aligned, owned by the caller. The library allocates no device memory and
 *   keeps no state besides the process-wide switches below (coefficient override,
 *   force algorithm, kernel timing); scratch space is the caller's workspace ws of at
 *   least sym_workspace_bytes(L, prec) bytes.
 *   All work is enqueued on `stream` (a hipStream_t; NULL = default stream) and the
 *   calls return without synchronising; results such as S_dev are device doubles.
 *   Arguments are validated on the host before anything is launched; a negative
 *   sym_status is returned and nothing is enqueued. The device regions of one call
 *   (fields it writes, fields it reads, the scalar outputs and the part of ws it uses)
 *   must not overlap, since kernels read neighbouring links while writing; overlapping
 *   regions give SYM_EINVAL (fields that are only read may coincide). A failed launch returns SYM_EHIP;
 *   faults inside kernels surface at the caller's next synchronisation. Nothing throws
 *   or aborts across this interface. Calls on different streams with different
 *   workspaces may run concurrently.
 */
#ifndef SYM_H
#define SYM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* sym_stream_t; /* hipStream_t */

typedef enum {
  SYM_OK = 0,
  SYM_EINVAL = -1,       /* bad dimension, precision, scalar, algorithm or alignment */
  SYM_ENULL = -2,        /* a required pointer is NULL */
  SYM_EWORKSPACE = -3,   /* ws_bytes < sym_workspace_bytes(L, prec) */
  SYM_EHIP = -4,         /* a HIP launch failed (e.g. no gfx950 device) */
  SYM_EUNSUPPORTED = -5  /* valid request this library does not implement */
} sym_status;

typedef enum { SYM_F32 = 1, SYM_F64 = 2 } sym_prec;

/* Force algorithms (both compute the same G; see sym_set_force_algorithm). */
typedef enum { SYM_ALG_AUTO = 0, SYM_ALG_DIRECT = 1, SYM_ALG_FACTORED = 2 } sym_algorithm;

/*
 * Tadpole-improved loop coefficients from u0 (Sec. II, eq. 18_3_27_30 and the line
 * after eq. 18_6_6_3_0): alpha_s = -4 ln(u0) / 3.06839, c_out = {c_plaq, c_rect,
 * c_cube} = {1, -(1 + 0.4805 alpha_s)/(20 u0^2), -2 * 0.03325 alpha_s / u0^2}.
 * Host pointers; alpha_s_out may be NULL. SYM_EINVAL unless u0 > 0 and finite.
 */
int sym_coeffs(double u0, double c_out[3], double* alpha_s_out);

/* Bytes of workspace every entry point below needs for lattice L and precision prec
 * (0 if L or prec is invalid). */
size_t sym_workspace_bytes(const int32_t L[4], int prec);

/*
 * S_G = beta/3 sum_n sum_P c_P [3 - Re tr P_n] over the 34 loops per site
 * (eq. 18_6_4_1), accumulated in double. U: link field (read). S_dev: 4 device
 * doubles, written {S_G, W_P, W_R, W_C} with W_X = sum_n sum_{P in X} Re tr P_n.
 */
int sym_action(const int32_t L[4], double u0, double beta, int prec, const void* U, double* S_dev, void* ws,
               size_t ws_bytes, sym_stream_t stream);

/*
 * Gauge force of S_G on every link (Sec. II, eq. 18_7_25_2 and the algorithm after
 * eq. 18_6_6_13): G_{k,rho} = (beta/6) (U_{k,rho} t_{k,rho})_TA, with t the c_P-weighted
 * sum of the 48 staples of the link and TA of eq. 18_6_6_11. G is traceless and
 * antihermitian; the paper's Hermitian force -sum_i T_i dS/domega^i is iG, and
 * dS/domega^a = -2i tr(T_a G) for U -> exp(i omega.T) U. U: link field (read);
 * F: output, same layout, disjoint from U (else SYM_EINVAL). S_dev: NULL, or 4 device
 * doubles that receive the action as in sym_action, computed from the same staple sums
 * (each loop of class X is seen once from each of its L_X = 4, 6, 6 links); when the
 * factored algorithm runs with c_cube = 0 (u0 = 1, or an override) those sums do not
 * separate W_C, and the action kernel of sym_action fills S_dev after the force pass.
 * The factored algorithm (the default) requires special-unitary links; see
 * sym_set_force_algorithm and sym_check_links.
 */
int sym_force(const int32_t L[4], double u0, double beta, int prec, const void* U, void* F, double* S_dev, void* ws,
              size_t ws_bytes, sym_stream_t stream);

/*
 * sym_force for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same computation
 * and result as sym_force with the same arguments, with no ws argument. Its workspace is
 * a fixed 64 MiB array inside the library's device image, one per GPU, created with the
 * library's device code on that GPU and held until the process ends; no call allocates.
 * A lattice whose sym_workspace_bytes(L, prec) exceeds 64 MiB gives SYM_EWORKSPACE (about
 * 384 bytes per link in FP32 and 768 in FP64: up to 14^4 in FP32 and 12^4 in FP64; larger
 * lattices use sym_force with a caller workspace). Every call on one GPU uses that
 * GPU's array, whatever the stream: calls that overlap in time on one GPU race and give
 * wrong results; serialise them (e.g. one stream). The array needs no clearing: every
 * call overwrites what it reads.
 */
int sym_force_static(const int32_t L[4], double u0, double beta, int prec, const void* U, void* F, double* S_dev,
                     sym_stream_t stream);

/*
 * Gradient of S_G with respect to the link field, for automatic differentiation:
 * grad = 2 G U per link (G as in sym_force), the representative of dS/dU on the tangent
 * space of SU(3) at U. It satisfies dS = Re tr(grad^dagger dU) for every dU = i X U
 * with X Hermitian and traceless, hence dS/domega^a = -2i tr(T_a G) through any
 * parametrisation of the links that stays in SU(3) (e.g. U = exp(i omega.T) U0).
 * Same layout as U; S_dev as in sym_force.
 */
int sym_action_grad(const int32_t L[4], double u0, double beta, int prec, const void* U, void* grad, double* S_dev,
                    void* ws, size_t ws_bytes, sym_stream_t stream);

/*
 * nsteps leapfrog steps of the molecular dynamics of H = sum_links -tr(Pi^2) + S_G,
 * with U-dot = Pi U and Pi-dot = -G (U = exp(i omega.T), dU/domega = iTU; Sec. II):
 * per step Pi -= dt/2 G(U); U <- exp(dt Pi) U; Pi -= dt/2 G(U), consecutive half kicks
 * merged. The exponential and U update are in double. U: links (in/out); P: momenta
 * Pi = i sum_a p_a T_a, antihermitian (in/out), disjoint from U. H_dev: NULL or 2 device
 * doubles, {H before, H after}. SYM_F64: the updated links are stored as computed
 * (unitary to double rounding, no reunitarisation). SYM_F32: each updated link is
 * projected onto SU(3) in double (Gram-Schmidt of the first two rows, third row their
 * conjugate cross product) before it is rounded to float, so the unitarity defect stays
 * at float rounding (about 1e-7) however many steps are taken; the projection moves a
 * link by its defect, far below the FP32 force tolerance. The call returns before the
 * trajectory runs, so it cannot return a status for a trajectory that diverges (dt too
 * large): H then comes back non-finite or with a large H after - H before, and
 * sym_check_links counts the non-finite link elements; callers check either.
 */
int md_leapfrog(const int32_t L[4], double u0, double beta, int prec, void* U, void* P, double dt, int32_t nsteps,
                double* H_dev, void* ws, size_t ws_bytes, sym_stream_t stream);

/*
 * Batched force: the forces (and optionally the actions) of n independent lattices of
 * any valid shapes, sharing u0, beta and prec, with one launch per pass for every 64
 * lattices: workgroups walk the concatenated link tiles of all lattices with a static
 * schedule (one tile per workgroup, or a persistent grid that loops over tiles), so the
 * result does not depend on timing and each link's force is the same as sym_force's
 * with SYM_ALG_FACTORED. The work table is passed by value in
 * the kernel arguments, so a call may be captured into a HIP graph (with the same
 * workspace) and replayed. L: host array of n x 4 dims. U, F: host arrays of n device
 * pointers (fields as in sym_force). S_dev: NULL or 4n device doubles, {S, W_P, W_R, W_C}
 * per lattice. ws: at least sym_batch_workspace_bytes(n, L, prec) bytes (0 if invalid).
 * The schedule (number of persistent workgroups, or one workgroup per tile; tile order;
 * links per workgroup; occupancy cap) is the one sym_batch_autotune chose for these
 * shapes and precision in this process, else one workgroup of 256 links per tile in an
 * XCD-contiguous order at the occupancy of sym_force. Every schedule gives the same
 * forces; the actions agree to rounding (the partial sums are grouped by workgroup).
 */
size_t sym_batch_workspace_bytes(int n, const int32_t* L, int prec);
int sym_force_batch(int n, const int32_t* L, double u0, double beta, int prec, const void* const* U, void* const* F,
                    double* S_dev, void* ws, size_t ws_bytes, sym_stream_t stream);

/*
 * Autotuner for sym_force_batch: times (mean of 3 runs after a warm-up) every candidate
 * schedule of the force pass, 48 in all:
 *   links per workgroup {256, 128} x LDS reserved per workgroup {0, the sym_force default,
 *   96 KiB (one workgroup per CU)}, which caps the resident waves per SIMD, x grid {one
 *   workgroup per tile (reported as 0), 2048, 1024, 512 persistent workgroups} x tile
 *   order {strided, XCD-contiguous},
 * on the caller's fields (F is overwritten: it ends with the forces of the last schedule
 * timed), synchronising the stream, keeps the fastest for later sym_force_batch calls with
 * the same shapes and precision (in-process cache), and writes it to schedule_out
 * (nullable; 4 ints: grid, order, links per workgroup, LDS KiB with -1 = default). The
 * first max_log candidates are logged: log_schedules (nullable, 4 ints each, as
 * schedule_out) and log_ms (nullable, milliseconds per batch); n_log_out (nullable)
 * receives their number. SYM_EINVAL if max_log < 0. Not for use under graph capture.
 */
int sym_batch_autotune(int n, const int32_t* L, double u0, double beta, int prec, const void* const* U, void* const* F,
                       void* ws, size_t ws_bytes, sym_stream_t stream, int32_t* schedule_out, int32_t max_log,
                       int32_t* log_schedules, float* log_ms, int32_t* n_log_out);

/*
 * Fat-link smearing of the asqtad and HISQ actions and the force it induces on the thin
 * links (Sec. "Asqtad fermion": fat link V of eq. 18_6_6_7_2 with the Lepage term of
 * eq. 18_6_6_7, Naik term of eq. 18_6_6_3; Sec. "HISQ fermion": the pull-back F~ of
 * eq. 18_7_24_7 and B = U F~^T of eq. 18_7_24_6).
 *
 * c: host array {c_1, c_3, c_5, c_7, c_L, c_N}, finite (tadpole factors included by
 * the caller; the paper gives no values). Per link (x, mu):
 *   V_{x,mu} = c_1 U_{x,mu} + c_3 (6 three-staples) + c_5 (24 five-staples)
 *            + c_7 (48 seven-staples) + c_L (6 Lepage paths),  every path x -> x+mu;
 *   W_{x,mu} = c_N U_{x,mu} U_{x+mu,mu} U_{x+2mu,mu}.
 * The staggered phases of the fermion matrix are not applied (they belong to the
 * caller's adjoint fields below). All fields have the link layout of sym_force.
 *
 * sym_fat_links: U (read) -> V, W (W may be NULL).
 *
 * sym_fat_force: for given adjoint fields GV, GW (device, link layout; GW may be NULL:
 * no Naik term) differentiates Phi(U) = Re sum tr(GV^dagger V) + Re sum tr(GW^dagger W).
 * GV is the complex conjugate of the paper's F (eq. 18_7_24_4): F^T = GV^dagger.
 *   mode SYM_FAT_GRAD:  out = grad with dPhi = Re sum tr(grad^dagger dU) for every
 *                       complex variation dU (grad = dPhi/dRe U + i dPhi/dIm U, the
 *                       complex conjugate of the paper's F~): the input of the next
 *                       level of a smearing chain, and what autograd expects;
 *   mode SYM_FAT_FORCE: out = G = -(1/2) (U grad^dagger)_TA, traceless antihermitian,
 *                       with dPhi/domega^a = -2i tr(T_a G) for U -> exp(i omega.T) U:
 *                       the same convention as the gauge force G of sym_force, so the
 *                       two add.
 *   flag SYM_FAT_REUSE_LINKS (or-ed into the mode): ws already holds the forward
 *                       intermediates of a sym_fat_links call with the same L, prec, c
 *                       and U, made on this stream with no other use of ws since; the
 *                       two forward passes are then skipped (the caller vouches for
 *                       this: it cannot be checked). Other mode values: SYM_EINVAL.
 * ws: at least sym_fat_workspace_bytes(L, prec) bytes (19 matrices per link of
 * intermediate fields, of which sym_fat_links leaves 9 that the force reads).
 * Errors and asynchrony as for sym_force.
 */
typedef enum { SYM_FAT_GRAD = 0, SYM_FAT_FORCE = 1, SYM_FAT_REUSE_LINKS = 2 } sym_fat_mode;
size_t sym_fat_workspace_bytes(const int32_t L[4], int prec);
int sym_fat_links(const int32_t L[4], int prec, const double c[6], const void* U, void* V, void* W, void* ws,
                  size_t ws_bytes, sym_stream_t stream);
int sym_fat_force(const int32_t L[4], int prec, const double c[6], const void* U, const void* GV, const void* GW,
                  void* out, int mode, void* ws, size_t ws_bytes, sym_stream_t stream);

/*
 * Wilson fermion force with clover term for given vectors X, Y (Sec. "Wilson fermion
 * action with clover term"): D = A - kappa Dh (eq. 18_7_17_2) with the hopping part of
 * eq. 18_7_17_4, (1 - gamma_mu) U_{n,mu} forwards and (1 + gamma_mu) U_{n,-mu} backwards,
 * and the clover diagonal A_n = 1 - (c_sw kappa/16) sum_{mu != nu} [gamma_mu, gamma_nu]
 * Q_{n;mu nu} (eq. 18_7_18_0, kappa = 1/(2(m+4)); Q the clover leaves of eq. 17_7_20_8).
 * Gamma matrices are Hermitian in the DeGrand-Rossi basis, gamma_1..4 along x, y, z, t.
 *
 * sym_wilson_force writes, for every link, G = -(1/2) M_TA where
 * dPsi/domega^a = Re tr(i T_a M) = -2i tr(T_a G) for Psi(U) = Y^+ D X + c.c. (the
 * derivative of eq. 18_6_24_0; X = (D^+ D)^{-1} phi and Y = D X in an HMC, any fixed
 * vectors here). G is traceless antihermitian in the convention of sym_force; the
 * pseudofermion action at fixed X, Y changes by -dPsi, so its force is -G.
 * kappa, c_sw: finite. U: link field, special unitary to working precision (links are
 * read as two rows and the third rebuilt); X, Y: spinor fields (read); G: link layout
 * (out). ws: at least sym_wilson_workspace_bytes(L, prec) bytes (six anti-Hermitian
 * colour matrices per site, 9 reals each).
 *
 * Spinor layout: field[p][3*spin + colour][V/2] complex (T re, T im), parity p and
 * checkerboard index as for links; sym_pack_spinor / sym_unpack_spinor convert from / to
 * the canonical complex array (Lt,Lz,Ly,Lx,4,3).
 */
size_t sym_wilson_workspace_bytes(const int32_t L[4], int prec);
int sym_wilson_force(const int32_t L[4], int prec, double kappa, double csw, const void* U, const void* X,
                     const void* Y, void* G, void* ws, size_t ws_bytes, sym_stream_t stream);
int sym_pack_spinor(const int32_t L[4], int prec, const void* aos_lex, void* soa, sym_stream_t stream);
int sym_unpack_spinor(const int32_t L[4], int prec, const void* soa, void* aos_lex, sym_stream_t stream);

/*
 * Link-field check, the precondition of the factored force (links in SU(3)): writes 3
 * device doubles to out_dev, {max over links of ||U^dagger U - 1||_F, max over links of
 * |det U - 1|, number of links with a non-finite element}, computed in double (links with
 * a non-finite element are left out of the two maxima). U: link field (read). ws: at
 * least sym_workspace_bytes(L, prec) bytes (per-workgroup partials). Asynchronous like
 * every other call; a caller that guards a force evaluation compares out_dev[0] and
 * out_dev[1] with its tolerance (e.g. 1e-5 for FP32 fields) and out_dev[2] with 0.
 */
int sym_check_links(const int32_t L[4], int prec, const void* U, double* out_dev, void* ws, size_t ws_bytes,
                    sym_stream_t stream);

/*
 * Link-field repair for the same precondition: every link of U (in place) is replaced by
 * its projection onto SU(3), computed in double: the first row normalised, the second
 * orthogonalised against it (Gram-Schmidt) and normalised, the third set to the complex
 * conjugate of the cross product of the first two (det = 1), then rounded to the field's
 * precision. A link within rounding of SU(3) moves by its unitarity defect; a link with a
 * zero-norm row or a non-finite element comes out non-finite (sym_check_links counts
 * it). For fields that come from elsewhere (files, other codes); md_leapfrog keeps its own
 * links in SU(3). No workspace.
 */
int sym_reunitarise(const int32_t L[4], int prec, void* U, sym_stream_t stream);

/* Canonical (Lt,Lz,Ly,Lx,4,3,3) complex array -> SoA even-odd layout, and back. */
int sym_pack(const int32_t L[4], int prec, const void* aos_lex, void* soa, sym_stream_t stream);
int sym_unpack(const int32_t L[4], int prec, const void* soa, void* aos_lex, sym_stream_t stream);

/*
 * Process-wide test switch: use these three loop coefficients instead of the ones
 * derived from u0 (e.g. {1, 0, 0} gives the Wilson plaquette action). c = NULL
 * restores the u0 coefficients. Not meant to be flipped while calls are in flight.
 */
int sym_set_coeffs_override(const double c[3]);

/*
 * Process-wide choice of force algorithm: SYM_ALG_DIRECT multiplies out all 48
 * staples of each link (181 SU(3) products per link) and makes no assumption on the
 * matrices; SYM_ALG_FACTORED first forms the 6 plaquette staples of every link in the
 * workspace and builds rectangles and cube loops from them (67.5 products per link); it
 * reads links and stores staples as two rows and rebuilds the third, which requires
 * the links to be special unitary to working precision, as the paper's link variables
 * are: for a link off SU(3) by delta (||U^dagger U - 1||), the rebuilt row differs from
 * the stored one by O(delta), and so does the force. md_leapfrog keeps its links within
 * float rounding of SU(3) in SYM_F32 and within double rounding in SYM_F64; fields
 * from elsewhere can be checked with sym_check_links and repaired with sym_reunitarise.
 * SYM_ALG_AUTO (default) is SYM_ALG_FACTORED. SYM_EINVAL for other values.
 */
int sym_set_force_algorithm(int algorithm);

/* Static description of a status code. */
const char* sym_strerror(int status);

/*
 * Per-kernel timing for profiling and benchmarks. With profiling on, every kernel the
 * library launches is bracketed by two HIP timing events recorded on the launch stream
 * (the events are created lazily and reused; no device memory is allocated).
 * sym_profile_collect waits for the recorded events, writes at most max_kinds entries
 * -- kernel name (NUL-terminated, 32 bytes per entry in names), summed milliseconds and
 * launch count -- in order of first launch, forgets them, and returns the number of
 * entries (or a negative sym_status). Host pointers. Process-wide; not for use while
 * other threads launch work through the library.
 */
int sym_profile_enable(int on);
int sym_profile_collect(int max_kinds, char* names, double* total_ms, int32_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* SYM_H */
