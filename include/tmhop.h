/*
 * tmhop.h -- C-ABI of libtmhop.so: the Wilson hopping matrix between the two
 * checkerboards of a 4D lattice, the even-odd preconditioned twisted-mass
 * operator built on it, and CG on that operator, on one MI355X (gfx950).
 *
 * The operation follows Deuzeman, Jansen, Kostrzewa, Urbach, "Experiences
 * with OpenMP in tmLQCD" (LATTICE 2013): the hopping matrix Hopping_Matrix
 * between even and odd sites (Section 2, "Optimizing the Hopping Matrix", and
 * the introduction, which names the half-spinor and full-spinor bodies), the
 * twisted-mass Wilson fermions it serves (introduction), and the real scalar
 * product scalar_prod_r used by the inverter (Section 3, "Measuring and
 * Reducing Overheads").  The paper does not write the operator down; this
 * library takes the standard definitions:
 *
 *   lattice   Z_T x Z_LX x Z_LY x Z_LZ, dims = {T, LX, LY, LZ}, mu = 0..3 =
 *             t,x,y,z; every extent even and >= 2.  lex = ((t*LX+x)*LY+y)*LZ+z,
 *             parity = (t+x+y+z) mod 2 (0 = even).  A site's even-odd index is
 *             lex >> 1 (its rank among the sites of its parity in lex order).
 *   gammas    chiral basis: gamma_mu = [[0, e_mu], [e_mu^+, 0]] with e_0 = -1,
 *             e_k = -i sigma_k, so gamma_5 = gamma_0 gamma_1 gamma_2 gamma_3 =
 *             diag(1, 1, -1, -1).
 *   hopping   (H psi)(x) = kappa sum_mu [ eta+_mu(x) (1 - gamma_mu) U_mu(x) psi(x+mu)
 *                                       + eta-_mu(x) (1 + gamma_mu) U_mu(x-mu)^+ psi(x-mu) ]
 *             eta+ = exp(+i pi theta_mu) if the forward hop wraps from L_mu-1
 *             to 0, eta- = exp(-i pi theta_mu) if the backward hop wraps from
 *             0 to L_mu-1, else 1.  theta = {1,0,0,0} is antiperiodic in time.
 *             H_eo (TMH_EO) maps odd to even sites, H_oe (TMH_OE) even to odd.
 *   twisted   mt = 2 kappa mu, A(s) = 1 + i s mt gamma_5 (s = +-1),
 *   mass      Mhat(s) = A(s) - H_oe A(s)^-1 H_eo on odd fields,
 *             Qhat(s) = gamma_5 Mhat(s); Qhat(+)^dagger = Qhat(-).
 *   CG        solves Qhat(+)^dagger Qhat(+) x = b on odd fields.
 *
 * Memory and ownership.  Every field buffer is a device pointer owned by the
 * caller (typically torch tensors on the device the lattice was created
 * for); the library never keeps a pointer past the call.  The library owns
 * only the lattice handle and its scratch (CG vectors, the intermediate even
 * field, reduction partials and, for mixed precision, low-precision copies),
 * allocated on first use and freed by tmh_lattice_destroy.
 *
 * Internal field layout ("site-coalesced structure of arrays").  S =
 * tmh_site_stride() is Vh = V/2 rounded up to a multiple of 64.  A complex
 * number is two reals (re, im) of the precision's storage type: double for
 * TMH_F64 and TMH_F64_R12, float for TMH_F32 and TMH_F32_R12, IEEE binary16
 * for TMH_F16 and TMH_F16_R12 (whose arithmetic is FP32).  Import rounds
 * FP64 values once, to nearest even, into the storage type.
 *   spinor (one parity): component c = 3*spin + colour of site i is the
 *             complex element c*S + i; tmh_spinor_bytes() = 12*S complexes.
 *   gauge (whole lattice): element (a, b) of U_mu(x), x of parity p with
 *             even-odd index i, is the complex element ((p*4+mu)*9 + 3a+b)*S + i;
 *             tmh_gauge_bytes() = 72*S complexes.
 *   gauge, two-row storage (TMH_F64_R12, TMH_F32_R12, TMH_F16_R12): only
 *             rows a = 0, 1 are stored, element (a, b) at
 *             ((p*4+mu)*6 + 3a+b)*S + i,
 *             tmh_gauge_bytes() = 48*S complexes.  The kernels rebuild row 2
 *             as the complex conjugate of the cross product of rows 0 and 1,
 *             which is exact for special unitary links (a unitary matrix with
 *             determinant 1 equals the conjugate of its cofactor matrix), so
 *             these formats represent SU(3) link fields only.  Spinors of an
 *             _R12 precision are those of its base precision.
 * Elements i in [Vh, S) are padding: never read as data, never written by
 * the operators.
 *
 * Canonical (import/export) layouts, FP64 complex interleaved, device memory:
 *   gauge   [4][V][3][3]  (mu, lex, row, column)
 *   spinor  [Vh][4][3]    (even-odd index, spin, colour) on one parity
 *
 * Streams.  Import, export, hop, qtm and the BLAS-1 calls enqueue on the
 * handle's stream (tmh_lattice_set_stream) and return without waiting.
 * tmh_cg_solve, tmh_scalar_prod_r and tmh_norm2 wait for their result.
 *
 * Errors.  Every entry point returns a status; nothing aborts or throws.
 * Kernel faults are asynchronous and surface as TMH_ERR_HIP at the next
 * call that waits.
 *
 * Threads.  A handle holds scratch, scalars and timing state that every call
 * on it uses: calls on one handle must not overlap (one handle per host
 * thread); calls on distinct handles are independent.
 */
#ifndef TMHOP_H
#define TMHOP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TMH_OK = 0,
    TMH_ERR_ARG = -1,           /* null pointer, bad enum, bad size          */
    TMH_ERR_GEOMETRY = -2,      /* an extent odd or < 2, or volume too large  */
    TMH_ERR_ALIAS = -3,         /* output buffer overlaps an input buffer     */
    TMH_ERR_HIP = -4,           /* a HIP runtime call failed                  */
    TMH_ERR_NOMEM = -5,         /* device allocation of scratch failed        */
    TMH_ERR_NOT_CONVERGED = -6, /* CG hit max_iter; x holds the last iterate  */
    TMH_ERR_UNSUPPORTED = -7,   /* precision or feature not built             */
    TMH_ERR_SCRATCH = -8        /* field exceeds the fixed scratch of an
                                   allocation-free call                        */
} tmh_status;

typedef enum { TMH_EO = 0 /* odd -> even */, TMH_OE = 1 /* even -> odd */ } tmh_dir;

/* Arithmetic and storage precision: spinor word and link storage (9 complex
 * entries, or the two-row storage described above). */
typedef enum {
    TMH_F64 = 0,     /* FP64 spinors and links                      */
    TMH_F32 = 1,     /* FP32 spinors and links                      */
    TMH_F64_R12 = 2, /* FP64 spinors, FP64 links as their two rows  */
    TMH_F32_R12 = 3, /* FP32 spinors, FP32 links as their two rows  */
    TMH_F16 = 4,     /* FP16 storage, FP32 arithmetic               */
    TMH_F16_R12 = 5  /* FP16 storage, links as their two rows       */
} tmh_prec;

typedef struct tmh_lattice tmh_lattice;

/* Creates a lattice handle for dims = {T, LX, LY, LZ} on HIP device `device`,
 * enqueueing on `hip_stream` (a hipStream_t, NULL = the null stream).
 * TMH_ERR_GEOMETRY if an extent is odd or < 2, or V = T*LX*LY*LZ >= 2^29 - 64
 * (one FP64 component array, 16 S bytes, must stay below 4 GiB).
 * TMH_ERR_HIP if the device does not exist. */
tmh_status tmh_lattice_create(tmh_lattice** out, const int dims[4], int device, void* hip_stream);
void tmh_lattice_destroy(tmh_lattice* lat);
tmh_status tmh_lattice_set_stream(tmh_lattice* lat, void* hip_stream);

/* Traversal order of the hopping-matrix kernels.  Each XCD works through one
 * contiguous range of time-slices; with xgroup > 0 it visits that range
 * x-group by x-group (all its time-slices for xgroup consecutive x values,
 * then the next group), which keeps the neighbours of the sites in flight
 * within fewer L2 lines.  0 = even-odd order.  TMH_TRAVERSAL_XSLAB splits x
 * instead of t among the 8 XCDs: XCD k owns x in [k LX/8, (k+1) LX/8) over
 * all time-slices and sweeps t, so that neighbouring XCDs read their shared
 * x boundaries at about the same time (needs LX a multiple of 8).  The
 * default is the largest xgroup with xgroup * LY * LZ / 2 <= 8192 when the
 * geometry tiles (LY*LZ/2 a multiple of 64, T a multiple of 8, xgroup
 * divides LX, V/2 a multiple of 2048); tmh_autotune_hop measures every
 * order instead (and the t-marching kernel below for the step counts whose
 * grids hold 64 to 4096 workgroups).  TMH_ERR_UNSUPPORTED if the geometry
 * does not tile for this order, TMH_ERR_ARG for other negative values.  tmh_lattice_traversal
 * returns the current value (-1 for a null handle). */
#define TMH_TRAVERSAL_XSLAB (-8)
/* t-marching hop kernel: the two sites (x, y, 2zp) and (x, y, 2zp+1) of one
 * time-slice are a pair whose sites alternate between the two parities with
 * t, so that the time neighbours of the output site of a pair at t are the
 * input sites of the same pair at t-1 and t+1.  Each thread owns a pair,
 * each workgroup a tile of 256 pairs, and walks `steps` consecutive
 * time-slices, keeping the input spinors of its pair at t-1, t and t+1 in
 * registers: the time neighbours are read from memory once, the spatial
 * ones from the caches while the neighbouring tiles of the same XCD work on
 * the same slice.  Valid when steps divides T and LX*LY*LZ/2 is a multiple
 * of 256. */
#define TMH_TRAVERSAL_TMARCH(steps) (-1024 - (steps))
tmh_status tmh_lattice_set_traversal(tmh_lattice* lat, int xgroup);
int tmh_lattice_traversal(const tmh_lattice* lat);

/* Even-odd half volume Vh and the padded site stride S. */
size_t tmh_half_volume(const tmh_lattice* lat);
size_t tmh_site_stride(const tmh_lattice* lat);
/* Bytes of one internal spinor (one parity) / gauge field (both parities);
 * 0 for an unknown precision. */
size_t tmh_spinor_bytes(const tmh_lattice* lat, tmh_prec prec);
size_t tmh_gauge_bytes(const tmh_lattice* lat, tmh_prec prec);

/* Canonical FP64 -> internal layout in precision `prec` (rounded once, to
 * nearest even, for FP32 and FP16), and back.  src and dst are device buffers and must not overlap
 * (TMH_ERR_ALIAS).  Two-row gauge import keeps rows 0 and 1 of each link and
 * export rebuilds row 2 from them. */
tmh_status tmh_gauge_import(tmh_lattice* lat, void* dst, const double* src, tmh_prec prec);
tmh_status tmh_spinor_import(tmh_lattice* lat, void* dst, const double* src, tmh_prec prec);
tmh_status tmh_spinor_export(tmh_lattice* lat, double* dst, const void* src, tmh_prec prec);

/* Hopping matrix (Section 2): out = H_eo in (TMH_EO: in odd, out even) or
 * out = H_oe in (TMH_OE: in even, out odd); kappa is folded in, theta[4] are
 * the boundary phases in units of pi.  gauge, in and out are internal-layout
 * buffers of precision `prec`; out must not overlap in or gauge. */
tmh_status tmh_hop_apply(tmh_lattice* lat, tmh_dir dir, void* out, const void* gauge,
                         const void* in, double kappa, const double theta[4], tmh_prec prec);

/* Even-odd twisted-mass operator (introduction): out = Qhat(sign) in on odd
 * fields, sign = +1 or -1, with mt = 2*kappa*mu.  Two fused hopping-matrix
 * launches: the first stores A^-1 H_eo in into the handle's even scratch, the
 * second forms gamma_5 [A in - H_oe (.)].  out must not overlap in or gauge. */
tmh_status tmh_qtm_apply(tmh_lattice* lat, void* out, const void* gauge, const void* in,
                         double kappa, double mu, const double theta[4], int sign,
                         tmh_prec prec);

/* Allocation-free tmh_qtm_apply, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same operation, arguments, checks and result (bitwise)
 * as tmh_qtm_apply, enqueued on the handle's stream, with no hipMalloc,
 * hipFree, event or other allocation inside the call, and no launch timing
 * (tmh_profile_* does not see it).  The intermediate even field lives in a
 * fixed device array of TMH_NOALLOC_MAX_BYTES bytes that the library holds
 * on every GPU it runs on until the process ends (its address is looked up
 * at tmh_lattice_create).  All calls on one GPU share that array: calls that
 * may overlap on one GPU (other streams, other host threads) race and must
 * not be issued.  The array needs no clearing: each call writes the field in
 * full before reading it.  TMH_ERR_SCRATCH if tmh_spinor_bytes(lat, prec)
 * exceeds TMH_NOALLOC_MAX_BYTES (64 MiB: FP64 up to 349,525 sites per
 * parity, e.g. 24^3x48). */
#define TMH_NOALLOC_MAX_BYTES (64u << 20)
tmh_status tmh_qtm_apply_noalloc(tmh_lattice* lat, void* out, const void* gauge, const void* in,
                                 double kappa, double mu, const double theta[4], int sign,
                                 tmh_prec prec);

/* CG (the paper's inverter, Section 3) on Qhat(+)^dagger Qhat(+) x = b.
 * x (FP64 internal layout, odd) holds the initial guess on entry and the
 * solution on return; b is FP64.  Stops when |r|^2 <= rel_tol^2 |b|^2 on the
 * recursive residual, then recomputes the true residual in FP64 and restarts
 * from x if it is above rel_tol (at most 3 restarts).
 *   inner = TMH_F64: plain FP64 CG.
 *   inner = TMH_F32: defect correction -- the FP64 outer loop forms the true
 *           residual, updates x and does every global reduction in FP64 on
 *           the device; each inner solve runs CG with the FP32 hopping matrix
 *           on an FP32 copy of the links made inside this call, on the
 *           residual scaled to unit mean square per real component (so the
 *           source's magnitude does not matter), and stops at a relative
 *           residual no smaller than 1e-5.
 *   inner = TMH_F16: defect correction as TMH_F32, with every field of
 *           the inner CG stored in FP16 (arithmetic and reductions in FP32 /
 *           FP64); the scaling keeps its vectors in FP16's normal range.
 *           Each inner solve stops at a relative residual no smaller than
 *           3e-3; more outer steps replace the precision FP16 lacks.
 *   inner = TMH_F64_R12 / TMH_F32_R12 / TMH_F16_R12: as without _R12, but
 *           the CG recursion reads a two-row copy of the links made inside
 *           this call, 1/3 fewer link bytes per hop, provided every link's
 *           stored third row matches the conjugate cross product of its
 *           first two to 1e-14 / 1e-7 / 1e-4 (SU(3) links to rounding);
 *           otherwise the 9-entry links are used.  The FP64 residuals
 *           (the initial one and the true residual after each inner or
 *           restarted solve) run on an FP64 two-row copy when the links
 *           pass the FP64 check (1e-14), else on the caller's 9-entry
 *           links; both are the same operator to rounding.
 *   gauge is always the 9-entry FP64 field.
 * *iters receives the number of operator (Qhat^dagger Qhat) applications in
 * CG recursions (inner ones for mixed precision), *true_rel_res the final
 * |b - A x| / |b|.  TMH_ERR_NOT_CONVERGED if max_iter is reached.  Blocks. */
tmh_status tmh_cg_solve(tmh_lattice* lat, void* x, const void* b, const void* gauge,
                        double kappa, double mu, const double theta[4], double rel_tol,
                        int max_iter, tmh_prec inner, int* iters, double* true_rel_res);

/* ------------------------------------------------------------------ batches
 * Several right-hand sides on one lattice share each link load; several
 * lattices share each launch.  A batch member is one lattice with nrhs
 * FP64 fields stored back to back (field r at base + r * tmh_spinor_bytes).
 * Tile shapes (sites x right-hand sides per workgroup): 0 = 256x1, 1 = 128x2,
 * 2 = 64x4, 3 = 128x4, 4 = 64x12, where each thread owns one (site, rhs) and
 * the right-hand sides of a workgroup share links through the caches; and
 * 5 = 128x2, 6 = 64x4, 7 = 128x4 with 2, 8 = 64x12, 9 = 128x6 with 3, and
 * 10 = 64x12, 11 = 128x4 with 4 right-hand sides per thread, which applies
 * each link it loads to all of them from registers; and 12 = 64x8 on the
 * matrix cores: per term, the colour products of two sites and 8
 * right-hand sides are three 16x16x4 MFMA products (FP64 or FP32) of the
 * block-diagonal real form of the two links against the half-spinors,
 * staged through LDS; 13 and 14 = t-march: a workgroup walks a range of
 * time-slices for one tile of 256 site pairs and one right-hand side,
 * keeping the projected time neighbours of its sites in registers (the
 * workgroups of a tile for all right-hand sides run together, sharing its
 * links), 14 with the loads of the next term issued before each term;
 * 15 = t-march with 64 site pairs and 4 right-hand sides per workgroup (its
 * four waves request the links of each step together), 16 the same with
 * each step's links loaded once into LDS (72 KB per workgroup in FP64, half
 * of them fetched while the other half is used) and read there by the four
 * right-hand sides; lattices whose LX*LY*LZ/2 is not
 * a multiple of 256 (64 for 15 and 16) get TMH_ERR_UNSUPPORTED for these
 * four.  -1 picks the autotuned shape of the handle
 * (tmh_autotune_mrhs) or a default. */
typedef struct {
    tmh_lattice* lat;      /* every member on the same device, distinct handles */
    int nrhs;              /* right-hand sides (>= 1) */
    void* x;               /* in: initial guesses, out: solutions (odd, FP64) */
    const void* b;         /* sources (odd, FP64) */
    const void* gauge;     /* FP64 internal links of this lattice */
    double kappa, mu;
    double theta[4];
} tmh_batch_member;

/* out_r = H in_r for r < nrhs (in/out: nrhs fields of precision prec back to
 * back), all in one launch; kappa folded in.  Enqueued on the stream.
 * TMH_F64 and TMH_F32 only (TMH_ERR_UNSUPPORTED for the _R12 codes). */
tmh_status tmh_hop_apply_mrhs(tmh_lattice* lat, tmh_dir dir, void* out, const void* gauge,
                              const void* in, int nrhs, double kappa, const double theta[4],
                              tmh_prec prec, int shape);

/* CG on Qhat(+)^dagger Qhat(+) for every (member, rhs) system at once (at most
 * 8 members): one launch per operator step for the whole batch, per-system
 * scalars and stopping flags on the device, and, with use_graph != 0, the 7
 * launches of an iteration captured once into a HIP graph and replayed.
 * Stopping rule, restarts and true residual as tmh_cg_solve, per system; a
 * system whose b is zero gets x = 0 and converges at once, as there.
 * iters[] and true_rel_res[] get one entry per system, members in order.
 * Runs on a private stream ordered after the first member's stream; blocks.
 * TMH_ERR_NOT_CONVERGED if any system missed rel_tol. */
tmh_status tmh_batch_cg_solve(const tmh_batch_member* members, int nmembers, double rel_tol,
                              int max_iter, int shape, int use_graph, int* iters,
                              double* true_rel_res);

/* Autotuner of the batch tile shape: times the multi-RHS hop of every shape on
 * this lattice for nrhs (<= 16) right-hand sides and keeps the fastest in the
 * handle (used by shape = -1).  It ranks the plain hop; in the batched CG the
 * last hop of an iteration also updates r and x of every right-hand side,
 * which favours fewer right-hand sides per thread, so a CG is best tuned by
 * timing tmh_batch_cg_solve itself for the few fastest shapes.  With cache_path, a line
 * "<arch> <T>x<LX>x<LY>x<LZ> <f64|f32> <nrhs> <shape> <us>" is looked up first
 * and appended after timing.  TMH_F64 and TMH_F32 only.  Blocks. */
tmh_status tmh_autotune_mrhs(tmh_lattice* lat, const void* gauge, int nrhs, tmh_prec prec,
                             const char* cache_path, int* best_shape, double* best_us);

/* Autotuner of the hop traversal: times chains of tmh_hop_apply (each hop
 * reading the previous one's output, as in the solvers) in precision prec
 * for xgroup = 0, TMH_TRAVERSAL_XSLAB, every valid group and the valid
 * TMH_TRAVERSAL_TMARCH step counts whose grids hold 64 to 4096 workgroups on
 * this lattice and returns the fastest.  The handle keeps it for every later launch of that
 * storage code (hop, qtm and the CG recursions, including the inner solves
 * of tmh_cg_solve) and as its order for the codes not tuned;
 * tmh_lattice_set_traversal discards the per-code choices.  With cache_path, a line "<arch> <T>x<LX>x<LY>x<LZ> <prec> hop
 * <xgroup> <us>" (prec one of f64, f32, f64r12, f32r12, f16, f16r12; gauge
 * in that storage) is looked up first and appended after timing.  Blocks. */
tmh_status tmh_autotune_hop(tmh_lattice* lat, const void* gauge, tmh_prec prec,
                            const char* cache_path, int* best_xgroup, double* best_us);

/* Full-lattice solve of M x = b, M = (1 + i mt gamma_5) - H the twisted-mass
 * Wilson operator on both checkerboards (what the inverter of the
 * introduction solves), through the even-odd split:
 *   bhat_o = b_o + H_oe A^-1 b_e,  Qhat(+)^+ Qhat(+) x_o = Qhat(-) gamma_5 bhat_o
 *   (tmh_cg_solve's system, x_odd holding the initial guess),
 *   x_e = A^-1 (b_e + H_eo x_o).
 * All buffers FP64 internal layout; x_even, x_odd must not overlap the inputs
 * or each other.  rel_tol, max_iter, inner, *iters and *true_rel_res are those
 * of the odd CG (its normal-equation residual).  Blocks. */
tmh_status tmh_solve_full(tmh_lattice* lat, void* x_even, void* x_odd, const void* b_even,
                          const void* b_odd, const void* gauge, double kappa, double mu,
                          const double theta[4], double rel_tol, int max_iter, tmh_prec inner,
                          int* iters, double* true_rel_res);

/* Gauge-link derivative, the paper's "fermionic derivative" (Section 2,
 * "Race conditions and Memory Locking", which updates it with atomics; here
 * every link has one writer).  For L = Re <left, H right> with H = H_eo
 * (TMH_EO: left even, right odd) or H_oe (TMH_OE: left odd, right even), every
 * link U = U_mu(x) of the lattice gets force[link] += coeff * P(link), where
 *   TMH_FORCE_SU3:    P = TA(M) = (M - M^+)/2 - tr(M - M^+)/6, the su(3)
 *                     force: under U -> exp(tZ) U, dL/dt = tr(Z TA(M));
 *   TMH_FORCE_EUCLID: P = G with dL = Re sum conj(G) dU for U a free complex
 *                     matrix (the gradient torch expects).
 * force, gauge, left and right are FP64 internal-layout buffers (force in the
 * gauge layout, tmh_gauge_bytes(TMH_F64)); force must not overlap the
 * inputs.  Enqueued on the handle's stream. */
typedef enum { TMH_FORCE_SU3 = 0, TMH_FORCE_EUCLID = 1 } tmh_force_kind;
tmh_status tmh_hop_force(tmh_lattice* lat, tmh_dir dir, void* force, const void* gauge,
                         const void* left, const void* right, double kappa,
                         const double theta[4], double coeff, tmh_force_kind kind);

/* The same for L = Re <chi, Qhat(sign) psi> (chi, psi odd, FP64): two
 * hopping-matrix launches into the handle's even scratch and one force
 * launch that adds the terms of both bilinears (through H_oe and H_eo) of
 * each link in one read-modify-write.  For L = |Qhat psi|^2 pass chi = 2 Qhat psi.  The psi-gradient
 * of L is Qhat(-sign) chi (tmh_qtm_apply). */
tmh_status tmh_qtm_force(tmh_lattice* lat, void* force, const void* gauge, const void* chi,
                         const void* psi, double kappa, double mu, const double theta[4],
                         int sign, double coeff, tmh_force_kind kind);

/* Internal gauge layout (precision prec) -> canonical FP64 [4][V][3][3]. */
tmh_status tmh_gauge_export(tmh_lattice* lat, double* dst, const void* src, tmh_prec prec);

/* scalar_prod_r (Section 3): *result = Re <a, b> = Re sum conj(a) b over one
 * parity, in FP64 with a deterministic two-pass reduction.  Blocks. */
tmh_status tmh_scalar_prod_r(tmh_lattice* lat, double* result, const void* a, const void* b,
                             tmh_prec prec);
/* *result = |a|^2, same reduction.  Blocks. */
tmh_status tmh_norm2(tmh_lattice* lat, double* result, const void* a, tmh_prec prec);

/* Bandwidth reference for the roofline: copies nbytes (a multiple of 16,
 * both buffers 16-byte aligned, not overlapping) from src to dst on the
 * handle's stream with a plain streaming kernel (non-temporal 16-byte loads
 * and stores).  Its measured rate is the achievable HBM bandwidth the hopping
 * matrix is compared with, and its hardware counters calibrate the measured
 * traffic of the other kernels. */
tmh_status tmh_stream_copy(tmh_lattice* lat, void* dst, const void* src, size_t nbytes);

/* Launch timing.  Section 3 of the paper measures where the hopping matrix
 * and the solver spend their time; this is the device-side equivalent.  With
 * timing enabled, every hopping-matrix launch made through the handle (by
 * tmh_hop_apply, tmh_qtm_apply and tmh_cg_solve) is bracketed by two HIP
 * events on the handle's stream.  tmh_profile_enable(on) resets the totals.
 * tmh_profile_read waits for the recorded launches and returns, for one
 * kernel kind, the number of launches that did work and the summed duration
 * of all its launches in ms since the last reset.  (The CG enqueues its
 * iterations 8 at a time; launches of iterations past convergence find the
 * stop flag set and return at once.  They are not counted; their few
 * microseconds each stay in the total.)  Kinds: 4*prec + mode, where prec
 * is the tmh_prec code of the launch (0..5: spinor precision and the link
 * storage it reads; the recursions of tmh_cg_solve report the copy they run
 * on) and mode is 0 (plain hop, or hop with the A^-1 store), 1 (hop with
 * the gamma_5 [A in - .] epilogue), 2 (as 1, plus the fused norm), 3 (as 1,
 * with the CG update fused in: r -= alpha q and |r|^2, and in the FP64
 * recursion also x += alpha p). */
#define TMH_PROFILE_KINDS 24
tmh_status tmh_profile_enable(tmh_lattice* lat, int on);
tmh_status tmh_profile_read(tmh_lattice* lat, int kind, long long* launches, double* total_ms);

const char* tmh_status_string(tmh_status st);

#ifdef __cplusplus
}
#endif

#endif /* TMHOP_H */
