/*
 * libigabem: fast isogeometric single-layer BEM for the 3D Laplace and
 * Helmholtz Dirichlet problems on NURBS multipatch surfaces, with the
 * Galerkin matrix compressed by interpolation-based (tensor Chebyshev,
 * nested / H2) fast multipole, after Doelz, Harbrecht, Kurz, Schoeps, Wolf,
 * "A Fast Isogeometric BEM for the Three Dimensional Laplace- and Helmholtz
 * Problems" (arXiv 1708.09162).  All compute runs in HIP kernels on one
 * gfx950 GPU in FP64.
 *
 * Conventions (apply to every entry point):
 *  - Host structs and arrays are read during the call and copied; the library
 *    keeps no host pointer of the caller.
 *  - "_dev" pointers are device (HBM) pointers owned by the caller.  Calls that
 *    take them are ordered on the operator's HIP stream and return before the
 *    work completes unless stated otherwise.
 *  - Real problems (Laplace) use double.  Helmholtz problems use interleaved
 *    (re, im) double pairs, the layout of complex128.
 *  - S = the spline space of Sec. 2.2 (eq. def::space), dimension
 *    n (2^m + p)^2; dof index patch*(2^m+p)^2 + j2*(2^m+p) + j1 (u fastest).
 *  - S* = the discontinuous Bernstein superspace of Sec. 4.3, dimension
 *    n (2^m (p+1))^2; external index E*(p+1)^2 + r2*(p+1) + r1 with element
 *    E = patch*4^m + e2*2^m + e1.
 *  - Cluster ids (Sec. 4.1, the tuple (i, j, k) of a cluster): within a level
 *    l, id = patch*4^l + k2*2^l + k1 for the parameter square
 *    [k1, k1+1] x [k2, k2+1] * 2^-l of patch `patch`.
 *  - Return value: IGB_OK (0), a negative error, or a positive warning.  On a
 *    non-zero return igb_last_error() gives a message (thread-local).
 */
#ifndef IGABEM_H
#define IGABEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t igb_status;

#define IGB_OK 0
#define IGB_ENOT_CONVERGED 1     /* warning: solver stopped at max_iter; w holds the last iterate */
#define IGB_EINVAL (-1)          /* invalid argument (null pointer, bad knots, weights, sizes ...) */
#define IGB_EHIP (-2)            /* a HIP runtime call or kernel launch failed */
#define IGB_ENOMEM (-3)          /* device or host allocation failed */
#define IGB_EUNSUPPORTED (-4)    /* valid request outside what this build implements */

#define IGB_LAPLACE 0            /* interior Laplace, kernel 1/(4 pi |x-y|) (Sec. 3.1, eq. fundament1) */
#define IGB_HELMHOLTZ 1          /* exterior Helmholtz, exp(i k |x-y|)/(4 pi |x-y|) (eq. fundament2) */

#define IGB_DENSE 0              /* every element pair by quadrature, no compression */
#define IGB_H2_STORED 1          /* near field + far field with coupling blocks stored in HBM */
#define IGB_H2_ONTHEFLY 2        /* near field stored; coupling blocks generated inside every matvec */

#define IGB_FP64 0
/* Single-precision far field (on-the-fly coupling; q <= 8 for Laplace, q <= 10
 * for Helmholtz).  Laplace: every coupling-kernel value 1/|x - y| is the
 * hardware reciprocal-square-root estimate without refinement (relative error
 * below 6e-8); distances, moments, transfers, sums and the near field stay
 * FP64.  Helmholtz: the kernel values exp(i k r)/r (hardware reciprocal square
 * root, sine and cosine of the phase in turns) and the sums inside each pair
 * of clusters are FP32 (about 1e-6 relative), and the near-field blocks
 * (integrated in FP64) are also kept rounded to FP32 for this operator's
 * products (leaves of up to 256 functions; half the bytes); moments,
 * transfers, the sums across pairs and the near-field sums stay FP64.
 * igb_matvec / igb_matvec_super apply this operator; igb_solve still solves
 * the FP64 system.  Laplace: CG
 * steps with this operator, the recursive residual replaced by the FP64
 * residual b - A w (full-precision far field) every 20 steps.  Helmholtz:
 * iterative refinement, each cycle a GMRES(restart) solve of A~ d = r with this
 * operator to relative 1e-4 (or what the last cycle needs), w += d, and the
 * FP64 residual r = b - A w.  Convergence is judged on the FP64 residual; the
 * iteration count includes both kinds of products. */
#define IGB_FP32 1

/* One NURBS patch F_j : [0,1]^2 -> Gamma_j (Sec. 2.2, eq. def::geom).
 * knots_u has n_u + deg_u + 1 entries, p-open (Sec. 2.1): deg_u+1 zeros first,
 * deg_u+1 ones last, non-decreasing; the same for v.  Interior knots must lie
 * on the refinement grid k/2^m of the operator built on it.
 * cpw holds n_v*n_u*4 doubles (x, y, z, w), u fastest, w > 0, points not
 * premultiplied by w.  Neighbouring patches must agree on shared edges up to
 * a rotation of the parameter square (Sec. 2.2). */
typedef struct {
    int32_t deg_u, deg_v;
    int32_t n_u, n_v;
    const double *knots_u;
    const double *knots_v;
    const double *cpw;
} igb_nurbs_patch;

/* Discretisation and compression parameters. */
typedef struct {
    int32_t kernel;          /* IGB_LAPLACE or IGB_HELMHOLTZ */
    double wavenumber;       /* kappa >= 0 (Helmholtz only) */
    int32_t p;               /* spline degree, 0 <= p <= 6 (Sec. 2.2) */
    int32_t m;               /* refinement level, 2^m x 2^m elements per patch, 0 <= m <= 10 */
    int32_t q;               /* Chebyshev nodes per parametric direction, 1 <= q <= 16 (Sec. 4.2) */
    double eta;              /* admissibility max(diam) < eta * dist, eta > 0 (Sec. 4.2 Def.) */
    int32_t leaf_depth;      /* levels between leaf clusters and elements; -1: smallest d with (p+1)^2 4^d >= q^2 */
    int32_t gauss_regular;   /* g0: Gauss points per direction for well separated pairs, 1..36 */
    int32_t gauss_singular;  /* points per variable in the regularised touching-pair rules; -1: g0+2 */
    int32_t gauss_rhs;       /* points per direction for right-hand side and potential; -1: max(g0, p+4) */
    int32_t mode;            /* IGB_DENSE, IGB_H2_STORED or IGB_H2_ONTHEFLY */
    int32_t far_precision;   /* IGB_FP64, or IGB_FP32 (see there) */
    double kappa_diam;       /* 0: the admissibility of Sec. 4.2 Def. as it stands (blind to the
                                wavenumber).  > 0 (Helmholtz): a block is admissible only if, in
                                addition, kappa * max(diam) <= kappa_diam, so that the interpolated
                                kernel oscillates at most kappa_diam / (2 pi) times across a cluster;
                                coarse blocks of high-wavenumber problems are then subdivided.  Not
                                from the paper: an option for accuracy at large kappa * size */
} igb_params;

/* Sizes of an assembled operator (host struct filled by igb_operator_info). */
typedef struct {
    int64_t n_dof;             /* dim S */
    int64_t n_dof_super;       /* dim S* */
    int64_t n_elements;
    int64_t n_rhs_points;      /* n_elements * gauss_rhs^2 */
    int32_t leaf_level;        /* L = m - leaf_depth */
    int32_t gauss_singular;
    int32_t gauss_rhs;
    int32_t layout_flags;      /* bit 0: near blocks stored once per mirrored leaf pair; bit 1: far
                                  field generated once per mirrored block pair; bit 2: both products
                                  (and both partial-row gathers) share one launch */
    int64_t n_near_blocks;     /* leaf pairs in the near field */
    int64_t n_far_blocks;      /* admissible cluster pairs, all levels */
    int64_t n_pairs[4];        /* element pairs by class: regular, identical, common edge, common vertex */
    int64_t near_bytes;        /* HBM bytes of the stored near-field blocks */
    int64_t coupling_bytes;    /* HBM bytes of the stored coupling blocks */
    int64_t matvec_bytes;      /* algorithmic HBM bytes of one superspace matvec */
    double setup_seconds;      /* host part of igb_operator_create (tree, partition, lists) */
    double assembly_seconds;   /* whole igb_operator_create, device work included */
    int64_t quad_points_regular;   /* quadrature points of the regular near-field pairs: g^4 per pair
                                      (g = g0, g0 + 2 or g0 + 4 by distance, at most 40) */
    int64_t quad_points_touching;  /* of the touching pairs: regions x gauss_singular^4 per pair
                                      (identical 4 integrated regions, common edge 6, vertex 4) */
    double quad_regular_ms;    /* kernel time of the regular-pair quadrature (operators only; 0 for plans) */
    double quad_touching_ms;   /* kernel time of the touching-pair quadrature (identical + adjacent) */
} igb_info;

typedef struct {
    int32_t iterations;        /* operator applications in the Krylov loop */
    int32_t converged;         /* 1 if the true relative residual reached rel_tol */
    double rel_residual;       /* final true relative residual ||b - A w|| / ||b|| */
    int32_t fallback;          /* igb_solve_fgmres with a network: 1 if it was dropped for Jacobi (stagnation) */
} igb_solve_info;

typedef struct igb_geometry igb_geometry;
typedef struct igb_operator igb_operator;

/* Message for the last non-zero status returned on this thread. */
const char *igb_last_error(void);

/* Validates and copies n_patches NURBS patches (Sec. 2.2).
 * IGB_EINVAL: null pointers, degrees outside 0..8, n < deg+1, knot vectors
 * that are not p-open or decrease, weights <= 0 or non-finite coordinates. */
igb_status igb_geometry_create(int32_t n_patches, const igb_nurbs_patch *patches, igb_geometry **out);
void igb_geometry_destroy(igb_geometry *geo);

/* Assembles the operator A (Sec. 4): Bezier extraction of the geometry onto
 * the 2^m x 2^m element grid, cluster tree and block partition (Sec. 4.1,
 * 4.2), near-field Galerkin quadrature (Sec. 3.2; Sec. 4 item 4), coupling
 * blocks and moment/transfer matrices (Sec. 4.2), Jacobi diagonal.  Device
 * memory is taken here (from the pool, else hipMalloc) and given back by
 * igb_operator_destroy.  `hip_stream`
 * is a hipStream_t (NULL = default stream) used by every later call on the
 * operator.  Synchronises the stream before returning.
 * IGB_EINVAL for parameters out of range, geometry whose interior knots are
 * off the refinement grid, or (Helmholtz) a wavenumber times the diagonal of
 * the control points' bounding box of 2^18 or more (the kernels reduce the
 * phase kappa |x - y| of surface points below 2^19); IGB_ENOMEM if HBM runs
 * out; IGB_EHIP otherwise. */
igb_status igb_operator_create(const igb_geometry *geo, const igb_params *prm, void *hip_stream,
                               igb_operator **out);
/* Synchronises the operator's stream, then gives its device buffers back to
 * the library's memory pool (see igb_release_cached_memory). */
void igb_operator_destroy(igb_operator *op);

/* Device memory pool.  The buffers of destroyed operators (and the scratch of
 * igb_potential) are kept per device, in size classes (4 KiB steps up to
 * 2 MiB, 2 MiB steps above), and handed to later allocations of the same
 * class, so an application that creates operators repeatedly calls hipMalloc
 * and hipFree only the first time.  An allocation that runs out of device
 * memory frees the cache and tries once more.  This call frees every cached
 * buffer on every device now (buffers of live operators are not touched).
 * Thread-safe.  Makes no HIP call when nothing is cached.  IGB_OK, or
 * IGB_EHIP if a hipFree fails. */
igb_status igb_release_cached_memory(void);

/* Fills `out` (host).  Synchronous. */
igb_status igb_operator_info(const igb_operator *op, igb_info *out);

/* Quadrature points where the Dirichlet data g must be sampled: n_rhs_points
 * x 3 doubles written to xyz_dev, element-major, then v-node outer, u-node
 * inner, Gauss order gauss_rhs per direction (Sec. 3.2, right-hand side). */
igb_status igb_rhs_points(const igb_operator *op, double *xyz_dev);

/* b = T g* with g*_a = int g(F x) kappa(x) phi_a(x) dx (Sec. 3.2; Sec. 4.3).
 * g_dev: n_rhs_points values at igb_rhs_points; b_dev: n_dof values. */
igb_status igb_rhs_assemble(const igb_operator *op, const void *g_dev, void *b_dev);

/* y = T A T^T x on S (Sec. 4.3): x_dev, y_dev n_dof values, must not alias. */
igb_status igb_matvec(const igb_operator *op, const void *x_dev, void *y_dev);

/* y* = A x* on S* (external S* order): xs_dev, ys_dev n_dof_super values, no aliasing. */
igb_status igb_matvec_super(const igb_operator *op, const void *xs_dev, void *ys_dev);

/* xs = T^T w (S -> S*) and y = T ys (S* -> S), Sec. 4.3; external S* order. */
igb_status igb_apply_Tt(const igb_operator *op, const void *w_dev, void *xs_dev);
igb_status igb_apply_T(const igb_operator *op, const void *ys_dev, void *y_dev);

/* Jacobi diagonal D_i = t_i^T A t_i, t_i = T^T e_i (far-field terms included): n_dof values. */
igb_status igb_jacobi_diag(const igb_operator *op, void *d_dev);

/* Solves T A T^T w = b (Sec. 4.3) with Jacobi-preconditioned CG (Laplace) or
 * restarted GMRES (Helmholtz) (Sec. 4 item 3).  w_dev holds the initial guess
 * on entry and the density coefficients on exit.  Stops when the true relative
 * residual ||b - A w|| <= rel_tol ||b|| or after max_iter operator
 * applications (then IGB_ENOT_CONVERGED, w = last iterate).  `restart` is the
 * GMRES cycle length, 1..2048 (ignored by CG); short cycles can stagnate on
 * oscillatory problems (the 16-patch torus at kappa = 8, 70k dofs, stalls near
 * 3e-5 with 100 and converges in about 560 applications with 300).  GMRES keeps
 * its Hessenberg matrix and rotations on the device and takes (2 restart + 1)
 * n_dof complex values of device memory.  Synchronous; `info` (host) may be
 * NULL. */
igb_status igb_solve(const igb_operator *op, const void *b_dev, void *w_dev, double rel_tol, int32_t max_iter,
                     int32_t restart, igb_solve_info *info);

/* ---- Learned preconditioner -------------------------------------------------
 * Motivation: Sec. 5 observes that diagonally preconditioned Krylov solves
 * grow costly on fine meshes with higher degrees.  A network acts patch by
 * patch on the (2^m+p) x (2^m+p) coefficient grid of S (Sec. 2.2) as an
 * approximate inverse of the Jacobi-scaled Galerkin matrix D^-1 A: the
 * preconditioner is M(r) = y + f(y), y = D^-1 r.  f is five 3x3 convolutions
 * with 1 -> 32 -> 32 -> 32 -> 32 -> 1 channels, an activation after the first
 * four (ReLU, or the identity: then f is a linear 11 x 11 stencil in factored
 * form), no biases, zero padding at patch edges.  Weights are FP32 for the optimiser and
 * rounded to BF16 (nearest even) for every pass; sums accumulate in FP32.
 * Weight layout: layers in order, each [c_out][c_in][3][3] (row dy, column
 * dx; tap (dy, dx) reads pixel (y + dy - 1, x + dx - 1)).  An igb_cnn lives on
 * the device current at igb_cnn_create; calls on one network must not
 * overlap. */
#define IGB_CNN_NUM_WEIGHTS 28224  /* 9 * (1*32 + 3*32*32 + 32*1) */
#define IGB_CNN_RELU 0
#define IGB_CNN_LINEAR 1
typedef struct igb_cnn igb_cnn;

/* Creates a network with the given FP32 weights (host, IGB_CNN_NUM_WEIGHTS
 * values, copied) and activation IGB_CNN_RELU or IGB_CNN_LINEAR.  Work is
 * ordered on hip_stream (NULL = default stream).  IGB_EINVAL for null
 * pointers, non-finite weights or another activation; IGB_ENOMEM. */
igb_status igb_cnn_create(const float *weights_host, int32_t activation, void *hip_stream, igb_cnn **out);
void igb_cnn_destroy(igb_cnn *net);

/* Copies the current FP32 weights to the host.  Synchronous. */
igb_status igb_cnn_get_weights(const igb_cnn *net, float *weights_host);

/* out = in + f(in) for n_img images of h x w (FP32 device arrays, image-major,
 * rows of w values).  Asynchronous on the network's stream.  IGB_EINVAL for
 * null pointers, sizes < 1, more than 65535 images or sides above 4096. */
igb_status igb_cnn_forward(const igb_cnn *net, const float *in_dev, int32_t n_img, int32_t h, int32_t w,
                           float *out_dev);

/* Loss L = sum (in + f(in) - target)^2 / (2 N) over the N = n_img h w values
 * and its gradient with respect to the BF16 weights (host, IGB_CNN_NUM_WEIGHTS
 * floats, weight layout).  Synchronous.  Errors as igb_cnn_forward. */
igb_status igb_cnn_gradient(igb_cnn *net, const float *in_dev, const float *target_dev, int32_t n_img, int32_t h,
                            int32_t w, double *loss_host, float *grad_host);

/* Training pairs from the operator (Laplace only): for each of the n_pairs
 * FP64 coefficient vectors x_s in x_dev (n_pairs x n_dof, device), y_s =
 * D^-1 A x_s and x_s, both rounded to FP32, into y_dev and x32_dev (n_pairs x
 * n_dof floats each).  A vector of S is n_patches images of (2^m+p)^2.
 * Asynchronous.  IGB_EUNSUPPORTED for Helmholtz operators. */
igb_status igb_cnn_training_pairs(const igb_operator *op, const double *x_dev, int64_t n_pairs, float *y_dev,
                                  float *x32_dev);

/* Adam (beta1 0.9, beta2 0.999, eps 1e-8, rate lr) on the loss of
 * igb_cnn_gradient over the pairs in order, `batch` pairs per step (the last
 * step of an epoch takes the rest), `epochs` passes.  Each pair is
 * imgs_per_pair images of h x w.  loss_host (may be NULL) receives the mean
 * loss of each epoch (epochs doubles).  Synchronous. */
igb_status igb_cnn_train(igb_cnn *net, const float *y_dev, const float *x_dev, int64_t n_pairs, int32_t imgs_per_pair,
                         int32_t h, int32_t w, int32_t epochs, int32_t batch, float lr, double *loss_host);

/* Adam as igb_cnn_train, but on the loss measured by the operator: for the
 * pairs (y_s, x_s) of igb_cnn_training_pairs (y_s = D^-1 A x_s),
 * L = sum_s |D^-1 A (M(y_s) - x_s)|^2 / (2 N), M(y) = y + f(y), N = n_pairs
 * n_dof: the residual of the preconditioned system (Laplace only).  Two FP64
 * operator applications per pair and step.  Uses the operator's solver work
 * vectors, so it must not overlap a solve on the same operator.  Synchronous. */
igb_status igb_cnn_train_operator(igb_cnn *net, const igb_operator *op, const float *y_dev, const float *x_dev,
                                  int64_t n_pairs, int32_t epochs, int32_t batch, float lr, double *loss_host);

/* Flexible GMRES (right preconditioned, restarted after `restart` steps) for
 * T A T^T w = b with the preconditioner M(v) = D^-1 v + f(D^-1 v) of `net`, or
 * plain Jacobi D^-1 v when net is NULL.  With a network, a restart cycle of k
 * steps that fails to cut the true relative residual by 0.9^k drops the network
 * for Jacobi for the rest of the solve (info->fallback = 1).  Laplace operators only
 * (IGB_EUNSUPPORTED otherwise).  Stopping rule, initial guess and return
 * values as igb_solve, judged on the true residual of the FP64 operator.
 * restart in 1..2048 (IGB_EINVAL otherwise).  The bases take (2 restart + 1)
 * n_dof doubles of device memory.  Synchronous. */
igb_status igb_solve_fgmres(const igb_operator *op, const igb_cnn *net, const void *b_dev, void *w_dev,
                            double rel_tol, int32_t max_iter, int32_t restart, igb_solve_info *info);

/* Model selection for the learned preconditioner, then the solve.  Runs
 * igb_solve_fgmres on the validation right-hand side v_dev (n_dof doubles, a
 * problem of the same operator with other data), from a zero guess and with the
 * same rel_tol, max_iter and restart, first with plain Jacobi and then with
 * each of the n_nets networks (n_nets >= 0, none NULL).  A network is kept if
 * it converged without falling back and in fewer steps than Jacobi and every
 * network before it; *chosen (host) receives its index, or -1 for Jacobi.
 * Then solves for b_dev into w_dev (initial guess on entry) with the kept
 * preconditioner, exactly as igb_solve_fgmres; `info` describes that solve.
 * The validation iterate lives in the operator's CG work vector, so the call
 * must not overlap another solve on the same operator.  Neither b nor v may
 * alias w (IGB_EINVAL).  Laplace only (IGB_EUNSUPPORTED otherwise).
 * Synchronous. */
igb_status igb_solve_fgmres_select(const igb_operator *op, const igb_cnn *const *nets, int32_t n_nets,
                                   const void *v_dev, const void *b_dev, void *w_dev, double rel_tol,
                                   int32_t max_iter, int32_t restart, int32_t *chosen, igb_solve_info *info);

/* Solves n independent systems at once (the Krylov solve of Sec. 4 item 3
 * for each instance), each as igb_solve on ops[i] with
 * b_devs[i], w_devs[i] (same rel_tol, max_iter, restart for all).  Solve i
 * runs on operator i's stream, driven by one of up to 16 host threads, so
 * instances given their own streams overlap on the GPU (instances sharing a
 * stream run one after another, still correct).  An operator may appear in
 * several entries (several right-hand sides of one problem): its entries are
 * solved one after another in list order by one thread, since a solve uses
 * its operator's buffers; distinct operators run concurrently.  Every entry
 * needs its own w_dev (IGB_EINVAL otherwise).
 * infos (host, n entries) may be NULL.  Returns IGB_OK, or the most severe
 * status of any instance with its index in igb_last_error().  Synchronous.
 * This batches whole solves over streams; it is not a single fused launch. */
igb_status igb_solve_many(int32_t n, igb_operator *const *ops, const void *const *b_devs, void *const *w_devs,
                          double rel_tol, int32_t max_iter, int32_t restart, igb_solve_info *infos);

/* Potential u(x) = (V~ mu_h)(x) for x off Gamma (Sec. 3.1, eq. eq::repform),
 * mu_h the density with S coefficients w_dev; Gauss order gauss_rhs per
 * element.  xyz_dev: n_pts x 3 doubles; u_dev: n_pts values. */
igb_status igb_potential(const igb_operator *op, const void *w_dev, int64_t n_pts, const double *xyz_dev,
                         void *u_dev);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the potential of
 * igb_potential without any allocation.  The partial sums of the direct sum
 * live in a fixed 32 MiB device array of the library, one per device, held
 * until the process ends; n_pts may be at most 4,194,304 (Laplace) or
 * 2,097,152 (Helmholtz), IGB_EINVAL above.  Every call on one device shares
 * that array (each call overwrites the part it uses; nothing needs clearing),
 * so calls that overlap in time on one device race: order them on one stream
 * or synchronise between them.  Otherwise as igb_potential, but asynchronous
 * (ordered on the operator's stream, returns before the work completes).  The
 * first call on a device looks up the array's address (hipGetSymbolAddress);
 * no call allocates. */
igb_status igb_potential_noalloc(const igb_operator *op, const void *w_dev, int64_t n_pts, const double *xyz_dev,
                                 void *u_dev);

/* The potential of igb_potential with the far field interpolated (Sec. 4.2
 * applied to eq. eq::repform), for large point sets: the density's moments at
 * the Chebyshev nodes of every cluster come from the operator's upward pass;
 * from the coarsest far-field level down, a cluster s is used through its
 * nodes when diam(s) < eta (|x - c_s| - r_s) (c_s, r_s: centre and radius of
 * its surface grid, eta the operator's) and, for Helmholtz, kappa diam(s)
 * <= 4 (or the operator's kappa_diam if smaller), so that the phase is
 * interpolated over at most 2/3 of a wavelength; else its children are
 * visited, and
 * leaves never admitted are summed directly over their quadrature points
 * (Gauss order gauss_rhs).  The error against igb_potential is that of the
 * interpolation, falling with q.  Same arguments, layout and errors as
 * igb_potential; synchronous.  An operator without far-field levels (dense,
 * or a tree too shallow) and a point whose traversal would hold more than
 * 1024 clusters of one level fall back to the direct sum of igb_potential.
 * The first call on an operator uploads its cluster bounds (5 doubles per
 * cluster), kept until igb_operator_destroy. */
igb_status igb_potential_h2(const igb_operator *op, const void *w_dev, int64_t n_pts, const double *xyz_dev,
                            void *u_dev);

/* Timing of the superspace matvec by stage: runs `reps` products on the
 * operator's internal work vectors with HIP events recorded on its stream
 * between stages and writes the mean milliseconds per stage to
 * stage_ms_host[IGB_NUM_MATVEC_STAGES]: 0 upward pass (leaf moments and
 * transfers), 1 coupling blocks (stored GEMV, or generated on the fly),
 * 2 gather of the coupling partial rows (on the fly with q^2 <= 64: each pair
 * of mirrored blocks is evaluated once; 0 otherwise), 3 near-field block
 * GEMV, 4 gather of the near-field partial rows (symmetric near storage: only
 * blocks (t, s) with t <= s are kept; 0 otherwise), 5 downward pass
 * (transfers and leaf back-moments) (Sec. 4.2).  With flags = 0 the products
 * are launched as in igb_matvec: when igb_info.layout_flags bit 2 is set, the
 * near-field products and gathers share the far-field launches (stages 1 and
 * 2) and stages 3 and 4 are empty; when the near-field GEMV runs on the
 * operator's side stream, concurrent with stages 0-2 (symmetric near storage
 * without the shared launch), stage 3 is its duration there.  With
 * IGB_PROFILE_SEPARATE they run as separate launches, one kernel per stage,
 * on the operator's stream.  Synchronous. */
#define IGB_NUM_MATVEC_STAGES 6
#define IGB_PROFILE_SEPARATE 1
igb_status igb_matvec_profile(const igb_operator *op, int32_t reps, int32_t flags, double *stage_ms_host);

/* Host-only planning: the cluster tree, block partition (Sec. 4.1, Sec. 4.2
 * Def.) and near-field element-pair classification that igb_operator_create
 * would build for the same geometry and parameters, without any GPU work.
 * Same errors as igb_operator_create's parameter checks. */
typedef struct igb_plan igb_plan;
igb_status igb_plan_create(const igb_geometry *geo, const igb_params *prm, igb_plan **out);
void igb_plan_destroy(igb_plan *plan);
/* sizes (device byte counts are those the operator would allocate) */
igb_status igb_plan_info(const igb_plan *plan, igb_info *out);
/* same layouts as igb_export_partition / igb_export_pair_classes */
igb_status igb_plan_export_partition(const igb_plan *plan, int32_t *near_host, int32_t *far_host);
igb_status igb_plan_export_pair_classes(const igb_plan *plan, int32_t *pairs_host);

/* Diagnostics for parity checks (host outputs, synchronous). */
/* near_host: n_near_blocks x 2 (target leaf, source leaf), far_host:
 * n_far_blocks x 3 (level, target, source); both sorted lexicographically. */
igb_status igb_export_partition(const igb_operator *op, int32_t *near_host, int32_t *far_host);
/* element-pair classes of the near field: for each of n_pairs_total computed
 * pairs (E <= F), 4 int32: E, F, class (0 regular, 1 identical, 2 edge,
 * 3 vertex), Gauss order. Sorted by (E, F). */
igb_status igb_export_pair_classes(const igb_operator *op, int32_t *pairs_host);
/* the stored near-field block of elements (E, F) (row = E's functions): nloc^2 values */
igb_status igb_export_near_block(const igb_operator *op, int32_t E, int32_t F, double *blk_host);
/* the stored coupling block of a far pair, q^2 x q^2 row-major (row = target node) */
igb_status igb_export_coupling_block(const igb_operator *op, int32_t level, int32_t tgt, int32_t src,
                                     double *blk_host);

#ifdef __cplusplus
}
#endif
#endif /* IGABEM_H */
