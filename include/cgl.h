/*
 * cgl.h -- C ABI of an MI355X (gfx950) exponential time stepper for the
 * cubic and cubic-quintic complex Ginzburg--Landau equation
 *
 *   d_t u = (a1 + i b1) Lap u + a2 u + (a3 + i b3)|u|^2 u + (a4 + i b4)|u|^4 u
 *
 * (Caliari & Cassini, eq. cqCGL) on Cartesian grids with homogeneous
 * Dirichlet or Neumann boundaries.  After a finite-difference
 * semi-discretisation the system is u' = K u + g(u) with K the Kronecker sum
 * of the 1-D operators A_mu (eq. ODEs).  The action of exp(t K) is computed as
 * the Tucker operator U x_1 exp(t A_1) x_2 ... x_d exp(t A_d) (eq. Tucker) of
 * dense mu-mode products; it is interleaved with the pointwise nonlinear flow
 * inside Strang (eq. Strang), split4 (eq. Richardson), Lawson2b (eq.
 * lawson2b) and Lawson4 (eq. lawson4) steps with a constant step size tau, so
 * the small exponentials are computed once per plan (Section 3.1).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Status codes are returned; nothing aborts.  Argument errors are detected
 *   synchronously on the host.  Conditions that arise on the device
 *   (non-finite state, exact-flow domain violated) are latched in a device
 *   flag and reported by cgl_run at its check points and by cgl_status.
 * - State tensors are device pointers to interleaved complex numbers, index 1
 *   fastest (the column-stacking vec of eq. kronsumv): element (i1,..,id)
 *   lives at i1 + n1*(i2 + n2*(i3 ...)).  Their type follows the plan's
 *   precision: complex128 (double re, double im) for CGL_FP64; complex64
 *   (float re, float im) for CGL_SPLIT_BF16, or complex128 when that plan was
 *   made with CGL_FLAG_FP64_MASTER.  The caller owns state memory; the plan
 *   owns everything else (operators, stage tensors, graphs, flags).
 * - Matrices passed on the host are complex128, column-major, n x n
 *   (element (i, j) at 2*(i + n*j) re, +1 im).
 * - All device work is enqueued on the plan's HIP stream (the one given to
 *   cgl_plan; NULL means the legacy default stream) and is stream-ordered;
 *   only cgl_run check points, cgl_status, cgl_get_operator of device data and
 *   cgl_destroy synchronise.  One plan must not be used from two host threads
 *   at once.
 */
#ifndef CGL_ABI_H_
#define CGL_ABI_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cgl_plan_s* cgl_plan_t;

/* Coefficients of eq. (cqCGL).  a4 = b4 = 0 is the cubic equation.  The
 * paper assumes a1 > 0 (Section 1); cgl_plan rejects a1 <= 0. */
typedef struct {
  double a1, b1, a2, a3, b3, a4, b4;
} cgl_coeffs;

enum {
  CGL_OK = 0,
  CGL_EINVAL = -1,     /* bad argument (sizes, pointers, tau, mu, method) */
  CGL_ENOMEM = -2,     /* host or device allocation failed */
  CGL_EDEVICE = -3,    /* a HIP runtime call failed */
  CGL_ENOTREADY = -4,  /* a step was requested before every mu has operators */
  CGL_ENONFINITE = -5, /* the state became NaN/Inf (the paper's "x" entries) */
  CGL_EBLOWUP = -6,    /* 1 - 2 a3 |u|^2 t <= 0 in the exact cubic flow (or
                          1 - 4 a4 |u|^4 t <= 0 in the exact quintic flow) */
  CGL_EGATE = -7,      /* a surrogate jump failed its a-posteriori check */
  CGL_ESCRATCH = -8    /* the grid does not fit cgl_tucker_noalloc's fixed scratch */
};

/* precision form.  CGL_SPLIT_BF16: complex64 stage tensors, operands split
 * into three bf16 terms (six term products kept), FP32 accumulation.  Its
 * stated accuracy (one mu-mode product or one step within 1e-6 relative of
 * the FP64 result, 2-norm and max-norm) holds for directions of up to 512
 * points: the FP32 accumulation error grows like sqrt(n_mu) (one product
 * with random operands measured 7.2e-7 / 1.25e-6 (2-norm / max-norm) at
 * n_mu = 1024 and 1.45e-6 / 2.5e-6 at n_mu = 4096). */
enum { CGL_FP64 = 0, CGL_SPLIT_BF16 = 1 };
/* time stepper: Strang (eq. Strang), Lawson4 (eq. lawson4), split4 = the
 * Richardson extrapolation of Strang (eq. richextrap / Richardson), Lawson2b
 * (eq. lawson2b) */
enum { CGL_STRANG = 0, CGL_LAWSON4 = 1, CGL_SPLIT4 = 2, CGL_LAWSON2 = 3 };
enum { CGL_DIRICHLET = 0, CGL_NEUMANN = 1 };       /* boundary type */
enum { CGL_E = 0, CGL_H = 1 };                     /* exp(tau A) or exp(tau A / 2) */

/* plan flags */
#define CGL_FLAG_FP64_MASTER 1u /* split form: the caller's state is complex128 and
                                   every step's final update is made in FP64 */
#define CGL_FLAG_RK4_FLOW 2u    /* Strang: use the RK4 sub-flow even when the
                                   nonlinearity is cubic (default: exact flow) */
#define CGL_FLAG_THREE_TERM 4u  /* Strang / split4 become strang_3t / split4_3t
                                   (Section 4.3): the sub-flow entering a step is
                                   phi^c o phi^q, the one leaving it phi^q o phi^c,
                                   both exact; excludes CGL_FLAG_RK4_FLOW */

/* Create a plan for a d-dimensional grid n[0..d-1] (n[mu] >= 3, d in 1..3),
 * coefficients c, constant step tau > 0 and a precision form.  hip_stream is
 * a hipStream_t (may be NULL).  On success *out receives the plan; the plan is
 * not ready to step until cgl_set_operators was called for every mu.
 * Errors: CGL_EINVAL (d, n, tau, a1 <= 0, precision, flags, null pointers),
 * CGL_ENOMEM, CGL_EDEVICE. */
int cgl_plan(cgl_plan_t* out, int d, const int64_t* n, const cgl_coeffs* c, double tau,
             int precision, unsigned flags, void* hip_stream);

/* Give the 1-D operator A_mu (host, complex128 column-major n_mu x n_mu;
 * copied).  The plan computes E_mu = exp(tau A_mu) and H_mu = exp(tau A_mu/2)
 * in FP64 by Pade approximation with scaling and squaring (the route the
 * paper uses for its small exponentials, Section 3.1), converts them to the
 * plan's device form and uploads them on the plan stream.  mu is 0-based.
 * Errors: CGL_EINVAL (mu out of range, null A, non-finite A), CGL_EDEVICE. */
int cgl_set_operators(cgl_plan_t p, int mu, const double* A);

/* Give exp(tau A_mu) and exp(tau A_mu / 2) directly (host, complex128
 * column-major), bypassing the Pade route.  Same errors as cgl_set_operators. */
int cgl_set_exponentials(cgl_plan_t p, int mu, const double* E, const double* H);

/* Build the 2nd-order central finite-difference operator
 * A = (a1 + i b1) D2 + (a2/d) I of one direction (display after eq. ODEs):
 * Dirichlet on interior nodes, h = (b-a)/(n+1), D2 = tridiag(1,-2,1)/h^2;
 * Neumann on the vertex grid, h = (b-a)/(n-1), boundary rows (-2,2)/h^2 and
 * (2,-2)/h^2 from the centred u' = 0 ghost value.  A_out: host, 2*n*n
 * doubles, complex128 column-major.  Errors: CGL_EINVAL. */
int cgl_fd_operator(int64_t n, double a, double b, int bc, const cgl_coeffs* c, int d,
                    double* A_out);

/* Build the finite-difference operator A = (a1 + i b1) D2 + (a2/d) I of one
 * direction with a condition bc_lo at a and bc_hi at b (CGL_DIRICHLET or
 * CGL_NEUMANN each) and order 2 or 4.  Grid: a Dirichlet end is not a node
 * (its value is 0), a Neumann end is the first or last node, so n unknowns
 * have h = (b-a)/(n+1) (both Dirichlet, the interior points of Section
 * 4.1.1), (b-a)/n (one of each, the semi-internal points of Section 4.2) or
 * (b-a)/(n-1) (both Neumann).  Order 2: rows (1,-2,1)/h^2, a Neumann end row
 * (-2,2)/h^2 (centred ghost value).  Order 4 (the matrices displayed in
 * Sections 4.1.1 and 4.2, n >= 6): centred rows (-1,16,-30,16,-1)/(12h^2);
 * next to a Dirichlet end the one-sided row (-15,-4,14,-6,1)/(12h^2); at a
 * Neumann end the rows (1,-6,14,-4,-15,10) and (1,-8/3,-6,56,-145/3) over
 * 12h^2 (the left end mirrored).  A_out: host, 2*n*n doubles, complex128
 * column-major.  Errors: CGL_EINVAL (order, n, bc, d, b <= a, null). */
int cgl_fd_operator_ex(int64_t n, double a, double b, int bc_lo, int bc_hi, int order,
                       const cgl_coeffs* c, int d, double* A_out);

/* Make direction mu periodic on (a, b) with the Fourier pseudospectral
 * discretisation of Section 3.2: n_mu equispaced nodes x_j = a + j (b-a)/n_mu,
 * A_mu diagonal in the transform's coefficients with entries
 * (a1 + i b1)(-k^2) + a2/d over the wave numbers k = 2 pi q / (b - a),
 * q = 0, 1, .., n/2, -n/2 + 1, .., -1.  The plan keeps the diagonals of
 * exp(tau A_mu) and exp(tau A_mu / 2) (FP64, computed on the host).  When n_mu
 * is a power of two from 8 to 1024 every pass of direction mu is a Fourier
 * pass: each fibre is transformed, multiplied by the diagonal and transformed
 * back in one read and one write of the tensor (FP64 arithmetic in the
 * CGL_FP64 form, FP32 in the CGL_SPLIT_BF16 form), and the plan's Lawson
 * rounds run as two actions; otherwise the dense n x n exponential
 * F^{-1} diag F is applied by the mu-mode product kernels.  cgl_get_operator
 * returns that dense exponential.  Plain plans only.
 * Errors: CGL_EINVAL (mu, b <= a, batched plan), CGL_ENOMEM, CGL_EDEVICE. */
int cgl_set_periodic(cgl_plan_t p, int mu, double a, double b);

/* The diagonal of exp(tau A_mu) (which = CGL_E) or exp(tau A_mu / 2) (CGL_H)
 * of a periodic direction, n_mu complex128 values in the transform's
 * coefficient order (out_host: 2 n_mu doubles).  Errors: CGL_EINVAL,
 * CGL_ENOTREADY (mu is not periodic). */
int cgl_get_periodic_factor(cgl_plan_t p, int mu, int which, double* out_host);

/* exp(t A) of a host complex128 column-major n x n matrix by the plan's Pade
 * routine (no plan needed).  out: host, 2*n*n doubles.  Errors: CGL_EINVAL. */
int cgl_expm(int64_t n, const double* A, double t, double* out);

/* Copy the FP64 exponential the plan holds for direction mu (which = CGL_E
 * or CGL_H) to out_host (2*n_mu*n_mu doubles, complex128 column-major).
 * Errors: CGL_EINVAL, CGL_ENOTREADY. */
int cgl_get_operator(cgl_plan_t p, int mu, int which, double* out_host);

/* One mu-mode product out = in x_mu M with M = E_mu or H_mu (Section 3.1):
 * out[.., i_mu, ..] = sum_j M[i_mu, j] in[.., j, ..].  in_dev/out_dev are
 * device state tensors of the plan's stage type (complex128 for CGL_FP64,
 * complex64 for CGL_SPLIT_BF16); they must not overlap.  Asynchronous.
 * Errors: CGL_EINVAL, CGL_ENOTREADY, CGL_EDEVICE. */
int cgl_mode_product(cgl_plan_t p, int mu, int which, const void* in_dev, void* out_dev);

/* The Tucker operator out = in x_1 M_1 ... x_d M_d (eq. Tucker), i.e.
 * exp(tau K) (which = CGL_E) or exp(tau K/2) (CGL_H) applied to in.  Same
 * types and errors as cgl_mode_product; in_dev may equal out_dev. */
int cgl_tucker(cgl_plan_t p, int which, const void* in_dev, void* out_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * Tucker operator as cgl_tucker, out = in x_1 M_1 ... x_d M_d, but its
 * intermediate tensors live in a fixed 32 MiB device array of the library
 * (two halves of 16 MiB; one copy per GPU, held until the process ends)
 * instead of the plan's stage buffers, and it enqueues no tile tuning (it
 * uses the shape an earlier call of the plan chose, else the default one).
 * It allocates nothing.  Plain plans only; the grid must fit a half:
 * N * 8 bytes (split form) or N * 16 bytes (FP64 form) <= 16 MiB, else
 * CGL_ESCRATCH and nothing is enqueued.  Every call on a GPU shares that GPU's
 * array: calls that overlap in time on one GPU (other streams, other host
 * threads) race and give wrong results.  Same argument rules and other errors
 * as cgl_tucker. */
int cgl_tucker_noalloc(cgl_plan_t p, int which, const void* in_dev, void* out_dev);

/* Advance u_dev in place by nsteps >= 0 Strang steps (eq. Strang),
 * u <- phi_{tau/2}(exp(tau K) phi_{tau/2}(u)).  phi is the exact cubic flow
 * (eq. exsolcub) when a4 = b4 = 0 and CGL_FLAG_RK4_FLOW is not set, otherwise
 * one classical RK4 step of u' = g(u) (eq. RK4 with K = 0).  Asynchronous;
 * device conditions are latched (see cgl_status).
 * Errors: CGL_EINVAL, CGL_ENOTREADY, CGL_EDEVICE. */
int cgl_step_strang(cgl_plan_t p, void* u_dev, int64_t nsteps);

/* Advance u_dev in place by nsteps Lawson4 steps (eq. lawson4).  The six
 * exponential actions of the scheme are evaluated as four actions of
 * exp(tau K/2), using exp(tau K) = exp(tau K/2) exp(tau K/2):
 * P = e^{tau K/2} u and Q = e^{tau K/2} g(u), from which the stages
 * X = P + tau g(u3), Y = P + tau/6 Q + tau/3 (g(u2) + g(u3)) are formed in
 * the last pass; then u4 = e^{tau K/2} X and
 * u_{n+1} = e^{tau K/2} Y + tau/6 g(u4).  The split form applies each
 * direction of the two actions of a pair (P with Q, then X with Y) in one
 * pass, both products sharing the operator; the FP64 form runs the two
 * actions side by side.  Same errors as cgl_step_strang. */
int cgl_step_lawson4(cgl_plan_t p, void* u_dev, int64_t nsteps);

/* Advance u_dev in place by nsteps steps of method (CGL_STRANG,
 * CGL_LAWSON4, CGL_SPLIT4, CGL_LAWSON2), enqueued eagerly.
 * split4 (eq. Richardson) runs three exponential actions per step:
 * S = phi_{tau/2}(e^{tau K} phi_{tau/2}(u)); V = phi_{tau/2}(e^{tau K/2}
 * phi_{tau/4}(u)) (one sub-flow over tau/2 between the half steps, as the
 * scheme is printed; the three-term form composes the exact flows);
 * u <- 4/3 phi_{tau/4}(e^{tau K/2} V) - 1/3 S, the combination fused into the
 * last pass.  Lawson2b (eq. lawson2b) runs the two actions P = e^{tau K} u and
 * Q = e^{tau K} g(u) (paired in the split form) and forms
 * u_{n+1} = P + tau/2 Q + tau/2 g(P + tau Q) in the last pass.
 * Same errors as cgl_step_strang. */
int cgl_step(cgl_plan_t p, int method, void* u_dev, int64_t nsteps);

/* Advance u_dev by nsteps steps of method (CGL_STRANG ... CGL_LAWSON2),
 * replaying a captured HIP graph of check_every steps (check_every <= 0:
 * one chunk of nsteps).  After every chunk the device flags are read; the
 * run stops early and returns CGL_ENONFINITE or CGL_EBLOWUP when one is set.
 * Synchronises the plan stream at each check point.  Since tau is constant
 * and the plan holds the exponentials, (u, step count) is a complete
 * checkpoint: a stopped run can be resumed by calling again. */
int cgl_run(cgl_plan_t p, int method, void* u_dev, int64_t nsteps, int64_t check_every);

/* Synchronise the plan stream and return the latched device condition
 * (CGL_OK, CGL_ENONFINITE or CGL_EBLOWUP); clears it. */
int cgl_status(cgl_plan_t p);

/* Enqueue a clear of the latched device condition on the plan stream. */
int cgl_clear_status(cgl_plan_t p);

/* Synchronise and free everything the plan owns.  NULL is accepted. */
void cgl_destroy(cgl_plan_t p);

/* Static message for a status code. */
const char* cgl_strerror(int status);

/* Number of bf16 terms used per operator entry by a CGL_SPLIT_BF16 plan. */
int cgl_split_terms(cgl_plan_t p, int* op_terms, int* state_terms);

/* Give every operator at once: A[mu] for mu < d (plain plan) or A[j*d + mu]
 * (batched plan), each host complex128 column-major.  The exponentials
 * H = exp(tau A / 2) (Pade-13 with scaling and squaring) and E = H H are
 * computed in parallel host threads.  Errors as cgl_set_operators. */
int cgl_set_operators_all(cgl_plan_t p, const double* const* A);

/* ---- batched plans: many independent instances stepped together ----
 * Instance j (0 <= j < batch) has its own grid n[j*d .. j*d+d-1] and
 * coefficients c[j] (the shared step tau and precision).  Every state tensor
 * of the plan concatenates the instances: instance j occupies the complex
 * elements [off_j, off_j + prod_mu n[j*d+mu]) (cgl_instance_offset), each
 * column-major as in a plain plan.  cgl_step_strang, cgl_step_lawson4,
 * cgl_run, cgl_tucker, cgl_status and cgl_destroy accept batched plans; in the
 * split form each mu-mode pass of all instances is ONE persistent launch over
 * a device table of (instance, row tile, fibre tile) work items, with the tile
 * shape chosen by timing at the first step.  The FP64 form launches one pass
 * per instance.  cgl_mode_product, cgl_set_operators, cgl_set_exponentials and
 * cgl_get_operator reject batched plans (CGL_EINVAL). */
int cgl_plan_batched(cgl_plan_t* out, int batch, int d, const int64_t* n /*[batch*d]*/,
                     const cgl_coeffs* c /*[batch]*/, double tau, int precision, unsigned flags,
                     void* hip_stream);
int cgl_batch_size(cgl_plan_t p, int* batch); /* 0 for a plain plan */
int cgl_instance_offset(cgl_plan_t p, int j, int64_t* off);
/* operator A_mu of instance j (host complex128 column-major, copied) */
int cgl_set_instance_operators(cgl_plan_t p, int j, int mu, const double* A);
/* FP64 exponential (which = CGL_E / CGL_H) of direction mu of instance j */
int cgl_get_instance_operator(cgl_plan_t p, int j, int mu, int which, double* out_host);

/* ---- the coupled two-field system (Section 4.4, eq. coupled) ----
 * Two fields u, v on one 2-D grid with periodic boundaries:
 *   u_t =  a0 d_1 u + (a1 + i b1) Lap u + a2 u + (a3 + i b3)|u|^2 u
 *          + (a4 + i b4)|u|^4 u + a5 |v|^2 u,
 *   v_t = -a0 d_1 v + ... + a5 |u|^2 v   (the same terms with u and v swapped).
 * K is block diagonal: each field's exponential is that of its own Kronecker
 * sum (the Fourier route of Section 3.2; the first derivative's symbol is
 * i k, 0 for the Nyquist mode of an even n), applied by the mu-mode product
 * or Fourier kernels of a single-field plan per field.  The nonlinear part
 * couples the fields pointwise; its sub-flow is one classical RK4 step.
 * A state is 2 N elements, u then v (N = n1 n2, index 1 fastest), complex128
 * for CGL_FP64 and complex64 for CGL_SPLIT_BF16. */
typedef struct {
  double a0, a1, b1, a2, a3, b3, a4, b4, a5;
} cgl_coupled_coeffs;
typedef struct cgl_coupled_s* cgl_coupled_t;

/* Plan for an n[0] x n[1] grid (3 <= n_mu <= 4096), step tau, precision
 * CGL_FP64 or CGL_SPLIT_BF16, on the caller's HIP stream; allocates five
 * stage tensors of 2 N elements.  CGL_EINVAL, CGL_ENOMEM. */
int cgl_coupled_plan(cgl_coupled_t* out, const int64_t* n, const cgl_coupled_coeffs* c,
                     double tau, int precision, void* hip_stream);
/* Periodic direction mu on (a, b) for both fields (u with +a0 d_1 and v with
 * -a0 d_1 in direction 0).  Both directions must be set before a step. */
int cgl_coupled_set_periodic(cgl_coupled_t p, int mu, double a, double b);
/* The diagonal of exp(t A_mu) of field 0 (u) or 1 (v), t = tau (CGL_E) or
 * tau/2 (CGL_H): 2 n_mu doubles (complex128, the transform's order). */
int cgl_coupled_get_factor(cgl_coupled_t p, int field, int mu, int which, double* out_host);
/* nsteps steps of CGL_STRANG, CGL_LAWSON4, CGL_SPLIT4 or CGL_LAWSON2
 * (asynchronous, on the plan's stream).  CGL_ENOTREADY before both
 * directions are set. */
int cgl_coupled_step(cgl_coupled_t p, int method, void* w_dev, int64_t nsteps);
/* Synchronise; CGL_ENONFINITE if a step produced a non-finite value since
 * the last call (then cleared), else CGL_OK. */
int cgl_coupled_status(cgl_coupled_t p);
/* Synchronise and free.  NULL is accepted. */
void cgl_coupled_destroy(cgl_coupled_t p);

/* ---- learned surrogate of the stepper (no counterpart in the paper) ----
 * A residual convolutional network on a 2-D grid n1 x n2 that maps a state
 * u(t) to an estimate of u(t + M tau) in one jump:
 *   x   = [Re u, Im u, c_1 .. c_5]  (7 planes; c = the five coefficients
 *         (a1, b1, a2, a3, b3) of eq. cqCGL standardised by the caller)
 *   h0  = silu(conv_in x)                      7 -> 48 channels
 *   h_k = h_{k-1} + silu(conv_k h_{k-1})        48 -> 48, k = 1..4
 *   y   = (Re b, Im b) + s conv_out h_4         48 -> 2
 * where the base b is u itself or a base state the caller gives (a cheap
 * propagation of u over the jump: the network then learns the correction to
 * it) and s is the output scale (1 unless set: the typical size of the
 * correction, so that the layers work on unit-size values), with 3x3
 * kernels, zero padding, silu(a) = a / (1 + e^{-a}).  Parameters are
 * FP32 on the device, packed as W_in, b_in, W_1, b_1, ..., W_out, b_out with
 * W[co][ci][ky][kx] (ky along index 2, kx along index 1); the convolutions
 * run on bf16 MFMA with the weights and activations rounded to bf16 and FP32
 * accumulation.  Training minimises a loss (cgl_sur_set_loss) with Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8).
 * States are complex64 device arrays, index 1 fastest; sample s of a batch
 * lives at complex offset s * n1 * n2.  Work is enqueued on the stream given
 * to cgl_sur_create; entry points returning host data synchronise it. */
typedef struct cgl_sur_s* cgl_sur_t;

/* Number of FP32 parameters (87 074). */
int cgl_sur_param_count(int64_t* count);

/* Network for grids n1 x n2 (n1 a multiple of 64, 64 <= n1 <= 4096,
 * 1 <= n2 <= 4096) and batches of at most max_batch samples; allocates the
 * activations of a training batch (about 2.6 KB per point and sample).
 * CGL_EINVAL for bad sizes, CGL_ENOMEM when allocation fails. */
int cgl_sur_create(cgl_sur_t* out, int64_t n1, int64_t n2, int max_batch, void* hip_stream);

/* Copy count FP32 parameters from the host (synchronous) and reset the Adam
 * moments and step count.  CGL_EINVAL if any parameter is not finite. */
int cgl_sur_set_params(cgl_sur_t s, const float* params_host);
/* Training loss: CGL_SUR_LOSS_MSE (the default) is the mean over samples,
 * planes and points of (y - target)^2; CGL_SUR_LOSS_REL is the mean over
 * samples of sum (y - target)^2 / sum target^2, the square of the relative
 * L2 error that the gated run checks (a sample with a zero target counts 0). */
enum { CGL_SUR_LOSS_MSE = 0, CGL_SUR_LOSS_REL = 1 };
int cgl_sur_set_loss(cgl_sur_t s, int kind);

/* Output scale s of the network (finite, > 0; 1 after cgl_sur_create).
 * CGL_EINVAL otherwise. */
int cgl_sur_set_output_scale(cgl_sur_t s, float scale);

/* Copy the current parameters to the host (synchronous). */
int cgl_sur_get_params(cgl_sur_t s, float* params_host);

/* out = network(u) for batch samples (1 <= batch <= max_batch); cstd_dev is a
 * device float array [batch][5]; base_dev (complex64 [batch][P]) gives the
 * base states, NULL takes u.  out may equal u or base.  CGL_ENOTREADY before
 * cgl_sur_set_params. */
int cgl_sur_forward(cgl_sur_t s, int batch, const void* u_dev, const float* cstd_dev,
                    const void* base_dev, void* out_dev);

/* Training batch: sample s is input src[i_s] with coefficients cstd[i_s]
 * (device [*][5]) and target src[i_s + target_offset], where i_s = idx[s]
 * (device int32 array) or s when idx_dev is NULL, and base state
 * base[i_s] (complex64, indexed like src) or src[i_s] when base_dev is NULL.
 * cgl_sur_grad writes the
 * loss gradient to grad_host[count] and the loss to *loss_host (if not NULL)
 * without changing the parameters (synchronous).  cgl_sur_train_step takes
 * one Adam step with learning rate lr (asynchronous); the mean loss of the
 * steps since the last call is returned by cgl_sur_take_loss (synchronous). */
int cgl_sur_grad(cgl_sur_t s, int batch, const void* src_dev, const float* cstd_dev,
                 const int32_t* idx_dev, int64_t target_offset, const void* base_dev,
                 float* grad_host, double* loss_host);
int cgl_sur_train_step(cgl_sur_t s, int batch, const void* src_dev, const float* cstd_dev,
                       const int32_t* idx_dev, int64_t target_offset, const void* base_dev,
                       float lr);
int cgl_sur_take_loss(cgl_sur_t s, double* mean_loss);

/* Synchronise and free the network.  NULL is accepted. */
void cgl_sur_destroy(cgl_sur_t s);

/* Bases of a gated run's jumps: the state itself; the exact linear flow
 * e^{M tau K} u (the change of variables behind the Lawson schemes,
 * Section 2.2), as the E exponential of a coarse plan whose step is M tau;
 * one Strang step (eq. Strang) of the coarse plan. */
enum { CGL_SUR_BASE_INPUT = 0, CGL_SUR_BASE_LINEAR = 1, CGL_SUR_BASE_STRANG = 2 };

/* Gated run of njumps jumps of steps_per_jump Lawson4 steps each on the
 * complex64 state u_dev of plan p (a 2-D CGL_SPLIT_BF16 plan without
 * CGL_FLAG_FP64_MASTER on the network's grid), with standardised
 * coefficients cstd[5].  A jump is network(u) with the base given by base
 * (CGL_SUR_BASE_*): for LINEAR and STRANG, coarse is a plan of the same
 * shape, precision and stream as p holding the same problem with step
 * steps_per_jump * tau (the caller builds it; the run only applies it);
 * coarse may be NULL for CGL_SUR_BASE_INPUT.  Jumps j = check_every,
 * 2 check_every, ... and the last one are checked: the plain stepper
 * advances the state the jump started from by steps_per_jump steps; if the
 * relative L2 distance of the
 * jump's result from it is <= tol, the jumps since the previous check are
 * accepted and the run continues from the plain result; otherwise they are
 * rejected, the state is rolled back to the last verified state and the
 * span is redone with the plain stepper, so the result then equals the
 * plain stepper's.  stats (if not NULL) receives [accepted jumps, rejected
 * jumps, checks, plain steps taken].  Runs on the plan's stream and
 * synchronises at every check. */
int cgl_run_surrogate(cgl_plan_t p, cgl_sur_t s, void* u_dev, const double* cstd,
                      int64_t njumps, int64_t steps_per_jump, int64_t check_every, double tol,
                      cgl_plan_t coarse, int base, int64_t* stats);

#ifdef __cplusplus
}
#endif

#endif /* CGL_ABI_H_ */
