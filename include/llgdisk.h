/*
 * lib_llgdisk: the thin-film LLG disk hot path on one AMD Instinct MI355X (gfx950).
 *
 * Method: G. M. Wysin and W. Figueiredo, "Thermal vortex dynamics in thin
 * circular ferromagnetic nanodisks" (2012).  A disk of radius R and thickness
 * L is cut into a x a x L cells on a square grid (Sec. II.A); each cell holds
 * a unit vector m_i.  The demagnetisation field is the convolution of m with
 * the 2-D thin-film Green's kernels (Sec. II.B), evaluated by zero-padded FFT;
 * the induction b adds the nearest-neighbour exchange sum (eq. Bi); the
 * dynamics is dm/dtau = m x b - alpha m x (m x b) (Sec. III.A), stepped by RK4
 * at T = 0 (Sec. III.A) and by the Heun (H2) scheme with thermal noise at
 * T > 0 (Sec. III.B-C).
 *
 * Conventions for every entry point
 * ---------------------------------
 * Handle.  An llg_disk owns one disk or a batch of disks (replicas included),
 *   with their kernel spectra, twiddle tables, workspaces and barrier counters
 *   in device memory on the device that was current when it was created.  It
 *   is not thread-safe; calls on one handle must not overlap.
 * State layout.  The magnetisation of disk k is float32 [3][D_k][D_k]
 *   (component x, y, z; row = y cell index, column = x cell index); cell
 *   (iy, ix) sits at ((ix-(D-1)/2) a, (iy-(D-1)/2) a) from the disk centre and
 *   belongs to the disk when that point lies inside the circle of radius R.
 *   For a batch the disks are packed back to back in creation order; disk k
 *   starts at float offset llg_disk_offset(h, k).  Values outside the disk are
 *   ignored on input and written as 0 on output.
 * Pointers.  Every float and double array argument is a caller-owned DEVICE
 *   pointer on the handle's device, unless the comment says "host".  The
 *   library never frees or keeps them past the call.  llg_params arrays are
 *   host memory (one entry per disk of the handle).
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the default
 *   stream).  All work is enqueued asynchronously on it; results are ready
 *   when the stream reaches them.  Only llg_build_kernels, llg_batch_create
 *   and llg_check synchronise.
 * Units.  Lengths cross the ABI in nm.  Fields are in units of Ms, the
 *   induction b in units of B0 = 2A/(a^2 Ms), time in units of
 *   t0 = 1/(gamma B0), energies in units of J = 2AL of each disk.
 * Errors.  Every int-returning call returns 0 on success or a negative LLG_E*
 *   code; the message is available from llg_last_error() (per thread).  A
 *   device-side failure (a group barrier that timed out, a non-finite state)
 *   is recorded on the device and reported by the next llg_check().
 */
#ifndef LLGDISK_H
#define LLGDISK_H

#ifdef __cplusplus
extern "C" {
#endif

#define LLG_OK 0
#define LLG_EINVAL (-1)    /* bad argument (geometry, sizes, null pointer) */
#define LLG_EHIP (-2)      /* a HIP runtime call failed */
#define LLG_ENOMEM (-3)    /* device or host allocation failed */
#define LLG_EDEVICE (-4)   /* device-side failure flag raised (llg_check) */
#define LLG_EUNSUPPORTED (-5)

typedef struct llg_disk_s* llg_disk;

/* Dimensionless parameters of one disk (Sec. II.A, Sec. III).
 *   alpha     Gilbert damping.
 *   c         a^2/lambda_ex^2; multiplies the demag and external fields in b (eq. Bi).
 *   hext      external field / Ms (its constant part).
 *   temp      scaled temperature kT/(2AL) (Sec. III.B).
 *   dtau      time step in units of t0.
 *   renorm    nonzero: reset |m| = 1 after every full step.
 *   fd_factor nonzero: noise variance 2 alpha T dtau / (1 + alpha^2) instead of
 *             the paper's 2 alpha T dtau (Sec. III.C).
 * Time-dependent driving field (the h_ext of eq. Hmm and eq. Bi as a function of
 * time; all zero = a constant field):
 *   h_ext(tau) = hext + hac sin(2 pi freq tau + phase)
 *                     + hpulse exp(-(tau - tpulse)^2 / (2 wpulse^2))
 *   hac, freq, phase  oscillating part: amplitude / Ms, cycles per unit of tau, radians;
 *   hpulse, tpulse, wpulse  Gaussian pulse: amplitude / Ms, centre and width in tau
 *             (wpulse > 0 whenever hpulse is nonzero);
 *   tau0      the time at the start of the call.  Step n of a call runs from
 *             tau0 + n dtau; RK4 evaluates the field at its stage times (fractions
 *             0, 1/2, 1/2, 1 of the step), Heun at the start (predictor) and the
 *             end (corrector) of the step; llg_demag_field, llg_rhs, llg_energy and
 *             llg_relax use h_ext(tau0). */
typedef struct {
    double alpha;
    double c;
    double hext[3];
    double temp;
    double dtau;
    int renorm;
    int fd_factor;
    double hac[3];
    double freq;
    double phase;
    double hpulse[3];
    double tpulse;
    double wpulse;
    double tau0;
} llg_params;

/* Fill *out (host) from SI material data: exchange stiffness A (J/m), Ms (A/m),
 * gamma (1/(T s)), cell edge a and thickness L (nm), time step dt (ps),
 * temperature T (K) and damping alpha; hext is set to 0, renorm and fd_factor
 * to 0.  Also returns lambda_ex in nm through *lambda_ex_nm (host, may be NULL).
 * Formulas of Sec. II.A and Sec. III.A-B. */
int llg_params_from_si(double A, double Ms, double gamma, double a_nm, double L_nm,
                       double dt_ps, double T_K, double alpha, llg_params* out,
                       double* lambda_ex_nm);

/* Build one disk: D = 2R/a cells across (must be an integer within 1e-9),
 * mask, and the FFT size P (P_override = 0: the smallest power of two >= 2D,
 * at least 64; otherwise a power of two in [64, 512] with P >= 2D-1).  The
 * thin-film kernels (Sec. II.B: G_xx, G_yy, G_xy, G_zz at cell-centre
 * displacements, self terms -N_x, -N_x, 0, -N_z of the cell cylinder of radius
 * a/sqrt(pi)) are laid out at wrapped displacements on the P x P grid and
 * transformed once in float64 on the host; the real spectra are stored as
 * float32 quarter planes.  Synchronises the current device. */
int llg_build_kernels(double R_nm, double L_nm, double a_nm, int P_override, llg_disk* out);

/* Build a batch of n disks (a ragged ensemble and/or replicas): disk k has
 * radius R_nm[k] and thickness L_nm[k] (host arrays), all with cell edge a.
 * Equal geometries share one set of spectra.  wg_per_disk (host, may be NULL)
 * fixes the number of workgroups that step each disk; NULL lets the library
 * choose from the disk's cost and the device size. */
int llg_batch_create(int n, const double* R_nm, const double* L_nm, double a_nm,
                     const int* wg_per_disk, llg_disk* out);

/* Host queries: number of disks; D, P and masked-cell count of disk k; float
 * offset of disk k in a packed state; total floats of a packed state. */
int llg_disk_count(llg_disk h);
int llg_disk_info(llg_disk h, int k, int* D, int* P, int* n_cells);
long long llg_disk_offset(llg_disk h, int k);
long long llg_state_size(llg_disk h);
/* Workgroups assigned to disk k (host). */
int llg_disk_workgroups(llg_disk h, int k);

/* Re-plan the persistent launch of h (host; synchronises the device):
 * unit_groups = 1, 2 or 4 groups of three wavefronts per workgroup (each
 * group carries one transform per field component at a time), the transform
 * policy radix_policy = 0..3 (bit 0: radix-8 LDS stages everywhere, else
 * radix 4 below P = 512; bit 1: each lane group transforms all three
 * components of one spectral column, else one wavefront per component; the
 * adjoint and relaxation kernels ignore bit 1), and the number of workgroups
 * per disk (wg_per_disk, host, n entries; NULL = the library's choice).
 * The plan keeps the kernels of every mode co-resident (the adjoint and
 * relaxation kernels hold fewer workgroups per CU than the integrators), so
 * explicit counts are trimmed, largest first, to that limit; llg_autotune
 * plans for its integrator and the field kernel only, and a mode launched
 * later under such a plan is checked and refused if it cannot hold the plan.
 * Results do not depend on the plan beyond float rounding of the radix
 * schedule. */
int llg_tune(llg_disk h, int unit_groups, int radix_policy, const int* wg_per_disk);

/* Spectra on chip (the small-disk plan of the ragged batch): every disk of h
 * with FFT size P <= max_P (64 or 128; 0 = none) is stepped by one workgroup
 * that keeps the disk's row/column spectra (3 (P/2+1) D' complex floats, D'
 * = D rounded up to 8: 25 KB at P = 64, up to 100 KB at P = 128) in its LDS
 * for the whole launch of the field kernel and the integrators, so the two
 * transform phases of a field evaluation exchange them without leaving the
 * CU; the adjoint and relaxation kernels keep them in global memory, as every
 * disk of a larger P does.  Every workgroup of those launches reserves the
 * largest on-chip workspace of the handle.  The on-chip kernel instances have
 * one group of three wavefronts per workgroup.  Re-plans like llg_tune with
 * the current unit groups and transform policy and the library's workgroup
 * counts (host; synchronises the device); llg_tune and llg_autotune keep the
 * setting.  Fails with LLG_EUNSUPPORTED, leaving the previous plan, when the
 * current plan has more than one unit group (and so does llg_tune asking for
 * more than one while a limit is set).
 * Results are bitwise those of the same plan with the spectra in global
 * memory.  llg_get_on_chip returns the current max_P. */
int llg_set_on_chip(llg_disk h, int max_P);
int llg_get_on_chip(llg_disk h);

/* Autotuner: times llg_rk4_step (integrator 0) or llg_heun_step (1) for
 * probe_steps steps on a private copy of m (device) under every candidate plan
 * (unit groups 1/2/4 x transform policy 0..3 x the library's workgroup counts
 * scaled by 1, 1/2, 1/4, with the spectra in global memory; and where the
 * handle has disks of P <= 64 / P <= 128, those disks on chip with one unit
 * group, transform policy 0..3 and the full budget) and keeps the fastest.
 * *best_us (host) receives its time per step in microseconds.  Synchronises;
 * m is not modified. */
int llg_autotune(llg_disk h, const float* m, const llg_params* p, int integrator, long long probe_steps,
                 void* stream, double* best_us);

/* Current launch shape (host): unit groups, total workgroups, threads per
 * workgroup, transform policy (any pointer may be NULL). */
int llg_launch_shape(llg_disk h, int* unit_groups, int* workgroups, int* threads, int* radix_policy);

/* Demagnetisation field H^M / Ms of state m (Sec. II.B): H[k] = sum over the
 * disk of K(r_i - r_j) m_j, written to H (packed like m). */
int llg_demag_field(llg_disk h, const float* m, float* H, void* stream);

/* Right-hand side dm/dtau = m x b - alpha m x (m x b) with
 * b = exchange sum + c (hext + H^M) (eq. Bi, Sec. III.A); p: one entry per disk. */
int llg_rhs(llg_disk h, const float* m, float* dmdtau, const llg_params* p, void* stream);

/* nsteps classical RK4 steps in place (Sec. III.A), the full field evaluated
 * at all four stages; |m| reset to 1 after each step when p->renorm is set. */
int llg_rk4_step(llg_disk h, float* m, long long nsteps, const llg_params* p, void* stream);

/* nsteps Heun (H2) steps in place (Sec. III.C): g = b dtau + sigma w,
 * Delta(m) = m x [g - alpha (m x g)], predictor m~ = m + Delta(m), corrector
 * m' = m + (Delta(m) + Delta(m~))/2 with the same w, sigma = sqrt(2 alpha T dtau)
 * (over 1 + alpha^2 when fd_factor is set).  At step s (= step0 + n) the two
 * cells (2p, ix) and (2p+1, ix) of row pair p of disk k draw their noise from
 * two Philox4x32-10 blocks with counters (s mod 2^32, s div 2^32, 2q + h,
 * replica + k), h = 0, 1, q = p*D + ix, and key (seed mod 2^32, seed div 2^32):
 * every 32-bit output x gives u = ((x >> 8) + 0.5) 2^-24, the uniforms
 * U0..U5 (block 0, then the first two of block 1) give three Box-Muller pairs
 * n_2k = sqrt(-2 ln U_2k) cos(2 pi U_2k+1), n_2k+1 = sqrt(-2 ln U_2k) sin(2 pi U_2k+1);
 * the even row takes w = (n0, n1, n2), the odd row (n3, n4, n5). */
int llg_heun_step(llg_disk h, float* m, long long nsteps, unsigned long long seed,
                  unsigned long long step0, unsigned int replica, const llg_params* p,
                  void* stream);

/* The integrators with an observable series (float64, on the device): like
 * llg_rk4_step / llg_heun_step, and in addition, for every step n of the call
 * with n mod sample_every = 0, the state at the start of that step gives
 * series[((n / sample_every) * n_disks + k) * 4 + q] = (<m_x>, <m_y>, <m_z>, E)
 * of disk k (Sec. IV: spatial average over the disk cells; eq. Hmm: the energy
 * in units of J at the field of that instant).  series (device) needs
 * ceil(nsteps / sample_every) * n_disks * 4 doubles; sample_every >= 1.  The
 * sums are reduced in a fixed order (deterministic).  These sequences are the
 * input of the power spectra of Sec. V.B (llg_power_spectrum). */
int llg_rk4_series(llg_disk h, float* m, long long nsteps, const llg_params* p, long long sample_every,
                   double* series, void* stream);
int llg_heun_series(llg_disk h, float* m, long long nsteps, unsigned long long seed, unsigned long long step0,
                    unsigned int replica, const llg_params* p, long long sample_every, double* series,
                    void* stream);

/* Power spectra of real float64 sequences (Sec. V.B: spectra of <m_x>(tau)).
 * Sequence b (0 <= b < n_seq) has elements x_b[t] = x[b * bstride + t * tstride],
 * t = 0 .. len-1 (device array).  With remove_mean set the sequence's mean is
 * subtracted; window 0 = none, 1 = Hann, w[t] = sin^2(pi t / len).  Then
 * X_b[k] = sum_t w[t] x_b[t] exp(-2 pi i t k / len) and
 * out[b * (len/2 + 1) + k] = |X_b[k]|^2 / len for k = 0 .. len/2 (device).
 * len must be a power of two in [16, 2^24].  work (device) holds 4 * len * n_seq
 * doubles.  float64 radix-2 Stockham passes through work. */
int llg_power_spectrum(const double* x, int n_seq, long long bstride, long long len, long long tstride,
                       int remove_mean, int window, double* work, double* out, void* stream);

/* step0 value for llg_heun_step: take the first step index from the handle's
 * device-side step counter and advance the counter by nsteps afterwards (in
 * stream order), so that repeated calls, and replays of a graph, continue one
 * noise stream without host involvement. */
#define LLG_STEP_COUNTER (~0ull)

/* Set the handle's step counter (enqueued on stream) / read it (host,
 * synchronises the stream). */
int llg_step_counter_set(llg_disk h, unsigned long long step, void* stream);
int llg_step_counter_get(llg_disk h, unsigned long long* step, void* stream);

/* Ragged batches as an executable hipGraph: one graph runs nsteps RK4
 * (integrator 0) or Heun (integrator 1) steps of every disk of h on the state
 * m (device, packed like the handle's disks), exactly like llg_rk4_step /
 * llg_heun_step with step0 = LLG_STEP_COUNTER: a barrier-reset kernel node,
 * the persistent launch as a cooperative kernel node, and for Heun a node that
 * advances the step counter.  The graph copies the parameters p (host, one per
 * disk) at creation and keeps the handle's launch plan of that moment; the
 * handle must outlive the graph, and replays must not overlap other calls on
 * the same handle.  Creation synchronises the device. */
typedef struct llg_graph_s* llg_graph;
int llg_graph_create(llg_disk h, int integrator, float* m, long long nsteps, const llg_params* p,
                     unsigned long long seed, unsigned int replica, llg_graph* out);
int llg_graph_launch(llg_graph g, void* stream);
void llg_graph_destroy(llg_graph g);

/* Lagrange-constrained alignment relaxation (Sec. IV) in place: every sweep
 * evaluates the full induction b and sets m_i <- (b_i + b^lam_i + kappa m_i)/|.|
 * for all cells at once, with the fictitious field b^lam_i = 2 m_z,i
 * (lambda . (r_i - X)) z-hat of the constraint sum_i m_z,i^2 (r_i - X) = 0
 * over the disk cells with |r_i - X| < cutoff_nm (cutoff_nm = 0: every disk
 * cell; 4 lambda_ex matches the core-position definition);
 * after each sweep the two multipliers take one Newton step in float64 on the
 * device (Jacobian of the aligned state at fixed b).  Stops when the largest
 * |m_i x (b_i + b^lam_i)| and |C| drop below tol, or after max_sweeps.
 * X_nm (host, 2 per disk): target vortex positions in nm from the disk centre.
 * out (device, 8 doubles per disk): lambda_x, lambda_y, sweeps, residual,
 * C_x, C_y, 0, 0.  The relaxed state's energy U(X) comes from llg_energy. */
int llg_relax(llg_disk h, float* m, const double* X_nm, double cutoff_nm, double kappa, double tol,
              long long max_sweeps, const llg_params* p, double* out, void* stream);

/* Adjoint support (the paper integrates forward only; this is the hand-written
 * reverse mode of its RK4 step, Sec. III.A).
 *
 * llg_rk4_record: nsteps RK4 steps in place like llg_rk4_step (renorm must be
 * off) that also store, for every step n and stage s, the stage state and its
 * demag field into rec: disk k's block starts at float offset
 * 8 * nsteps * llg_disk_offset(h, k) and holds [nsteps][4][2][3][D][D]
 * (stage state, demag field).  rec needs 8 * nsteps * llg_state_size(h) floats.
 *
 * llg_rk4_vjp: reverse pass over the same nsteps: on entry ybar holds the
 * cotangent of the state after the last step, on exit the cotangent of the
 * state before the first step.  pgrad (2 doubles per disk) is incremented by
 * d/d alpha and d/d c of the same scalar.  The demag and exchange operators are
 * symmetric, so the reverse pass applies the forward field machinery to the
 * cotangent of the induction at every stage.  rec must come from
 * llg_rk4_record with the same nsteps and params. */
int llg_rk4_record(llg_disk h, float* m, long long nsteps, const llg_params* p, float* rec, void* stream);
int llg_rk4_vjp(llg_disk h, const float* rec, long long nsteps, float* ybar, double* pgrad,
                const llg_params* p, void* stream);

/* Adjoint of the Heun (H2) step with the noise replayed (Sec. III.C; the
 * reverse mode is this library's, the paper integrates forward only).
 *
 * llg_heun_record: nsteps Heun steps in place like llg_heun_step (explicit
 * step0; renorm allowed) that also store, for every step n and both stages
 * (the field at m_n and at the predictor m~), the stage state and its demag
 * field into rec: disk k's block starts at float offset
 * 4 * nsteps * llg_disk_offset(h, k) and holds [nsteps][2][2][3][D][D].
 * rec needs 4 * nsteps * llg_state_size(h) floats.
 *
 * llg_heun_vjp: reverse pass over the same steps (same seed, step0, replica
 * and params): on entry ybar holds the cotangent of the state after the last
 * step, on exit the cotangent of the state before the first step.  pgrad (2
 * doubles per disk) is incremented by d/d alpha (through the torque and
 * through sigma(alpha) of the noise) and d/d c of the same scalar; the noise
 * w itself is regenerated from the counter, not stored. */
int llg_heun_record(llg_disk h, float* m, long long nsteps, unsigned long long seed, unsigned long long step0,
                    unsigned int replica, const llg_params* p, float* rec, void* stream);
int llg_heun_vjp(llg_disk h, const float* rec, long long nsteps, unsigned long long seed, unsigned long long step0,
                 unsigned int replica, float* ybar, double* pgrad, const llg_params* p, void* stream);

/* Cotangent of the core position: with the plaquette r_v and the cutoff set
 * frozen at `core` (the out array llg_vortex_core_position returned for the
 * same m), adds d(rbar . r_c)/dm to mbar (packed like m).  rbar: 2 doubles per
 * disk (device), in 1/nm. */
int llg_core_position_vjp(llg_disk h, const float* m, double lambda_ex_nm, const double* core,
                          const double* rbar, float* mbar, void* stream);

/* Opt-in launch timing (host): with enable set, every later persistent
 * launch of h (the field kernel, the integrators, their series, adjoint and
 * relaxation forms; not graph replays) is bracketed by two HIP events on its
 * stream, just around the cooperative kernel (after the barrier reset), kept
 * per kind of launch.  llg_last_launch_ms waits for the last launch of one
 * kind (mode: 0 field, 1 right-hand side, 2 energy, 3 RK4, 4 Heun, 5 RK4
 * adjoint, 6 relaxation, 7 Heun adjoint) and returns its duration in ms;
 * LLG_EINVAL when no launch of that kind was timed since timing was
 * (re-)enabled.  Costs two event records per launch; off by default. */
int llg_timing(llg_disk h, int enable);
int llg_last_launch_ms(llg_disk h, int mode, float* ms);

/* Failure-path test hook (host): every later launch of h gives a group-
 * barrier wait `polls` polls (each a device-coherent load, about a
 * microsecond) before it records
 * LLG_EDEVICE "group barrier timed out" for llg_check and leaves the kernel,
 * as it would after a lost workgroup; 0 restores the default budget of 2^22
 * polls (seconds).  Graphs keep the budget of their creation.  States written by a
 * launch that timed out are unspecified. */
int llg_debug_spin_limit(llg_disk h, unsigned int polls);

/* The noise w that llg_heun_step uses at one time step (test hook), packed
 * like m (zero outside the disks). */
int llg_noise(llg_disk h, unsigned long long seed, unsigned long long step,
              unsigned int replica, float* w, void* stream);

/* Energy of eq. Hmm in units of J, float64 sums on the device:
 * out[4k..4k+3] = (E, E_exchange, E_demag, E_external) for disk k with
 * E_exchange = -sum over neighbour pairs m_i.m_j, E_demag = -(c/2) sum H.m,
 * E_external = -c sum hext.m. */
int llg_energy(llg_disk h, const float* m, const llg_params* p, double* out, void* stream);

/* Vortex core position (Sec. IV), float64 on the device.  out[5k..5k+4] =
 * (x_c, y_c, x_v, y_v, n_plus) in nm from the disk centre: r_v is the shared
 * corner of a 2x2 plaquette of disk cells whose in-plane angle winds by +1
 * (angle differences wrapped into [-pi, pi)); with several, the one nearest
 * hint_nm[2k..2k+1] (host, may be NULL) or else the one with the largest
 * sum of m_z^2 over its corners, ties to the lowest row then column;
 * r_c = sum (m_z)^2 r_i / sum (m_z)^2 over disk cells with |r_i - r_v| <
 * 4 lambda_ex.  With no such plaquette n_plus = 0, r_v = NaN and r_c is the
 * weighted mean over the whole disk. */
int llg_vortex_core_position(llg_disk h, const float* m, double lambda_ex_nm,
                             const double* hint_nm, double* out, void* stream);

/* Spatial average <m> per disk (Sec. IV): out[3k..3k+2], float64. */
int llg_mean_m(llg_disk h, const float* m, double* out, void* stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): llg_rk4_step whose
 * workspaces (stage states, RK4 accumulator, row/column spectra, barrier
 * counters, descriptor table) live in a fixed array of LLG_NOALLOC_BYTES
 * bytes inside the library instead of the handle's own buffers.  The array
 * exists once per GPU for the life of the process; its address is looked up
 * on the first call on a device.  The call allocates nothing (the handle,
 * created earlier, supplies the geometry, kernel spectra and launch plan) and
 * returns LLG_EINVAL, before enqueueing anything, when the handle needs more
 * than LLG_NOALLOC_BYTES (llg_noalloc_bytes tells how much; a single disk up
 * to D = 256 needs at most about 5 MB).  Results equal llg_rk4_step's.  All
 * calls on one GPU share the array: calls that overlap on one GPU (several
 * streams, several threads) race and must be serialised by the caller. */
#define LLG_NOALLOC_BYTES (32ll << 20)
long long llg_noalloc_bytes(llg_disk h);
int llg_rk4_step_noalloc(llg_disk h, float* m, long long nsteps, const llg_params* p, void* stream);

/* Synchronise the stream and report a device-side failure recorded since the
 * last check (LLG_EDEVICE) or 0. */
int llg_check(llg_disk h, void* stream);

void llg_destroy(llg_disk h);
const char* llg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LLGDISK_H */
