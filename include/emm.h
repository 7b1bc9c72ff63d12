/*
 * emm.h -- C ABI of the MI355X fictitious-wave-domain CSEM FDTD library.
 *
 * What it computes (Yang, "libEMM", arXiv:2304.00233):
 *   Given a resistivity model on a rectilinear (possibly non-uniform) mesh,
 *   electric dipole sources, receivers and frequencies, it returns the complex
 *   frequency-domain Green's functions G^EE and G^HE of the diffusive Maxwell
 *   equations (Section 2.1, eq. 1) at the receivers.  It does so in Mittet's
 *   fictitious wave domain (Section 2.2, eqs. mittet/correspondence): a
 *   leap-frog staggered-grid (Yee) FDTD of the lossless wave equations with
 *   eps = sigma/(2 omega0), high-order finite differences on the non-uniform
 *   grid (Section 3.1, eqs. HFD1/HFD2), CPML absorbing layers (Section 3.4),
 *   time step dt = cfl/eta (Section 3.2), and an on-the-fly DTFT of the
 *   receiver samples (Section 3.5) normalised by the source spectrum
 *   (Section 2.2, eq. greenfunction).
 *
 * Conventions shared by every call:
 *   - every function returns emm_status: EMM_OK = 0, errors are negative; no
 *     C++ exception crosses the ABI;
 *   - all pointers are host pointers; inputs are borrowed for the duration of
 *     the call and copied, never written; outputs are caller-allocated;
 *   - 3D arrays are [n3][n2][n1] with x (index 1) fastest (Section 3.8);
 *   - the time-domain hot loop runs entirely on the GPU, with no host
 *     involvement between steps; the device is the current HIP device at
 *     emm_create time;
 *   - one emm_model per host thread at a time (not thread-safe).
 */
#ifndef EMM_H
#define EMM_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct emm_model emm_model;   /* opaque; owned by the caller between create and destroy */

typedef enum {
    EMM_OK            =  0,
    EMM_ERR_ARG       = -1,  /* NULL pointer, count out of range, bad option, bad channel mask */
    EMM_ERR_GRID      = -2,  /* n_d < 2*rd+1, coordinates not finite / not strictly increasing, or
                                a padded field array of 2^31 cells or more (see emm_create) */
    EMM_ERR_MODEL     = -3,  /* a resistivity <= 0 or not finite */
    EMM_ERR_GEOMETRY  = -4,  /* a source/receiver 2*rd stencil leaves the unpadded interior */
    EMM_ERR_FREQ      = -5,  /* a frequency <= 0 or not finite, or nfreq < 1 */
    EMM_ERR_CFL       = -6,  /* dt_override > 1/eta without allow_unstable */
    EMM_ERR_NONFINITE = -7,  /* a DTFT accumulator ended non-finite (unstable run), or a misfit /
                                cotangent of emm_gradient is not finite */
    EMM_ERR_OOM       = -8,  /* device memory request larger than what is free */
    EMM_ERR_DEVICE    = -9   /* a HIP call failed; emm_last_error() has the HIP message */
} emm_status;

/* The model mesh (Section 5, "Physical domain, grid dimensions and
 * coordinates" and "Resistivity files").  Node coordinates x_d[0..n_d-1] in
 * metres, strictly increasing, any spacing (the paper allows a non-uniform
 * z axis; all three axes are accepted here).  rho11/rho22/rho33 are the
 * homogenized resistivities (ohm-m) at the Ex/Ey/Ez positions, i.e. shifted
 * by half a cell along x/y/z: rho11[k][j][i] sits at (x_{i+1/2}, y_j, z_k). */
typedef struct {
    int n1, n2, n3;
    const double *x1, *x2, *x3;
    const float *rho11, *rho22, *rho33;
} emm_grid;

/* Options; emm_default_options() fills the defaults given in brackets. */
typedef struct {
    int    rd;             /* half stencil length r, 1..4: order 2r in space [2] (Section 5, rd) */
    int    nb;             /* CPML layers per side [10] (Section 3.4) */
    int    ne;             /* buffer layers between CPML and interior [rd+5 when < 0] */
    double f0;             /* omega0 = 2 pi f0 of the wave-domain transform, Hz [1.0] */
    double cfl;            /* dt = cfl/eta [0.99] (Section 3.2) */
    double dt_override;    /* > 0: use this dt; above 1/eta it is an EMM_ERR_CFL unless allow_unstable [0] */
    int    nt;             /* time steps; 0 = automatic (wavelet length + DFT kernel decay) [0] */
    int    dft_mode;       /* 0 = FP64 accumulators, 1 = FP32 with Kahan compensation [0] */
    double cpml_R;         /* theoretical reflection coefficient [1e-5] */
    double cpml_npow;      /* profile power N [2] */
    double cpml_alpha_max; /* frequency-shift maximum; 0 = pi * f_peak [0] */
    double wavelet_fpeak;  /* source wavelet peak frequency; 0 = 2 sqrt(f_max f0) [0] */
    int    allow_unstable; /* test hook: accept dt_override above the CFL limit [0] */
    int    profile;        /* 1 = time stencil launches with HIP events that the dispatch
                              stamps at kernel start and end (hipExtLaunchKernel): one E/H pair
                              in 16 direct steps; with graph_steps, every 8th block of steps runs
                              as direct launches and one pair in 4 of them is timed (emm_query) [0] */
    int    tile_kz;        /* z planes per thread block; 0 = chosen from the grid, -1 = autotuned
                              together with the nontemporal hint on the first forward (timing
                              candidates on this model) [0] */
    int    checkpoint_every; /* > 0: emm_forward keeps full-state checkpoints every this many
                              steps for a following emm_gradient, and emm_gradient uses this
                              outer interval; 0: emm_gradient plans it (see below) [0] */
    int    graph_steps;    /* > 0: capture this many time steps in one hipGraph and replay it
                              (a device step counter advances between replays) [0] */
    int    checkpoint_inner; /* > 0 and < the outer interval: emm_gradient re-runs each outer
                              segment once to lay inner checkpoints this many steps apart
                              (two levels); 0: planned [0] */
    int    nontemporal;    /* stencil kernels move the arrays they touch once with nontemporal
                              hints: 1 = yes, 0 = no, -1 = autotuned with tile_kz = -1, else
                              yes when the fields and dt/eps exceed 160 MiB [-1] */
    int    airwave;        /* 1: the first z node is the sea (or land) surface with air above it
                              (Section 3.3): no cell above it is updated and the ghost planes the
                              stencils reach are filled after each half step from 2-D Fourier
                              transforms of the surface plane (H as a potential field, E
                              harmonic); needs uniform x and y spacing (EMM_ERR_GRID otherwise);
                              with graph_steps the fills are captured in the step graphs;
                              emm_gradient and emm_forward_batch refuse it (EMM_ERR_ARG).
                              The transforms: 1 = chosen by plane size (the direct kernels while
                              both padded horizontal axes have at most 512 points, hipFFT above),
                              2 = hipFFT in FP32, 3 = the direct kernels: three per fill, in FP64
                              (each axis split once as n = f m and summed directly), accurate
                              where the surface field spans many orders of magnitude across the
                              plane; EMM_ERR_DEVICE above 512 points per axis [0] */
    double converge_tol;   /* > 0: stop early (Section 3.5, Section 4.1) once the lowest-frequency
                              DTFT of E1 at the 8 corner nodes of the interior changes, between two
                              checks converge_every steps apart, by at most converge_tol times its
                              largest corner magnitude, for every source; nt is then the maximum.
                              With graph_steps, graphs replay only if they divide converge_every.
                              emm_gradient and emm_forward_batch refuse it [0] */
    int    converge_every; /* steps between convergence checks [100] */
    int    fused;          /* 1: emm_forward runs one launch per time step (the E update, then
                              the H update of the same tile, with E recomputed on the x/y halo;
                              E, H and the E-step CPML memories in ping-pong buffers: 60 instead
                              of 84 B per cell and step) when no checkpoints, air boundary or
                              convergence stop are asked for; 0: two half-step launches [0] */
    int    ce_table;       /* compact dt/eps for the E step: per cell one 32-bit word of three
                              8-bit indices into a table of the model's distinct FP32 values
                              (the same values: 4 instead of 12 B per cell), possible when the
                              three components together hold at most 256 distinct values; then
                              4 B per padded cell of device memory. -1: used whenever possible
                              unless the autotuner (tile_kz = -1) measures the FP32 arrays
                              faster; 1: whenever possible; 0: never [-1] */
    int    src_group;      /* sources per time loop of emm_forward, which runs the loops one after
                              another (results are the same bit for bit): 0 = as many as keep the
                              arrays of one step within 160 MiB, so they stay in the 256 MB
                              Infinity Cache between steps, or all when one source alone does
                              not fit; -1 = all; k > 0 = k. With checkpoint_every or converge_tol
                              set, all sources run in one loop. emm_gradient groups its sources
                              too (0 = the most whose checkpoints fit one level, see there) [0] */
    int    tile_x;         /* columns per block of the stencil kernels: 64 (x 4 rows) or 32 (x 8
                              rows); 0 = autotuned with tile_kz = -1, else 32 where it leaves
                              fewer idle lanes in the last x tile of a row or at rd >= 3 [0] */
    int    tile_rows;      /* grid rows each wavefront of a stencil block updates: 1, or 2 / 4
                              (64-wide tiles of 8 / 16 rows, register-blocked: less staged halo
                              per cell, more loads per thread, but 2-3 waves per SIMD; needs
                              tile_x 0 or 64); 0 = 1, and the autotuner (tile_kz = -1) then
                              tries only the one-row shapes.  Every shape gives the same bits [0] */
    int    src_order;      /* order of the stencil blocks of several sources in one launch: 0 =
                              source fastest (the blocks of all sources for one spatial tile run
                              together and share dt/eps through L2), 1 = source slowest (each XCD
                              streams whole sources, so neighbouring tiles of one source share their
                              halos in L2); -1 = autotuned with tile_kz = -1, else 0.  Both give
                              the same bits [-1] */
} emm_options;

/* A point electric dipole (the acquisition of Section 5): position in
 * metres, component 0/1/2 = Jx/Jy/Jz, moment in A.m (G is per unit moment). */
typedef struct { double x, y, z; int comp; double moment; } emm_source;

/* A receiver position in metres; every receiver is live for every source. */
typedef struct { double x, y, z; } emm_receiver;

/* Model and last-run facts. */
typedef struct {
    double dt;               /* time step, s */
    int    nt;               /* steps of the last forward (or the fixed option; 0 before a forward if automatic) */
    int    n1pad, n2pad, n3pad;
    long long cells;         /* n1pad * n2pad * n3pad */
    double bytes_per_step;   /* algorithmic HBM bytes of one e-step + h-step, one source, as the
                                last forward ran them (FP32 dt/eps before the first) */
    double e_bytes, h_bytes; /* split of bytes_per_step over the two stencil kernels */
    /* filled when options.profile = 1: totals over the timed launches of the last forward */
    double e_kernel_ms, h_kernel_ms;   /* summed kernel durations (HIP events) */
    long long e_launches, h_launches;  /* number of launches timed */
    double forward_ms;       /* device time of the whole time loop (HIP events) */
    int    tile_kz;          /* z planes per block actually used */
    /* checkpoint schedule of the last emm_gradient */
    int    ckpt_outer;       /* steps between the forward's checkpoints */
    int    ckpt_inner;       /* steps between inner checkpoints (== ckpt_outer: one level) */
    double ckpt_bytes;       /* device bytes of checkpoints and per-step E snapshots */
    int    nontemporal;      /* 1: the stencil kernels of the last run used nontemporal hints */
    int    converged;        /* 1: the last forward stopped at a convergence check (nt = its step) */
    int    fused;            /* 1: the last forward ran the fused step kernel; e_kernel_ms,
                                e_launches then time that kernel and leap_bytes is its traffic */
    double leap_bytes;       /* algorithmic bytes of one fused step, one source */
    int    ce_table;         /* 1: the last forward's E step read dt/eps in the compact form */
    int    src_group;        /* sources per time loop of the last emm_forward (jobs per graph
                                after emm_forward_batch) */
    int    tile_x;           /* columns per block of the last forward's stencil kernels */
    int    tile_rows;        /* grid rows per wavefront of the last forward's stencil kernels */
    int    src_order;        /* tile order of the sources in the last forward's launches */
    int    air_transform;    /* ghost-fill transforms of the last forward: 0 = no air boundary,
                                1 = hipFFT, 2 = direct kernels */
} emm_info;

/* Fill *o with the defaults above: the paper's values where it states them
 * (rd = 2, the order of its GPU code, Section 4; dt = 0.99/eta, Section 3.2;
 * the CPML form of Section 3.4), this library's readings where it is silent
 * (f0 of Section 2.2, the wavelet, the CPML constants).  Errors: ARG (o is
 * NULL). */
emm_status emm_default_options(emm_options *o);

/* The set-up half of the init/close pairing of Section 3.8 (every module has
 * an xxx_init that allocates and an xxx_close that frees; Algorithm 1
 * set-up phase).  Validate the mesh and model, build the padded grid
 * (Section 3.4: nb + ne layers per side, coordinates extended with the end
 * interval, resistivity replicated), the FD coefficient tables by solving the
 * transposed Vandermonde system (Section 3.1, Bjorck-Pereyra), dt
 * (Section 3.2) and dt/eps per cell, then allocate device memory and upload.
 * Size limit: one field array of the padded grid, (n1 + 2(nb+ne) rounded up
 * to a multiple of 64) x (n2 + 2(nb+ne)) x (n3 + 2(nb+ne)) cells, must stay
 * below 2^31 (the kernels use 32-bit offsets within it), else EMM_ERR_GRID
 * before the resistivity arrays are read.  On success *out owns device memory
 * until emm_destroy.  Errors: ARG, GRID, MODEL, CFL, OOM, DEVICE; on error
 * *out is NULL. */
emm_status emm_create(const emm_grid *g, const emm_options *o, emm_model **out);

/* Copy model facts into *info: the padded grid (Section 3.4), dt
 * (Section 3.2), the step count of the last forward (Section 3.5) and the
 * launch and timing facts of the last run.  Errors: ARG. */
emm_status emm_query(const emm_model *m, emm_info *info);

/* Run the forward modelling for nsrc independent sources (batched in one
 * launch per half step) and write
 *   green[((s*nrec + r)*nchan + c)*nfreq + f] = (re, im)   (2 doubles)
 * for the channels c enumerated in bit order of chan_mask (bit 0..5 =
 * Ex, Ey, Ez, Hx, Hy, Hz; the order of the paper's output listing,
 * Section 5): G^EE in V/(A m^2) for E channels, G^HE in 1/m^2 for H
 * channels.  green must hold 2*nsrc*nrec*popcount(chan_mask)*nfreq doubles;
 * nsrc >= 1 and nrec >= 1 (else ARG), any number nfreq >= 1 of frequencies
 * (Section 3.5: one DTFT each; else FREQ).
 * hip_stream: a hipStream_t to run on, or NULL for the library's own stream.
 * Errors: ARG, GEOMETRY, FREQ, NONFINITE, OOM, DEVICE. */
emm_status emm_forward(emm_model *m, const emm_source *src, int nsrc,
                       const emm_receiver *rec, int nrec, unsigned chan_mask,
                       const double *freq_hz, int nfreq, double *green,
                       void *hip_stream);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): emm_forward with the
 * same arguments, results and errors, whose per-call device buffers (fields,
 * CPML memories, DTFT accumulators, source / receiver / CPML / phase tables)
 * all live in one static device workspace of 128 MiB per device (held from
 * the library's first use on a device until the process ends); it calls no
 * hipMalloc / hipFree, creates no event or graph, and clears what must start
 * at zero with a fill kernel.  It runs every source in one time loop of
 * direct launches (graph_steps and profile are ignored for the call; tiles:
 * the model's option or earlier autotuned choice, no autotuning).  A call
 * whose buffers exceed 128 MiB fails with EMM_ERR_OOM and a message giving
 * the bytes it needs (about 30 MB per source on a 48^3 grid with 10 CPML
 * layers); the air boundary and checkpoints (options airwave,
 * checkpoint_every) are refused with EMM_ERR_ARG.  The model itself must
 * exist (emm_create allocates its arrays once).  All calls on one device
 * share its workspace: calls that overlap in time on one device (any
 * models, any host threads or streams) race and give wrong results; the
 * workspace keeps the last call's contents.  A following emm_gradient does
 * not reuse anything from this call. */
emm_status emm_forward_noalloc(emm_model *m, const emm_source *src, int nsrc,
                               const emm_receiver *rec, int nrec, unsigned chan_mask,
                               const double *freq_hz, int nfreq, double *green,
                               void *hip_stream);

/* One forward modelling of emm_forward_batch: a model with its acquisition
 * and output, all as in emm_forward. */
typedef struct {
    emm_model *model;
    const emm_source *src;
    int nsrc;
    const emm_receiver *rec;
    int nrec;
    unsigned chan_mask;
    const double *freq_hz;
    int nfreq;
    double *green;
} emm_job;

/* Run the forward modellings of njobs jobs on different models (any grid
 * sizes; each keeps its own dt, step count and autotuned tiles) side by
 * side: each job gets its own stream and its own captured hipGraph of
 * graph_steps time steps (0 = 64), replayed with a device step counter per
 * model, and its last nt % graph_steps steps as direct launches; the
 * replays of all jobs of a group are issued in turn, so small grids share
 * the chip instead of running one after another (the paper runs one
 * transmitter per process, Section 5; here many models and sources share one
 * device).  Each job's green is exactly what emm_forward writes for it
 * (bitwise).  Jobs run in consecutive groups, group after group, by the
 * src_group option of the first job's model: -1 = all jobs together,
 * k > 0 = k jobs per group, 0 = as many jobs as keep their arrays within
 * 160 MiB (the Infinity Cache rule of emm_forward; a job that alone exceeds
 * it runs by itself), except that a group takes more jobs while its grids
 * hold fewer than 4 Mi cells in all (too few to fill the chip);
 * info.src_group of each model then holds the number of jobs in its group.
 * A model may appear in one job only; every model must live on the same
 * device.  hip_stream: the work starts after what is queued on it and it
 * waits for all jobs (NULL = the first model's stream).  Errors: as
 * emm_forward; the first failing job stops the call (emm_last_error of that
 * model). */
emm_status emm_forward_batch(const emm_job *jobs, int njobs, int graph_steps, void *hip_stream);

/* Discrete adjoint of the whole time loop (the exact gradient of the
 * FP32 time stepping as written: reverse of every E and H update with the
 * transposed finite-difference operators, reverse of the CPML memory-variable
 * recursion, reverse of the receiver DTFT), evaluated from full-state
 * checkpoints with forward recomputation.  The reverse sweep walks the
 * segments between checkpoints backwards; each segment is recomputed once
 * with the E field of every step kept, then reversed.  Memory, with S the
 * state of all nsrc sources (E, H, CPML memories) and F their E fields:
 *   one level  (inner == outer = C):  ceil(nt/C) S + (C+1) F
 *   two levels (inner C2 < outer C1): ceil(nt/C1) S + ceil(C1/C2) S + (C2+1) F
 * at the price of one more forward pass.  Intervals left at 0 are planned:
 * the one-level interval of least memory if it fits in the free device
 * memory (after the adjoint's own arrays), else the two-level pair of least
 * memory; EMM_ERR_OOM if neither fits (run fewer sources per call).  The
 * sources run in groups, one forward + reverse sweep per group, by the
 * src_group option: 0 = the most sources whose planned checkpoints fit one
 * level (a second level costs one more forward pass, batching saves only a
 * few per cent), else the most that fit two levels; -1 = all; k > 0 = k;
 * all of them when checkpoint_every is set or the last forward's
 * checkpoints are reused (info.src_group: the group size).  The result
 * does not depend on the schedule or the grouping (bitwise).  The scalar L is either
 *   g_obs != NULL: L = 1/2 sum over all results of |log(G/G_obs)|^2 (real
 *                  part: log-amplitude residual, imaginary part: phase
 *                  residual), returned in *misfit (may be NULL), or
 *   g_bar != NULL: any L given by its cotangent dL/dRe G + i dL/dIm G;
 * both laid out like `green`; exactly one must be given.  Output
 *   grad[(c*n3 + k)*n2 + j)*n1 + i] = dL/d log sigma_c at input cell (i,j,k),
 *   c = 0, 1, 2 for the conductivities behind rho11, rho22, rho33,
 * summed over sources (3*n1*n2*n3 doubles, caller-owned), with dt, the step
 * count and the CPML profile held fixed (they depend on the largest
 * resistivities).  green (may be NULL) receives G.  If the previous call on
 * this model left checkpoints of the same acquisition (an emm_forward with
 * checkpoint_every > 0, or an emm_gradient, whose own forward stores them),
 * they are reused and only the reverse sweep runs; otherwise the forward is
 * run here.  The sum over sources and the fold of the padding onto the
 * input cells run on the device.  The fields are FP32: a log misfit over
 * data far below the largest |G| (near the fields' rounding) amplifies that
 * rounding into the gradient; floor or down-weight such data and pass the
 * cotangent as g_bar.
 * This is the gradient that CSEM inversion needs (the paper's stated
 * horizon, Section 9).  Errors: as emm_forward, plus ARG. */
emm_status emm_gradient(emm_model *m, const emm_source *src, int nsrc,
                        const emm_receiver *rec, int nrec, unsigned chan_mask,
                        const double *freq_hz, int nfreq, const double *g_obs,
                        const double *g_bar, double *green, double *misfit,
                        double *grad, void *hip_stream);

/* The close half of the init/close pairing of Section 3.8: free the device
 * and host memory emm_create and the runs allocated. NULL-safe. */
void emm_destroy(emm_model *m);

/* Static name of a status code (the input classes of the problem statement
 * of Section 5: grid, model, geometry, frequencies; plus run-time failures). */
const char *emm_status_str(emm_status s);

/* Detail of the last failure on this thread (a validation message naming
 * the offending input of Section 5, or the HIP error string); empty if none.
 * m may be NULL. */
const char *emm_last_error(const emm_model *m);

#ifdef __cplusplus
}
#endif
#endif /* EMM_H */
