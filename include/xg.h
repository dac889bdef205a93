/* xg -- batched evaluation of straight-line scalar programs on one MI355X.
 *
 * A program is the paper's representation of a closed-form symbolic
 * function (section "Code Generation"): a work vector of scalar slots and
 * a list of instructions, each with an operation id, operand indices and
 * an output index, evaluated by walking the list in order.  Inputs and
 * outputs are dense vectors of structural non-zeros (background section on
 * sparse SX functions).  The library compiles one program into HIP kernels
 * (one thread per instance, as in the paper's generated-kernel listing)
 * and evaluates it for N independent instances whose data stay on the GPU
 * (the section on data residency: no host<->device transfer per call).
 *
 * Data layout of every argument: structure of arrays, instance fastest.
 * Element e of instance i of argument a is at ptr[a][e * ld[a] + i], with
 * ld[a] >= N.  Pointers passed to the evaluation calls are device pointers.
 *
 * Conventions: every call returns an xg_status; XG_OK is 0 and errors are
 * negative.  On error, xg_last_error() returns a message for the calling
 * thread.  No call throws.  Evaluation calls are asynchronous on the given
 * stream (a hipStream_t, or NULL for the default stream); they neither
 * allocate nor synchronise.  A launch failure is reported by the call; a
 * fault during execution surfaces at the caller's next synchronisation.
 */
#ifndef XG_H
#define XG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  XG_OK = 0,
  XG_EINVAL = -1,        /* invalid argument or malformed program */
  XG_EALIAS = -2,        /* an output range overlaps an input range */
  XG_ENOMEM = -3,        /* host allocation failed / workspace too small */
  XG_ECOMPILE = -4,      /* the runtime compiler rejected generated code */
  XG_EDEVICE = -5,       /* a HIP runtime call failed */
  XG_EUNSUPPORTED = -6   /* valid request the library does not implement */
} xg_status;

typedef enum { XG_F32 = 32, XG_F64 = 64 } xg_dtype;

/* Operation ids.  Arity and semantics (C99 / IEEE-754, round to nearest):
 *   INPUT  out=slot, a=argument, b=element      work[out] = x_a[b]
 *   OUTPUT out=argument, a=slot, b=element      y_out[b] = work[a]
 *   CONST  out=slot, a=constant index           work[out] = c[a]
 *   ASSIGN out=slot, a=slot                     copy
 *   ADD SUB MUL DIV                             a op b
 *   NEG SQ                                      -a, a*a
 *   SQRT EXP LOG SIN COS TAN TANH ATAN FABS     library function of a
 *   FMIN FMAX                                   C99 fmin / fmax
 *   LT LE                                       a < b ? 1 : 0, a <= b ? 1 : 0
 *   POW ATAN2                                   pow(a, b), atan2(a, b)
 * Every instruction reads all of its operands before writing its output
 * (an instruction may overwrite one of its operands' slots, as the paper's
 * generated-kernel listing does).  Constants are given in double and are
 * rounded once to float in an XG_F32 program.  The set follows the paper's
 * mapping table (assign, add, sub, mul, div, neg, exp, log, pow, ...) and
 * the functions its text names (log, cos, sqrt, atan2, min/max). */
typedef enum {
  XG_OP_INPUT = 0, XG_OP_OUTPUT, XG_OP_CONST, XG_OP_ASSIGN,
  XG_OP_ADD, XG_OP_SUB, XG_OP_MUL, XG_OP_DIV,
  XG_OP_NEG, XG_OP_SQ, XG_OP_SQRT, XG_OP_EXP, XG_OP_LOG,
  XG_OP_SIN, XG_OP_COS, XG_OP_TAN, XG_OP_TANH, XG_OP_ATAN,
  XG_OP_FABS, XG_OP_FMIN, XG_OP_FMAX, XG_OP_LT, XG_OP_LE,
  XG_OP_POW, XG_OP_ATAN2,
  XG_OP_COUNT
} xg_op;

typedef struct {
  int32_t op;  /* xg_op */
  int32_t out;
  int32_t a;
  int32_t b;   /* -1 where unused */
} xg_instr;

/* A program as the caller holds it.  The library copies everything it
 * needs during xg_program_load; the caller keeps ownership of the arrays. */
typedef struct {
  int32_t n_in;             /* number of input arguments */
  const int32_t* nnz_in;    /* [n_in] elements per input argument */
  int32_t n_out;            /* number of output arguments */
  const int32_t* nnz_out;   /* [n_out] elements per output argument */
  int32_t n_work;           /* work-vector slots */
  int64_t n_instr;
  const xg_instr* instr;    /* [n_instr] */
  int32_t n_const;
  const double* consts;     /* [n_const] */
  int32_t dtype;            /* xg_dtype: arithmetic of the whole program */
  const int8_t* prec;       /* [n_instr] or NULL: per-instruction precision
                               in an XG_F64 program: 0 = the program's, 32 =
                               binary32 (operands rounded to float, operation
                               in float, result widened exactly).  Keeps
                               e.g. dynamics in fp32 and a KKT factorisation
                               in fp64 inside one program. */
} xg_program_desc;

/* Compilation and launch options.  Zero means "library default". */
typedef struct {
  int32_t block;       /* threads per workgroup: 64, 128, 256 (default 64) */
  int32_t ipt;         /* instances per thread: 1, 2, 4 (default 1) */
  int32_t chunk_ops;   /* max operations per kernel of a chunked program */
  int32_t reg_budget;  /* max live values held in registers before the
                          planner spills to LDS (per instance) */
  int32_t lds_slots;   /* max LDS spill slots per lane */
  int32_t strict;      /* 1: no FMA contraction (bitwise-reproducible basic ops) */
  int32_t eager;       /* 1: compile during xg_program_load */
  int32_t adj_seg_ops; /* adjoint: operations per recomputed leaf range
                          (default 250; <= 0 would keep every value) */
  int32_t verbose;     /* 1: log planning and compile times to stderr */
  int32_t prefetch;    /* reloads are issued this many operations ahead of
                          their use (default 24; -1 disables) */
  int32_t waves;       /* cooperative tiles: 1 (default), 2, 4, 8 or 16
                          waves of one workgroup evaluate the same 64
                          instances, the program split by dependency level
                          (forward mode; needs block 64 and ipt 1) */
  int32_t inline_math; /* SIN, COS, EXP, TANH: 0 or 1 (default) inline
                          branch-free evaluation in fp64 (argument
                          reduction, polynomials; sin/cos within 2 ulp for
                          |x| <= 2^50 and NaN beyond); -1 calls the device
                          library */
  int32_t adj_fanout;  /* adjoint: a range of more than adj_seg_ops
                          operations is cut into up to this many parts at
                          small live sets, reversed part by part from the
                          states at the cuts (recursively); 2 ... 16,
                          default 2 */
  int32_t coop_phase;  /* cooperative tiles (waves > 1): 0 (default) splits
                          the program by dependency level with a barrier per
                          level (wide programs); > 0 plans phases of about
                          this much work per wave (operation-cost units, ~1
                          per arithmetic operation) for narrow programs:
                          reduction trees kept whole on one wave, values
                          kept in registers, exchanged values through LDS.
                          Forward mode only (the adjoint modes ignore it);
                          inside a batch every program then needs the
                          same workgroup size, 64 x waves. */
} xg_options;

typedef struct xg_program xg_program;
typedef struct xg_batch xg_batch;
typedef struct xg_graph xg_graph;

/* Facts about a loaded program (per evaluation mode). */
typedef struct {
  int64_t n_nodes;      /* SSA values after common-subexpression merging and DCE */
  int64_t n_ops;        /* arithmetic operations (no INPUT/OUTPUT/CONST/ASSIGN) */
  int64_t max_live;     /* largest live set of the chosen schedule */
  int32_t n_chunks;     /* kernels per evaluation */
  int32_t n_ws_slots;   /* workspace values per instance (chunk boundaries, spills) */
  int32_t n_lds_slots;  /* LDS spill slots per lane (largest chunk) */
  int32_t n_spills;     /* spill stores emitted */
  double compile_ms;    /* last compile (0 if served from the cache) */
  int32_t cache_hits;   /* code objects served from the on-disk cache */
  int32_t vgprs;        /* registers (VGPRs + AGPRs) a wave of the largest kernel is
                           allocated (granules of 8), from its kernel descriptor;
                           0 until compiled */
  uint64_t code_hash;   /* FNV-1a of the generated sources and compile options:
                           identifies the kernels a measurement was taken on */
  int32_t lds_bytes;    /* static LDS per workgroup of the largest kernel (bytes),
                           from its kernel descriptor; 0 until compiled */
  int32_t scratch_bytes;/* scratch (compiler register spills) per lane of the
                           largest kernel, from its kernel descriptor */
} xg_info;

/* Load, validate and plan a program (copying the description).  Errors:
 * XG_EINVAL with the offending instruction index in the message for an
 * unknown op, an index out of range, a read of a slot never written, or an
 * output element never written.  If an output element is written twice the
 * last write wins.  Compilation happens at the first evaluation unless
 * opts->eager.  `opts` may be NULL.  The representation is the paper's
 * ("Code Generation": work vector, instruction list, nnz inputs/outputs);
 * the paper generates and compiles code offline, this library at load. */
xg_status xg_program_load(const xg_program_desc* desc, const xg_options* opts,
                          xg_program** out);
/* Frees the program and unloads its kernels, first waiting for the devices
 * that hold them to finish queued work (launches are asynchronous). */
void xg_program_free(xg_program* p);

/* mode: 0 forward, 1 adjoint (gradient), 2 fused forward + adjoint. */
xg_status xg_program_info(xg_program* p, int32_t mode, xg_info* info);

/* The options `mode` is planned and launched with (library defaults
 * resolved).  Mode 0 (forward) and the adjoint modes 1 and 2 start from the
 * load options; xg_autotune replaces those of mode 0, xg_autotune_adjoint
 * those of modes 1 and 2. */
xg_status xg_program_options(xg_program* p, int32_t mode, xg_options* out);

/* Device workspace (bytes) an evaluation of n instances needs: values that
 * cross kernel boundaries of a chunked program.  The caller allocates it
 * (e.g. as a torch tensor) and passes it to the evaluation; 0 means none is
 * needed and NULL may be passed. */
xg_status xg_workspace_bytes(xg_program* p, int64_t n, int32_t mode, size_t* bytes);

/* Compile (if not yet compiled) the kernels of `mode` for the current
 * device.  Optional: evaluation compiles on first use. */
xg_status xg_compile(xg_program* p, int32_t mode);

/* Generate and compile the code objects of `mode` into the on-disk cache
 * without touching any device (works on a machine without a GPU).  The
 * cache directory is $XG_CACHE_DIR, else "_kcache" next to the library. */
xg_status xg_precompile(xg_program* p, int32_t mode);

/* Forward evaluation for n instances: y = P(x).  d_in[a] / d_out[a] are
 * device pointers with pitches ld_in[a] / ld_out[a] (elements, >= n).
 * n == 0 is a no-op.  Output ranges must not overlap input ranges
 * (XG_EALIAS).  Inputs are read-only.  d_workspace: xg_workspace_bytes(mode 0).
 * The evaluation of the paper's generated kernel (one instance per GPU
 * thread, every instruction in order; "Code Generation" listing), with
 * instance-fastest layouts and registers instead of a global work vector. */
xg_status xg_eval(xg_program* p, int64_t n,
                  const void* const* d_in, const int64_t* ld_in,
                  void* const* d_out, const int64_t* ld_out,
                  void* d_workspace, void* stream);

/* Reverse-mode adjoint: x_bar = J_P(x)^T y_bar, written (not accumulated)
 * to d_in_bar (same shapes as the inputs).  d_out_bar holds the seeds y_bar
 * (same shapes as the outputs).  If d_out is non-NULL the forward outputs
 * are written too (fused forward + adjoint, mode 2); otherwise mode 1.
 * Derivative rules: those of calculus; FMIN/FMAX pass the derivative to the
 * first operand on a tie; FABS'(0) = 0; LT/LE have zero derivative.
 * Extension beyond the paper, which differentiates symbolically in CasADi
 * before generating code: here the library derives the adjoint program. */
xg_status xg_eval_adjoint(xg_program* p, int64_t n,
                          const void* const* d_in, const int64_t* ld_in,
                          const void* const* d_out_bar, const int64_t* ld_out_bar,
                          void* const* d_out, const int64_t* ld_out,
                          void* const* d_in_bar, const int64_t* ld_in_bar,
                          void* d_workspace, void* stream);

/* Size of the fixed device array xg_eval_adjoint_noalloc uses as its
 * workspace: 128 MiB on every GPU the library runs on (the 7-link
 * pendulum's fused adjoint at 65,536 instances in binary64 needs 78 MiB in
 * its tuned plan: 156 slots of 8 bytes per instance). */
#define XG_NOALLOC_SCRATCH_BYTES (128u << 20)

/* xg_eval_adjoint for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Arguments and results are those of xg_eval_adjoint without
 * d_workspace: the workspace is a fixed array of XG_NOALLOC_SCRATCH_BYTES
 * inside this library, one per GPU, held from the first call on that GPU
 * until the process ends.  The call compiles, loads and allocates nothing:
 * the mode's kernels must already be loaded on the current device
 * (xg_compile(p, 1) for the gradient, xg_compile(p, 2) for the fused
 * forward + adjoint), else XG_EINVAL.  The first call on a device looks up
 * the array's device address (this can load the library's device code onto
 * the GPU, the one allocation: make that first call outside graph capture).
 * XG_ENOMEM if n instances need more workspace than the array holds (the
 * message gives both sizes).  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (two streams, two threads) race and
 * must be serialised by the caller.  Extension beyond the paper. */
xg_status xg_eval_adjoint_noalloc(xg_program* p, int64_t n,
                                  const void* const* d_in, const int64_t* ld_in,
                                  const void* const* d_out_bar, const int64_t* ld_out_bar,
                                  void* const* d_out, const int64_t* ld_out,
                                  void* const* d_in_bar, const int64_t* ld_in_bar,
                                  void* stream);

/* Several distinct programs in ONE persistent launch.  The programs are
 * borrowed (they must outlive the batch).  Workgroups pull (program, tile)
 * jobs, longest tiles first, from a counter in the workspace.  Every program
 * needs the same workgroup size (its block, or 64 x waves for cooperative
 * tiles) and the same ipt (XG_EINVAL otherwise); XG_EUNSUPPORTED if the
 * compiled kernel needs more registers per wave than a workgroup of that
 * size can hold on one CU, or its arguments exceed one launch.  Extension
 * beyond the paper, which launches one kernel per function. */
typedef struct {
  int64_t n;
  const void* const* d_in;
  const int64_t* ld_in;
  void* const* d_out;
  const int64_t* ld_out;
} xg_batch_args;

xg_status xg_batch_create(xg_program* const* progs, int32_t k, const xg_options* opts,
                          xg_batch** out);
/* Frees the batch (not its programs), waiting as xg_program_free does. */
void xg_batch_free(xg_batch* b);
/* args: k entries.  Workspace: xg_batch_workspace_bytes for the same n's. */
xg_status xg_batch_workspace_bytes(xg_batch* b, const int64_t* n, size_t* bytes);
xg_status xg_batch_eval(xg_batch* b, const xg_batch_args* args, void* d_workspace,
                        void* stream);

/* Capture a steady-state forward evaluation (or batch evaluation) in a HIP
 * graph; pointers are baked into the graph (re-capture when they change).
 * While a graph lives, its program or batch keeps its kernels loaded and
 * refuses re-tuning.  Extension beyond the paper. */
xg_status xg_graph_capture_eval(xg_program* p, int64_t n,
                                const void* const* d_in, const int64_t* ld_in,
                                void* const* d_out, const int64_t* ld_out,
                                void* d_workspace, void* stream, xg_graph** out);
xg_status xg_graph_capture_batch(xg_batch* b, const xg_batch_args* args,
                                 void* d_workspace, void* stream, xg_graph** out);
/* Capture a closed-loop time loop of `steps` evaluations z <- P(z, ...),
 * for programs whose only output has the shape of their first input (a
 * simulation step, as in the paper's quadcopter rollouts): evaluation k
 * reads the state from d_state0 (k even) or d_state1 (k odd) and writes the
 * other buffer, so the final state is in d_state0 when steps is even and in
 * d_state1 when odd.  Both state buffers use pitch ld_state; d_in/ld_in give
 * the remaining inputs (entry 0 is ignored).  Extension beyond the paper. */
xg_status xg_graph_capture_rollout(xg_program* p, int64_t n, int32_t steps,
                                   void* d_state0, void* d_state1, int64_t ld_state,
                                   const void* const* d_in, const int64_t* ld_in,
                                   void* d_workspace, void* stream, xg_graph** out);
xg_status xg_graph_launch(xg_graph* g, void* stream);
void xg_graph_free(xg_graph* g);

/* Choose the forward launch plan for n instances by timing candidates with
 * HIP events on `stream`: register budget x reload prefetch distance x LDS
 * spill budget (the full one and the one that keeps every wave of an
 * n-instance launch resident), plus block 256, two instances per thread,
 * half-size chunks, a single chunk (programs of up to three chunks) and
 * cooperative tiles where n or the program makes them
 * matter.  Inputs and outputs are buffers the caller provides, as for
 * xg_eval; the workspace must hold xg_autotune_workspace_bytes(p, n, 0)
 * bytes (candidates needing more are skipped).  The chosen options replace
 * those of mode 0 and are cached on disk per (program, n).  Extension
 * beyond the paper. */
xg_status xg_autotune(xg_program* p, int64_t n,
                      const void* const* d_in, const int64_t* ld_in,
                      void* const* d_out, const int64_t* ld_out,
                      void* d_workspace, size_t workspace_bytes, void* stream,
                      xg_options* chosen);

/* The same for the adjoint evaluations: candidates of the same kinds
 * (no cooperative tiles) plus shorter and longer recomputed segments
 * (adj_seg_ops) are timed as xg_eval_adjoint calls on the caller's
 * buffers (arguments as for xg_eval_adjoint; with d_out the fused mode 2 is
 * timed, without it mode 1), and the fastest replaces the options of both
 * adjoint modes.  The workspace must hold
 * xg_autotune_workspace_bytes(p, n, 2 or 1) bytes.  Cached on disk per
 * (program, n, mode timed).  Extension beyond the paper. */
xg_status xg_autotune_adjoint(xg_program* p, int64_t n,
                              const void* const* d_in, const int64_t* ld_in,
                              const void* const* d_out_bar, const int64_t* ld_out_bar,
                              void* const* d_out, const int64_t* ld_out,
                              void* const* d_in_bar, const int64_t* ld_in_bar,
                              void* d_workspace, size_t workspace_bytes, void* stream,
                              xg_options* chosen);

/* Largest workspace any candidate of xg_autotune (mode 0) or
 * xg_autotune_adjoint (mode 1 or 2) for n instances needs. */
xg_status xg_autotune_workspace_bytes(xg_program* p, int64_t n, int32_t mode, size_t* bytes);

/* Plan and compile every candidate the autotuner would time for n
 * instances of `mode` into the code cache, without touching a device. */
xg_status xg_autotune_precompile(xg_program* p, int64_t n, int32_t mode);

/* Choose a persistent launch for these programs and instance counts (the
 * args' n) by timing candidates on the caller's buffers: one workgroup size
 * B in {64, 256, 512, 1024} for the launch, each program with few tiles
 * (under 4 per CU) and at least 32 x B/64 operations per dependency level
 * as B/64-wave cooperative tiles, every other program on B-lane
 * workgroups.  Candidates whose kernel cannot be resident or whose
 * workspace exceeds workspace_bytes are skipped.  Returns a new batch that
 * owns copies of the programs with the chosen options (the caller's
 * programs are not changed; free the batch with xg_batch_free) and the
 * chosen B; the choice is cached on disk per (programs, instance counts).
 * The workspace must hold xg_batch_autotune_workspace_bytes bytes; the
 * returned batch needs xg_batch_workspace_bytes of its own.  Extension
 * beyond the paper. */
xg_status xg_batch_autotune(xg_program* const* progs, int32_t k, const xg_batch_args* args,
                            void* d_workspace, size_t workspace_bytes, void* stream,
                            xg_batch** out, int32_t* chosen_block);
/* Largest workspace any xg_batch_autotune candidate needs (n: k counts). */
xg_status xg_batch_autotune_workspace_bytes(xg_program* const* progs, int32_t k, const int64_t* n,
                                            size_t* bytes);
/* Compile every xg_batch_autotune candidate into the code cache (no device). */
xg_status xg_batch_autotune_precompile(xg_program* const* progs, int32_t k, const int64_t* n);

/* Thread-local message of the last error on this thread ("" if none). */
const char* xg_last_error(void);

/* Library version string. */
const char* xg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* XG_H */
