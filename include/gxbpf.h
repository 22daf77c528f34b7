/*
 * gxbpf — device-side eBPF runtime for AMD MI355X (gfx950).  Public C ABI.
 *
 * The runtime follows the paper's model of programs, hooks and maps (gpu_ext,
 * arXiv 2512.12615, sections 4.2–4.4 and 5.3): a control plane loads verified
 * policy bytecode and configures maps; the device runs the policy once per
 * hook event, one event per GPU lane, over batches of event records; policies
 * read and update shared maps (array, hash, ring buffer) and return an integer
 * decision per event.
 *
 * Conventions
 *   - Every call returns 0 (or a non-negative handle / count) on success and a
 *     negative Linux errno value on failure; nothing throws across the ABI.
 *   - Pointers named d_* are device pointers (e.g. torch tensor data_ptr());
 *     every other pointer is host memory.  The caller keeps ownership of all
 *     buffers it passes; the runtime copies what it needs to keep.
 *   - A gx_rt owns every map and program created through it; gx_close frees
 *     them.  One runtime drives one HIP device.  Calls on one runtime are not
 *     thread-safe; use one runtime per host thread, or serialise.
 *   - hipStream_t arguments are passed as void*; NULL is the default stream.
 */
#ifndef GXBPF_H
#define GXBPF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gx_rt gx_rt;

/* Map types (Linux numbering) and flags. */
enum {
  GX_MAP_HASH = 1,
  GX_MAP_ARRAY = 2,
  GX_MAP_RINGBUF = 27,
};
enum {
  /* Shared across streams within a run: lookups and commutative atomics
   * (ADD/OR/AND/XOR without fetch) only. */
  GX_F_SHARED = 1u,
  /* Written by the host only: lookups and loads only. */
  GX_F_READ_ONLY = 2u,
  /* With GX_F_READ_ONLY: the map lives in host memory (pinned, mapped into
   * the device's address space) instead of device memory: the cold tier of
   * section 4.4's hierarchical maps, for large host-written state that the
   * device reads rarely (each device read crosses the host link). */
  GX_F_HOST = 4u,
};

/* Hook types: select the event record layout and the stream key.
 *   GX_HOOK_MEM_ACCESS    24 B {u64 addr; u32 stream_id; u32 pad; u64 ts}
 *                         stream key = stream_id (modelled on the paper's
 *                         device memory-access hook, section 4.3.1)
 *   GX_HOOK_KERNEL_TIMING 16 B {u32 kernel_id; u32 pad; u64 latency_ns}
 *                         stream key = kernel_id (modelled on the paper's
 *                         device observability tools, Table 2)
 *   GX_HOOK_WAVE_MEM      warp-leader hook (section 4.4, "Warp-level
 *                         Execution Optimizations"): input records as
 *                         GX_HOOK_MEM_ACCESS, but the program runs once per
 *                         tile of 64 consecutive records (one wave) on the
 *                         tile's aggregate ctx {u64 lo = smallest addr;
 *                         u64 hi = largest addr; u32 n = records; u32
 *                         stream_id of the tile's first record}, and every
 *                         record of the tile gets its return code.  Its
 *                         maps must be shared, read-only or ring buffers.
 *   GX_HOOK_SIMT_MEM      SIMT-aware per-lane hook (section 4.4, "SIMT-aware
 *                         Verification"): input records as
 *                         GX_HOOK_MEM_ACCESS, one invocation per record,
 *                         whose ctx is the record (bytes 0..23, lane-
 *                         varying) followed by its tile's aggregate as for
 *                         GX_HOOK_WAVE_MEM (bytes 24..47, warp-uniform).
 *                         The verifier tracks uniformity from these fields
 *                         and rejects lane-varying branch conditions (loop
 *                         exits included), map keys, ring records and
 *                         flags, map-update addresses and fetching map
 *                         atomics; maps must be shared, read-only or ring
 *                         buffers.  Waves then never split, and a wave's
 *                         shared-map updates (one word) are combined into
 *                         one.
 *   GX_HOOK_SCHED         steal decision of the device block scheduler
 *                         (section 4.3.2, should_try_steal): run by
 *                         gx_run_sched only, once per decision of a
 *                         persistent worker, on 32 B {u32 worker; u32 done
 *                         (units run so far); u64 elapsed_ns (since the
 *                         worker started); u64 steal_ns (since it began
 *                         stealing); u32 stolen (units stolen so far); u32
 *                         left (units left in the victim's range)}; a
 *                         non-zero return code takes one more unit.  Maps
 *                         must be shared, read-only or ring buffers.
 * The record (or aggregate) is the program's read-only ctx (r1).  The
 * memory hooks (1, 3, 4) can also sit inside an application kernel
 * (gx_run_app_vadd). */
enum {
  GX_HOOK_MEM_ACCESS = 1,
  GX_HOOK_KERNEL_TIMING = 2,
  GX_HOOK_WAVE_MEM = 3,
  GX_HOOK_SIMT_MEM = 4,
  GX_HOOK_SCHED = 5,
};

/* Execution modes chosen by the verifier.  They follow from this runtime's
 * deterministic map contract, which replaces the relaxed, eventually
 * consistent maps of section 4.4 (each stream's events run in index order;
 * shared maps take commutative atomics only): a program that touches only
 * shared, read-only and ring maps is event-parallel; any other program
 * runs each stream's events in order. */
enum {
  GX_MODE_EVENT_PARALLEL = 0,
  GX_MODE_STREAM_SEQUENTIAL = 1,
};

typedef struct gx_prog_info {
  uint32_t mode;          /* GX_MODE_* */
  uint32_t hook;
  uint32_t n_insns;       /* bytecode slots */
  uint32_t stack_bytes;   /* stack frame the program uses (multiple of 8) */
  uint64_t max_insns;     /* longest path, loops counted by trip count */
  uint64_t max_calls;     /* helper calls per invocation, worst case */
  uint64_t max_ring_bytes;/* ring bytes per invocation, worst case */
} gx_prog_info;

typedef struct gx_stats {
  uint64_t launches;      /* kernel launches issued */
  uint64_t events;        /* events submitted */
  uint64_t ring_drops;    /* ringbuf_output calls that found no space */
  uint64_t hash_e2big;    /* hash inserts refused because the map was full */
  uint64_t vm_errors;     /* runaway-program aborts (should stay 0) */
  uint64_t bytes_drained; /* ring bytes copied to the host */
} gx_stats;

/* Open a runtime on HIP device ``hip_device``.  -ENODEV if it does not
 * exist, -ENOMEM on allocation failure. */
int gx_open(int hip_device, gx_rt** out);
/* Free every map and program of the runtime, then the runtime. */
void gx_close(gx_rt* rt);

/* Create a map (section 4.4, "Hierarchical Cross-layer Maps": device memory,
 * or host memory for GX_F_HOST; LDS shards are the kernels' own, and host
 * snapshots are gx_snapshot_*).  Returns a map fd >= 0.
 *   ARRAY:   key_size 4 (u32 index), value_size 1..4096, max_entries >= 1;
 *            values start zeroed.
 *   HASH:    key_size 1..64, value_size 1..4096, max_entries >= 1.
 *   RINGBUF: key_size = value_size = 0, max_entries = data bytes, a power of
 *            two >= 4096.
 * flags: GX_F_SHARED or GX_F_READ_ONLY (not both; not on a ring);
 * GX_F_HOST only together with GX_F_READ_ONLY, on arrays and hashes.
 * Errors: -EINVAL bad sizes or flags; -ENOMEM. */
int gx_create_map(gx_rt* rt, uint32_t type, uint32_t key_size, uint32_t value_size,
                  uint32_t max_entries, uint32_t flags);

/* Control-plane map access (the paper's user-space control plane, section
 * 4.2).  Synchronous with respect to the device: they wait for all work the
 * runtime has launched.  Same error codes as the eBPF helpers:
 *   update: flags 0 ANY / 1 NOEXIST / 2 EXIST; -EEXIST, -ENOENT, -E2BIG,
 *           -EINVAL; key/val are key_size / value_size host bytes.
 *   lookup: copies the value into val_out; -ENOENT if absent.
 *   delete: -ENOENT if absent; -EINVAL on arrays. */
int gx_map_update(gx_rt* rt, int map_fd, const void* key, const void* val, uint64_t flags);
int gx_map_lookup(gx_rt* rt, int map_fd, const void* key, void* val_out);
int gx_map_delete(gx_rt* rt, int map_fd, const void* key);
/* Snapshot of a map: writes up to ``cap`` (key, value) pairs (arrays: every
 * index in order; hashes: live entries in slot order) to keys / vals (either
 * may be NULL) and returns the number of entries the map holds. */
int64_t gx_map_dump(gx_rt* rt, int map_fd, void* keys, void* vals, uint64_t cap);
/* Zero an array map, or empty a hash map or a ring buffer. */
int gx_map_clear(gx_rt* rt, int map_fd);

/* Verify and load a program (section 4.4 "SIMT-aware Verification"; section
 * 5.3).  ``insns`` holds n_insns 8-byte eBPF slots; map references are
 * `lddw rX` with src=5 (imm = index into map_fds) or src=1 (imm = a map fd
 * listed in map_fds).  Returns a program fd >= 0.  On rejection returns
 * -EACCES and writes the reason to ``log`` (if log_size > 0).  -E2BIG if
 * n_insns > 4096, -EINVAL for a bad hook or map table. */
int gx_load_program(gx_rt* rt, const uint64_t* insns, uint32_t n_insns, uint32_t hook_type,
                    const int* map_fds, uint32_t n_maps, char* log, uint32_t log_size);
int gx_prog_info_get(gx_rt* rt, int prog_fd, gx_prog_info* out);

/* Verify without loading (no device needed).  ``map_shapes`` holds 5 u32 per
 * map: type, key_size, value_size, max_entries, flags; the program's map
 * table is the identity over them.  Returns 0 if accepted, -EACCES if
 * rejected (reason in log), and fills *info when accepted. */
int gx_verify(const uint64_t* insns, uint32_t n_insns, uint32_t hook_type, const uint32_t* map_shapes,
              uint32_t n_maps, char* log, uint32_t log_size, gx_prog_info* info);

/* Compile a loaded program to native gfx950 code (the paper lowers verified
 * bytecode through LLVM and inlines helpers and map accesses: sections 5.1, 5.3,
 * section 4.4 "Warp-level Execution Optimizations").  The micro-ops become
 * HIP source compiled with hipRTC; later gx_run_batch calls of this program
 * launch the compiled kernels (gx_run_batches keeps interpreting).  Results
 * are identical to the interpreter's.  Returns 0 (also if already
 * compiled), -EINVAL for a bad fd, -EIO if compilation or module loading
 * fails (compiler log in ``log``).  Takes seconds: call it at load time. */
int gx_jit_program(gx_rt* rt, int prog_fd, char* log, uint32_t log_size);

/* Autotuner: the launch shape of a program's runs (stream-sequential:
 * queues per wave and queue count; compiled event-parallel: block count) is
 * chosen by timing each candidate on a sample batch (the default shape
 * stays unless a candidate is at least 3 % faster; d_events, n_events
 * records of record_size bytes in device memory; d_rc receives return codes
 * and may be NULL) on ``stream``.  Map and ring contents are saved first
 * and restored before every trial and at the end, so the only lasting
 * effect is the choice, which later gx_run_batch / gx_run_batches calls of
 * the program use.  Synchronous.  Fills *out (may be NULL).  Returns 0,
 * -EINVAL for bad arguments, -ENOMEM. */
typedef struct gx_tune {
  uint32_t lanes;     /* stream-sequential: queues per wave */
  uint32_t qbits;     /* stream-sequential: log2 queue count */
  uint32_t blocks;    /* compiled event-parallel: blocks (0: sized per run) */
  uint32_t trials;    /* candidates timed */
  double best_ms;     /* time of the chosen shape on the sample */
  double default_ms;  /* time of the default shape on the sample */
} gx_tune;
int gx_autotune(gx_rt* rt, int prog_fd, const void* d_events, uint64_t n_events, uint32_t record_size, uint32_t* d_rc,
                void* stream, gx_tune* out);

/* Compile several loaded programs (at most 64, each once) into one module
 * whose persistent kernel serves the batched form: in later gx_run_batches
 * calls (and in the served form), the runs of all programs of a set in one
 * phase share one persistent launch, as the interpreter's runs do, instead
 * of one launch per run.  Instances of one program with same-shaped maps
 * share one copy of the code.  A program belongs to the set of its latest
 * call.
 * Plain gx_run_batch runs keep using gx_jit_program's form or the
 * interpreter.  Results are identical to the interpreter's.  Returns the set
 * id (>= 0), -EINVAL for a bad or repeated fd, -EIO if compilation fails (log
 * in ``log``).  Thread-safe against concurrent gx_jit_program /
 * gx_jit_program_set calls on other programs, not against gx_load_program. */
int gx_jit_program_set(gx_rt* rt, const int* prog_fds, uint32_t n, char* log, uint32_t log_size);

/* The HIP source gx_jit_program would compile for a program (no device
 * needed; map descriptors get stand-in addresses).  Same program and shape
 * arguments as gx_verify.  With bit 0 of ``compile`` set the source is also
 * compiled for gfx950; with bit 1 set it is the source of the instrumented
 * vector add's kernel (gx_run_app_vadd; event-parallel memory hooks only,
 * else -EINVAL) instead of the run kernels.  A GX_HOOK_SCHED program's
 * source holds the block scheduler's worker kernel (gx_run_sched).  Writes up to cap - 1 bytes of source (NUL-terminated) to
 * ``out`` (may be NULL) and returns the full length; -EACCES if the
 * verifier rejects (reason in out), -EIO if compilation fails (compiler log
 * in out). */
int64_t gx_jit_source(const uint64_t* insns, uint32_t n_insns, uint32_t hook_type, const uint32_t* map_shapes,
                      uint32_t n_maps, int compile, char* out, uint64_t cap);
/* The same for a program set (gx_jit_program_set): n_progs programs whose
 * slots are concatenated in ``insns`` (n_insns[i] each), hooks[i], and map
 * shapes concatenated in ``map_shapes`` (5 u32 per map, n_maps[i] maps). */
int64_t gx_jit_set_source(const uint64_t* insns, const uint32_t* n_insns, const uint32_t* hooks,
                          const uint32_t* map_shapes, const uint32_t* n_maps, uint32_t n_progs, int compile, char* out,
                          uint64_t cap);

/* Run a program over n_events records at d_events (device memory, record
 * size given by the hook; the hook's invocation of section 4.3.1, one per
 * event, here one GPU lane per event) asynchronously on ``stream``; writes the u32 return
 * code of event i to d_rc[i] if d_rc is not NULL.  Maps change in place.
 * The caller keeps d_events / d_rc alive until the stream reaches this point.
 * Errors: -EINVAL (bad fd, record_size mismatch), -ENOMEM. */
int gx_run_batch(gx_rt* rt, int prog_fd, const void* d_events, uint64_t n_events,
                 uint32_t record_size, uint32_t* d_rc, void* stream);

/* gx_run_batch for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * arguments, kernels and results, but nothing is allocated - no hipMalloc,
 * hipFree, events, streams or staging.  The run's workspace (the stream
 * partition of a stream-sequential program; a compiled event-parallel
 * program's cache spill, which flushes to the map directly when it does not
 * fit) lives in a fixed 16 MiB array per device, found at gx_open and held
 * until the process ends.  Every call on a device shares that array and
 * nothing in it carries over between calls, so calls on one device must not
 * overlap: issue them on one stream or order them.  No profile brackets are
 * recorded.  Errors: as gx_run_batch, and -E2BIG when a stream-sequential
 * run's workspace exceeds the array (about 480 k events with 4096 queues,
 * the default launch shape). */
int gx_run_batch_noalloc(gx_rt* rt, int prog_fd, const void* d_events, uint64_t n_events,
                         uint32_t record_size, uint32_t* d_rc, void* stream);

/* A hook inside an application kernel (section 5.3: trampolines at a
 * kernel's memory instructions; section 6.2.1's vector add with a stride
 * access pattern): the HIP kernel computes d_c[j] = d_a[j] + d_b[j] for j =
 * (i * stride) mod n over iterations i < n (device arrays of n doubles; j
 * visits every element once since gcd(stride, n) = 1), and at its load of
 * d_a[j] runs the event-parallel memory-hook program prog_fd on the access's
 * record {addr = 8 j (byte offset in d_a), stream_id = i / 64 (the 64-
 * iteration tile, one wave's), ts = i}: per lane for GX_HOOK_MEM_ACCESS and
 * GX_HOOK_SIMT_MEM (with the tile's aggregate), once per tile for
 * GX_HOOK_WAVE_MEM.  The results equal gx_run_batch over those records in
 * iteration order.  The return code d of iteration i goes to d_rc[i] if
 * d_rc is not NULL and, when non-zero, is a prefetch hint: the lane also
 * loads d_a[(j + d) mod n] ahead of its own loads (gfx950 has no data
 * prefetch instruction).  prog_fd < 0 runs the kernel without the hook.
 * Compiled programs run in a compiled copy of the kernel (built at the
 * first call), others in the interpreter.  Asynchronous on ``stream``.
 * Errors: -EINVAL (n = 0 or n > 2^32, stride >= n, gcd(stride, n) != 1,
 * a program of another hook or a stream-sequential one), -ENOMEM, -EIO. */
int gx_run_app_vadd(gx_rt* rt, int prog_fd, const double* d_a, const double* d_b, double* d_c, uint64_t n,
                    uint64_t stride, uint32_t* d_rc, void* stream);

/* Device block scheduler (section 4.3.2's work-stealing thread-block
 * scheduler with persistent workers; section 6.2.1's policies): ``workers``
 * persistent workers (one wave each) run n_units work units of d_cost[u]
 * iterations each (d_out[64 u + l] = 64 u + l after d_cost[u] steps of the
 * 64-bit MMIX linear congruential generator; d_out holds 64 n_units words).
 * Worker w owns units [w n_units / workers, (w + 1) n_units / workers) and
 * claims them in order; with a GX_HOOK_SCHED program, once its range is
 * empty the worker asks the program before each steal whether to take one
 * more unit from the first worker after it (cyclically) with units left,
 * and stops at the first "no" or when no unit is left anywhere.  prog_fd <
 * 0: static assignment (no stealing).  Every unit runs exactly once, so
 * d_out never depends on the policy.  Each decision's 32-byte context (the
 * GX_HOOK_SCHED record) goes to d_log[4 k .. 4 k + 3] and its return code
 * to d_log_rc[k], k < log_cap (decision k in the order they were made; each
 * worker's own decisions keep their order); *d_log_n (device, may be NULL)
 * receives the number of decisions, which may exceed log_cap.  Compiled
 * programs run in a compiled worker kernel (gx_jit_program), others in the
 * interpreter.  Asynchronous on ``stream``; the runtime zeroes its counters
 * on the stream.  Errors: -EINVAL (n_units or workers 0, workers > 65536,
 * log_cap > 0 without log arrays, a program of another hook), -ENOMEM. */
int gx_run_sched(gx_rt* rt, int prog_fd, const uint32_t* d_cost, uint32_t n_units, uint32_t workers,
                 uint64_t* d_out, uint64_t* d_log, uint32_t* d_log_rc, uint32_t log_cap, uint32_t* d_log_n,
                 void* stream);

/* Batched form: the work of n gx_run_batch calls in one persistent launch
 * (persistent workers claiming work units, as the paper's device scheduler
 * policies use them, section 5.3).  The results are those of the n calls
 * made in order. */
typedef struct gx_batch {
  int32_t prog_fd;
  uint32_t record_size;
  const void* d_events;
  uint64_t n_events;
  uint32_t* d_rc;
} gx_batch;
int gx_run_batches(gx_rt* rt, const gx_batch* descs, uint32_t n, void* stream);

/* Autotuner of the batched form (the persistent launch's waves per compute
 * unit, 2-32): times gx_run_batches over ``descs`` with each candidate, maps
 * saved and restored as gx_autotune does, and keeps the fastest (the default
 * unless a candidate is at least 3 % faster) for later batched launches of
 * this runtime.  *out: blocks = the chosen waves per CU, trials, best_ms,
 * default_ms.  Synchronous.  Errors as gx_run_batches, -ENOMEM. */
int gx_autotune_batches(gx_rt* rt, const gx_batch* descs, uint32_t n, void* stream, gx_tune* out);

/* A batch captured into a HIP graph (the batched form's launches, replayed
 * without host work).  gx_graph_create runs the batch once to size a
 * workspace of the graph's own (the maps it touches are saved first and put
 * back, so that run leaves no trace), then captures the same launches.
 * gx_graph_launch replays them on ``stream``: the same programs over the
 * same device buffers (events, return codes) as given to create, whose
 * contents the caller may change between launches; each replay has the
 * effect of one gx_run_batches call with those descriptors.  Launches of
 * one graph must be ordered (one stream, or synchronized), like batches
 * over the same maps.  Errors: -EINVAL, -E2BIG as gx_run_batches, -ENOMEM,
 * -EIO if capture or instantiation fails. */
typedef struct gx_graph gx_graph;
int gx_graph_create(gx_rt* rt, const gx_batch* descs, uint32_t n, gx_graph** out);
int gx_graph_launch(gx_graph* g, void* stream);
void gx_graph_destroy(gx_graph* g);

/* Copy committed ring records to host memory as {u32 len; u32 flags;
 * payload padded to 8} and release their space.  Returns the bytes written
 * (whole records only) and the record count in *n_records.  Waits for work
 * already launched on the runtime's streams that may still write the ring. */
int64_t gx_drain_ringbuf(gx_rt* rt, int ring_fd, void* host_buf, uint64_t buf_bytes,
                         uint64_t* n_records);

/* As gx_drain_ringbuf without the copy into caller memory: *view points at
 * the drained range in the runtime's pinned staging buffer for this ring
 * (*view_bytes bytes, valid until the next drain of this ring or
 * gx_destroy_map), which still holds the discard records (flags bit 0; len
 * bytes of padding) that close unused chunk space; readers skip them.
 * Returns the bytes of the kept records (headers included) and their
 * count in *n_records; releases the whole range.  When the previous drain
 * took its whole range, both figures come from counts the device keeps
 * (discard bytes and records written), without a host pass over the
 * records.  Errors as gx_drain_ringbuf. */
int64_t gx_drain_ringbuf_view(gx_rt* rt, int ring_fd, const void** view, uint64_t* view_bytes,
                              uint64_t* n_records);

/* The drain of gx_drain_ringbuf_view in two halves, so that the copy to
 * the host overlaps the caller's next launches (section 5.3's host side
 * draining the ring while the device keeps producing).  _start waits for
 * the runtime's launches, reads the ring's position and queues, on a copy
 * stream of the runtime, the copy of the committed range into the ring's
 * pinned staging buffer and then the move of the ring's tail past it; it
 * returns 0 without waiting for them.  Until _finish: launches of
 * gx_run_batch that may write this ring wait on the device for the copy
 * before their VM kernel (their partition kernels do not); the other
 * launching entry points and the autotuners wait for it on the host (a
 * server's own launches do not: rings of served programs are drained by
 * their callers after the requests complete); gx_drain_ringbuf,
 * gx_drain_ringbuf_view and a second _start on the ring return -EBUSY.
 * When the range needs a host pass (records some writer did not count, a
 * cut-back head) _start drains it synchronously instead.  _finish waits
 * for the copy and returns what gx_drain_ringbuf_view would have: *view
 * (valid until the next drain of this ring), *view_bytes, *n_records and
 * the kept bytes; -EINVAL without a started drain. */
int gx_drain_ringbuf_start(gx_rt* rt, int ring_fd);
int64_t gx_drain_ringbuf_finish(gx_rt* rt, int ring_fd, const void** view, uint64_t* view_bytes,
                                uint64_t* n_records);

/* Position of a ring: *head = bytes reserved since the ring was created
 * (records, their padding and discard records), *tail = bytes drained.
 * Both only grow; head - tail is the backlog a drain would read, and
 * head / capacity the number of times the writers went round the ring.
 * Waits for the runtime's launches like a drain; -EINVAL if ring_fd is not
 * a ring or an output pointer is null. */
int gx_ringbuf_pos(gx_rt* rt, int ring_fd, uint64_t* head, uint64_t* tail);

/* Host snapshots of device maps (section 4.4, "Hierarchical Cross-layer
 * Maps": GPU-resident state flushed asynchronously to host-visible
 * instances at kernel completion boundaries, so that host-side readers get
 * a coherent view without synchronising with the device).
 *
 * gx_snapshot_start: a daemon thread copies the n maps (arrays or hashes)
 * every interval_us microseconds into pinned host buffers.  Each copy is
 * issued on ``stream`` (the stream the maps' runs go to) between two runs
 * (never inside one), so a snapshot is the maps' state after some prefix
 * of the runs issued on that stream, identical for all n maps.  One daemon
 * per runtime: -EBUSY if one runs, -EINVAL for a bad fd or a ring, -ENOMEM.
 *
 * gx_snapshot_read: the latest snapshot of one map, without touching the
 * device (relaxed consistency: up to an interval plus the runs in flight
 * behind the exact state that gx_map_dump returns).  Same output as
 * gx_map_dump; *version (may be NULL) is the snapshot's sequence number,
 * 0 before the first.  -ENOENT if the map is not snapshotted.
 *
 * gx_snapshot_flush: take a snapshot now, after every run issued on the
 * daemon's stream so far, and wait for it (after it, gx_snapshot_read
 * equals gx_map_dump if nothing else ran).  -ENOENT if no daemon runs.
 *
 * gx_snapshot_stop: stop the daemon and free its buffers (also done by
 * gx_close). */
int gx_snapshot_start(gx_rt* rt, const int* map_fds, uint32_t n, uint64_t interval_us, void* stream);
int64_t gx_snapshot_read(gx_rt* rt, int map_fd, void* keys, void* vals, uint64_t cap, uint64_t* version);
int gx_snapshot_flush(gx_rt* rt);
void gx_snapshot_stop(gx_rt* rt);

/* Counters accumulated since gx_open (synchronises the device). */
int gx_stats_get(gx_rt* rt, gx_stats* out);

/* Measurement support.  While enabled, each gx_run_batch brackets its VM
 * kernel launch with HIP events on the caller's stream (the stable stream
 * partition of stream-sequential programs is outside the bracket).
 * gx_profile_read waits for those events, returns the summed VM-kernel time
 * in milliseconds and the number of bracketed launches since the last read,
 * and resets both. */
int gx_profile_enable(gx_rt* rt, int on);
int gx_profile_read(gx_rt* rt, double* vm_ms, uint64_t* vm_launches);

/* ---------------------------------------------------------------------------
 * Served form: continuous batching of tenant requests (multi-tenant policy
 * coordination, paper sections 3 and 6.3).  A request is (tenant, program,
 * host event batch).  Requests of one tenant run in submission order (a
 * tenant's programs own its maps): all of them go to one of ``streams`` HIP
 * streams (tenant mod streams).  Requests are admitted whenever device
 * memory for their buffers (events + return codes) fits in the budget; a
 * stream with fewer than four unfinished launches takes the head request of
 * each of its tenants as one batched launch, so a tenant's next request is
 * queued on the device before its previous one is done, requests gather
 * into larger launches while the device is busy, and launches on different
 * streams overlap.  GX_SERVE_PER_REQUEST
 * runs every request as its own plain launch, one request per tenant in
 * flight (the baseline the continuous mode is compared with).  The server drives the
 * runtime from its own host thread: while a server exists, make no other
 * calls on its runtime except map snapshots after gx_server_drain. */
typedef struct gx_server gx_server;
enum {
  GX_SERVE_CONTINUOUS = 0,
  GX_SERVE_PER_REQUEST = 1,
};
typedef struct gx_server_cfg {
  uint64_t hbm_budget_bytes; /* device bytes for in-flight request buffers */
  uint32_t streams;          /* launch streams (>= 1; per-request mode uses 1) */
  uint32_t mode;             /* GX_SERVE_* */
  uint32_t max_group;        /* most requests per launch (0: no limit) */
  uint32_t pad;
} gx_server_cfg;
typedef struct gx_completion {
  uint64_t req_id;
  int32_t tenant;
  int32_t status;        /* 0, or -errno of the launch */
  uint64_t n_events;
  const uint32_t* rc;    /* n_events return codes, valid until gx_server_release */
  double t_submit;       /* host monotonic seconds */
  double t_admit;
  double t_done;
  void* priv;
} gx_completion;

/* Create a server on ``rt``.  -EINVAL for a zero budget; -ENOMEM. */
int gx_server_create(gx_rt* rt, const gx_server_cfg* cfg, gx_server** out);
/* Queue a request; the events (n_events records of record_size bytes in host
 * memory) are copied before the call returns.  -E2BIG if the request alone
 * exceeds the budget, -EINVAL for a bad program or record size. */
int gx_server_submit(gx_server* srv, int32_t tenant, int prog_fd, const void* host_events, uint64_t n_events,
                     uint32_t record_size, uint64_t req_id);
/* As gx_server_submit, without the copy: the server reads ``host_events``
 * when it admits the request, so the caller keeps that memory valid and
 * unchanged until the request's completion has been returned by
 * gx_server_poll.  Pinned memory (hipHostMalloc) makes the transfer
 * asynchronous; pageable memory works but is staged by the HIP runtime. */
int gx_server_submit_borrowed(gx_server* srv, int32_t tenant, int prog_fd, const void* host_events,
                              uint64_t n_events, uint32_t record_size, uint64_t req_id);
/* Take up to ``max`` completions, waiting up to wait_ms for the first one.
 * Returns the number written. */
int gx_server_poll(gx_server* srv, gx_completion* out, uint32_t max, int wait_ms);
/* Return a completion's return-code buffer to the server. */
void gx_server_release(gx_server* srv, gx_completion* c);
/* Wait until every submitted request has completed (they remain to be
 * polled). */
int gx_server_drain(gx_server* srv);
/* Stop the server thread (after draining) and free its buffers. */
void gx_server_destroy(gx_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* GXBPF_H */
