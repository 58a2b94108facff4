// libatfd host side: argument validation, workspace layout, launch sequencing
// and HIP graph capture behind the C ABI of include/atfd.h.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "atfd_internal.hpp"
#include "adjoint.hpp"
#include "delays.hpp"
#include "host_common.hpp"

using namespace atfd;

std::string& atfd::thread_error() {
  thread_local std::string err;
  return err;
}

namespace {

constexpr int kNormBlocks = 1024;
static_assert(kNormBlocks <= kNormStaticBlocks, "the static norm scratch holds every workgroup's partials");

struct Layout {
  size_t field_bytes = 0, ring_bytes = 0, host_tab_bytes = 0;
  size_t off_u[2] = {0, 0}, off_f[2] = {0, 0}, off_ustar = 0, off_ring = 0, off_sring = 0;
  bool pe_major = false;   // fields stored PE after PE (the 32 x 32 path's problems)
  size_t off_counter = 0, off_partial = 0, off_result = 0, off_delays = 0, off_host = 0;
  size_t total = 0;
  int nslots = 0;
  int64_t pe_block = 0;
  int64_t face_off[6] = {0, 0, 0, 0, 0, 0};
  int64_t face_chunk[6] = {1, 1, 1, 1, 1, 1};
  int nfbuf = 0;
  bool star = false;
};

constexpr int64_t kDelayScratch = 1 << 16;   // bytes for at_get_delays chunks

struct Geometry {
  int ndim, s, T;
  int scheme, sd;     // AT family and face-strip depth (s, or 2 / 3 for the space-expanded schemes)
  int64_t n[3];
  int pe[3], b[3];
  int64_t npts;
  int npe;
  bool f64;
};

}  // namespace

struct at_ctx {
  at_problem prob;
  at_delay delay;
  Geometry g;
  Layout lay;
  StepParams sp;
  unsigned char* ws = nullptr;
  hipStream_t stream = nullptr;
  int device = 0;            // current device at at_create
  int sweep_parity = 0;      // z sweep direction of the next step (alternating variants)
  int64_t n = 0;
  bool state_set = false;
  std::string err;
  // graph replay
  int graph_chunk = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  hipStream_t cap_stream = nullptr;
  // the adjoint's recomputation stream (default priority)
  hipStream_t aux_stream = nullptr;
};

namespace {

at_status fail(at_ctx* ctx, at_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  thread_error() = buf;
  return st;
}

#define HIP_TRY(ctx, call)                                                              \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) return fail(ctx, AT_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

at_status validate(const at_problem* p, const at_delay* d, Geometry* g) {
  if (!p || !d) return fail(nullptr, AT_EINVAL, "null problem or delay");
  if (p->ndim < 1 || p->ndim > 3) return fail(nullptr, AT_EINVAL, "ndim must be 1..3");
  if (p->order != 2 && p->order != 4 && p->order != 6)
    return fail(nullptr, AT_EINVAL, "order must be 2, 4 or 6");
  if (p->equation != AT_ADVDIFF && p->equation != AT_BURGERS)
    return fail(nullptr, AT_EINVAL, "unknown equation");
  if (p->integrator < AT_EULER || p->integrator > AT_RK2)
    return fail(nullptr, AT_EINVAL, "unknown integrator");
  if (p->precision != AT_F64 && p->precision != AT_F32_F64B)
    return fail(nullptr, AT_EINVAL, "unknown precision");
  if (!(p->dt > 0) || !(p->length > 0)) return fail(nullptr, AT_EINVAL, "dt and length must be > 0");
  if (d->mode < AT_DELAY_RNG || d->mode > AT_SYNC) return fail(nullptr, AT_EINVAL, "unknown delay mode");
  g->ndim = p->ndim;
  g->s = p->order / 2;
  if (d->scheme < AT_SCHEME_TIME || d->scheme > AT_SCHEME_NONUNIFORM_212)
    return fail(nullptr, AT_EINVAL, "unknown AT scheme");
  g->scheme = d->scheme;
  if (d->scheme != AT_SCHEME_TIME) {
    if (p->order != 2) return fail(nullptr, AT_EINVAL, "the single-level AT schemes need order 2");
    if (d->T != 0 && d->T != 1) return fail(nullptr, AT_EINVAL, "the single-level AT schemes use one level (T = 1)");
  }
  if (d->scheme == AT_SCHEME_NONUNIFORM_212 && d->mode == AT_DELAY_HOST)
    return fail(nullptr, AT_EINVAL, "the non-uniform-delay scheme draws its per-point delays (no host table)");
  g->T = d->scheme != AT_SCHEME_TIME ? 1 : d->T == 0 ? p->order / 2 + 1 : d->T;
  g->sd = d->scheme == AT_SCHEME_SPACE_222 ? 3 : d->scheme != AT_SCHEME_TIME ? 2 : g->s;
  g->f64 = p->precision == AT_F64;
  if (d->mode != AT_SYNC) {
    if (d->L < 1 || d->L > kMaxL) return fail(nullptr, AT_EINVAL, "L must be 1..%d", kMaxL);
    if (g->T < 1 || g->T > kMaxT) return fail(nullptr, AT_EINVAL, "T must be 1..%d", kMaxT);
  }
  g->npts = 1;
  g->npe = 1;
  for (int a = 0; a < 3; ++a) {
    g->n[a] = p->n[a];
    g->pe[a] = p->pe[a];
    if (a >= p->ndim) {
      if (p->n[a] != 1 || p->pe[a] != 1)
        return fail(nullptr, AT_EINVAL, "unused axis %d must have n = 1 and pe = 1", a);
    }
    if (p->n[a] < 1 || p->pe[a] < 1 || p->n[a] % p->pe[a])
      return fail(nullptr, AT_EINVAL, "axis %d: n must be a positive multiple of pe", a);
    if (p->n[a] > (int64_t(1) << 30)) return fail(nullptr, AT_EINVAL, "axis %d too long", a);
    g->b[a] = static_cast<int>(p->n[a] / p->pe[a]);
    if (a < p->ndim && g->b[a] < 2 * g->s)
      return fail(nullptr, AT_EINVAL, "axis %d: PE edge %d < 2s = %d", a, g->b[a], 2 * g->s);
    if (a < p->ndim && g->b[a] < g->sd)
      return fail(nullptr, AT_EINVAL, "axis %d: PE edge %d below the strip depth %d", a, g->b[a], g->sd);
    g->npts *= p->n[a];
    g->npe *= p->pe[a];
  }
  if (static_cast<int64_t>(g->b[0]) * g->b[1] > 64 * 64)
    return fail(nullptr, AT_EINVAL, "PE x*y extent above 4096 points");
  if (d->mode == AT_DELAY_HOST) {
    if (!d->host_delays || d->host_nsteps < 1)
      return fail(nullptr, AT_EINVAL, "AT_DELAY_HOST needs a delay table");
    const int64_t cnt = d->host_nsteps * g->npe * 2 * g->ndim;
    for (int64_t i = 0; i < cnt; ++i)
      if (d->host_delays[i] < 0 || d->host_delays[i] >= d->L)
        return fail(nullptr, AT_EINVAL, "host delay %d at entry %lld outside [0, L-1]",
                    int(d->host_delays[i]), (long long)i);
  }
  if (d->weights) {
    for (int j = 0; j < d->L; ++j) (void)d->weights[j];
  }
  return AT_OK;
}

Layout make_layout(const at_problem* p, const at_delay* d, const Geometry& g) {
  Layout l;
  const size_t w = g.f64 ? 8 : 4;
  l.field_bytes = static_cast<size_t>(g.npts) * w;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  // Every delay mode except the synchronous arm reads neighbours only through
  // the ring, and each sweep reads a point's own level-n values before it
  // writes them: the solution is updated in place (one buffer; a smaller
  // working set stays in the Infinity Cache). The synchronous arm reads the
  // neighbours' level-n values directly and keeps two buffers.
  l.off_u[0] = take(l.field_bytes);
  // Two buffers as well for a 3-D problem that only the generic sweep can
  // take (no 32 x 32 cross-section, or the non-uniform-delay scheme), with
  // fewer PEs than four workgroups per compute unit, and whose new level is
  // written over u^n (not RK2): that sweep then splits a PE's planes over
  // several workgroups, which read their neighbours' planes.
  const bool generic3d = g.ndim == 3 && g.npe < 4 * 256 &&
                         (g.b[0] != 32 || g.b[1] != 32 || g.scheme == AT_SCHEME_NONUNIFORM_212);
  const bool two = d->mode == AT_SYNC || (generic3d && p->integrator != AT_RK2);
  l.off_u[1] = two ? take(l.field_bytes) : l.off_u[0];
  l.pe_major = fast3d_shape(g.ndim, g.b[0], g.b[1], g.scheme, d->mode, g.T, g.s,
                            static_cast<int64_t>(l.field_bytes));
  l.nfbuf = p->integrator == AT_AB2 ? 1 : p->integrator == AT_AB3 ? 2 : 0;
  for (int i = 0; i < l.nfbuf; ++i) l.off_f[i] = take(l.field_bytes);
  l.star = p->integrator == AT_RK2;
  if (l.star) l.off_ustar = take(l.field_bytes);
  // face strips: faces 2a, 2a+1 of a PE hold sd * (product of the other
  // edges) values (sd = s, or the 2 or 3 buffer points of the
  // space-expanded stencils), as planes of face_chunk values (x, y faces:
  // one plane per z-plane; z faces: one per depth); a slot stores every
  // face's planes of all PEs side by side (ring_index)
  const int s = g.sd;
  int64_t fo = 0, pe_block = 0;
  for (int a = 0; a < 3; ++a) {
    int64_t area = 1;
    for (int c = 0; c < 3; ++c)
      if (c != a) area *= g.b[c];
    const int64_t sz = a < g.ndim ? s * area : 0;
    const int64_t chunk = a == 2 ? static_cast<int64_t>(g.b[0]) * g.b[1] : static_cast<int64_t>(s) * g.b[1 - a];
    for (int side = 0; side < 2; ++side) {
      l.face_off[2 * a + side] = fo;
      l.face_chunk[2 * a + side] = chunk > 0 ? chunk : 1;
      fo += sz * g.npe;
      pe_block += sz;
    }
  }
  l.pe_block = pe_block;
  if (d->mode != AT_SYNC) {
    l.nslots = d->L + g.T;
    l.ring_bytes = static_cast<size_t>(l.nslots) * g.npe * l.pe_block * w;
    l.off_ring = take(l.ring_bytes);
    if (l.star) l.off_sring = take(l.ring_bytes);
  }
  l.off_counter = take(kCounterWords * sizeof(int64_t));
  l.off_partial = take(static_cast<size_t>(kNormBlocks) * 8 * sizeof(double));
  l.off_result = take(16 * sizeof(double));
  l.off_delays = take(kDelayScratch);
  if (d->mode == AT_DELAY_HOST) {
    l.host_tab_bytes = static_cast<size_t>(d->host_nsteps) * g.npe * 2 * g.ndim;
    l.off_host = take(l.host_tab_bytes);
  }
  l.total = off;
  return l;
}

// The library's schedule variant: the 32 x 32 path's default, or variant 1
// (one plane in flight) where the default's planes in flight do not divide
// the PE depth.
int default_variant(const StepParams& p, bool f64) {
  StepParams t = p;
  t.depth = fast3d_default_depth(f64);
  if (p.pe_major && !fast3d_applies(t, f64)) return 1;
  return t.depth;
}

void fill_params(at_ctx* c) {
  StepParams& p = c->sp;
  std::memset(&p, 0, sizeof(p));
  const Geometry& g = c->g;
  p.nx = int(g.n[0]); p.ny = int(g.n[1]); p.nz = int(g.n[2]);
  p.bx = g.b[0]; p.by = g.b[1]; p.bz = g.b[2];
  p.px = g.pe[0]; p.py = g.pe[1]; p.pz = g.pe[2];
  p.ndim = g.ndim;
  p.npe = g.npe;
  p.s = g.s;
  p.scheme = g.scheme;
  p.sd = g.sd;
  for (int a = 0; a < 3; ++a) {
    double t1[2 * kMaxS + 1] = {0}, t2[2 * kMaxS + 1] = {0};
    cd_taps(1, c->prob.order, t1);
    cd_taps(2, c->prob.order, t2);
    const double dx = c->prob.length / double(g.n[a]);
    p.vel[a] = a < g.ndim ? c->prob.c[a] : 0.0;
    for (int o = 0; o <= 2 * g.s; ++o) {
      p.c1[a][o] = t1[o] / dx;
      p.c2[a][o] = t2[o] / (dx * dx);
      p.d2a[a][o] = c->prob.alpha * p.c2[a][o];
      p.kad[a][o] = p.d2a[a][o] - p.vel[a] * p.c1[a][o];
      p.c1f[a][o] = static_cast<float>(p.c1[a][o]);
      p.d2af[a][o] = static_cast<float>(p.d2a[a][o]);
      p.kadf[a][o] = static_cast<float>(p.kad[a][o]);
    }
    double l1[2 * kMaxS + 1] = {0}, l2[2 * kMaxS + 1] = {0};
    if (g.scheme != AT_SCHEME_TIME) {
      space_taps(1, g.scheme, l1);
      space_taps(2, g.scheme, l2);
    }
    for (int o = 0; o <= 2 * kMaxS; ++o) {
      p.sl1[a][o] = l1[o] / dx;
      p.sl2[a][o] = l2[o] / (dx * dx);
    }
    if (g.scheme == AT_SCHEME_NONUNIFORM_212) {
      // the sweep derives this scheme's taps from the step's delays; the
      // tables carry only the axis scales, in their centre entry
      p.sl1[a][kMaxS] = 1.0 / dx;
      p.sl2[a][kMaxS] = 1.0 / (dx * dx);
    }
  }
  p.alpha = c->prob.alpha;
  p.dt = c->prob.dt;
  p.equation = c->prob.equation;
  p.integrator = c->prob.integrator;
  p.stage = kStageSingle;
  p.mode = c->delay.mode;
  p.L = c->delay.mode == AT_SYNC ? 1 : c->delay.L;
  p.T = g.T;
  p.key = c->delay.seed;
  make_thresholds(p.L, c->delay.weights, p.thr);
  unsigned char* ws = c->ws;
  const Layout& l = c->lay;
  p.host_delays = c->delay.mode == AT_DELAY_HOST ? reinterpret_cast<const int8_t*>(ws + l.off_host) : nullptr;
  p.ubuf[0] = ws + l.off_u[0];
  p.ubuf[1] = ws + l.off_u[1];
  p.fbuf[0] = l.nfbuf > 0 ? ws + l.off_f[0] : nullptr;
  p.fbuf[1] = l.nfbuf > 1 ? ws + l.off_f[1] : nullptr;
  p.ustar = l.star ? ws + l.off_ustar : nullptr;
  p.ring = l.nslots ? ws + l.off_ring : nullptr;
  p.sring = (l.nslots && l.star) ? ws + l.off_sring : nullptr;
  p.nslots = l.nslots;
  p.pe_block = l.pe_block;
  for (int f = 0; f < 6; ++f) {
    p.face_off[f] = l.face_off[f];
    p.face_chunk[f] = l.face_chunk[f];
  }
  p.counter = reinterpret_cast<int64_t*>(ws + l.off_counter);
  p.advance = 1;
  p.pe_major = l.pe_major ? 1 : 0;
  p.depth = default_variant(p, g.f64);
}

// Queue the kernels of one time step on `st`, with the context's parameters
// or with `p` (the same problem, other solution buffers).
at_status enqueue_step_p(at_ctx* c, StepParams p, hipStream_t st) {
  // alternating schedule variants: every launch sweeps z the other way from
  // the one before it (the direction is a schedule choice only)
  const bool alt = (p.depth & 16) != 0;
  if (c->prob.integrator == AT_RK2) {
    p.stage = kStageRk1;
    p.advance = 0;
    p.sweep_down = 0;
    HIP_TRY(c, launch_step(p, c->g.f64, c->g.s, st));
    p.stage = kStageRk2;
    p.advance = 1;
    p.sweep_down = alt ? 1 : 0;
    HIP_TRY(c, launch_step(p, c->g.f64, c->g.s, st));
  } else {
    p.sweep_down = alt ? c->sweep_parity : 0;
    c->sweep_parity ^= 1;
    HIP_TRY(c, launch_step(p, c->g.f64, c->g.s, st));
  }
  return AT_OK;
}

at_status enqueue_step(at_ctx* c, hipStream_t st) { return enqueue_step_p(c, c->sp, st); }

// Teardown calls below: a failure to release leaves nothing to recover, so
// their status is deliberately discarded.
void drop_graph(at_ctx* c) {
  if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->graph_exec = nullptr;
  c->graph = nullptr;
}

}  // namespace

extern "C" {

const char* at_version(void) { return "atfd 0.1 (gfx950)"; }

at_status at_workspace_size(const at_problem* prob, const at_delay* delay, size_t* bytes) {
  Geometry g;
  at_status st = validate(prob, delay, &g);
  if (st != AT_OK) return st;
  if (!bytes) return fail(nullptr, AT_EINVAL, "null bytes");
  *bytes = make_layout(prob, delay, g).total;
  return AT_OK;
}

at_status at_create(const at_problem* prob, const at_delay* delay, void* ws_dev, size_t ws_bytes,
                    void* hip_stream, at_ctx** out) {
  if (!out) return fail(nullptr, AT_EINVAL, "null out");
  *out = nullptr;
  Geometry g;
  at_status st = validate(prob, delay, &g);
  if (st != AT_OK) return st;
  Layout l = make_layout(prob, delay, g);
  if (!ws_dev) return fail(nullptr, AT_EINVAL, "null workspace");
  if (reinterpret_cast<uintptr_t>(ws_dev) % kAlign)
    return fail(nullptr, AT_EINVAL, "workspace must be %zu-byte aligned", kAlign);
  if (ws_bytes < l.total)
    return fail(nullptr, AT_ENOMEM, "workspace %zu bytes < %zu needed", ws_bytes, l.total);
  at_ctx* c = new (std::nothrow) at_ctx();
  if (!c) return fail(nullptr, AT_ENOMEM, "host allocation failed");
  c->prob = *prob;
  c->delay = *delay;
  c->delay.weights = nullptr;
  c->delay.host_delays = nullptr;
  c->g = g;
  c->lay = l;
  c->ws = static_cast<unsigned char*>(ws_dev);
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
  // thresholds are derived from the caller's weights now; keep a private copy
  {
    at_delay tmp = *delay;
    c->delay = tmp;
    fill_params(c);          // uses delay.weights for the thresholds
    c->delay.weights = nullptr;
    c->delay.host_delays = nullptr;
  }
  const size_t lds = step_lds_bytes(c->sp, g.f64, g.s);
  if (lds > kLdsLimit) {
    delete c;
    return fail(nullptr, AT_EINVAL, "PE tile needs %zu B of LDS (> %zu)", lds, kLdsLimit);
  }
  if (delay->mode == AT_DELAY_HOST) {
    hipError_t e = hipMemcpyAsync(c->ws + l.off_host, delay->host_delays, l.host_tab_bytes,
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
      delete c;
      return fail(nullptr, AT_EHIP, "copy of host delays: %s", hipGetErrorString(e));
    }
  }
  hipError_t e = launch_set_counter(c->sp.counter, 0, c->stream);
  if (e != hipSuccess) {
    delete c;
    return fail(nullptr, AT_EHIP, "counter init: %s", hipGetErrorString(e));
  }
  *out = c;
  return AT_OK;
}

at_status at_set_state(at_ctx* c, const void* u0_dev) {
  if (!c || !u0_dev) return fail(c, AT_EINVAL, "null argument");
  HIP_TRY(c, launch_field_copy(c->sp, c->g.f64, u0_dev, c->sp.ubuf[0], true, c->stream));
  HIP_TRY(c, launch_set_counter(c->sp.counter, 0, c->stream));
  if (c->delay.mode != AT_SYNC) HIP_TRY(c, launch_publish_all(c->sp, c->g.f64, c->g.sd, c->stream));
  c->n = 0;
  c->state_set = true;
  return AT_OK;
}

at_status at_set_graph(at_ctx* c, int32_t chunk) {
  if (!c || chunk < 0) return fail(c, AT_EINVAL, "bad graph chunk");
  if (chunk != c->graph_chunk) drop_graph(c);
  c->graph_chunk = chunk;
  return AT_OK;
}

at_status at_step(at_ctx* c, int64_t nsteps) {
  if (!c || nsteps < 0) return fail(c, AT_EINVAL, "bad arguments");
  if (!c->state_set) return fail(c, AT_ESTATE, "at_step before at_set_state");
  if (c->delay.mode == AT_DELAY_HOST && c->n + nsteps > c->delay.host_nsteps)
    return fail(c, AT_EINVAL, "host delay table covers %lld steps", (long long)c->delay.host_nsteps);
  int64_t done = 0;
  if (c->graph_chunk > 0 && nsteps >= c->graph_chunk) {
    if (!c->graph_exec) {
      if (!c->cap_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
      HIP_TRY(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
      at_status st = AT_OK;
      for (int i = 0; i < c->graph_chunk && st == AT_OK; ++i) st = enqueue_step(c, c->cap_stream);
      hipGraph_t gr = nullptr;
      hipError_t e = hipStreamEndCapture(c->cap_stream, &gr);
      if (st != AT_OK) {
        if (gr) (void)hipGraphDestroy(gr);
        return st;
      }
      if (e != hipSuccess) return fail(c, AT_EHIP, "graph capture: %s", hipGetErrorString(e));
      c->graph = gr;
      HIP_TRY(c, hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
    }
    while (nsteps - done >= c->graph_chunk) {
      HIP_TRY(c, hipGraphLaunch(c->graph_exec, c->stream));
      done += c->graph_chunk;
    }
  }
  for (; done < nsteps; ++done) {
    at_status st = enqueue_step(c, c->stream);
    if (st != AT_OK) return st;
  }
  c->n += nsteps;
  return AT_OK;
}

at_status at_set_tuning(at_ctx* c, int32_t depth) {
  if (!c) return fail(nullptr, AT_EINVAL, "null context");
  if (depth == 0) depth = default_variant(c->sp, c->g.f64);
  if (!fast3d_valid_variant(depth) && !chunk_variant(depth))
    return fail(c, AT_EINVAL, "schedule variant must be 1, 2, 4, 9, 10, 12, 17, 18, 20, 33, 34, 36, 40 or 48");
  if (c->sp.pe_major) {
    StepParams trial = c->sp;
    trial.depth = depth;
    if (!fast3d_applies(trial, c->g.f64))
      return fail(c, AT_EINVAL, "schedule variant %d does not apply to this problem (32 x 32 path: the planes in "
                  "flight must divide the PE depth %d; the space-expanded schemes take 1 and 2)", depth, c->g.b[2]);
  }
  if (depth != c->sp.depth) drop_graph(c);
  c->sp.depth = depth;
  return AT_OK;
}

at_status at_get_tuning(const at_ctx* c, int32_t* depth) {
  if (!c || !depth) return fail(nullptr, AT_EINVAL, "null argument");
  *depth = c->sp.depth;
  return AT_OK;
}

at_status at_autotune(at_ctx* c, void* scratch_dev, size_t scratch_bytes, int32_t nsteps,
                      int32_t* best_depth, double* ms_out) {
  if (!c || !scratch_dev || nsteps < 1) return fail(c, AT_EINVAL, "bad arguments");
  if (!c->state_set) return fail(c, AT_ESTATE, "autotune before at_set_state");
  size_t need = 0;
  at_checkpoint_size(c, &need);
  if (scratch_bytes < need) return fail(c, AT_ENOMEM, "scratch %zu < %zu bytes", scratch_bytes, need);
  if (c->delay.mode == AT_DELAY_HOST && c->n + nsteps > c->delay.host_nsteps)
    return fail(c, AT_EINVAL, "host delay table too short for autotuning");
  at_status st = at_save(c, scratch_dev);
  if (st != AT_OK) return st;
  const int cand[AT_TUNE_CANDIDATES] = {1, 2, 4, 9, 10, 12, 17, 18, 20, 33, 34, 36, 40, 48};
  // the z-chunk variants are timed only for problems the 32 x 32 path does
  // not take by default and whose planes the generic sweep may split
  const bool chunks_apply = !c->sp.pe_major && sweep_can_chunk(c->sp);
  const int keep = c->sp.depth, keep_chunk = c->graph_chunk;
  double best_ms = 1e300;
  int best = keep;
  hipEvent_t e0, e1;
  HIP_TRY(c, hipEventCreate(&e0));
  HIP_TRY(c, hipEventCreate(&e1));
  c->graph_chunk = 0;
  for (int i = 0; i < AT_TUNE_CANDIDATES; ++i) {
    double ms = -1.0;
    StepParams trial = c->sp;
    trial.depth = cand[i];
    if (chunk_variant(cand[i]) ? chunks_apply : fast3d_applies(trial, c->g.f64)) {
      c->sp.depth = cand[i];
      st = at_load(c, scratch_dev);
      if (st == AT_OK) st = enqueue_step(c, c->stream);          // warm-up
      if (st == AT_OK && hipEventRecord(e0, c->stream) != hipSuccess) st = AT_EHIP;
      for (int k = 0; k < nsteps && st == AT_OK; ++k) st = enqueue_step(c, c->stream);
      if (st == AT_OK && hipEventRecord(e1, c->stream) != hipSuccess) st = AT_EHIP;
      if (st == AT_OK && hipEventSynchronize(e1) != hipSuccess) st = AT_EHIP;
      float t = 0.f;
      if (st == AT_OK && hipEventElapsedTime(&t, e0, e1) == hipSuccess) ms = t / nsteps;
      if (st != AT_OK) break;
      if (ms >= 0 && ms < best_ms) {
        best_ms = ms;
        best = cand[i];
      }
    }
    if (ms_out) ms_out[i] = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->graph_chunk = keep_chunk;
  c->sp.depth = keep;
  at_status st2 = at_load(c, scratch_dev);
  if (st != AT_OK) return st;
  if (st2 != AT_OK) return st2;
  if (best != keep) drop_graph(c);
  c->sp.depth = best;
  if (best_depth) *best_depth = best;
  return AT_OK;
}

at_status at_get_state(at_ctx* c, void* u_dev) {
  if (!c || !u_dev) return fail(c, AT_EINVAL, "null argument");
  if (!c->state_set) return fail(c, AT_ESTATE, "no state");
  HIP_TRY(c, launch_field_copy(c->sp, c->g.f64, c->sp.ubuf[c->n & 1], u_dev, false, c->stream));
  return AT_OK;
}

at_status at_get_step(const at_ctx* c, int64_t* n) {
  if (!c || !n) return fail(nullptr, AT_EINVAL, "null argument");
  *n = c->n;
  return AT_OK;
}

at_status at_get_delays(at_ctx* c, int64_t n0, int64_t count, int8_t* host_out) {
  if (!c || !host_out || n0 < 0 || count < 0) return fail(c, AT_EINVAL, "bad arguments");
  if (c->delay.mode == AT_DELAY_HOST && n0 + count > c->delay.host_nsteps)
    return fail(c, AT_EINVAL, "beyond the host delay table");
  const int64_t per = static_cast<int64_t>(c->g.npe) * 2 * c->g.ndim;
  if (per > kDelayScratch) return fail(c, AT_EINVAL, "too many faces for one step of scratch");
  const int64_t chunk = kDelayScratch / per;
  int8_t* scratch = reinterpret_cast<int8_t*>(c->ws + c->lay.off_delays);
  for (int64_t s = 0; s < count; s += chunk) {
    const int64_t m = count - s < chunk ? count - s : chunk;
    HIP_TRY(c, launch_delays(c->sp, n0 + s, m, scratch, c->stream));
    HIP_TRY(c, hipMemcpyAsync(host_out + s * per, scratch, m * per, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  return AT_OK;
}

at_status at_get_point_delays(at_ctx* c, int64_t n0, int64_t count, int8_t* host_out) {
  if (!c || !host_out || n0 < 0 || count < 0) return fail(c, AT_EINVAL, "bad arguments");
  if (c->g.scheme != AT_SCHEME_NONUNIFORM_212)
    return fail(c, AT_EINVAL, "only the non-uniform-delay scheme has per-point delays");
  const int64_t per = static_cast<int64_t>(c->g.npe) * 2 * c->g.ndim;
  if (per > kDelayScratch) return fail(c, AT_EINVAL, "too many faces for one step of scratch");
  const int64_t chunk = kDelayScratch / per;
  int8_t* scratch = reinterpret_cast<int8_t*>(c->ws + c->lay.off_delays);
  for (int64_t s = 0; s < count; s += chunk) {
    const int64_t m = count - s < chunk ? count - s : chunk;
    HIP_TRY(c, launch_point_delays(c->sp, n0 + s, m, scratch, c->stream));
    HIP_TRY(c, hipMemcpyAsync(host_out + s * per, scratch, m * per, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  return AT_OK;
}

namespace {

// Validation and parameters shared by at_norms and at_norms_noalloc.
at_status norm_params(at_ctx* c, int32_t nmodes, const int32_t* kappa, const double* amp, const double* phase,
                      const double* ref_dev, double* out, NormParams* p, int* blocks) {
  if (!c || !out) return fail(c, AT_EINVAL, "null argument");
  if (!c->state_set) return fail(c, AT_ESTATE, "no state");
  if (nmodes < 0 || nmodes > kMaxModes) return fail(c, AT_EINVAL, "nmodes must be 0..%d", kMaxModes);
  if (nmodes == 0 && !ref_dev) return fail(c, AT_EINVAL, "need modes or a reference field");
  if (nmodes > 0 && (!kappa || !amp || !phase)) return fail(c, AT_EINVAL, "null mode arrays");
  std::memset(p, 0, sizeof(*p));
  p->nx = int(c->g.n[0]); p->ny = int(c->g.n[1]); p->nz = int(c->g.n[2]);
  p->bx = c->g.b[0]; p->by = c->g.b[1]; p->bz = c->g.b[2];
  p->ndim = c->g.ndim;
  p->s = c->g.s;
  p->length = c->prob.length;
  p->alpha = c->prob.alpha;
  p->dt = c->prob.dt;
  for (int a = 0; a < 3; ++a) p->vel[a] = a < c->g.ndim ? c->prob.c[a] : 0.0;
  p->nmodes = nmodes;
  for (int m = 0; m < nmodes; ++m) {
    for (int a = 0; a < 3; ++a) p->kap[m][a] = kappa[3 * m + a];
    p->amp[m] = amp[m];
    p->phase[m] = phase[m];
  }
  p->u = c->sp.ubuf[c->n & 1];
  p->pe_major = c->sp.pe_major;
  p->px = c->g.pe[0];
  p->py = c->g.pe[1];
  p->ref = ref_dev;
  p->counter = c->sp.counter;
  int nb = static_cast<int>((c->g.npts + 255) / 256);
  if (nb > kNormBlocks) nb = kNormBlocks;
  *blocks = nb;
  return AT_OK;
}

at_status norm_result(at_ctx* c, const double* res, double* out) {
  double host[10];
  HIP_TRY(c, hipMemcpyAsync(host, res, sizeof(host), hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int j = 0; j < 9; ++j) out[j] = host[j];
  if (host[9] > 0 || !std::isfinite(host[1]))
    return fail(c, AT_EUNSTABLE, "%.0f non-finite values in the field at step %lld", host[9],
                (long long)c->n);
  return AT_OK;
}

}  // namespace

at_status at_norms(at_ctx* c, int32_t nmodes, const int32_t* kappa, const double* amp,
                   const double* phase, const double* ref_dev, double* out) {
  NormParams p;
  int blocks = 0;
  at_status st = norm_params(c, nmodes, kappa, amp, phase, ref_dev, out, &p, &blocks);
  if (st != AT_OK) return st;
  p.partial = reinterpret_cast<double*>(c->ws + c->lay.off_partial);
  double* res = reinterpret_cast<double*>(c->ws + c->lay.off_result);
  HIP_TRY(c, launch_norms(p, c->g.f64, blocks, res, c->stream));
  return norm_result(c, res, out);
}

at_status at_norms_noalloc(at_ctx* c, int32_t nmodes, const int32_t* kappa, const double* amp,
                           const double* phase, const double* ref_dev, double* out) {
  NormParams p;
  int blocks = 0;
  at_status st = norm_params(c, nmodes, kappa, amp, phase, ref_dev, out, &p, &blocks);
  if (st != AT_OK) return st;
  if (blocks > kNormStaticBlocks)
    return fail(c, AT_EINVAL, "%d norm workgroups exceed the static scratch (%d)", blocks, kNormStaticBlocks);
  int dev = -1;
  HIP_TRY(c, hipGetDevice(&dev));
  if (dev != c->device)
    return fail(c, AT_EINVAL, "current device %d is not the context's device %d", dev, c->device);
  double* scr = nullptr;
  HIP_TRY(c, norms_static_scratch(dev, &scr));
  p.partial = scr;                                          // kNormStaticBlocks x 8 partials
  double* res = scr + static_cast<size_t>(kNormStaticBlocks) * 8;   // 16 doubles
  HIP_TRY(c, launch_norms(p, c->g.f64, blocks, res, c->stream));
  return norm_result(c, res, out);
}

at_status at_checkpoint_size(const at_ctx* c, size_t* bytes) {
  if (!c || !bytes) return fail(nullptr, AT_EINVAL, "null argument");
  const Layout& l = c->lay;
  *bytes = align_up(l.field_bytes) * (1 + l.nfbuf + (l.star ? 1 : 0)) +
           align_up(l.ring_bytes) * (l.star ? 2 : 1) + kAlign;
  return AT_OK;
}

namespace {
at_status ckpt_copy(at_ctx* c, unsigned char* dst_base, const unsigned char* src_base, bool save,
                    hipStream_t st) {
  const Layout& l = c->lay;
  size_t off = 0;
  auto cp = [&](size_t ws_off, size_t bytes) -> hipError_t {
    unsigned char* wsp = c->ws + ws_off;
    hipError_t e = save ? hipMemcpyAsync(dst_base + off, wsp, bytes, hipMemcpyDeviceToDevice, st)
                        : hipMemcpyAsync(wsp, src_base + off, bytes, hipMemcpyDeviceToDevice, st);
    off += align_up(bytes);
    return e;
  };
  // the current solution is stored as slot 0 of the checkpoint
  HIP_TRY(c, cp(l.off_u[c->n & 1], l.field_bytes));
  for (int i = 0; i < l.nfbuf; ++i) HIP_TRY(c, cp(l.off_f[i], l.field_bytes));
  if (l.star) HIP_TRY(c, cp(l.off_ustar, l.field_bytes));
  if (l.ring_bytes) HIP_TRY(c, cp(l.off_ring, l.ring_bytes));
  if (l.ring_bytes && l.star) HIP_TRY(c, cp(l.off_sring, l.ring_bytes));
  HIP_TRY(c, cp(l.off_counter, 2 * sizeof(int64_t)));
  return AT_OK;
}
}  // namespace

at_status at_save(at_ctx* c, void* ckpt_dev) {
  if (!c || !ckpt_dev) return fail(c, AT_EINVAL, "null argument");
  if (!c->state_set) return fail(c, AT_ESTATE, "no state");
  return ckpt_copy(c, static_cast<unsigned char*>(ckpt_dev), nullptr, true, c->stream);
}

at_status at_load(at_ctx* c, const void* ckpt_dev) {
  if (!c || !ckpt_dev) return fail(c, AT_EINVAL, "null argument");
  // the step number travels in the checkpoint's counter; read it back
  const Layout& l = c->lay;
  size_t coff = align_up(l.field_bytes) * (1 + l.nfbuf + (l.star ? 1 : 0)) +
                align_up(l.ring_bytes) * (l.star ? 2 : 1);
  int64_t cnt[2];
  HIP_TRY(c, hipMemcpyAsync(cnt, static_cast<const unsigned char*>(ckpt_dev) + coff, sizeof(cnt),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (cnt[0] < 0) return fail(c, AT_EINVAL, "corrupt checkpoint");
  c->n = cnt[0];
  // the saved solution goes to the buffer of its level's parity
  at_status st = ckpt_copy(c, nullptr, static_cast<const unsigned char*>(ckpt_dev), false, c->stream);
  c->state_set = st == AT_OK;
  return st;
}

at_status at_destroy(at_ctx* c) {
  if (!c) return AT_OK;
  drop_graph(c);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->aux_stream) (void)hipStreamDestroy(c->aux_stream);
  delete c;
  return AT_OK;
}

const char* at_last_error(const at_ctx* c) {
  if (c) return c->err.c_str();
  return thread_error().c_str();
}

}  // extern "C"

namespace {

// Scratch layout of at_adjoint: nck + 1 checkpoints; the levels of one
// segment (contiguous fields: u^seg .. u^{seg+every}, and for RK2 the
// predictors u*^seg .. u*^{seg+every-1}) with the forward rings at the
// segment start, twice when the two sets fit kOverlapBytes (then segment s-1
// is recomputed on a second stream while segment s is reversed); the adjoint
// fields (lambda x3, sigma); the forward halo buffer; the adjoint ring (two
// for RK2); alpha partial sums.
constexpr size_t kOverlapBytes = size_t(4) << 30;

struct AdjSet {
  size_t levels = 0, slevels = 0, ring0 = 0, sring0 = 0;
};

struct AdjLayout {
  size_t ck = 0, off_lam[3] = {0, 0, 0}, off_sigma = 0;
  size_t off_hbuf = 0, off_aring = 0, off_bring = 0;
  size_t off_partial = 0, off_out = 0, total = 0, aring_bytes = 0;
  AdjSet set[2];
  int nsets = 1;
  int64_t nck = 0;
  int anslots = 0;
  bool rk2 = false;
};

AdjLayout adj_layout(const at_ctx* c, int64_t nsteps, int every) {
  AdjLayout a;
  size_t ck = 0;
  at_checkpoint_size(c, &ck);
  a.ck = align_up(ck);
  a.nck = (nsteps + every - 1) / every;
  a.rk2 = c->prob.integrator == AT_RK2;
  size_t off = a.ck * static_cast<size_t>(a.nck + 1);
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const Layout& l = c->lay;
  const size_t w = c->g.f64 ? 8 : 4;
  const size_t seg_bytes = l.field_bytes * static_cast<size_t>(every + 1) +
                           (a.rk2 ? l.field_bytes * static_cast<size_t>(every) + l.ring_bytes : 0) + l.ring_bytes;
  a.nsets = a.nck > 1 && seg_bytes <= kOverlapBytes ? 2 : 1;
  for (int k = 0; k < a.nsets; ++k) {
    a.set[k].levels = take(l.field_bytes * static_cast<size_t>(every + 1));
    if (a.rk2) a.set[k].slevels = take(l.field_bytes * static_cast<size_t>(every));
    a.set[k].ring0 = take(l.ring_bytes);
    if (a.rk2) a.set[k].sring0 = take(l.ring_bytes);
  }
  for (int i = 0; i < 3; ++i) a.off_lam[i] = take(l.field_bytes);
  if (a.rk2) a.off_sigma = take(l.field_bytes);
  a.off_hbuf = take(static_cast<size_t>(c->g.npe) * l.pe_block * w);
  a.anslots = c->delay.mode == AT_SYNC ? 1 : l.nslots;
  a.aring_bytes = static_cast<size_t>(a.anslots) * c->g.npe * l.pe_block * w;
  a.off_aring = take(a.aring_bytes);
  if (a.rk2) a.off_bring = take(a.aring_bytes);
  a.off_partial = take(static_cast<size_t>(adj_partials(c->sp)) * sizeof(double));
  a.off_out = take(sizeof(double));
  a.total = off;
  return a;
}

at_status adj_check(at_ctx* c, int64_t nsteps, int32_t every) {
  if (!c) return fail(nullptr, AT_EINVAL, "null context");
  if (nsteps < 1 || every < 1) return fail(c, AT_EINVAL, "nsteps and the checkpoint interval must be >= 1");
  if (c->prob.integrator == AT_AB3) return fail(c, AT_EINVAL, "the adjoint covers Euler, AB2 and RK2");
  if (c->delay.scheme != AT_SCHEME_TIME)
    return fail(c, AT_EINVAL, "the adjoint covers the time-expanded schemes");
  if (c->delay.mode == AT_DELAY_HOST && nsteps > c->delay.host_nsteps)
    return fail(c, AT_EINVAL, "host delay table covers %lld steps", (long long)c->delay.host_nsteps);
  if (c->g.npts >= (int64_t(1) << 31) || c->g.npe * c->lay.pe_block >= (int64_t(1) << 31))
    return fail(c, AT_EINVAL, "the adjoint covers fields and strip sets below 2^31 values");
  return AT_OK;
}

}  // namespace

extern "C" {

at_status at_adjoint_scratch_size(at_ctx* c, int64_t nsteps, int32_t every, size_t* bytes) {
  at_status st = adj_check(c, nsteps, every);
  if (st != AT_OK) return st;
  if (!bytes) return fail(c, AT_EINVAL, "null argument");
  *bytes = adj_layout(c, nsteps, every).total;
  return AT_OK;
}

at_status at_adjoint(at_ctx* c, int64_t nsteps, int32_t every, const void* seed_dev, void* scratch_dev,
                     size_t scratch_bytes, void* grad_u0_dev, double* grad_alpha) {
  at_status st = adj_check(c, nsteps, every);
  if (st != AT_OK) return st;
  if (!seed_dev || !scratch_dev || !grad_u0_dev || !grad_alpha) return fail(c, AT_EINVAL, "null argument");
  if (!c->state_set || c->n != 0) return fail(c, AT_ESTATE, "the adjoint starts from a state set at step 0");
  const AdjLayout a = adj_layout(c, nsteps, every);
  if (scratch_bytes < a.total) return fail(c, AT_ENOMEM, "scratch %zu < %zu bytes", scratch_bytes, a.total);
  if (reinterpret_cast<uintptr_t>(scratch_dev) % kAlign)
    return fail(c, AT_EINVAL, "scratch must be %zu-byte aligned", kAlign);
  unsigned char* sc = static_cast<unsigned char*>(scratch_dev);
  const Layout& l = c->lay;
  const int64_t N = nsteps;
  // forward run, checkpoint at the start of every segment and at the end
  for (int64_t s = 0; s < a.nck; ++s) {
    st = at_save(c, sc + a.ck * s);
    if (st != AT_OK) return st;
    const int64_t len = std::min<int64_t>(every, N - s * every);
    st = at_step(c, len);
    if (st != AT_OK) return st;
  }
  st = at_save(c, sc + a.ck * a.nck);
  if (st != AT_OK) return st;
  // reverse sweep from lambda^N = seed
  unsigned char* lam[3] = {sc + a.off_lam[0], sc + a.off_lam[1], sc + a.off_lam[2]};
  int i1 = 0, i2 = 1, i0 = 2;   // roles: lambda^{n+1}, lambda^{n+2}, lambda^n
  HIP_TRY(c, hipMemcpyAsync(lam[i1], seed_dev, l.field_bytes, hipMemcpyDeviceToDevice, c->stream));
  HIP_TRY(c, hipMemsetAsync(lam[i2], 0, l.field_bytes, c->stream));
  HIP_TRY(c, hipMemsetAsync(sc + a.off_aring, 0, a.aring_bytes, c->stream));
  if (a.rk2) HIP_TRY(c, hipMemsetAsync(sc + a.off_bring, 0, a.aring_bytes, c->stream));
  HIP_TRY(c, hipMemsetAsync(sc + a.off_partial, 0, static_cast<size_t>(adj_partials(c->sp)) * sizeof(double),
                            c->stream));
  const double dt = c->prob.dt;
  // Recompute segment s into level set k on stream st: restore its
  // checkpoint into the context, keep the forward rings at its start and
  // step through it with every level kept.
  auto recompute = [&](int64_t s, int k, hipStream_t st) -> at_status {
    const AdjSet& z = a.set[k];
    unsigned char* levels = sc + z.levels;
    unsigned char* slevels = a.rk2 ? sc + z.slevels : nullptr;
    const int64_t seg = s * every;
    const int64_t len = std::min<int64_t>(every, N - seg);
    c->n = seg;
    at_status r = ckpt_copy(c, nullptr, sc + a.ck * s, false, st);
    if (r != AT_OK) return r;
    // the adjoint kernels take the levels in the [z][y][x] layout
    HIP_TRY(c, launch_field_copy(c->sp, c->g.f64, c->sp.ubuf[c->n & 1], levels, false, st));
    if (l.ring_bytes) {
      HIP_TRY(c, hipMemcpyAsync(sc + z.ring0, c->sp.ring, l.ring_bytes, hipMemcpyDeviceToDevice, st));
      if (a.rk2) HIP_TRY(c, hipMemcpyAsync(sc + z.sring0, c->sp.sring, l.ring_bytes, hipMemcpyDeviceToDevice, st));
    }
    for (int64_t j = 1; j <= len; ++j) {
      if (c->sp.pe_major) {
        // the 32 x 32 path keeps its fields PE-major: step, then copy the
        // levels out in the [z][y][x] layout
        r = enqueue_step(c, st);
        if (r != AT_OK) return r;
        c->n += 1;
        HIP_TRY(c, launch_field_copy(c->sp, c->g.f64, c->sp.ubuf[c->n & 1], levels + l.field_bytes * j, false, st));
        if (a.rk2)
          HIP_TRY(c, launch_field_copy(c->sp, c->g.f64, c->sp.ustar, slevels + l.field_bytes * (j - 1), false, st));
      } else {
        // the step reads level seg+j-1 from the segment's levels and writes
        // level seg+j (and the RK2 predictor) straight into them: no copies
        // (the generic sweep takes two solution buffers as well as one)
        StepParams p = c->sp;
        p.ubuf[c->n & 1] = levels + l.field_bytes * (j - 1);
        p.ubuf[(c->n + 1) & 1] = levels + l.field_bytes * j;
        if (a.rk2) p.ustar = slevels + l.field_bytes * (j - 1);
        r = enqueue_step_p(c, p, st);
        if (r != AT_OK) return r;
        c->n += 1;
      }
    }
    return AT_OK;
  };
  // Two level sets: segment s-1 is recomputed on the auxiliary stream while
  // segment s is reversed on the context's stream. Events order the reuse of
  // a set (the recomputation of s-1 waits for the reversal of s+1, which
  // read the same set) and the start of each reversal (it waits for its
  // recomputation). The reversal reads only the level set, the ring copies
  // and the adjoint's own buffers, never the context's live fields, which
  // the recomputation overwrites.
  const bool overlap = a.nsets == 2;
  hipEvent_t ev_start = nullptr, ev_rec[2] = {nullptr, nullptr}, ev_rev[2] = {nullptr, nullptr};
  struct EventGuard {
    hipEvent_t* e[5];
    ~EventGuard() {
      for (hipEvent_t* p : e)
        if (*p) (void)hipEventDestroy(*p);
    }
  } guard{{&ev_start, &ev_rec[0], &ev_rec[1], &ev_rev[0], &ev_rev[1]}};
  hipStream_t aux = c->stream;
  if (overlap) {
    if (!c->aux_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->aux_stream, hipStreamNonBlocking));
    aux = c->aux_stream;
    for (hipEvent_t* e : guard.e) HIP_TRY(c, hipEventCreateWithFlags(e, hipEventDisableTiming));
    // the recomputations start after the forward run and the initialisation
    HIP_TRY(c, hipEventRecord(ev_start, c->stream));
    HIP_TRY(c, hipStreamWaitEvent(aux, ev_start, 0));
    st = recompute(a.nck - 1, (a.nck - 1) & 1, aux);
    if (st != AT_OK) return st;
    HIP_TRY(c, hipEventRecord(ev_rec[(a.nck - 1) & 1], aux));
  }
  for (int64_t s = a.nck - 1; s >= 0; --s) {
    const int k = overlap ? static_cast<int>(s & 1) : 0;
    if (overlap) {
      HIP_TRY(c, hipStreamWaitEvent(c->stream, ev_rec[k], 0));
      if (s >= 1) {
        // set (s-1) & 1 was last read by the reversal of segment s+1
        if (s + 1 <= a.nck - 1) HIP_TRY(c, hipStreamWaitEvent(aux, ev_rev[(s + 1) & 1], 0));
        st = recompute(s - 1, static_cast<int>((s - 1) & 1), aux);
        if (st != AT_OK) return st;
        HIP_TRY(c, hipEventRecord(ev_rec[(s - 1) & 1], aux));
      }
    } else {
      st = recompute(s, 0, c->stream);
      if (st != AT_OK) return st;
    }
    unsigned char* levels = sc + a.set[k].levels;
    unsigned char* slevels = a.rk2 ? sc + a.set[k].slevels : nullptr;
    const int64_t seg = s * every;
    const int64_t len = std::min<int64_t>(every, N - seg);
    for (int64_t n = seg + len - 1; n >= seg; --n) {
      AdjParams q;
      std::memset(&q, 0, sizeof(q));
      q.sp = c->sp;
      q.n = n;
      q.npts = c->g.npts;
      q.burgers = c->prob.equation == AT_BURGERS;
      q.hbuf = sc + a.off_hbuf;
      q.anslots = a.anslots;
      q.seg_start = seg;
      q.partial = reinterpret_cast<double*>(sc + a.off_partial);
      for (int k = 0; k < kMaxL; ++k) {
        double w[kMaxT] = {0.0, 0.0, 0.0, 0.0};
        level_weights(k, c->delay.mode == AT_SYNC ? 1 : c->g.T, w);
        for (int m = 0; m < kMaxT; ++m) q.wt[k][m] = w[m];
      }
      for (int f = 0; f < 6; ++f) q.pfo[f] = c->lay.face_off[f] / c->g.npe;
      if (a.rk2) {
        // stage 2: sigma = dJ/du*^n from mu = dt/2 lambda^{n+1}
        AdjParams q2 = q;
        q2.y0 = lam[i1];
        q2.m0 = 0.5 * dt;
        q2.x0 = lam[i1];
        q2.b0 = 0.5;
        q2.out = sc + a.off_sigma;
        q2.levels = slevels;
        q2.ring0 = sc + a.set[k].sring0;
        q2.aring = sc + a.off_bring;
        HIP_TRY(c, launch_adj_step(q2, c->g.f64, c->stream));
        // stage 1: lambda^n from mu = dt sigma
        q.y0 = sc + a.off_sigma;
        q.m0 = dt;
        q.x0 = lam[i1];
        q.b0 = 0.5;
        q.x1 = sc + a.off_sigma;
        q.b1 = 1.0;
      } else {
        const bool ab2 = c->prob.integrator == AT_AB2;
        q.y0 = lam[i1];
        q.m0 = dt * ((ab2 && n > 0) ? 1.5 : 1.0);
        q.y1 = lam[i2];
        q.m1 = (ab2 && n + 1 <= N - 1) ? -0.5 * dt : 0.0;
        q.x0 = lam[i1];
        q.b0 = 1.0;
      }
      q.out = lam[i0];
      q.levels = levels;
      q.ring0 = sc + a.set[k].ring0;
      q.aring = sc + a.off_aring;
      HIP_TRY(c, launch_adj_step(q, c->g.f64, c->stream));
      const int t = i2;
      i2 = i1;
      i1 = i0;
      i0 = t;
    }
    if (overlap) HIP_TRY(c, hipEventRecord(ev_rev[k], c->stream));
  }
  HIP_TRY(c, hipMemcpyAsync(grad_u0_dev, lam[i1], l.field_bytes, hipMemcpyDeviceToDevice, c->stream));
  double* out = reinterpret_cast<double*>(sc + a.off_out);
  HIP_TRY(c, launch_adj_sum(reinterpret_cast<double*>(sc + a.off_partial), adj_partials(c->sp), out, c->stream));
  HIP_TRY(c, hipMemcpyAsync(grad_alpha, out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  // leave the context at the end of the forward run
  st = at_load(c, sc + a.ck * a.nck);
  if (st != AT_OK) return st;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return AT_OK;
}

}  // extern "C"
