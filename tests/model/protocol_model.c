/*
 * Protocol model of the sweep's reservation state machine: test
 * infrastructure only. The test suite loads it; the library never does, and
 * the two share no code.
 *
 * What it models. Every lane of the GPU sweep walks the lists of its sources
 * and, for a candidate edge (x, y), runs the reservation of Algorithm 1 with
 * u = min(x, y), v = max(x, y): take u, take v, then mark u matched or give
 * u back. On the GPU the lanes of a wavefront share one instruction stream,
 * so the model follows the library's form of the protocol, not a thread's:
 *   * a wavefront advances in trips; a trip first consumes, for every lane of
 *     the wavefront, the result of the memory operation the lane issued on the
 *     previous trip, then lets every lane issue its next operation;
 *   * a wait of Algorithm 1 is "stay in this phase and poll again next trip";
 *   * the memory operations of all wavefronts are applied to memory one at a
 *     time, in an order the scheduler (the adversary) chooses, each before the
 *     next trip of the wavefront that issued it (a trip waits for everything
 *     its wavefront issued before);
 *   * a cached read may return the value a state word had before its last
 *     change (a stale line); an atomic or a coherent read returns the current
 *     value.
 *
 * Variants (the options the library offers):
 *   layout       word (one 32-bit word per vertex that is also the output),
 *                8-bit or 2-bit fields packed into 32-bit words (a CAS on v
 *                that fails only because another field of its word changed
 *                is retried with the word it saw);
 *   two_phase    v is reserved like u and both are then marked matched,
 *                instead of one CAS moving v from accessible to matched;
 *   wait_release a lane that finds v reserved gives u back while it waits,
 *                then takes u again;
 *   lazy         symmetric input only: a source whose list ends with every
 *                neighbour matched writes its own "unmatched" output;
 *   upper        symmetric input only: a lane examines only the neighbours
 *                above its source (each undirected edge from its lower end);
 *                upper = 2 also ends a scan at the first neighbour below the
 *                source, which is sound when every list holds the neighbours
 *                above its vertex first.
 *
 * Two drivers: pm_run follows one schedule drawn by a seeded generator under
 * a strategy; pm_explore visits every state reachable under every schedule
 * (small graphs) and reports whether each can still reach the end, and the
 * distinct outputs at the end.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define PM_MAXN 8
#define PM_MAXM 64
#define PM_MAXL 4
#define PM_MAXS 8
#define PM_MAXOPS 16

enum { LAY_WORD = 0, LAY_U8 = 1, LAY_U2 = 2 };
enum { S_ACC = 0, S_RSVD = 1, S_MCHD = 2 };
enum { P_IDLE = 0, P_SRC, P_IDS, P_STS, P_RES, P_CHK, P_MAT, P_MATW, P_VW, P_FIN };
enum { K_LD_CACHED = 1, K_LD_COH, K_RESERVE, K_CAS, K_OR, K_AND, K_STORE_W, K_STORE_MATE };
enum { D_NONE = 0, D_RW0, D_RW1, D_RW2, D_RW3, D_XW, D_RES, D_CHKU, D_CHKV, D_MAT, D_MATW, D_FIN };

typedef struct {
  int layout, two_phase, wait_release, lazy, scan_width, stale, upper;
  int probe;  /* 1: a source's first state read takes one candidate; 2: every one does */
  int mutant; /* planted mistakes, to show the model notices them: 1 no id
                 order (u is always the source), 2 u is never given back,
                 3 v is taken by a plain store after a read saw it free */
} Variant;

typedef struct {
  int n;
  int off[PM_MAXN + 1];
  int nbr[PM_MAXM];
} Graph;

typedef struct {
  uint8_t kind, dest;
  int8_t at;  /* word index, or vertex for a mate store */
  uint8_t pad;
  uint32_t a, b;
} Op;

typedef struct {
  uint8_t phase, nsrc, si, k, nids, nops;
  uint8_t kr;     /* the buffered ids [k, kr) have their states read */
  uint8_t probe1; /* the next state read is the source's first */
  int8_t x, u, v, pad2;
  int16_t i, e;
  int8_t ids[4];
  uint32_t rw[4];
  uint32_t xword, vguess, res_w, chk_u, chk_v, mat_w, matw_w, fin_w;
  int8_t src[PM_MAXS];
  Op ops[PM_MAXOPS];
} Lane;

typedef struct {
  uint32_t w[PM_MAXN];   /* state words */
  uint32_t pw[PM_MAXN];  /* each word's value before its last change */
  int32_t mate[PM_MAXN]; /* mate array of the packed layouts */
  Lane lane[PM_MAXL];
} State;

typedef struct {
  const Graph *g;
  Variant var;
  int lanes, waves;
  int wave_of[PM_MAXL];
  uint32_t acc, rsvd; /* word layout: the values of ACC and RSVD */
  int per_word, bits;
} Ctx;

/* ------------------------------------------------------------------ layouts */

static int word_of(const Ctx *c, int v) { return c->var.layout == LAY_WORD ? v : v / c->per_word; }
static uint32_t shift_of(const Ctx *c, int v) { return (uint32_t)((v % c->per_word) * c->bits); }
static uint32_t field_mask(const Ctx *c) { return c->bits == 8 ? 0xffu : 0x3u; }

static int decode(const Ctx *c, uint32_t word, int v) {
  if (c->var.layout == LAY_WORD) return word == c->acc ? S_ACC : word == c->rsvd ? S_RSVD : S_MCHD;
  const uint32_t f = (word >> shift_of(c, v)) & field_mask(c);
  return f == 0 ? S_ACC : (f & 2u) ? S_MCHD : S_RSVD;
}

static void push(Lane *L, uint8_t kind, uint8_t dest, int at, uint32_t a, uint32_t b) {
  Op *o = &L->ops[L->nops++];
  o->kind = kind;
  o->dest = dest;
  o->at = (int8_t)at;
  o->pad = 0;
  o->a = a;
  o->b = b;
}

/* take u, or (two-phase) v */
static void issue_reserve(const Ctx *c, Lane *L, int t, uint8_t dest) {
  if (c->var.layout == LAY_WORD) {
    if (c->var.two_phase)
      push(L, K_RESERVE, dest, t, 0, 0); /* atomic min with RSVD */
    else
      push(L, K_CAS, dest, t, c->acc, c->rsvd);
  } else {
    push(L, K_OR, dest, word_of(c, t), 1u << shift_of(c, t), 0);
  }
}

static void issue_commit(const Ctx *c, Lane *L) {
  const int u = L->u, v = L->v;
  if (c->var.layout == LAY_WORD) {
    push(L, K_STORE_W, D_NONE, u, (uint32_t)v, 0);
    if (c->var.two_phase) push(L, K_STORE_W, D_NONE, v, (uint32_t)u, 0);
  } else {
    push(L, K_OR, D_NONE, word_of(c, u), 2u << shift_of(c, u), 0);
    if (c->var.two_phase) push(L, K_OR, D_NONE, word_of(c, v), 2u << shift_of(c, v), 0);
    push(L, K_STORE_MATE, D_NONE, u, (uint32_t)v, 0);
    push(L, K_STORE_MATE, D_NONE, v, (uint32_t)u, 0);
  }
}

static void issue_release(const Ctx *c, Lane *L) {
  if (c->var.mutant == 2) return;
  if (c->var.layout == LAY_WORD)
    push(L, K_STORE_W, D_NONE, L->u, c->acc, 0);
  else
    push(L, K_AND, D_NONE, word_of(c, L->u), ~(1u << shift_of(c, L->u)), 0);
}

/* "x can never be matched": its output is -1 */
static void issue_unmatched(const Ctx *c, Lane *L, int x) {
  if (c->var.layout == LAY_WORD) {
    if (c->var.two_phase) push(L, K_STORE_W, D_NONE, x, 0xffffffffu, 0);
  } else {
    push(L, K_STORE_MATE, D_NONE, x, 0xffffffffu, 0);
  }
}

/* ------------------------------------------------------------------ one lane */

static void advance(const Ctx *c, Lane *L) {
  int found = -1;
  for (int j = L->k; j < L->kr; ++j)
    if (L->ids[j] != L->x && (!c->var.upper || L->ids[j] > L->x) &&
        decode(c, L->rw[j], L->ids[j]) != S_MCHD) {
      found = j;
      break;
    }
  if (found >= 0) {
    const int y = L->ids[found];
    L->k = (uint8_t)(found + 1);
    L->u = (int8_t)(L->x < y ? L->x : y);
    L->v = (int8_t)(L->x < y ? y : L->x);
    if (c->var.mutant == 1) {
      L->u = L->x;
      L->v = (int8_t)y;
    }
    L->vguess = (L->x < y) ? L->rw[found] : L->xword;
    L->phase = P_RES;
  } else if (L->kr < L->nids) { /* the rest of the step's ids: their states next */
    L->k = L->kr;
    L->phase = P_STS;
  } else {
    L->k = L->nids;
    L->phase = L->i < L->e ? P_IDS : (c->var.lazy ? P_FIN : P_IDLE);
  }
}

static void edge_dead(const Ctx *c, Lane *L, int w) {
  if (w == L->x) L->phase = P_IDLE;
  else advance(c, L);
}

/* Consumes the result of the operation issued on the previous trip. */
static void consume(const Ctx *c, Lane *L) {
  const Graph *g = c->g;
  switch (L->phase) {
    case P_SRC: {
      const int x = L->x;
      if (decode(c, L->xword, x) == S_MCHD) {
        L->phase = P_IDLE; /* matched already: its list is skipped (Fig. 6g) */
      } else {
        L->i = (int16_t)g->off[x];
        L->e = (int16_t)g->off[x + 1];
        L->probe1 = (uint8_t)(c->var.probe != 0);
        L->phase = P_IDS;
      }
      break;
    }
    case P_IDS: {
      const int rem = L->e - L->i;
      L->nids = (uint8_t)(rem < c->var.scan_width ? rem : c->var.scan_width);
      for (int j = 0; j < 4; ++j) {
        L->ids[j] = j < L->nids ? (int8_t)g->nbr[L->i + j] : 0;
        L->rw[j] = 0;
      }
      L->i = (int16_t)(L->i + L->nids);
      L->k = 0;
      L->phase = P_STS;
      if (c->var.upper) {
        int any = 0, low = 0;
        for (int j = 0; j < L->nids; ++j) {
          any |= L->ids[j] > L->x;
          low |= L->ids[j] < L->x;
        }
        if (c->var.upper == 2 && low) L->e = L->i; /* the rest is below the source */
        if (!any) { /* nothing above the source here: read on without states */
          L->k = L->nids;
          L->phase = L->i < L->e ? P_IDS : (c->var.lazy ? P_FIN : P_IDLE);
        }
      }
      break;
    }
    case P_STS:
      advance(c, L);
      break;
    case P_RES: {
      const int s = decode(c, L->res_w, L->u);
      if (s == S_ACC) L->phase = P_MAT;
      else if (s == S_MCHD) edge_dead(c, L, L->u);
      else L->phase = P_CHK;
      break;
    }
    case P_CHK: {
      const int su = decode(c, L->chk_u, L->u), sv = decode(c, L->chk_v, L->v);
      if (sv == S_MCHD) edge_dead(c, L, L->v);
      else if (su == S_MCHD) edge_dead(c, L, L->u);
      else if (su == S_ACC) L->phase = P_RES;
      break;
    }
    case P_MAT: {
      int won, s;
      if (c->var.two_phase || c->var.layout == LAY_WORD) {
        s = decode(c, L->mat_w, L->v);
        won = s == S_ACC;
      } else {
        const uint32_t exp = L->vguess & ~(field_mask(c) << shift_of(c, L->v));
        won = L->mat_w == exp;
        s = won ? S_ACC : decode(c, L->mat_w, L->v);
      }
      if (won) {
        if (c->var.mutant == 3 && c->var.layout == LAY_WORD && !c->var.two_phase)
          push(L, K_STORE_W, D_NONE, L->v, (uint32_t)L->u, 0);
        issue_commit(c, L);
        L->phase = P_IDLE;
      } else if (s == S_ACC) {
        L->vguess = L->mat_w; /* another field of v's word changed: try again */
      } else if (s == S_RSVD) {
        if (c->var.wait_release) {
          issue_release(c, L);
          L->phase = P_VW;
        } else {
          L->phase = P_MATW;
        }
      } else {
        issue_release(c, L);
        edge_dead(c, L, L->v);
      }
      break;
    }
    case P_MATW: {
      const int s = decode(c, L->matw_w, L->v);
      if (s == S_ACC) {
        L->vguess = L->matw_w;
        L->phase = P_MAT;
      } else if (s == S_MCHD) {
        issue_release(c, L);
        edge_dead(c, L, L->v);
      }
      break;
    }
    case P_VW: {
      const int s = decode(c, L->matw_w, L->v);
      if (s == S_ACC) {
        L->vguess = L->matw_w;
        L->phase = P_RES;
      } else if (s == S_MCHD) {
        edge_dead(c, L, L->v);
      }
      break;
    }
    case P_FIN: {
      const int s = decode(c, L->fin_w, L->x);
      if (s == S_ACC) {
        if (c->var.layout != LAY_WORD) issue_unmatched(c, L, L->x);
        L->phase = P_IDLE;
      } else if (s == S_MCHD) {
        L->phase = P_IDLE;
      }
      break;
    }
    default:
      break;
  }
  /* results are consumed: clear them, so that equal situations are equal states */
  L->res_w = L->chk_u = L->chk_v = L->mat_w = L->matw_w = L->fin_w = 0;
  if (L->phase != P_STS && L->phase != P_RES && L->phase != P_CHK && L->phase != P_MAT &&
      L->phase != P_MATW && L->phase != P_VW)
    for (int j = 0; j < 4; ++j) L->rw[j] = 0;
  if (L->phase == P_IDLE || L->phase == P_IDS || L->phase == P_FIN) L->vguess = 0;
}

/* An idle lane takes its next source (sources without entries are skipped;
   their output is written at once under lazy output). */
static void hand_out(const Ctx *c, Lane *L) {
  if (L->phase != P_IDLE) return;
  while (L->si < L->nsrc) {
    const int x = L->src[L->si++];
    if (c->g->off[x] == c->g->off[x + 1]) {
      if (c->var.lazy) issue_unmatched(c, L, x);
      continue;
    }
    L->x = (int8_t)x;
    L->u = L->v = 0;
    L->i = L->e = 0;
    L->nids = L->k = 0;
    L->xword = 0;
    for (int j = 0; j < 4; ++j) L->ids[j] = 0;
    L->phase = P_SRC;
    return;
  }
  L->x = L->u = L->v = 0;
  L->i = L->e = 0;
  L->nids = L->k = 0;
  L->xword = 0;
  for (int j = 0; j < 4; ++j) L->ids[j] = 0;
}

static void issue(const Ctx *c, Lane *L) {
  switch (L->phase) {
    case P_SRC:
      push(L, K_LD_CACHED, D_XW, word_of(c, L->x), 0, 0);
      break;
    case P_STS: {
      int lim = L->nids;
      for (int j = L->k; j < lim; ++j)
        if (L->ids[j] != L->x && (!c->var.upper || L->ids[j] > L->x)) {
          push(L, K_LD_CACHED, (uint8_t)(D_RW0 + j), word_of(c, L->ids[j]), 0, 0);
          if (L->probe1 || c->var.probe == 2) lim = j + 1;
        }
      L->kr = (uint8_t)lim;
      L->probe1 = 0;
      break;
    }
    case P_RES:
      issue_reserve(c, L, L->u, D_RES);
      break;
    case P_CHK:
      push(L, K_LD_COH, D_CHKU, word_of(c, L->u), 0, 0);
      push(L, K_LD_COH, D_CHKV, word_of(c, L->v), 0, 0);
      break;
    case P_MAT:
      if (c->var.two_phase) {
        issue_reserve(c, L, L->v, D_MAT);
      } else if (c->var.layout == LAY_WORD) {
        if (c->var.mutant == 3)
          push(L, K_LD_COH, D_MAT, L->v, 0, 0); /* consume stores u if it read ACC */
        else
          push(L, K_CAS, D_MAT, L->v, c->acc, (uint32_t)L->u);
      } else {
        const uint32_t sh = shift_of(c, L->v);
        const uint32_t exp = L->vguess & ~(field_mask(c) << sh);
        push(L, K_CAS, D_MAT, word_of(c, L->v), exp, exp | (3u << sh));
      }
      break;
    case P_MATW:
    case P_VW:
      push(L, K_LD_COH, D_MATW, word_of(c, L->v), 0, 0);
      break;
    case P_FIN:
      if (c->var.layout == LAY_WORD && c->var.two_phase)
        push(L, K_CAS, D_FIN, L->x, c->acc, 0xffffffffu); /* ACC -> -1, or the state met */
      else
        push(L, K_LD_COH, D_FIN, word_of(c, L->x), 0, 0);
      break;
    default:
      break;
  }
}

static int lane_done(const Lane *L) { return L->phase == P_IDLE && L->si >= L->nsrc && L->nops == 0; }

static int wave_ready(const Ctx *c, const State *s, int w) {
  int any_work = 0;
  for (int l = 0; l < c->lanes; ++l) {
    if (c->wave_of[l] != w) continue;
    if (s->lane[l].nops) return 0;
    if (!lane_done(&s->lane[l])) any_work = 1;
  }
  return any_work;
}

/* One trip of wavefront w: consume, hand out, issue (every lane of it). */
static void trip(const Ctx *c, State *s, int w) {
  for (int l = 0; l < c->lanes; ++l)
    if (c->wave_of[l] == w) consume(c, &s->lane[l]);
  for (int l = 0; l < c->lanes; ++l)
    if (c->wave_of[l] == w) hand_out(c, &s->lane[l]);
  for (int l = 0; l < c->lanes; ++l)
    if (c->wave_of[l] == w) issue(c, &s->lane[l]);
}

static void deliver(Lane *L, uint8_t dest, uint32_t val) {
  switch (dest) {
    case D_RW0: case D_RW1: case D_RW2: case D_RW3: L->rw[dest - D_RW0] = val; break;
    case D_XW: L->xword = val; break;
    case D_RES: L->res_w = val; break;
    case D_CHKU: L->chk_u = val; break;
    case D_CHKV: L->chk_v = val; break;
    case D_MAT: L->mat_w = val; break;
    case D_MATW: L->matw_w = val; break;
    case D_FIN: L->fin_w = val; break;
    default: break;
  }
}

static void set_word(State *s, int at, uint32_t nv) {
  if (s->w[at] != nv) {
    s->pw[at] = s->w[at];
    s->w[at] = nv;
  }
}

/* Applies pending operation k of lane l; a cached read returns the word's
   previous value when `stale` is set (and it differs). */
static void apply(const Ctx *c, State *s, int l, int k, int stale) {
  Lane *L = &s->lane[l];
  const Op o = L->ops[k];
  L->ops[k] = L->ops[--L->nops];
  memset(&L->ops[L->nops], 0, sizeof(Op));
  const uint32_t old = o.kind == K_STORE_MATE ? 0 : s->w[o.at];
  switch (o.kind) {
    case K_LD_CACHED: deliver(L, o.dest, stale ? s->pw[o.at] : old); break;
    case K_LD_COH: deliver(L, o.dest, old); break;
    case K_RESERVE:
      if ((int32_t)old > (int32_t)c->rsvd) set_word(s, o.at, c->rsvd);
      deliver(L, o.dest, old);
      break;
    case K_CAS:
      if (old == o.a) set_word(s, o.at, o.b);
      deliver(L, o.dest, old);
      break;
    case K_OR: set_word(s, o.at, old | o.a); deliver(L, o.dest, old); break;
    case K_AND: set_word(s, o.at, old & o.a); deliver(L, o.dest, old); break;
    case K_STORE_W: set_word(s, o.at, o.a); break;
    case K_STORE_MATE: s->mate[o.at] = (int32_t)o.a; break;
    default: break;
  }
}

/* ------------------------------------------------------------------ set-up */

static int setup(Ctx *c, State *s, const Graph *g, const int *var6, int lanes, const int *wave_of,
                 const int *src, int max_src) {
  memset(c, 0, sizeof(*c));
  memset(s, 0, sizeof(*s));
  c->g = g;
  c->var.layout = var6[0];
  c->var.two_phase = var6[1];
  c->var.wait_release = var6[2];
  c->var.lazy = var6[3];
  c->var.scan_width = var6[4] < 1 ? 1 : (var6[4] > 4 ? 4 : var6[4]);
  c->var.stale = var6[5];
  c->var.upper = var6[6];
  c->var.mutant = var6[7];
  c->var.probe = var6[8];
  if (g->n > PM_MAXN || lanes < 1 || lanes > PM_MAXL || max_src > PM_MAXS) return -1;
  c->lanes = lanes;
  c->waves = 0;
  for (int l = 0; l < lanes; ++l) {
    c->wave_of[l] = wave_of[l];
    if (wave_of[l] + 1 > c->waves) c->waves = wave_of[l] + 1;
  }
  c->acc = c->var.two_phase ? 0x7fffffffu : 0xffffffffu;
  c->rsvd = c->var.two_phase ? 0x7ffffffeu : 0xfffffffeu;
  c->per_word = c->var.layout == LAY_U8 ? 4 : c->var.layout == LAY_U2 ? 16 : 1;
  c->bits = c->var.layout == LAY_U8 ? 8 : c->var.layout == LAY_U2 ? 2 : 32;
  for (int v = 0; v < PM_MAXN; ++v) {
    s->w[v] = c->var.layout == LAY_WORD ? c->acc : 0u;
    s->pw[v] = s->w[v];
    /* lazy output leaves -1 to the sweep: start from a value no output has */
    s->mate[v] = (c->var.lazy && c->var.layout != LAY_WORD) ? 0x40000000 : -1;
  }
  for (int l = 0; l < lanes; ++l) {
    Lane *L = &s->lane[l];
    for (int j = 0; j < max_src; ++j) {
      const int x = src[l * max_src + j];
      if (x < 0) break;
      if (x >= g->n) return -1;
      L->src[L->nsrc++] = (int8_t)x;
    }
    L->phase = P_IDLE;
  }
  /* every wavefront's first trip hands out sources and issues */
  for (int w = 0; w < c->waves; ++w) trip(c, s, w);
  return 0;
}

static int finished(const Ctx *c, const State *s) {
  for (int l = 0; l < c->lanes; ++l)
    if (!lane_done(&s->lane[l])) return 0;
  return 1;
}

/* The output mate array; returns the number of vertices left accessible
   or reserved under lazy output of the word layout (the sweep must have
   written every output). */
static int output(const Ctx *c, const State *s, int32_t *mate) {
  int bad = 0;
  for (int v = 0; v < c->g->n; ++v) {
    if (c->var.layout == LAY_WORD) {
      const uint32_t w = s->w[v];
      if (c->var.two_phase && w == c->acc) {
        if (c->var.lazy) ++bad;
        mate[v] = -1; /* the eager pass rewrites leftover ACC as -1 */
      } else {
        mate[v] = (int32_t)w;
      }
    } else {
      mate[v] = s->mate[v];
    }
  }
  return bad;
}

/* ------------------------------------------------------------------ one schedule */

static uint64_t rng_next(uint64_t *x) {
  uint64_t z = (*x += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

/*
 * Runs one schedule. var6 = {layout, two_phase, wait_release, lazy,
 * scan_width, stale, upper, mutant, probe}; lanes in wavefronts wave_of[l]; src: lanes x max_src
 * source ids (-1 ends a lane's list). strategy: 0 every choice equally
 * likely; 1 wavefronts advance before pending operations are applied where
 * possible (operations stay in flight long, reads are stale); 2 operations
 * are applied before wavefronts advance (near lockstep); 3 wavefront 0 is
 * starved (it moves only when nothing else can). mate_out: n entries.
 * Returns the total number of trips, -1 on bad arguments, -2 if max_trips
 * passed without the sweep ending, -3 if an output was left unwritten.
 */
int64_t pm_run(const Graph *g, const int *var6, int lanes, const int *wave_of, const int *src,
               int max_src, int strategy, uint64_t seed, int64_t max_trips, int32_t *mate_out) {
  Ctx c;
  State s;
  if (setup(&c, &s, g, var6, lanes, wave_of, src, max_src)) return -1;
  uint64_t r = seed;
  int64_t trips = c.waves;
  while (!finished(&c, &s)) {
    /* the choices: advance a wavefront whose operations are all applied, or
       apply one pending operation; under strategy 3 wavefront 0's choices
       are taken only when no other exists (fair, but as late as possible) */
    int ready[PM_MAXL], nready = 0, opl[PM_MAXL * PM_MAXOPS], opk[PM_MAXL * PM_MAXOPS], nops = 0;
    for (int pass = 0; pass < 2 && nready + nops == 0; ++pass) {
      const int skip0 = strategy == 3 && pass == 0;
      for (int w = 0; w < c.waves; ++w)
        if (!(skip0 && w == 0) && wave_ready(&c, &s, w)) ready[nready++] = w;
      for (int l = 0; l < c.lanes; ++l)
        if (!(skip0 && c.wave_of[l] == 0))
          for (int k = 0; k < s.lane[l].nops; ++k) {
            opl[nops] = l;
            opk[nops++] = k;
          }
    }
    if (nready + nops == 0) return -1; /* cannot happen: a lane with work is ready or waits */
    int do_trip;
    if (nops == 0) do_trip = 1;
    else if (nready == 0) do_trip = 0;
    else if (strategy == 1) do_trip = (rng_next(&r) % 8) != 0;
    else if (strategy == 2) do_trip = (rng_next(&r) % 8) == 0;
    else do_trip = (int)(rng_next(&r) % (uint64_t)(nops + nready)) < nready;
    if (do_trip) {
      trip(&c, &s, ready[rng_next(&r) % (uint64_t)nready]);
      ++trips;
    } else {
      const int q = (int)(rng_next(&r) % (uint64_t)nops);
      const Op o = s.lane[opl[q]].ops[opk[q]];
      const int stale = c.var.stale && o.kind == K_LD_CACHED && s.pw[o.at] != s.w[o.at] &&
                        (rng_next(&r) & 1);
      apply(&c, &s, opl[q], opk[q], stale);
    }
    if (trips > max_trips) return -2;
  }
  if (output(&c, &s, mate_out)) return -3;
  return trips;
}

/* ------------------------------------------------------------------ every schedule */

/* A state's canonical bytes: the pending operations of a lane form a set, so
   they are sorted. */
static void canon(State *s, int lanes) {
  for (int l = 0; l < lanes; ++l) {
    Lane *L = &s->lane[l];
    for (int a = 1; a < L->nops; ++a)
      for (int b = a; b > 0 && memcmp(&L->ops[b - 1], &L->ops[b], sizeof(Op)) > 0; --b) {
        Op t = L->ops[b];
        L->ops[b] = L->ops[b - 1];
        L->ops[b - 1] = t;
      }
  }
}

typedef struct {
  State *st;
  int64_t n, cap;
  int64_t *slot; /* hash table of state indices, -1 empty */
  int64_t tcap;
  int64_t *succ, nsucc, succ_cap; /* successor lists */
  int64_t *first;                 /* first successor of each state (n + 1 entries when done) */
} Graphs;

static uint64_t hash_state(const State *s) {
  const unsigned char *p = (const unsigned char *)s;
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < sizeof(State); ++i) h = (h ^ p[i]) * 1099511628211ull;
  return h;
}

static int grow(void **p, int64_t *cap, int64_t need, size_t elem) {
  if (need <= *cap) return 0;
  int64_t nc = *cap ? *cap : 1024;
  while (nc < need) nc *= 2;
  void *q = realloc(*p, (size_t)nc * elem);
  if (!q) return -1;
  *p = q;
  *cap = nc;
  return 0;
}

static int64_t find_or_add(Graphs *G, const State *s, int *added) {
  if (G->n * 2 >= G->tcap) {
    const int64_t nt = G->tcap ? G->tcap * 2 : 1 << 16;
    int64_t *ns = (int64_t *)malloc((size_t)nt * sizeof(int64_t));
    if (!ns) return -1;
    for (int64_t i = 0; i < nt; ++i) ns[i] = -1;
    for (int64_t i = 0; i < G->n; ++i) {
      uint64_t h = hash_state(&G->st[i]) & (uint64_t)(nt - 1);
      while (ns[h] >= 0) h = (h + 1) & (uint64_t)(nt - 1);
      ns[h] = i;
    }
    free(G->slot);
    G->slot = ns;
    G->tcap = nt;
  }
  uint64_t h = hash_state(s) & (uint64_t)(G->tcap - 1);
  while (G->slot[h] >= 0) {
    if (!memcmp(&G->st[G->slot[h]], s, sizeof(State))) {
      *added = 0;
      return G->slot[h];
    }
    h = (h + 1) & (uint64_t)(G->tcap - 1);
  }
  if (grow((void **)&G->st, &G->cap, G->n + 1, sizeof(State))) return -1;
  G->st[G->n] = *s;
  G->slot[h] = G->n;
  *added = 1;
  return G->n++;
}

/*
 * Visits every state reachable under every schedule (every order of applying
 * the pending operations, every choice of a wavefront to advance, and, with
 * stale reads, both values a cached read may return). Returns the number of
 * states, or -1 on bad arguments or lack of memory, or -2 if more than
 * max_states. *stuck receives the number of reachable states from which no
 * schedule reaches the end (a deadlock or livelock under fair scheduling);
 * outs (max_outs x n) receives the distinct outputs at the end, *n_outs their
 * number (-3 in *n_outs if an output was left unwritten).
 */
int64_t pm_explore(const Graph *g, const int *var6, int lanes, const int *wave_of, const int *src,
                   int max_src, int64_t max_states, int64_t *stuck, int32_t *outs, int max_outs,
                   int *n_outs) {
  Ctx c;
  State s0;
  if (setup(&c, &s0, g, var6, lanes, wave_of, src, max_src)) return -1;
  canon(&s0, c.lanes);
  Graphs G;
  memset(&G, 0, sizeof(G));
  int added;
  if (find_or_add(&G, &s0, &added) < 0) return -1;
  int64_t *q_first = NULL, qf_cap = 0;
  int64_t ret = 0;
  *n_outs = 0;
  /* breadth-first: state i's successors are appended in order of discovery */
  for (int64_t i = 0; i < G.n; ++i) {
    if (grow((void **)&q_first, &qf_cap, i + 2, sizeof(int64_t))) { ret = -1; goto out; }
    q_first[i] = G.nsucc;
    const State cur = G.st[i];
    if (finished(&c, &cur)) {
      int32_t mate[PM_MAXN];
      if (output(&c, &cur, mate)) *n_outs = -3;
      if (*n_outs >= 0) {
        int seen = 0;
        for (int k = 0; k < *n_outs && !seen; ++k)
          seen = !memcmp(outs + (int64_t)k * g->n, mate, sizeof(int32_t) * (size_t)g->n);
        if (!seen && *n_outs < max_outs) {
          memcpy(outs + (int64_t)(*n_outs) * g->n, mate, sizeof(int32_t) * (size_t)g->n);
          ++*n_outs;
        }
      }
      continue;
    }
    for (int w = 0; w < c.waves; ++w) {
      if (!wave_ready(&c, &cur, w)) continue;
      State nx = cur;
      trip(&c, &nx, w);
      canon(&nx, c.lanes);
      const int64_t j = find_or_add(&G, &nx, &added);
      if (j < 0) { ret = -1; goto out; }
      if (grow((void **)&G.succ, &G.succ_cap, G.nsucc + 1, sizeof(int64_t))) { ret = -1; goto out; }
      G.succ[G.nsucc++] = j;
    }
    for (int l = 0; l < c.lanes; ++l)
      for (int k = 0; k < cur.lane[l].nops; ++k) {
        const Op o = cur.lane[l].ops[k];
        const int outcomes = (c.var.stale && o.kind == K_LD_CACHED && cur.pw[o.at] != cur.w[o.at]) ? 2 : 1;
        for (int stale = 0; stale < outcomes; ++stale) {
          State nx = cur;
          apply(&c, &nx, l, k, stale);
          canon(&nx, c.lanes);
          const int64_t j = find_or_add(&G, &nx, &added);
          if (j < 0) { ret = -1; goto out; }
          if (grow((void **)&G.succ, &G.succ_cap, G.nsucc + 1, sizeof(int64_t))) { ret = -1; goto out; }
          G.succ[G.nsucc++] = j;
        }
      }
    if (G.n > max_states) { ret = -2; goto out; }
  }
  q_first[G.n] = G.nsucc;
  {
    /* states that reach the end: a fixed point from the finished ones */
    char *good = G.n > 0 ? (char *)calloc((size_t)G.n, 1) : NULL;
    if (!good) { ret = -1; goto out; }
    for (int64_t i = 0; i < G.n; ++i) good[i] = (char)finished(&c, &G.st[i]);
    int changed = 1;
    while (changed) {
      changed = 0;
      for (int64_t i = G.n - 1; i >= 0; --i) {
        if (good[i]) continue;
        for (int64_t e = q_first[i]; e < q_first[i + 1]; ++e)
          if (good[G.succ[e]]) {
            good[i] = 1;
            changed = 1;
            break;
          }
      }
    }
    int64_t bad = 0;
    for (int64_t i = 0; i < G.n; ++i) bad += !good[i];
    *stuck = bad;
    free(good);
    ret = G.n;
  }
out:
  free(q_first);
  free(G.st);
  free(G.slot);
  free(G.succ);
  return ret;
}

int pm_sizeof_graph(void) { return (int)sizeof(Graph); }
int pm_max_vertices(void) { return PM_MAXN; }
