/*
 * neat_oracle.c -- plain CPU oracle for the population forward of tensorized
 * NEAT (Wang et al., "Tensorized NeuroEvolution of Augmenting Topologies for
 * GPU Acceleration", GECCO 2024).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this library.  It shares no source,
 * header, table or helper with the GPU library, and the GPU library never
 * calls it.
 *
 * What it computes is the plain definition behind Section 3.3 ("Tensorized
 * Network Inference"): a feedforward evaluation of each genome's graph.  The
 * paper's tensors (node order N_order, expanded connections C_exp) are only a
 * fast way of doing that, so this file works on adjacency lists instead:
 *
 *   - Section 3.1 (Tensorized Encodings): a node row is
 *     (key, bias, response, act, agg); a connection row is
 *     (in key, out key, enabled, weight); rows padded with NaN are absent.
 *   - Section 3.3: the transformation topologically sorts the nodes and keeps
 *     the enabled connections' attributes; disabled rows become absent (NaN)
 *     cells.  The calculation sets v[input] = I, then walks the order and
 *     sets v[k] = f_n(f_c(v | incoming)), with f_c(x | w) = w x and
 *     f_n(x | b, agg, act) = act(agg(x) + b); the outputs are v[output].
 *   - Appendix (genome interface): input keys are 0..I-1 and output keys are
 *     I..I+O-1.
 *
 * Readings where the paper is silent or ambiguous (each listed with its
 * reason in the design notes):
 *   - connection ends are node KEYS (historical markers), resolved to rows;
 *   - the topological order is the level-synchronous Kahn order, ties broken
 *     by key: nodes sorted by (level, key), level = longest path from a node
 *     without incoming enabled edges;
 *   - node value = act(bias + response * agg(incoming)), agg of nothing = 0
 *     (response is a node attribute in the paper's hyper-parameters; every
 *     experiment there keeps it at 1, where this equals f_n);
 *   - act codes: 0 identity, 1 tanh, 2 sigmoid, 3 relu, 4 sin, 5 gaussian
 *     exp(-z^2), 6 abs; agg codes: 0 sum, 1 product, 2 max, 3 min, 4 mean.
 *     NaN propagates through every one of them (max/min/relu included);
 *   - incoming values are aggregated in ascending source-key order;
 *   - malformed genomes are flagged in a status bit-mask and produce NaN;
 *   - recurrent networks (Section 3.3 and Appendix A name them; only the
 *     feedforward calculation is defined): cycles are allowed, the nodes keep
 *     key order, and K synchronous sweeps update every non-input node from the
 *     previous sweep's values, starting from the inputs and 0 elsewhere.
 *
 * Floating point: the reference arithmetic is IEEE double (oracle_forward_f64).
 * The same code is also instantiated in float (oracle_forward_f32) so the
 * tests can check the first-order error bound beta that the f64 version
 * propagates for an fp32 evaluation of the same graph.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* status bits (per genome) */
enum {
    ST_BAD_VALUE = 1u,   /* non-integer / out-of-range key, code or flag */
    ST_DUP_KEY = 2u,     /* two valid nodes share a key                  */
    ST_MISSING_IO = 4u,  /* an input or output key is absent             */
    ST_BAD_REF = 8u,     /* enabled connection names an absent key       */
    ST_INTO_INPUT = 16u, /* enabled connection ends at an input node     */
    ST_DUP_EDGE = 32u,   /* two enabled connections with the same ends   */
    ST_CYCLE = 64u       /* the enabled connections contain a cycle      */
};

#define NODE_W 5
#define CONN_W 4
#define KEY_LIMIT 16777216.0 /* 2^24: keys stay exact in float */
#define N_ACT 7
#define N_AGG 5

#define ORACLE_E_INVALID (-1)
#define ORACLE_E_NOMEM (-3)
#define ORACLE_E_SELFCHECK (-100)

typedef struct {
    int src, dst; /* node rows */
    float w;
} o_edge;

/* Everything the transformation of one genome produces. */
typedef struct {
    uint32_t status;
    int nvalid;
    int *order;  /* [N_max] rows by (level, key), -1 padded */
    int *level;  /* [N_max] level per row, -1 for absent rows */
    o_edge *edges; /* resolved enabled edges */
    int nedges;
} o_genome;

static int is_int_in(double x, double lo, double hi_excl) {
    return !isnan(x) && x == floor(x) && x >= lo && x < hi_excl;
}

/* Row of the valid, well-keyed node whose key equals k, or -1. */
static int find_row(const float *nodes, int N_max, float k) {
    for (int r = 0; r < N_max; ++r) {
        float key = nodes[r * NODE_W + 0];
        if (isnan(key) || !is_int_in(key, 0.0, KEY_LIMIT)) continue;
        if (key == k) return r;
    }
    return -1;
}

static void genome_free(o_genome *g) {
    free(g->order);
    free(g->level);
    free(g->edges);
    memset(g, 0, sizeof(*g));
}

/*
 * Transformation of one genome (Section 3.3, first stage), plus the validity
 * checks that make the encoding of Section 3.1 well defined.
 */
static int genome_transform(const float *nodes, const float *conns, int N_max,
                            int C_max, int I, int O, int recurrent, o_genome *g) {
    memset(g, 0, sizeof(*g));
    g->order = (int *)malloc(sizeof(int) * (size_t)N_max);
    g->level = (int *)malloc(sizeof(int) * (size_t)N_max);
    g->edges = (o_edge *)malloc(sizeof(o_edge) * (size_t)(C_max > 0 ? C_max : 1));
    if (!g->order || !g->level || !g->edges) return ORACLE_E_NOMEM;
    for (int r = 0; r < N_max; ++r) {
        g->order[r] = -1;
        g->level[r] = -1;
    }
    uint32_t st = 0;

    /* 1. node rows: a row is present iff its key (column 0) is not NaN */
    for (int r = 0; r < N_max; ++r) {
        const float *n = nodes + (size_t)r * NODE_W;
        if (isnan(n[0])) continue;
        g->nvalid++;
        if (!is_int_in(n[0], 0.0, KEY_LIMIT)) st |= ST_BAD_VALUE;
        if (!is_int_in(n[3], 0.0, (double)N_ACT)) st |= ST_BAD_VALUE;
        if (!is_int_in(n[4], 0.0, (double)N_AGG)) st |= ST_BAD_VALUE;
    }
    /* duplicate keys among well-formed keys */
    for (int r = 0; r < N_max; ++r) {
        float kr = nodes[r * NODE_W];
        if (isnan(kr) || !is_int_in(kr, 0.0, KEY_LIMIT)) continue;
        for (int q = r + 1; q < N_max; ++q) {
            float kq = nodes[q * NODE_W];
            if (isnan(kq) || !is_int_in(kq, 0.0, KEY_LIMIT)) continue;
            if (kq == kr) st |= ST_DUP_KEY;
        }
    }
    /* input keys 0..I-1 and output keys I..I+O-1 must exist */
    for (int k = 0; k < I + O; ++k)
        if (find_row(nodes, N_max, (float)k) < 0) st |= ST_MISSING_IO;

    /* 2. connection rows: padding iff column 0 is NaN; disabled rows ignored */
    for (int r = 0; r < C_max; ++r) {
        const float *c = conns + (size_t)r * CONN_W;
        if (isnan(c[0])) continue;
        if (c[2] == 0.0f) continue;
        if (c[2] != 1.0f) {
            st |= ST_BAD_VALUE;
            continue;
        }
        int s = find_row(nodes, N_max, c[0]);
        int d = find_row(nodes, N_max, c[1]);
        if (s < 0 || d < 0) {
            st |= ST_BAD_REF;
            continue;
        }
        if (nodes[d * NODE_W] < (float)I) st |= ST_INTO_INPUT;
        if (s == d && !recurrent) st |= ST_CYCLE;
        for (int e = 0; e < g->nedges; ++e)
            if (g->edges[e].src == s && g->edges[e].dst == d) st |= ST_DUP_EDGE;
        g->edges[g->nedges].src = s;
        g->edges[g->nedges].dst = d;
        g->edges[g->nedges].w = c[3];
        g->nedges++;
    }

    /* 3. levels by level-synchronous Kahn, only for an otherwise clean genome.
     * A recurrent network has no levels: every valid node gets level 0, so
     * the order below is plain key order. */
    if (st == 0 && recurrent) {
        for (int r = 0; r < N_max; ++r)
            if (!isnan(nodes[r * NODE_W])) g->level[r] = 0;
    }
    if (st == 0 && !recurrent) {
        int *indeg = (int *)calloc((size_t)N_max, sizeof(int));
        char *emitted = (char *)calloc((size_t)N_max, 1);
        char *ready = (char *)calloc((size_t)N_max, 1);
        if (!indeg || !emitted || !ready) {
            free(indeg), free(emitted), free(ready);
            return ORACLE_E_NOMEM;
        }
        for (int e = 0; e < g->nedges; ++e) indeg[g->edges[e].dst]++;
        int done = 0;
        for (int lvl = 0;; ++lvl) {
            int nready = 0;
            for (int r = 0; r < N_max; ++r) {
                ready[r] = 0;
                if (isnan(nodes[r * NODE_W]) || emitted[r]) continue;
                if (indeg[r] == 0) {
                    ready[r] = 1;
                    nready++;
                }
            }
            if (nready == 0) break;
            for (int r = 0; r < N_max; ++r) {
                if (!ready[r]) continue;
                emitted[r] = 1;
                g->level[r] = lvl;
                done++;
            }
            for (int e = 0; e < g->nedges; ++e)
                if (ready[g->edges[e].src]) indeg[g->edges[e].dst]--;
        }
        if (done < g->nvalid) st |= ST_CYCLE;
        free(indeg), free(emitted), free(ready);
    }

    /* 4. order: valid rows sorted by (level, key); all -1 when rejected */
    if (st == 0) {
        int n = 0;
        for (int r = 0; r < N_max; ++r)
            if (!isnan(nodes[r * NODE_W])) g->order[n++] = r;
        for (int i = 1; i < n; ++i) { /* insertion sort, plain and stable */
            int x = g->order[i];
            int j = i - 1;
            while (j >= 0) {
                int y = g->order[j];
                int before = g->level[x] < g->level[y] ||
                             (g->level[x] == g->level[y] &&
                              nodes[x * NODE_W] < nodes[y * NODE_W]);
                if (!before) break;
                g->order[j + 1] = y;
                --j;
            }
            g->order[j + 1] = x;
        }
    } else {
        for (int r = 0; r < N_max; ++r) {
            g->order[r] = -1;
            g->level[r] = -1;
        }
    }
    g->status = st;
    return 0;
}

static int check_dims(int P, int N_max, int C_max, int I, int O) {
    if (P < 0 || N_max < 1 || C_max < 0 || I < 1 || O < 1) return 0;
    if (I + O > N_max) return 0;
    return 1;
}

static int transform_population(int P, int N_max, int C_max, int I, int O,
                                const float *nodes, const float *conns, int recurrent,
                                int32_t *order, int32_t *level, uint32_t *status) {
    if (!check_dims(P, N_max, C_max, I, O)) return ORACLE_E_INVALID;
    for (int p = 0; p < P; ++p) {
        o_genome g;
        int rc = genome_transform(nodes + (size_t)p * N_max * NODE_W,
                                  conns + (size_t)p * C_max * CONN_W, N_max,
                                  C_max, I, O, recurrent, &g);
        if (rc != 0) {
            genome_free(&g);
            return rc;
        }
        for (int r = 0; r < N_max; ++r) {
            order[(size_t)p * N_max + r] = g.order[r];
            level[(size_t)p * N_max + r] = g.level[r];
        }
        status[p] = g.status;
        genome_free(&g);
    }
    return 0;
}

/* Public: transformation of a whole population (order, level, status). */
int oracle_transform(int P, int N_max, int C_max, int I, int O,
                     const float *nodes, const float *conns, int32_t *order,
                     int32_t *level, uint32_t *status) {
    return transform_population(P, N_max, C_max, I, O, nodes, conns, 0, order, level,
                                status);
}

/* Public: the same checks for a recurrent network (cycles and self-loops are
 * allowed, so CYCLE is never set); order is the valid rows in key order and
 * level is 0 for every valid row. */
int oracle_transform_recurrent(int P, int N_max, int C_max, int I, int O,
                               const float *nodes, const float *conns, int32_t *order,
                               int32_t *level, uint32_t *status) {
    return transform_population(P, N_max, C_max, I, O, nodes, conns, 1, order, level,
                                status);
}

/* Incoming edges of every row, each list sorted by ascending source key. */
typedef struct {
    int *off;   /* [N_max + 1] */
    int *src;   /* [nedges] */
    float *w;   /* [nedges] */
} o_incoming;

static int build_incoming(const float *nodes, int N_max, const o_genome *g,
                          o_incoming *in) {
    in->off = (int *)calloc((size_t)N_max + 1, sizeof(int));
    in->src = (int *)malloc(sizeof(int) * (size_t)(g->nedges > 0 ? g->nedges : 1));
    in->w = (float *)malloc(sizeof(float) * (size_t)(g->nedges > 0 ? g->nedges : 1));
    if (!in->off || !in->src || !in->w) return ORACLE_E_NOMEM;
    int k = 0;
    for (int d = 0; d < N_max; ++d) {
        in->off[d] = k;
        for (int e = 0; e < g->nedges; ++e) {
            if (g->edges[e].dst != d) continue;
            /* insert keeping ascending source key */
            int j = k;
            float key = nodes[g->edges[e].src * NODE_W];
            while (j > in->off[d] && nodes[in->src[j - 1] * NODE_W] > key) {
                in->src[j] = in->src[j - 1];
                in->w[j] = in->w[j - 1];
                --j;
            }
            in->src[j] = g->edges[e].src;
            in->w[j] = g->edges[e].w;
            ++k;
        }
    }
    in->off[N_max] = k;
    return 0;
}

static void incoming_free(o_incoming *in) {
    free(in->off);
    free(in->src);
    free(in->w);
}

/* The calculation stage, instantiated for double (with the fp32 error bound
 * beta) and for float. */
#define REAL double
#define SUFFIX(name) name##_f64
#define WITH_BETA 1
#define R_TANH tanh
#define R_EXP exp
#define R_SIN sin
#define R_FABS fabs
#include "neat_oracle_forward.inc"
#undef REAL
#undef SUFFIX
#undef WITH_BETA
#undef R_TANH
#undef R_EXP
#undef R_SIN
#undef R_FABS

#define REAL float
#define SUFFIX(name) name##_f32
#define WITH_BETA 0
#define R_TANH tanhf
#define R_EXP expf
#define R_SIN sinf
#define R_FABS fabsf
#include "neat_oracle_forward.inc"
#undef REAL
#undef SUFFIX
#undef WITH_BETA
#undef R_TANH
#undef R_EXP
#undef R_SIN
#undef R_FABS

/*
 * Compatibility distance (the step before the transformation in each
 * generation: speciation divides the population by distances between
 * networks, Appendix (NEAT algorithm); Appendix A names the coefficients
 * compatibility_disjoint and compatibility_homologous).  The form is NEAT's
 * (a reading; the paper gives no formula):
 *   genes: node rows with a key, connection rows with an in key (enabled or
 *   not); an A gene is homologous when B has a gene with the same key (node)
 *   or (in, out) keys (connection), its partner being the first such B row;
 *   node gene distance |bias - bias'| + |response - response'| + [act != act']
 *   + [agg != agg']; connection gene distance |w - w'| + [enabled != enabled'];
 *   per kind: (cd (|A| + |B| - 2 h) + ch sum of homologous distances) /
 *   max(|A|, |B|), 0 when both are empty; distance = node part + connection
 *   part.
 * out [P][Q] is the distance of genome p to representative q; bound [P][Q]
 * (nullable) a first-order bound on the error of an fp32 evaluation.
 */
static void kind_distance(const float *a, int na_rows, const float *b, int nb_rows, int w,
                          int node, double cd, double ch, double *d, double *e) {
    int na = 0, nb = 0, h = 0;
    double hsum = 0.0;
    for (int r = 0; r < nb_rows; ++r)
        if (!isnan(b[(size_t)r * w])) nb++;
    for (int r = 0; r < na_rows; ++r) {
        const float *x = a + (size_t)r * w;
        if (isnan(x[0])) continue;
        na++;
        for (int q = 0; q < nb_rows; ++q) {
            const float *y = b + (size_t)q * w;
            if (isnan(y[0])) continue;
            if (node ? (x[0] == y[0]) : (x[0] == y[0] && x[1] == y[1])) {
                h++;
                if (node)
                    hsum += fabs((double)x[1] - (double)y[1]) + fabs((double)x[2] - (double)y[2]) +
                            (x[3] != y[3]) + (x[4] != y[4]);
                else
                    hsum += fabs((double)x[3] - (double)y[3]) + (x[2] != y[2]);
                break;
            }
        }
    }
    const int m = na > nb ? na : nb;
    if (m == 0) {
        *d = 0.0;
        *e = 0.0;
        return;
    }
    const double num = cd * (double)(na + nb - 2 * h) + ch * hsum;
    *d = num / (double)m;
    /* fp32: each term rounded once, the sum of h terms, the products, the
     * division: (h + 6) u relative to the absolute numerator */
    const double u = 1.0 / 16777216.0;
    *e = (double)(h + 6) * u * (fabs(cd) * fabs((double)(na + nb - 2 * h)) + fabs(ch) * hsum) /
         (double)m;
}

int oracle_distance(int P, int Q, int N_max, int C_max, const float *nodes,
                    const float *conns, const float *rnodes, const float *rconns, double cd,
                    double ch, double *out, double *bound) {
    if (P < 0 || Q < 0 || N_max < 1 || C_max < 0) return ORACLE_E_INVALID;
    for (int p = 0; p < P; ++p)
        for (int q = 0; q < Q; ++q) {
            double dn, en, dc, ec;
            kind_distance(nodes + (size_t)p * N_max * NODE_W, N_max,
                          rnodes + (size_t)q * N_max * NODE_W, N_max, NODE_W, 1, cd, ch, &dn,
                          &en);
            kind_distance(conns + (size_t)p * C_max * CONN_W, C_max,
                          rconns + (size_t)q * C_max * CONN_W, C_max, CONN_W, 0, cd, ch, &dc,
                          &ec);
            out[(size_t)p * Q + q] = dn + dc;
            if (bound)
                bound[(size_t)p * Q + q] = en + ec + fabs(dn + dc) / 16777216.0;
        }
    return 0;
}

/*
 * Crossover (Section 3.2: mutation and crossover become tensor writes of
 * rows and attributes; the gene alignment is NEAT's, a reading): the child
 * of (p1, p2), p1 the fitter parent, keeps p1's rows (keys, and the
 * disjoint and excess genes of p1); a p1 gene that is homologous in p2
 * (same node key, or same (in, out) keys; the partner is p2's first such
 * row) takes all of its non-key columns from the partner when the gene's
 * random number r < 0.5, else from p1.  Rows absent in p1 stay NaN.
 *   parents: nodes [Pp][N][5], conns [Pp][C][4]; pairs [Pc][2] (p1, p2);
 *   rn [Pc][N], rc [Pc][C] uniform numbers per p1 row; children written to
 *   cn [Pc][N][5], cc [Pc][C][4].
 */
int oracle_crossover(int Pc, int N_max, int C_max, const float *nodes, const float *conns,
                     const int32_t *pairs, const float *rn, const float *rc, float *cn,
                     float *cc) {
    if (Pc < 0 || N_max < 1 || C_max < 0) return ORACLE_E_INVALID;
    for (int k = 0; k < Pc; ++k) {
        const int a = pairs[2 * k], b = pairs[2 * k + 1];
        const float *an = nodes + (size_t)a * N_max * NODE_W;
        const float *bn = nodes + (size_t)b * N_max * NODE_W;
        const float *ac = conns + (size_t)a * C_max * CONN_W;
        const float *bc = conns + (size_t)b * C_max * CONN_W;
        float *on = cn + (size_t)k * N_max * NODE_W;
        float *oc = cc + (size_t)k * C_max * CONN_W;
        for (int r = 0; r < N_max; ++r) {
            const float *x = an + (size_t)r * NODE_W;
            memcpy(on + (size_t)r * NODE_W, x, sizeof(float) * NODE_W);
            if (isnan(x[0]) || !(rn[(size_t)k * N_max + r] < 0.5f)) continue;
            for (int q = 0; q < N_max; ++q) {
                const float *y = bn + (size_t)q * NODE_W;
                if (!isnan(y[0]) && y[0] == x[0]) {
                    memcpy(on + (size_t)r * NODE_W + 1, y + 1, sizeof(float) * (NODE_W - 1));
                    break;
                }
            }
        }
        for (int r = 0; r < C_max; ++r) {
            const float *x = ac + (size_t)r * CONN_W;
            memcpy(oc + (size_t)r * CONN_W, x, sizeof(float) * CONN_W);
            if (isnan(x[0]) || !(rc[(size_t)k * C_max + r] < 0.5f)) continue;
            for (int q = 0; q < C_max; ++q) {
                const float *y = bc + (size_t)q * CONN_W;
                if (!isnan(y[0]) && y[0] == x[0] && y[1] == x[1]) {
                    memcpy(oc + (size_t)r * CONN_W + 2, y + 2, sizeof(float) * (CONN_W - 2));
                    break;
                }
            }
        }
    }
    return 0;
}

/*
 * Tensorized genome edits (Section 3.2): node addition writes the new row at
 * the first NaN row of the node tensor, node removal writes NaN over a row,
 * connection addition and removal do the same on the connection tensor,
 * and an attribute write sets one column of a row (node columns 1..4 after
 * the key; connection columns 2..3, the enabled flag and the weight).  The
 * edits of a genome apply in their order; genomes are independent.
 *   an edit is 9 words: genome, op, row, column (int32), then five floats
 *   v: the new row for an addition (node: key, bias, response, act, agg;
 *   connection: in, out, enabled, weight), v[0] for an attribute write;
 *   op: 0 node add, 1 node removal, 2 connection add, 3 connection
 *   removal, 4 node attribute, 5 connection attribute.
 *   applied [n] i32 (written): 1 when the edit changed the tensors, 0 when
 *   it could not apply (no NaN row left, a row, column, op or genome out of
 *   range).
 */
typedef struct {
    int32_t genome, op, row, column;
    float v[5];
} o_edit;

int oracle_edit(int P, int N_max, int C_max, float *nodes, float *conns, int n,
                const void *edits_, int32_t *applied) {
    if (P < 0 || N_max < 1 || C_max < 0 || n < 0) return ORACLE_E_INVALID;
    const o_edit *edits = (const o_edit *)edits_;
    for (int e = 0; e < n; ++e) {
        const o_edit *d = edits + e;
        applied[e] = 0;
        if (d->genome < 0 || d->genome >= P) continue;
        float *gn = nodes + (size_t)d->genome * N_max * NODE_W;
        float *gc = conns + (size_t)d->genome * C_max * CONN_W;
        if (d->op == 0 || d->op == 2) {
            float *t = d->op == 0 ? gn : gc;
            const int rows = d->op == 0 ? N_max : C_max, w = d->op == 0 ? NODE_W : CONN_W;
            int r = 0;
            while (r < rows && !isnan(t[(size_t)r * w])) ++r;
            if (r == rows) continue;
            for (int c = 0; c < w; ++c) t[(size_t)r * w + c] = d->v[c];
            applied[e] = 1;
        } else if (d->op == 1 || d->op == 3) {
            float *t = d->op == 1 ? gn : gc;
            const int rows = d->op == 1 ? N_max : C_max, w = d->op == 1 ? NODE_W : CONN_W;
            if (d->row < 0 || d->row >= rows) continue;
            for (int c = 0; c < w; ++c) t[(size_t)d->row * w + c] = NAN;
            applied[e] = 1;
        } else if (d->op == 4) {
            if (d->row < 0 || d->row >= N_max || d->column < 1 || d->column > 4) continue;
            gn[(size_t)d->row * NODE_W + d->column] = d->v[0];
            applied[e] = 1;
        } else if (d->op == 5) {
            if (d->row < 0 || d->row >= C_max || d->column < 2 || d->column > 3) continue;
            gc[(size_t)d->row * CONN_W + d->column] = d->v[0];
            applied[e] = 1;
        }
    }
    return 0;
}
