/*
 * Kripke census oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of what the census and
 * split paths compute.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the product path never calls it.  It shares
 * no code, header, table or constant generator with the HIP library: it has
 * its own bytecode decoder, its own frame and valuation decoding, and it
 * evaluates formulas by the recursive satisfaction definition of Section 2
 * over explicit boolean arrays (no bitmask arithmetic, Section 5: the
 * independent recursive checker over explicit sets).
 *
 * Definitions followed:
 *   - Satisfaction (Section 2): M,w |= BOX phi iff every R-successor v of w
 *     satisfies phi; M,w |= DIA phi iff some R-successor satisfies phi.
 *     Dead ends therefore make BOX true and DIA false.
 *   - Frame classes (Section 2): K all frames, T reflexive, S4 reflexive and
 *     transitive (preorders), S5 equivalence relations.  K4 (transitive only)
 *     is supported for tests; it appears in the paper's ablation table.
 *   - Census of one (class, n) layer (Algorithm 1): for every frame of the
 *     class and every valuation, a countermodel is a world where the formula
 *     is false; the failure count counts (frame, valuation) pairs with at
 *     least one falsifying world.
 *   - Certificate (Definition 1, Proposition 3): (phi, n, succ, V, w, C) is
 *     valid iff the frame is in C and M,w does not satisfy phi.
 *   - Split (Definition 2, Proposition 5): the first model where phi and psi
 *     take different truth values.
 *
 * Readings where the paper leaves the encoding open:
 *   - frame index f: bit (w*n + v) of f is R(w, v) (row-major adjacency);
 *   - valuation index val: bit (i*n + w) of val is "p_i true at w";
 *   - "first" countermodel: least (frame, valuation, world) in lexicographic
 *     order, packed as key = frame << (nvars*n + 4) | val << 4 | world;
 *   - filtered classes keep the raw frame index (not a rank in the class).
 *
 * Bytecode (postfix, one byte per node): 0 TOP, 1 BOT, 2+i VAR p_i (i < 4),
 * 6 NOT, 7 AND, 8 OR, 9 IMP, 10 BOX, 11 DIA, 12 IFF.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define ORC_MAXN 16
#define ORC_MAXNODES 512

enum { O_TOP = 0, O_BOT = 1, O_VAR = 2, O_NOT = 6, O_AND = 7, O_OR = 8, O_IMP = 9,
       O_BOX = 10, O_DIA = 11, O_IFF = 12 };
enum { C_K = 0, C_T = 1, C_S4 = 2, C_S5 = 3, C_K4 = 4 };

typedef struct {
    int op;    /* O_* ; variables use O_VAR with `var` set */
    int var;
    int left;  /* child indices into the node array, -1 if absent */
    int right;
} Node;

typedef struct {
    Node nodes[ORC_MAXNODES];
    int count;
    int root;
} Tree;

typedef struct {
    int n;
    int R[ORC_MAXN][ORC_MAXN];   /* R[w][v] = 1 iff w R v */
    int V[4][ORC_MAXN];          /* V[i][w] = 1 iff p_i holds at w */
} Model;

/* ------------------------------------------------------------ decoding */
/* Build a tree from postfix bytecode.  Returns 0, or -2 on a malformed
 * program (unknown opcode, stack underflow, leftover operands, var >= nvars). */
static int decode(const uint8_t *code, uint32_t len, uint32_t nvars, Tree *t) {
    int stack[ORC_MAXNODES];
    int sp = 0;
    if (len == 0 || len > ORC_MAXNODES) return -2;
    t->count = 0;
    for (uint32_t i = 0; i < len; ++i) {
        int b = code[i];
        Node nd;
        nd.var = -1;
        nd.left = nd.right = -1;
        if (b == O_TOP || b == O_BOT) {
            nd.op = b;
        } else if (b >= 2 && b <= 5) {
            nd.op = O_VAR;
            nd.var = b - 2;
            if ((uint32_t)nd.var >= nvars) return -2;
        } else if (b == O_NOT || b == O_BOX || b == O_DIA) {
            if (sp < 1) return -2;
            nd.op = b;
            nd.left = stack[--sp];
        } else if (b == O_AND || b == O_OR || b == O_IMP || b == O_IFF) {
            if (sp < 2) return -2;
            nd.op = b;
            nd.right = stack[--sp];
            nd.left = stack[--sp];
        } else {
            return -2;
        }
        t->nodes[t->count] = nd;
        stack[sp++] = t->count;
        t->count++;
    }
    if (sp != 1) return -2;
    t->root = stack[0];
    return 0;
}

static void frame_from_index(uint64_t f, int n, Model *m) {
    m->n = n;
    for (int w = 0; w < n; ++w)
        for (int v = 0; v < n; ++v)
            m->R[w][v] = (int)((f >> (w * n + v)) & 1u);
}

static void frame_from_succ(const uint32_t *succ, int n, Model *m) {
    m->n = n;
    for (int w = 0; w < n; ++w)
        for (int v = 0; v < n; ++v)
            m->R[w][v] = (int)((succ[w] >> v) & 1u);
}

static void valuation_from_index(uint64_t val, int nvars, Model *m) {
    for (int i = 0; i < nvars; ++i)
        for (int w = 0; w < m->n; ++w)
            m->V[i][w] = (int)((val >> (i * m->n + w)) & 1u);
}

/* --------------------------------------------------------- frame classes */
static int reflexive(const Model *m) {
    for (int w = 0; w < m->n; ++w)
        if (!m->R[w][w]) return 0;
    return 1;
}

static int transitive(const Model *m) {
    for (int u = 0; u < m->n; ++u)
        for (int v = 0; v < m->n; ++v)
            for (int w = 0; w < m->n; ++w)
                if (m->R[u][v] && m->R[v][w] && !m->R[u][w]) return 0;
    return 1;
}

static int symmetric(const Model *m) {
    for (int u = 0; u < m->n; ++u)
        for (int v = 0; v < m->n; ++v)
            if (m->R[u][v] != m->R[v][u]) return 0;
    return 1;
}

static int in_class(const Model *m, int cls) {
    switch (cls) {
    case C_K: return 1;
    case C_T: return reflexive(m);
    case C_S4: return reflexive(m) && transitive(m);
    case C_S5: return reflexive(m) && transitive(m) && symmetric(m);
    case C_K4: return transitive(m);
    default: return 0;
    }
}

/* ------------------------------------------------------------ semantics */
/* Truth set of node `i`: out[w] = 1 iff M,w |= node, computed recursively
 * from the children's truth sets by the satisfaction clauses. */
static void truth_set(const Model *m, const Tree *t, int i, int out[ORC_MAXN]) {
    const Node *nd = &t->nodes[i];
    int a[ORC_MAXN], b[ORC_MAXN];
    int n = m->n;
    switch (nd->op) {
    case O_TOP:
        for (int w = 0; w < n; ++w) out[w] = 1;
        return;
    case O_BOT:
        for (int w = 0; w < n; ++w) out[w] = 0;
        return;
    case O_VAR:
        for (int w = 0; w < n; ++w) out[w] = m->V[nd->var][w];
        return;
    case O_NOT:
        truth_set(m, t, nd->left, a);
        for (int w = 0; w < n; ++w) out[w] = !a[w];
        return;
    case O_BOX:
        truth_set(m, t, nd->left, a);
        for (int w = 0; w < n; ++w) {
            int all = 1;
            for (int v = 0; v < n; ++v)
                if (m->R[w][v] && !a[v]) all = 0;
            out[w] = all;
        }
        return;
    case O_DIA:
        truth_set(m, t, nd->left, a);
        for (int w = 0; w < n; ++w) {
            int some = 0;
            for (int v = 0; v < n; ++v)
                if (m->R[w][v] && a[v]) some = 1;
            out[w] = some;
        }
        return;
    default:
        break;
    }
    truth_set(m, t, nd->left, a);
    truth_set(m, t, nd->right, b);
    for (int w = 0; w < n; ++w) {
        switch (nd->op) {
        case O_AND: out[w] = a[w] && b[w]; break;
        case O_OR: out[w] = a[w] || b[w]; break;
        case O_IMP: out[w] = !a[w] || b[w]; break;
        case O_IFF: out[w] = (a[w] != 0) == (b[w] != 0); break;
        default: out[w] = 0; break;
        }
    }
}

/* Pointwise satisfaction M,w |= node, the literal recursive definition
 * (Proposition 3's checker).  Exponential in modal depth; used for single
 * pointed models only. */
static int sat_at(const Model *m, const Tree *t, int i, int w) {
    const Node *nd = &t->nodes[i];
    switch (nd->op) {
    case O_TOP: return 1;
    case O_BOT: return 0;
    case O_VAR: return m->V[nd->var][w];
    case O_NOT: return !sat_at(m, t, nd->left, w);
    case O_AND: return sat_at(m, t, nd->left, w) && sat_at(m, t, nd->right, w);
    case O_OR: return sat_at(m, t, nd->left, w) || sat_at(m, t, nd->right, w);
    case O_IMP: return !sat_at(m, t, nd->left, w) || sat_at(m, t, nd->right, w);
    case O_IFF: return sat_at(m, t, nd->left, w) == sat_at(m, t, nd->right, w);
    case O_BOX:
        for (int v = 0; v < m->n; ++v)
            if (m->R[w][v] && !sat_at(m, t, nd->left, v)) return 0;
        return 1;
    case O_DIA:
        for (int v = 0; v < m->n; ++v)
            if (m->R[w][v] && sat_at(m, t, nd->left, v)) return 1;
        return 0;
    default: return 0;
    }
}

/* -------------------------------------------------------------- census */
typedef struct {
    const Tree *tree;
    int n, cls, nvars, stop_at_first;
    uint64_t f0, f1;
    uint64_t first_key, fail_count;
} CensusJob;

static void census_range(CensusJob *job) {
    Model m;
    int truth[ORC_MAXN];
    int n = job->n;
    uint64_t nval = 1ull << (job->nvars * n);
    job->first_key = UINT64_MAX;
    job->fail_count = 0;
    for (uint64_t f = job->f0; f < job->f1; ++f) {
        frame_from_index(f, n, &m);
        if (!in_class(&m, job->cls)) continue;
        for (uint64_t val = 0; val < nval; ++val) {
            valuation_from_index(val, job->nvars, &m);
            truth_set(&m, job->tree, job->tree->root, truth);
            int bad = -1;
            for (int w = 0; w < n; ++w)
                if (!truth[w]) { bad = w; break; }
            if (bad < 0) continue;
            job->fail_count++;
            if (job->first_key == UINT64_MAX) {
                job->first_key = (f << (job->nvars * n + 4)) | (val << 4) | (uint64_t)bad;
                if (job->stop_at_first) return;
            }
        }
    }
}

static void *census_thread(void *p) {
    census_range((CensusJob *)p);
    return NULL;
}

int orc_hardware_threads(void) {
    long c = sysconf(_SC_NPROCESSORS_ONLN);
    return c > 0 ? (int)c : 1;
}

/* Census of one formula over frames [frame_begin, frame_end) of the class.
 * nthreads <= 0 uses every online core.  Returns the number of threads used,
 * or a negative status (-1 bad sizes, -2 malformed program). */
int orc_census(const uint8_t *code, uint32_t len, uint32_t n, uint32_t cls, uint32_t nvars,
               uint64_t frame_begin, uint64_t frame_end, int stop_at_first, int nthreads,
               uint64_t *first_key, uint64_t *fail_count) {
    Tree *tree = (Tree *)malloc(sizeof(Tree));
    if (!tree) return -1;
    if (n < 1 || n > 8 || nvars > 4 || cls > C_K4 || n * n + nvars * n + 4 > 64 ||
        frame_end > (n * n >= 64 ? UINT64_MAX : (1ull << (n * n))) || frame_begin > frame_end) {
        free(tree);
        return -1;
    }
    if (decode(code, len, nvars, tree) != 0) { free(tree); return -2; }
    if (nthreads <= 0) nthreads = orc_hardware_threads();
    uint64_t span = frame_end - frame_begin;
    if ((uint64_t)nthreads > span) nthreads = span ? (int)span : 1;
    CensusJob *jobs = (CensusJob *)calloc((size_t)nthreads, sizeof(CensusJob));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int i = 0; i < nthreads; ++i) {
        jobs[i].tree = tree;
        jobs[i].n = (int)n;
        jobs[i].cls = (int)cls;
        jobs[i].nvars = (int)nvars;
        jobs[i].stop_at_first = stop_at_first;
        jobs[i].f0 = frame_begin + span * (uint64_t)i / (uint64_t)nthreads;
        jobs[i].f1 = frame_begin + span * (uint64_t)(i + 1) / (uint64_t)nthreads;
    }
    if (nthreads == 1) {
        census_range(&jobs[0]);
    } else {
        for (int i = 0; i < nthreads; ++i) pthread_create(&th[i], NULL, census_thread, &jobs[i]);
        for (int i = 0; i < nthreads; ++i) pthread_join(th[i], NULL);
    }
    uint64_t key = UINT64_MAX, cnt = 0;
    for (int i = 0; i < nthreads; ++i) {
        if (jobs[i].first_key < key) key = jobs[i].first_key;
        cnt += jobs[i].fail_count;
    }
    *first_key = key;
    *fail_count = cnt;
    free(jobs);
    free(th);
    free(tree);
    return nthreads;
}

/* Number of frames on n worlds in the class (brute force over all indices). */
int64_t orc_class_size(uint32_t n, uint32_t cls) {
    Model m;
    if (n < 1 || n > 5) return -1;
    int64_t c = 0;
    for (uint64_t f = 0; f < (1ull << (n * n)); ++f) {
        frame_from_index(f, (int)n, &m);
        c += in_class(&m, (int)cls);
    }
    return c;
}

int orc_in_class(const uint32_t *succ, uint32_t n, uint32_t cls) {
    Model m;
    if (n < 1 || n > ORC_MAXN) return -1;
    frame_from_succ(succ, (int)n, &m);
    return in_class(&m, (int)cls);
}

/* Truth set of phi at the model (succ, val): out[w] in {0,1}. */
int orc_truth_set(const uint8_t *code, uint32_t len, uint32_t n, const uint32_t *succ,
                  uint32_t nvars, uint64_t val, uint8_t *out) {
    Tree *tree = (Tree *)malloc(sizeof(Tree));
    Model m;
    int truth[ORC_MAXN];
    if (!tree || n < 1 || n > ORC_MAXN || nvars > 4) { free(tree); return -1; }
    if (decode(code, len, nvars, tree) != 0) { free(tree); return -2; }
    frame_from_succ(succ, (int)n, &m);
    valuation_from_index(val, (int)nvars, &m);
    truth_set(&m, tree, tree->root, truth);
    for (uint32_t w = 0; w < n; ++w) out[w] = (uint8_t)truth[w];
    free(tree);
    return 0;
}

/* Pointwise satisfaction M,w |= phi by the literal recursive definition. */
int orc_sat_at(const uint8_t *code, uint32_t len, uint32_t n, const uint32_t *succ,
               uint32_t nvars, uint64_t val, uint32_t world) {
    Tree *tree = (Tree *)malloc(sizeof(Tree));
    Model m;
    if (!tree || n < 1 || n > ORC_MAXN || nvars > 4 || world >= n) { free(tree); return -1; }
    if (decode(code, len, nvars, tree) != 0) { free(tree); return -2; }
    frame_from_succ(succ, (int)n, &m);
    valuation_from_index(val, (int)nvars, &m);
    int r = sat_at(&m, tree, tree->root, (int)world);
    free(tree);
    return r;
}

/* Certificate check (Definition 1): 1 if the frame is in the class and
 * M,w does not satisfy phi, 0 if not, negative on bad input. */
int orc_check_certificate(const uint8_t *code, uint32_t len, uint32_t n, const uint32_t *succ,
                          uint32_t nvars, uint64_t val, uint32_t world, uint32_t cls) {
    Model m;
    if (n < 1 || n > ORC_MAXN) return -1;
    frame_from_succ(succ, (int)n, &m);
    if (!in_class(&m, (int)cls)) return 0;
    int s = orc_sat_at(code, len, n, succ, nvars, val, world);
    if (s < 0) return s;
    return s ? 0 : 1;
}

/* Split of (phi, psi) over an explicit frame list (uint32 succ[nframes][n]):
 * the least (position, valuation, world) where the two truth values differ,
 * packed as position << (nvars*n + 4) | val << 4 | world; UINT64_MAX if the
 * formulas agree everywhere on the list. */
int orc_split(const uint8_t *phi, uint32_t len_phi, const uint8_t *psi, uint32_t len_psi,
              const uint32_t *frames, uint64_t nframes, uint32_t n, uint32_t nvars,
              uint64_t *first_key) {
    Tree *a = (Tree *)malloc(sizeof(Tree));
    Tree *b = (Tree *)malloc(sizeof(Tree));
    Model m;
    int ta[ORC_MAXN], tb[ORC_MAXN];
    int rc = 0;
    *first_key = UINT64_MAX;
    if (!a || !b || n < 1 || n > ORC_MAXN || nvars > 4 || nvars * n > 40) { rc = -1; goto done; }
    if (decode(phi, len_phi, nvars, a) != 0 || decode(psi, len_psi, nvars, b) != 0) {
        rc = -2;
        goto done;
    }
    for (uint64_t k = 0; k < nframes; ++k) {
        frame_from_succ(frames + k * n, (int)n, &m);
        for (uint64_t val = 0; val < (1ull << (nvars * n)); ++val) {
            valuation_from_index(val, (int)nvars, &m);
            truth_set(&m, a, a->root, ta);
            truth_set(&m, b, b->root, tb);
            for (uint32_t w = 0; w < n; ++w) {
                if (ta[w] != tb[w]) {
                    *first_key = (k << (nvars * n + 4)) | (val << 4) | w;
                    goto done;
                }
            }
        }
    }
done:
    free(a);
    free(b);
    return rc;
}

/* Truth bits at sampled pointed models: sample s is (n, frame index, val,
 * world) packed as n << 60 | frame << 24 | val << 4 | world (n <= 3, so the
 * frame index fits 9 bits and the valuation 6 bits).  Bit s of sig row i is
 * M,w |= phi_i.  sig is uint64[nformulas][(nsamples + 63) / 64]. */
int orc_signatures(const uint8_t *code, const uint32_t *offsets, uint32_t nformulas,
                   uint32_t nvars, const uint64_t *samples, uint32_t nsamples, uint64_t *sig) {
    Tree *tree = (Tree *)malloc(sizeof(Tree));
    Model m;
    uint32_t words = (nsamples + 63) / 64;
    if (!tree) return -1;
    memset(sig, 0, sizeof(uint64_t) * (size_t)words * nformulas);
    for (uint32_t i = 0; i < nformulas; ++i) {
        if (decode(code + offsets[i], offsets[i + 1] - offsets[i], nvars, tree) != 0) {
            free(tree);
            return -2;
        }
        for (uint32_t s = 0; s < nsamples; ++s) {
            uint64_t smp = samples[s];
            int n = (int)(smp >> 60);
            uint64_t f = (smp >> 24) & 0xFFFFFFFFFull;
            uint64_t val = (smp >> 4) & 0xFFFFFu;
            int w = (int)(smp & 15u);
            frame_from_index(f, n, &m);
            valuation_from_index(val, (int)nvars, &m);
            if (sat_at(&m, tree, tree->root, w)) sig[(size_t)i * words + s / 64] |= 1ull << (s % 64);
        }
    }
    free(tree);
    return 0;
}
