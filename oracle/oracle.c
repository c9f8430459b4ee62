/*
 * Plain FP64 CPU oracle for the sample-many path of the frame-factored
 * near-Clifford simulator ("Clifft", Chase & Labib).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file.  Only tests/, the smoke check and the benchmark's
 * cpu_baseline leg use it.  It shares no code with the HIP path.
 *
 * It is written for clarity, not speed: bits are one byte each, every
 * virtual Clifford gate is applied on its own, the active vector is
 * renormalised after every expansion and measurement, and the global scalar
 * gamma is tracked exactly (Definition 2, Eq. 2).
 *
 * Paper passages followed (section / equation / appendix):
 *   Definition 1 (Heisenberg mapping, Eq. 1)          -> map_pauli()
 *   Definition 2 (frame-factored state, Eq. 2)        -> struct shot_state
 *   Lemma 1 + Appendix A (Pauli localization)         -> localize()
 *   Lemma 2 (dormant invariance)                      -> check_* asserts
 *   Section 2.4 + Appendix B.1 (rotations, 3 cases)   -> compile_rotation(), exec O_EXPAND/O_ROT/O_PHASE
 *   Section 2.4 + Appendix B.2 (measurements)         -> compile_measure(), exec O_M*
 *   Section 2.4 + Appendix B.3 (conditional Paulis)   -> exec O_NOISE/O_CPAULI
 *   Theorem 1 (coordinate/amplitude decoupling)       -> compile is shot-independent
 *   Section 3.2 (sparse error bottleneck: cumulative
 *                hazard, jump to next fault)          -> draw_faults()
 *
 * Stochastic contract (the readings of the paper this oracle follows):
 *   Philox4x32-10 (Salmon et al., SC'11), key = (seed_lo, seed_hi),
 *   counter = (index, purpose, shot_lo, shot_hi).
 *   Every recorded outcome is m = m_ref XOR pn, where pn is the commutation
 *   parity of the noise-only Pauli frame with the measured observable and
 *   m_ref is: the reference parity (deterministic measurement), a Philox bit
 *   (dormant random measurement), or [u < P(m_ref = 1)] (active measurement).
 */
#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define MAXQ 4096
#define CHUNK 4096

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).                  */
/* ------------------------------------------------------------------ */
static void philox(const uint32_t ctr[4], uint32_t k0, uint32_t k1, uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

#define PURPOSE_NOISE 0x4E000000u /* | chunk */
#define PURPOSE_RBIT 0x52000000u
#define PURPOSE_AMEAS 0x41000000u
#define PURPOSE_STRAT 0x53000000u /* stratified sampling: fault i of the shot */

static void draw(uint32_t index, uint32_t purpose, uint64_t shot, uint64_t seed, uint32_t out[4])
{
    uint32_t ctr[4] = {index, purpose, (uint32_t)shot, (uint32_t)(shot >> 32)};
    philox(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), out);
}

static double uniform53(const uint32_t w[4])
{
    uint64_t v = ((uint64_t)w[1] << 32) | (uint64_t)w[0];
    return (double)(v >> 11) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------ */
/* Hermitian Pauli strings: (-1)^r * prod_j sigma(x_j, z_j), with      */
/* sigma(1,0)=X, sigma(0,1)=Z, sigma(1,1)=Y.                           */
/* ------------------------------------------------------------------ */
typedef struct {
    int r;
    uint8_t *x, *z;
} pauli;

static pauli pauli_new(int n)
{
    pauli p;
    p.r = 0;
    p.x = (uint8_t *)calloc((size_t)n, 1);
    p.z = (uint8_t *)calloc((size_t)n, 1);
    return p;
}
static void pauli_free(pauli *p) { free(p->x); free(p->z); }
static void pauli_copy(pauli *dst, const pauli *src, int n)
{
    dst->r = src->r;
    memcpy(dst->x, src->x, (size_t)n);
    memcpy(dst->z, src->z, (size_t)n);
}

/* Exponent g of i in sigma(x1,z1) * sigma(x2,z2) = i^g sigma(x1^x2, z1^z2)
 * for one qubit (Aaronson & Gottesman 2004, function g). */
static int g_exp(int x1, int z1, int x2, int z2)
{
    if (!x1 && !z1) return 0;
    if (x1 && z1) return z2 - x2;
    if (x1 && !z1) return z2 * (2 * x2 - 1);
    return x2 * (1 - 2 * z2);
}

/* a <- i^extra * a * b ; returns the resulting power of i (0..3).  For a
 * product of two Hermitian Paulis times i^extra that is again Hermitian the
 * result is even and folded into a->r. */
static int pauli_mul_into(pauli *a, const pauli *b, int n, int extra)
{
    int e = extra + 2 * a->r + 2 * b->r;
    for (int j = 0; j < n; j++) {
        e += g_exp(a->x[j], a->z[j], b->x[j], b->z[j]);
        a->x[j] ^= b->x[j];
        a->z[j] ^= b->z[j];
    }
    e = ((e % 4) + 4) % 4;
    a->r = 0;
    return e;
}

/* Conjugation rules P -> G P G^dagger for the virtual gates used by the
 * localization sequences (Lemma 1, Appendix A), on one Hermitian Pauli. */
static void conj_cx(pauli *p, int c, int t)
{
    p->r ^= p->x[c] & p->z[t] & (p->x[t] ^ p->z[c] ^ 1);
    p->x[t] ^= p->x[c];
    p->z[c] ^= p->z[t];
}
static void conj_cz(pauli *p, int a, int b)
{
    p->r ^= p->x[a] & p->x[b] & (p->z[a] ^ p->z[b]);
    p->z[a] ^= p->x[b];
    p->z[b] ^= p->x[a];
}
static void conj_s(pauli *p, int a)
{
    p->r ^= p->x[a] & p->z[a];
    p->z[a] ^= p->x[a];
}
static void conj_h(pauli *p, int a)
{
    p->r ^= p->x[a] & p->z[a];
    uint8_t t = p->x[a];
    p->x[a] = p->z[a];
    p->z[a] = t;
}

/* ------------------------------------------------------------------ */
/* Parsed circuit (flat, REPEAT unrolled).                             */
/* ------------------------------------------------------------------ */
enum {
    P_H, P_S, P_SDAG, P_X, P_Y, P_Z, P_CX, P_CZ, P_SWAP,
    P_ROTZ,          /* exp(-i theta Z_q) */
    P_M, P_MX, P_MR, P_R,
    P_NOISE,
    P_DET, P_OBS,
    P_PROT,          /* exp(-i theta P) for a Pauli product P (pq, pl) */
    P_MPP,           /* measurement of a Pauli product P (pq, pl) */
    P_CFEED,         /* Pauli pl[0] on qubit a if record refs[0] is 1 */
    P_GPHASE,        /* global phase exp(-i theta) */
    P_EXPVAL         /* expectation value of a Pauli product (probe obs) */
};
enum { N_DEP1, N_DEP2, N_XERR, N_YERR, N_ZERR };

typedef struct {
    int kind;
    int a, b;
    double arg;     /* rotation angle theta, or noise probability */
    int ntype;      /* noise type */
    int nref;
    int *refs;      /* absolute record indices (DET / OBS / CFEED) */
    int obs;
    int np;         /* Pauli product: qubits pq[i] with letters pl[i] ('X', 'Y', 'Z') */
    int *pq;
    char *pl;
} pop;

typedef struct {
    pop *ops;
    int n, cap;
    int nq;
    int nrec;
    int ndet, nobs;
    int nprobes;
    char err[256];
} circuit;

static void circ_push(circuit *c, pop o)
{
    if (c->n == c->cap) {
        c->cap = c->cap ? 2 * c->cap : 256;
        c->ops = (pop *)realloc(c->ops, (size_t)c->cap * sizeof(pop));
    }
    c->ops[c->n++] = o;
}

typedef struct {
    const char *s;
    size_t len, pos;
    int line;
} lexer;

static int next_line(lexer *L, char *buf, size_t cap)
{
    if (L->pos >= L->len) return 0;
    size_t i = 0;
    while (L->pos < L->len && L->s[L->pos] != '\n') {
        if (i + 1 < cap) buf[i++] = L->s[L->pos];
        L->pos++;
    }
    if (L->pos < L->len) L->pos++;
    buf[i] = 0;
    L->line++;
    char *h = strchr(buf, '#');
    if (h) *h = 0;
    return 1;
}

static char *trim(char *s)
{
    while (*s == ' ' || *s == '\t' || *s == '\r') s++;
    size_t n = strlen(s);
    while (n && (s[n - 1] == ' ' || s[n - 1] == '\t' || s[n - 1] == '\r')) s[--n] = 0;
    return s;
}

/* Parse the lines of one block until "}" (or end of text).  Instructions are
 * appended to the flat list; REPEAT blocks are unrolled by re-parsing. */
static int parse_block(circuit *c, lexer *L, int depth);

static int parse_instruction(circuit *c, char *line, lexer *L, int depth)
{
    char name[64];
    int ni = 0;
    char *p = line;
    while (*p && *p != ' ' && *p != '\t' && *p != '(' && ni < 63) name[ni++] = *p++;
    name[ni] = 0;
    for (int i = 0; name[i]; i++)
        if (name[i] >= 'a' && name[i] <= 'z') name[i] = (char)(name[i] - 'a' + 'A');
    double arg = 0, args[3] = {0, 0, 0};
    int has_arg = 0, nargs = 0;
    while (*p == ' ' || *p == '\t') p++;
    if (*p == '(') {
        char *e = strchr(p, ')');
        if (!e) { snprintf(c->err, sizeof c->err, "line %d: missing ')'", L->line); return -1; }
        *e = 0;
        char *a = p + 1;
        while (nargs < 3) {
            char *end;
            args[nargs] = strtod(a, &end);
            if (end == a) break;
            nargs++;
            while (*end == ' ' || *end == '\t') end++;
            if (*end != ',') break;
            a = end + 1;
        }
        arg = args[0];
        has_arg = nargs > 0;
        p = e + 1;
    }
    if (!strcmp(name, "REPEAT")) {
        long count = strtol(p, &p, 10);
        while (*p == ' ' || *p == '\t') p++;
        if (*p != '{') { snprintf(c->err, sizeof c->err, "line %d: REPEAT needs '{'", L->line); return -1; }
        size_t body_start = L->pos;
        int line0 = L->line;
        for (long r = 0; r < count; r++) {
            L->pos = body_start;
            L->line = line0;
            if (parse_block(c, L, depth + 1) < 0) return -1;
        }
        if (count == 0) { /* skip the body */
            circuit tmp;
            memset(&tmp, 0, sizeof tmp);
            if (parse_block(&tmp, L, depth + 1) < 0) { snprintf(c->err, sizeof c->err, "%s", tmp.err); return -1; }
            free(tmp.ops);
        }
        return 0;
    }
    if (!strcmp(name, "TICK") || !strcmp(name, "QUBIT_COORDS") || !strcmp(name, "SHIFT_COORDS")) return 0;

    /* targets; a Pauli product target (MPP, R_PAULI) is letters and qubits
     * joined by '*', as X0*Y3*Z5 */
    int tg[8192];
    int nt = 0;
    int isrec[8192];
    char *prods[1024];
    int nprod = 0;
    char *tok = strtok(p, " \t");
    while (tok) {
        if (nt >= 8192) { snprintf(c->err, sizeof c->err, "line %d: too many targets", L->line); return -1; }
        if ((tok[0] == 'X' || tok[0] == 'Y' || tok[0] == 'Z' || tok[0] == 'x' || tok[0] == 'y' || tok[0] == 'z')) {
            if (nprod >= 1024) { snprintf(c->err, sizeof c->err, "line %d: too many products", L->line); return -1; }
            prods[nprod++] = tok;
            tok = strtok(NULL, " \t");
            continue;
        }
        if (!strncmp(tok, "rec[", 4)) {
            tg[nt] = (int)strtol(tok + 4, NULL, 10);
            isrec[nt++] = 1;
        } else {
            char *end;
            long v = strtol(tok, &end, 10);
            if (end == tok || v < 0 || v >= MAXQ) { snprintf(c->err, sizeof c->err, "line %d: bad target '%s'", L->line, tok); return -1; }
            tg[nt] = (int)v;
            isrec[nt++] = 0;
            if (v + 1 > c->nq) c->nq = (int)v + 1;
        }
        tok = strtok(NULL, " \t");
    }
    pop o;
    memset(&o, 0, sizeof o);
    int is_prod_gate = !strcmp(name, "MPP") || !strcmp(name, "R_PAULI") || !strcmp(name, "EXP_VAL");
    if (nprod && !is_prod_gate) { snprintf(c->err, sizeof c->err, "line %d: Pauli product target on %s", L->line, name); return -1; }
    if (is_prod_gate) {
        /* MPP P...: one measurement per product; R_PAULI(phi) P...:
         * exp(-i phi P / 2) per product */
        if (nt) { snprintf(c->err, sizeof c->err, "line %d: %s takes Pauli products", L->line, name); return -1; }
        if (!strcmp(name, "R_PAULI") && !has_arg) { snprintf(c->err, sizeof c->err, "line %d: R_PAULI needs an angle", L->line); return -1; }
        for (int k = 0; k < nprod; k++) {
            pop q;
            memset(&q, 0, sizeof q);
            q.kind = !strcmp(name, "MPP") ? P_MPP : !strcmp(name, "EXP_VAL") ? P_EXPVAL : P_PROT;
            q.arg = arg / 2;
            if (q.kind == P_EXPVAL) q.obs = c->nprobes++;
            q.pq = (int *)malloc(sizeof(int) * 256);
            q.pl = (char *)malloc(256);
            char *s = prods[k];
            while (*s) {
                char letter = (char)(*s >= 'a' ? *s - 'a' + 'A' : *s);
                if (letter != 'X' && letter != 'Y' && letter != 'Z') { snprintf(c->err, sizeof c->err, "line %d: bad Pauli product", L->line); free(q.pq); free(q.pl); return -1; }
                char *end;
                long v = strtol(s + 1, &end, 10);
                if (end == s + 1 || v < 0 || v >= MAXQ || (*end && *end != '*') || q.np >= 256) { snprintf(c->err, sizeof c->err, "line %d: bad Pauli product", L->line); free(q.pq); free(q.pl); return -1; }
                for (int i = 0; i < q.np; i++)
                    if (q.pq[i] == (int)v) { snprintf(c->err, sizeof c->err, "line %d: repeated qubit in a product", L->line); free(q.pq); free(q.pl); return -1; }
                q.pq[q.np] = (int)v;
                q.pl[q.np++] = letter;
                if (v + 1 > c->nq) c->nq = (int)v + 1;
                s = *end ? end + 1 : end;
            }
            if (!q.np) { snprintf(c->err, sizeof c->err, "line %d: empty Pauli product", L->line); free(q.pq); free(q.pl); return -1; }
            circ_push(c, q);
            if (q.kind == P_MPP) c->nrec++;
        }
        return 0;
    }
    /* Pauli X, Y or Z on a qubit controlled by a measurement record
     * (feed-forward, Appendix B.3): CX rec[-k] q, CY rec[-k] q, CZ rec[-k] q
     * (CZ also q rec[-k]) */
    if ((!strcmp(name, "CX") || !strcmp(name, "CNOT") || !strcmp(name, "ZCX") || !strcmp(name, "CY") ||
         !strcmp(name, "ZCY") || !strcmp(name, "CZ") || !strcmp(name, "ZCZ"))) {
        int anyrec = 0;
        for (int i = 0; i < nt; i++) anyrec |= isrec[i];
        if (anyrec) {
            char letter = name[strlen(name) - 1] == 'Y' ? 'Y' : (!strcmp(name, "CZ") || !strcmp(name, "ZCZ")) ? 'Z' : 'X';
            if (nt % 2) { snprintf(c->err, sizeof c->err, "line %d: %s needs target pairs", L->line, name); return -1; }
            for (int i = 0; i < nt; i += 2) {
                int r = i, q = i + 1;
                if (letter == 'Z' && !isrec[i] && isrec[i + 1]) { r = i + 1; q = i; }
                if (!isrec[r] || isrec[q]) { snprintf(c->err, sizeof c->err, "line %d: feed-forward needs rec[-k] then a qubit", L->line); return -1; }
                if (tg[r] >= 0 || c->nrec + tg[r] < 0) { snprintf(c->err, sizeof c->err, "line %d: bad rec target", L->line); return -1; }
                pop q2;
                memset(&q2, 0, sizeof q2);
                q2.kind = P_CFEED;
                q2.a = tg[q];
                q2.nref = 1;
                q2.refs = (int *)malloc(sizeof(int));
                q2.refs[0] = c->nrec + tg[r];
                q2.np = 1;
                q2.pq = (int *)malloc(sizeof(int));
                q2.pl = (char *)malloc(1);
                q2.pq[0] = tg[q];
                q2.pl[0] = letter;
                circ_push(c, q2);
            }
            return 0;
        }
    }
    struct { const char *nm; int kind; int arity; } gates[] = {
        {"H", P_H, 1}, {"S", P_S, 1}, {"S_DAG", P_SDAG, 1}, {"X", P_X, 1}, {"Y", P_Y, 1}, {"Z", P_Z, 1},
        {"CX", P_CX, 2}, {"CNOT", P_CX, 2}, {"ZCX", P_CX, 2}, {"CZ", P_CZ, 2}, {"SWAP", P_SWAP, 2},
        {"M", P_M, 1}, {"MZ", P_M, 1}, {"MX", P_MX, 1}, {"MR", P_MR, 1}, {"MRZ", P_MR, 1},
        {"R", P_R, 1}, {"RZ", P_R, 1}};
    for (size_t g = 0; g < sizeof gates / sizeof gates[0]; g++) {
        if (strcmp(name, gates[g].nm)) continue;
        if (nt % gates[g].arity) { snprintf(c->err, sizeof c->err, "line %d: %s needs target pairs", L->line, name); return -1; }
        for (int i = 0; i < nt; i += gates[g].arity) {
            if (isrec[i]) { snprintf(c->err, sizeof c->err, "line %d: rec target on gate", L->line); return -1; }
            o.kind = gates[g].kind;
            o.a = tg[i];
            o.b = gates[g].arity == 2 ? tg[i + 1] : -1;
            if (o.b == o.a) { snprintf(c->err, sizeof c->err, "line %d: repeated qubit", L->line); return -1; }
            circ_push(c, o);
            if (o.kind == P_M || o.kind == P_MX || o.kind == P_MR) c->nrec++;
        }
        return 0;
    }
    /* non-Clifford rotations: T = exp(-i pi/8 Z), T_DAG = exp(+i pi/8 Z),
     * R_Z(phi) = exp(-i phi Z / 2) */
    if (!strcmp(name, "T") || !strcmp(name, "T_DAG") || !strcmp(name, "R_Z") || !strcmp(name, "RZ_ROT")) {
        double th;
        if (!strcmp(name, "T")) th = M_PI / 8;
        else if (!strcmp(name, "T_DAG")) th = -M_PI / 8;
        else {
            if (!has_arg) { snprintf(c->err, sizeof c->err, "line %d: R_Z needs an angle", L->line); return -1; }
            th = arg / 2;
        }
        for (int i = 0; i < nt; i++) {
            o.kind = P_ROTZ;
            o.a = tg[i];
            o.b = -1;
            o.arg = th;
            circ_push(c, o);
        }
        return 0;
    }
    /* R_X(phi) = exp(-i phi X / 2), R_Y(phi) = exp(-i phi Y / 2) */
    if (!strcmp(name, "R_X") || !strcmp(name, "R_Y")) {
        if (!has_arg) { snprintf(c->err, sizeof c->err, "line %d: %s needs an angle", L->line, name); return -1; }
        for (int i = 0; i < nt; i++) {
            pop q;
            memset(&q, 0, sizeof q);
            q.kind = P_PROT;
            q.arg = arg / 2;
            q.np = 1;
            q.pq = (int *)malloc(sizeof(int));
            q.pl = (char *)malloc(1);
            q.pq[0] = tg[i];
            q.pl[0] = name[2];
            circ_push(c, q);
        }
        return 0;
    }
    /* U3(theta, phi, lambda) = [[cos t, -e^{i l} sin t], [e^{i p} sin t,
     * e^{i (p + l)} cos t]] with t = theta / 2, which is
     * e^{i (p + l) / 2} R_Z(phi) R_Y(theta) R_Z(lambda) */
    if (!strcmp(name, "U3")) {
        if (nargs != 3) { snprintf(c->err, sizeof c->err, "line %d: U3 needs three angles", L->line); return -1; }
        for (int i = 0; i < nt; i++) {
            pop q;
            memset(&q, 0, sizeof q);
            q.kind = P_ROTZ; q.a = tg[i]; q.b = -1; q.arg = args[2] / 2;
            circ_push(c, q);
            memset(&q, 0, sizeof q);
            q.kind = P_PROT; q.arg = args[0] / 2; q.np = 1;
            q.pq = (int *)malloc(sizeof(int)); q.pl = (char *)malloc(1);
            q.pq[0] = tg[i]; q.pl[0] = 'Y';
            circ_push(c, q);
            memset(&q, 0, sizeof q);
            q.kind = P_ROTZ; q.a = tg[i]; q.b = -1; q.arg = args[1] / 2;
            circ_push(c, q);
            memset(&q, 0, sizeof q);
            q.kind = P_GPHASE; q.arg = -(args[1] + args[2]) / 2;
            circ_push(c, q);
        }
        return 0;
    }
    struct { const char *nm; int nt; int arity; } noises[] = {
        {"DEPOLARIZE1", N_DEP1, 1}, {"DEPOLARIZE2", N_DEP2, 2}, {"X_ERROR", N_XERR, 1},
        {"Y_ERROR", N_YERR, 1}, {"Z_ERROR", N_ZERR, 1}};
    for (size_t g = 0; g < sizeof noises / sizeof noises[0]; g++) {
        if (strcmp(name, noises[g].nm)) continue;
        if (!has_arg || arg < 0 || arg > 1) { snprintf(c->err, sizeof c->err, "line %d: bad probability", L->line); return -1; }
        if (nt % noises[g].arity) { snprintf(c->err, sizeof c->err, "line %d: noise needs pairs", L->line); return -1; }
        if (arg == 0) return 0;
        for (int i = 0; i < nt; i += noises[g].arity) {
            o.kind = P_NOISE;
            o.ntype = noises[g].nt;
            o.a = tg[i];
            o.b = noises[g].arity == 2 ? tg[i + 1] : -1;
            o.arg = arg;
            if (o.b == o.a) { snprintf(c->err, sizeof c->err, "line %d: repeated qubit", L->line); return -1; }
            circ_push(c, o);
        }
        return 0;
    }
    if (!strcmp(name, "DETECTOR") || !strcmp(name, "OBSERVABLE_INCLUDE")) {
        o.kind = !strcmp(name, "DETECTOR") ? P_DET : P_OBS;
        o.obs = (int)arg;
        o.nref = nt;
        o.refs = (int *)malloc(sizeof(int) * (size_t)(nt ? nt : 1));
        for (int i = 0; i < nt; i++) {
            if (!isrec[i] || tg[i] >= 0 || c->nrec + tg[i] < 0) { snprintf(c->err, sizeof c->err, "line %d: bad rec target", L->line); return -1; }
            o.refs[i] = c->nrec + tg[i];
        }
        if (o.kind == P_DET) c->ndet++;
        else if (o.obs + 1 > c->nobs) c->nobs = o.obs + 1;
        circ_push(c, o);
        return 0;
    }
    snprintf(c->err, sizeof c->err, "line %d: unsupported instruction '%s'", L->line, name);
    return -2;
}

static int parse_block(circuit *c, lexer *L, int depth)
{
    char buf[65536];
    while (next_line(L, buf, sizeof buf)) {
        char *s = trim(buf);
        if (!*s) continue;
        if (*s == '}') {
            if (depth == 0) { snprintf(c->err, sizeof c->err, "line %d: unmatched '}'", L->line); return -1; }
            return 0;
        }
        int rc = parse_instruction(c, s, L, depth);
        if (rc < 0) return rc;
    }
    if (depth > 0) { snprintf(c->err, sizeof c->err, "missing '}'"); return -1; }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Compiled program: a shot-independent list of plain operations       */
/* (Theorem 1: the Clifford frame and active set do not depend on any   */
/* sample, so they are resolved here once).                            */
/* ------------------------------------------------------------------ */
enum {
    O_VCX,       /* virtual CNOT a->b */
    O_VCZ,       /* virtual CZ a,b */
    O_VS,        /* virtual S on a */
    O_VH,        /* virtual H on an active qubit a */
    O_EXPAND,    /* dormant a -> active (H on |0>) */
    O_ROT,       /* exp(-i theta Z_a) on active a, sign from frame */
    O_PHASE,     /* dormant Z-string rotation: scalar into gamma */
    O_MSTATIC,   /* deterministic measurement */
    O_MRANDOM,   /* dormant X_a measurement, then H absorbed */
    O_MACTIVE_Z, /* active Z_a measurement, demote */
    O_MACTIVE_X, /* active X_a measurement (interfere), demote */
    O_CPAULI,    /* conditional Pauli (reset correction) */
    O_NOISE,     /* stochastic Pauli site */
    O_DET,
    O_OBS,
    O_CFEED,     /* Pauli `mask` if record `rec` is 1 (feed-forward) */
    O_EXPVAL     /* expectation value of the virtual observable `mask` (probe `obs`) */
};

typedef struct {
    int kind;
    int a, b;
    double theta;
    int sign;        /* sign bit of the localized observable / generator */
    int event;       /* measurement event ordinal j */
    int rec;         /* record index or -1 */
    int site;        /* noise site */
    pauli mask;      /* O_MSTATIC / O_PHASE z-string; O_CPAULI image */
    int nref;
    int *refs;
    int obs;
    int k_after;     /* active dimension after this op */
} oop;

typedef struct {
    int type;        /* noise type */
    double p;
    int nimg;        /* 2 (one qubit) or 4 (two qubits) */
    pauli img[4];    /* virtual images of X_a, Z_a, X_b, Z_b */
} site_t;

typedef struct {
    int nq;
    int kmax;
    int nevents, nrec, ndet, nobs, nprobes;
    int nsites;
    oop *ops;
    int nops, capops;
    site_t *sites;
    int *event_class; /* 0 static, 1 random, 2 active */
    int *event_rec;
    /* survival tables per chunk: S[c][i], i = 0..len */
    int nchunks;
    double **surv;
    int *chunk_len;
    /* log of how U_C was built (for dense reconstruction in tests):
     * entries (side, gate, a, b): side 0 = left by a physical gate,
     * side 1 = right by V^dagger of a virtual gate. */
    int *uclog;
    int nuclog, capuclog;
    /* post-selected detectors (Section 3.2, post-selection): per detector 1
     * if a shot whose detector reads 1 is rejected there */
    uint8_t *det_post;
} program;

static void prog_push(program *P, oop o)
{
    if (P->nops == P->capops) {
        P->capops = P->capops ? 2 * P->capops : 256;
        P->ops = (oop *)realloc(P->ops, (size_t)P->capops * sizeof(oop));
    }
    P->ops[P->nops++] = o;
}

enum { G_H, G_S, G_SDAG, G_X, G_Y, G_Z, G_CX, G_CZ, G_SWAP };

static void uclog_push(program *P, int side, int gate, int a, int b)
{
    if (P->nuclog + 4 > P->capuclog) {
        P->capuclog = P->capuclog ? 2 * P->capuclog : 1024;
        P->uclog = (int *)realloc(P->uclog, (size_t)P->capuclog * sizeof(int));
    }
    P->uclog[P->nuclog++] = side;
    P->uclog[P->nuclog++] = gate;
    P->uclog[P->nuclog++] = a;
    P->uclog[P->nuclog++] = b;
}

/* Compile-time state: the Clifford frame U_C stored as the virtual images
 * U_C^dagger X_q U_C and U_C^dagger Z_q U_C of every physical Pauli, plus the
 * active set A (Definition 2). */
typedef struct {
    int n;
    pauli *ix, *iz;
    uint8_t *active;
    int k;
    program *P;
} compiler;

/* Definition 1 (Eq. 1): virtual generator of a physical Pauli
 * P = sigma on qubit q (letter 'X', 'Y', 'Z'). */
static void map_pauli(compiler *C, int q, char letter, pauli *out)
{
    int n = C->n;
    if (letter == 'X') pauli_copy(out, &C->ix[q], n);
    else if (letter == 'Z') pauli_copy(out, &C->iz[q], n);
    else { /* Y = i X Z */
        pauli_copy(out, &C->ix[q], n);
        int e = pauli_mul_into(out, &C->iz[q], n, 1);
        out->r = (e / 2) & 1;
    }
}

/* U_C <- G U_C for a physical Clifford gate G: each image becomes the image
 * of G^dagger P G (Definition 1 applied to the new frame). */
static void phys_gate(compiler *C, int g, int a, int b)
{
    int n = C->n;
    pauli t = pauli_new(n);
    switch (g) {
    case G_H: { pauli s = C->ix[a]; C->ix[a] = C->iz[a]; C->iz[a] = s; break; }
    case G_S:    /* S^dag X S = -Y */
        map_pauli(C, a, 'Y', &t); t.r ^= 1; pauli_copy(&C->ix[a], &t, n); break;
    case G_SDAG: /* S X S^dag = Y */
        map_pauli(C, a, 'Y', &t); pauli_copy(&C->ix[a], &t, n); break;
    case G_X: C->iz[a].r ^= 1; break;
    case G_Z: C->ix[a].r ^= 1; break;
    case G_Y: C->ix[a].r ^= 1; C->iz[a].r ^= 1; break;
    case G_CX: { /* X_a -> X_a X_b, Z_b -> Z_a Z_b */
        int e = pauli_mul_into(&C->ix[a], &C->ix[b], n, 0); C->ix[a].r = (e / 2) & 1;
        e = pauli_mul_into(&C->iz[b], &C->iz[a], n, 0); C->iz[b].r = (e / 2) & 1;
        break; }
    case G_CZ: { /* X_a -> X_a Z_b, X_b -> Z_a X_b */
        int e = pauli_mul_into(&C->ix[a], &C->iz[b], n, 0); C->ix[a].r = (e / 2) & 1;
        e = pauli_mul_into(&C->ix[b], &C->iz[a], n, 0); C->ix[b].r = (e / 2) & 1;
        break; }
    case G_SWAP: {
        pauli s = C->ix[a]; C->ix[a] = C->ix[b]; C->ix[b] = s;
        s = C->iz[a]; C->iz[a] = C->iz[b]; C->iz[b] = s;
        break; }
    }
    pauli_free(&t);
    uclog_push(C->P, 0, g, a, b);
}

/* U_C <- U_C V^dagger for a virtual gate V: every image P~ becomes V P~ V^dagger
 * (Section 2.3, distributing V). */
static void virt_gate(compiler *C, int g, int a, int b)
{
    for (int q = 0; q < C->n; q++) {
        pauli *rows[2] = {&C->ix[q], &C->iz[q]};
        for (int i = 0; i < 2; i++) {
            if (g == G_CX) conj_cx(rows[i], a, b);
            else if (g == G_CZ) conj_cz(rows[i], a, b);
            else if (g == G_S) conj_s(rows[i], a);
            else conj_h(rows[i], a);
        }
    }
    uclog_push(C->P, 1, g, a, b);
}

static void emit(compiler *C, oop o)
{
    o.k_after = C->k;
    if (C->k > C->P->kmax) C->P->kmax = C->k;
    prog_push(C->P, o);
}

/* Emit one virtual gate: update U_C, the generator being localized, and the
 * shot program.  Lemma 2: a controlled Pauli whose control is dormant acts
 * as identity on |phi>_A (x) |0>_D; the checks below make sure no emitted
 * gate would take the state out of that form. */
static void vgate(compiler *C, pauli *gen, int g, int a, int b)
{
    oop o;
    memset(&o, 0, sizeof o);
    o.a = a;
    o.b = b;
    if (g == G_CX) {
        if (C->active[a] && !C->active[b]) { fprintf(stderr, "oracle: CX from active to dormant\n"); abort(); }
        conj_cx(gen, a, b);
        o.kind = O_VCX;
    } else if (g == G_CZ) {
        conj_cz(gen, a, b);
        o.kind = O_VCZ;
    } else if (g == G_S) {
        conj_s(gen, a);
        o.kind = O_VS;
    } else {
        if (!C->active[a]) { fprintf(stderr, "oracle: H on dormant qubit outside expansion\n"); abort(); }
        conj_h(gen, a);
        o.kind = O_VH;
    }
    virt_gate(C, g, a, b);
    emit(C, o);
}

/* Lemma 1 / Appendix A, Case 1 (x != 0): pivot v with x_v = 1; CNOT v->q for
 * every other q in x, then CZ v,q for every other q in the remaining z; if
 * the result is Y_v, S_v maps it to -X_v.  Leaves gen = +-X_v. */
static void localize_case1(compiler *C, pauli *gen, int v)
{
    int n = C->n;
    for (int q = 0; q < n; q++)
        if (q != v && gen->x[q]) vgate(C, gen, G_CX, v, q);
    for (int q = 0; q < n; q++)
        if (q != v && gen->z[q]) vgate(C, gen, G_CZ, v, q);
    if (gen->z[v]) vgate(C, gen, G_S, v, -1);
}

/* Lemma 1 / Appendix A, Case 2 (x = 0): pivot v with z_v = 1; CNOT q->v for
 * every other q in z.  Leaves gen = +-Z_v. */
static void localize_case2(compiler *C, pauli *gen, int v)
{
    for (int q = 0; q < C->n; q++)
        if (q != v && gen->z[q]) vgate(C, gen, G_CX, q, v);
}

static int lowest(compiler *C, const uint8_t *bits, int want_active)
{
    for (int q = 0; q < C->n; q++)
        if (bits[q] && (C->active[q] != 0) == (want_active != 0)) return q;
    return -1;
}

static int any(const uint8_t *b, int n)
{
    for (int i = 0; i < n; i++)
        if (b[i]) return 1;
    return 0;
}

/* The virtual image U_C^dagger P U_C of a physical Pauli product (the
 * letters' images multiplied; letters on different qubits commute). */
static void map_product(compiler *C, int np, const int *pq, const char *pl, pauli *out)
{
    int n = C->n;
    memset(out->x, 0, (size_t)n);
    memset(out->z, 0, (size_t)n);
    out->r = 0;
    pauli t = pauli_new(n);
    for (int i = 0; i < np; i++) {
        map_pauli(C, pq[i], pl[i], &t);
        int e = pauli_mul_into(out, &t, n, 0);
        out->r = (e / 2) & 1;
    }
    pauli_free(&t);
}

static void compile_rotation_g(compiler *C, pauli g, double theta);

/* Section 2.4 / Appendix B.1: a rotation exp(-i theta P) on physical
 * qubit q with P = Z. */
static void compile_rotation(compiler *C, int q, double theta)
{
    pauli g = pauli_new(C->n);
    map_pauli(C, q, 'Z', &g);
    compile_rotation_g(C, g, theta);
}

/* The same for any virtual generator g (owned by the call): a rotation
 * exp(-i theta g). */
static void compile_rotation_g(compiler *C, pauli g, double theta)
{
    int n = C->n;
    int vd = lowest(C, g.x, 0);
    int va = lowest(C, g.x, 1);
    oop o;
    memset(&o, 0, sizeof o);
    if (vd >= 0) {
        /* dormant pivot with X support: localize to X_v, then H_v promotes v
         * (case 2 of Appendix B.1: subspace expansion) */
        localize_case1(C, &g, vd);
        conj_h(&g, vd);
        virt_gate(C, G_H, vd, -1);
        C->active[vd] = 1;
        C->k++;
        o.kind = O_EXPAND;
        o.a = vd;
        emit(C, o);
        o.kind = O_ROT;
        o.a = vd;
        o.theta = g.r ? -theta : theta;
        emit(C, o);
    } else if (va >= 0) {
        /* x inside A: active pivot, H on an active axis, then diagonal
         * rotation (case 3 of Appendix B.1) */
        localize_case1(C, &g, va);
        vgate(C, &g, G_H, va, -1);
        o.kind = O_ROT;
        o.a = va;
        o.theta = g.r ? -theta : theta;
        emit(C, o);
    } else {
        int vz = lowest(C, g.z, 1);
        if (vz >= 0) {
            localize_case2(C, &g, vz);
            o.kind = O_ROT;
            o.a = vz;
            o.theta = g.r ? -theta : theta;
            emit(C, o);
        } else {
            /* case 1 of Appendix B.1: diagonal on dormant qubits only */
            o.kind = O_PHASE;
            o.mask = pauli_new(n);
            pauli_copy(&o.mask, &g, n);
            o.theta = g.r ? -theta : theta;
            emit(C, o);
        }
    }
    pauli_free(&g);
}

static int compile_measure_g(compiler *C, pauli g, int rec);

/* Section 2.4 / Appendix B.2: a projective measurement of the physical
 * Pauli `letter` on qubit q.  Returns the measurement event ordinal. */
static int compile_measure(compiler *C, int q, char letter, int rec)
{
    pauli g = pauli_new(C->n);
    map_pauli(C, q, letter, &g);
    return compile_measure_g(C, g, rec);
}

/* The same for any virtual observable g (owned by the call). */
static int compile_measure_g(compiler *C, pauli g, int rec)
{
    int n = C->n;
    program *P = C->P;
    int j = P->nevents++;
    P->event_class = (int *)realloc(P->event_class, sizeof(int) * (size_t)P->nevents);
    P->event_rec = (int *)realloc(P->event_rec, sizeof(int) * (size_t)P->nevents);
    P->event_rec[j] = rec;
    oop o;
    memset(&o, 0, sizeof o);
    o.event = j;
    o.rec = rec;
    int xd = lowest(C, g.x, 0);
    if (!any(g.x, n) && lowest(C, g.z, 1) < 0) {
        /* commutes with Z_D and lies in it: deterministic */
        o.kind = O_MSTATIC;
        o.mask = pauli_new(n);
        pauli_copy(&o.mask, &g, n);
        o.sign = g.r;
        P->event_class[j] = 0;
        emit(C, o);
    } else if (xd >= 0) {
        /* conjugate to a dormant qubit: uniformly random; localize to X_v,
         * then absorb H_v into both frames */
        localize_case1(C, &g, xd);
        o.kind = O_MRANDOM;
        o.a = xd;
        o.sign = g.r;
        P->event_class[j] = 1;
        virt_gate(C, G_H, xd, -1);
        emit(C, o);
    } else {
        int v;
        if (any(g.x, n)) {
            v = lowest(C, g.x, 1);
            localize_case1(C, &g, v);
            o.kind = O_MACTIVE_X;
            virt_gate(C, G_H, v, -1);
        } else {
            v = lowest(C, g.z, 1);
            localize_case2(C, &g, v);
            o.kind = O_MACTIVE_Z;
        }
        o.a = v;
        o.sign = g.r;
        C->active[v] = 0;
        C->k--;
        P->event_class[j] = 2;
        emit(C, o);
    }
    pauli_free(&g);
    return j;
}

static void compile_reset_fix(compiler *C, int q, int event)
{
    oop o;
    memset(&o, 0, sizeof o);
    o.kind = O_CPAULI;
    o.event = event;
    o.mask = pauli_new(C->n);
    map_pauli(C, q, 'X', &o.mask);
    emit(C, o);
}

static void compile_noise(compiler *C, const pop *po)
{
    program *P = C->P;
    int s = P->nsites++;
    P->sites = (site_t *)realloc(P->sites, sizeof(site_t) * (size_t)P->nsites);
    site_t *st = &P->sites[s];
    st->type = po->ntype;
    st->p = po->arg;
    st->nimg = po->ntype == N_DEP2 ? 4 : 2;
    for (int i = 0; i < st->nimg; i++) st->img[i] = pauli_new(C->n);
    map_pauli(C, po->a, 'X', &st->img[0]);
    map_pauli(C, po->a, 'Z', &st->img[1]);
    if (st->nimg == 4) {
        map_pauli(C, po->b, 'X', &st->img[2]);
        map_pauli(C, po->b, 'Z', &st->img[3]);
    }
    oop o;
    memset(&o, 0, sizeof o);
    o.kind = O_NOISE;
    o.site = s;
    emit(C, o);
}

/* Survival products of the cumulative hazard (Section 3.2), one table per
 * chunk of CHUNK sites: S[0] = 1, S[i+1] = S[i] * (1 - p_i), FP64, no FMA. */
static void build_survival(program *P)
{
    P->nchunks = (P->nsites + CHUNK - 1) / CHUNK;
    P->surv = (double **)calloc((size_t)(P->nchunks ? P->nchunks : 1), sizeof(double *));
    P->chunk_len = (int *)calloc((size_t)(P->nchunks ? P->nchunks : 1), sizeof(int));
    for (int c = 0; c < P->nchunks; c++) {
        int lo = c * CHUNK, hi = lo + CHUNK < P->nsites ? lo + CHUNK : P->nsites;
        P->chunk_len[c] = hi - lo;
        P->surv[c] = (double *)malloc(sizeof(double) * (size_t)(hi - lo + 1));
        volatile double s = 1.0;
        P->surv[c][0] = s;
        for (int i = lo; i < hi; i++) {
            volatile double q = 1.0 - P->sites[i].p;
            s = s * q;
            P->surv[c][i - lo + 1] = s;
        }
    }
}

static void prog_free(program *P)
{
    if (!P) return;
    for (int i = 0; i < P->nops; i++) {
        if (P->ops[i].mask.x) pauli_free(&P->ops[i].mask);
        free(P->ops[i].refs);
    }
    free(P->ops);
    for (int s = 0; s < P->nsites; s++)
        for (int i = 0; i < P->sites[s].nimg; i++) pauli_free(&P->sites[s].img[i]);
    free(P->sites);
    free(P->event_class);
    free(P->event_rec);
    free(P->det_post);
    for (int c = 0; c < P->nchunks; c++) free(P->surv[c]);
    free(P->surv);
    free(P->chunk_len);
    free(P->uclog);
    free(P);
}

static program *compile_circuit(circuit *ci)
{
    program *P = (program *)calloc(1, sizeof(program));
    int n = ci->nq > 0 ? ci->nq : 1;
    P->nq = n;
    compiler C;
    C.n = n;
    C.P = P;
    C.k = 0;
    C.active = (uint8_t *)calloc((size_t)n, 1);
    C.ix = (pauli *)malloc(sizeof(pauli) * (size_t)n);
    C.iz = (pauli *)malloc(sizeof(pauli) * (size_t)n);
    for (int q = 0; q < n; q++) { /* U_C = I */
        C.ix[q] = pauli_new(n);
        C.iz[q] = pauli_new(n);
        C.ix[q].x[q] = 1;
        C.iz[q].z[q] = 1;
    }
    int rec = 0;
    for (int i = 0; i < ci->n; i++) {
        pop *po = &ci->ops[i];
        switch (po->kind) {
        case P_H: phys_gate(&C, G_H, po->a, -1); break;
        case P_S: phys_gate(&C, G_S, po->a, -1); break;
        case P_SDAG: phys_gate(&C, G_SDAG, po->a, -1); break;
        case P_X: phys_gate(&C, G_X, po->a, -1); break;
        case P_Y: phys_gate(&C, G_Y, po->a, -1); break;
        case P_Z: phys_gate(&C, G_Z, po->a, -1); break;
        case P_CX: phys_gate(&C, G_CX, po->a, po->b); break;
        case P_CZ: phys_gate(&C, G_CZ, po->a, po->b); break;
        case P_SWAP: phys_gate(&C, G_SWAP, po->a, po->b); break;
        case P_ROTZ: compile_rotation(&C, po->a, po->arg); break;
        case P_M: compile_measure(&C, po->a, 'Z', rec++); break;
        case P_MX: compile_measure(&C, po->a, 'X', rec++); break;
        case P_MR: { int j = compile_measure(&C, po->a, 'Z', rec++); compile_reset_fix(&C, po->a, j); break; }
        case P_R: { int j = compile_measure(&C, po->a, 'Z', -1); compile_reset_fix(&C, po->a, j); break; }
        case P_NOISE: compile_noise(&C, po); break;
        case P_PROT: {
            pauli g = pauli_new(n);
            map_product(&C, po->np, po->pq, po->pl, &g);
            compile_rotation_g(&C, g, po->arg);
            break; }
        case P_MPP: {
            pauli g = pauli_new(n);
            map_product(&C, po->np, po->pq, po->pl, &g);
            compile_measure_g(&C, g, rec++);
            break; }
        case P_CFEED: {
            oop o;
            memset(&o, 0, sizeof o);
            o.kind = O_CFEED;
            o.rec = po->refs[0];
            o.mask = pauli_new(n);
            map_pauli(&C, po->a, po->pl[0], &o.mask);
            emit(&C, o);
            break; }
        case P_EXPVAL: {
            oop o;
            memset(&o, 0, sizeof o);
            o.kind = O_EXPVAL;
            o.obs = po->obs;
            o.mask = pauli_new(n);
            map_product(&C, po->np, po->pq, po->pl, &o.mask);
            emit(&C, o);
            break; }
        case P_GPHASE: {
            oop o;
            memset(&o, 0, sizeof o);
            o.kind = O_PHASE;  /* empty Z string: parity 0 */
            o.mask = pauli_new(n);
            o.theta = po->arg;
            emit(&C, o);
            break; }
        case P_DET:
        case P_OBS: {
            oop o;
            memset(&o, 0, sizeof o);
            o.kind = po->kind == P_DET ? O_DET : O_OBS;
            o.nref = po->nref;
            o.refs = (int *)malloc(sizeof(int) * (size_t)(po->nref ? po->nref : 1));
            memcpy(o.refs, po->refs, sizeof(int) * (size_t)po->nref);
            o.obs = po->obs;
            if (o.kind == O_DET) o.rec = P->ndet++;
            emit(&C, o);
            break; }
        }
    }
    P->nrec = rec;
    P->nobs = ci->nobs;
    P->nprobes = ci->nprobes;
    build_survival(P);
    for (int q = 0; q < n; q++) { pauli_free(&C.ix[q]); pauli_free(&C.iz[q]); }
    free(C.ix);
    free(C.iz);
    free(C.active);
    return P;
}

/* ------------------------------------------------------------------ */
/* Per-shot state (Definition 2, Eq. 2):                               */
/*   |psi> = gamma U_C P~ (|phi>_A (x) |0>_D)                          */
/* P~ = prod_j X_j^{x_j} Z_j^{z_j} (phase free).  tx/tz is the full     */
/* frame; nx/nz is the part contributed by noise only (readings).       */
/* ------------------------------------------------------------------ */
typedef struct {
    int n, kmax;
    uint8_t *tx, *tz, *nx, *nz;
    double complex *phi, *tmp;
    int k;
    int *slot_q;   /* virtual qubit held by each slot */
    int *q_slot;   /* slot of each virtual qubit, -1 if dormant */
    double complex gamma;
    uint8_t *rec;   /* per record */
    uint8_t *ev_m;  /* per event: outcome m */
    uint8_t *ev_pn; /* per event: noise parity */
    uint8_t *det;
    uint8_t *obs;
    double *probe;  /* per probe: expectation value */
    int rejected;   /* a post-selected detector read 1 */
} shot_state;

static double complex ipow(int e)
{
    e = ((e % 4) + 4) % 4;
    static const double complex t[4] = {1, I, -1, -I};
    return t[e];
}

/* Conjugate the phase-free frame X^x Z^z by a virtual gate and return the
 * phase picked up (as a power of i): X^x Z^z = (-i)^{|x&z|} sigma(x,z). */
static int frame_conj(uint8_t *x, uint8_t *z, int g, int a, int b)
{
    int q[2] = {a, b};
    int nq = (g == G_CX || g == G_CZ) ? 2 : 1;
    int e = 0;
    for (int i = 0; i < nq; i++) e -= x[q[i]] & z[q[i]];
    /* single-frame Hermitian conjugation on the touched qubits */
    int r = 0;
    if (g == G_CX) {
        r = x[a] & z[b] & (x[b] ^ z[a] ^ 1);
        x[b] ^= x[a];
        z[a] ^= z[b];
    } else if (g == G_CZ) {
        r = x[a] & x[b] & (z[a] ^ z[b]);
        z[a] ^= x[b];
        z[b] ^= x[a];
    } else if (g == G_S) {
        r = x[a] & z[a];
        z[a] ^= x[a];
    } else {
        r = x[a] & z[a];
        uint8_t t = x[a];
        x[a] = z[a];
        z[a] = t;
    }
    e += 2 * r;
    for (int i = 0; i < nq; i++) e += x[q[i]] & z[q[i]];
    return e;
}

/* P~ <- E~ P~ for a Hermitian virtual Pauli E~ (Appendix B.3); returns the
 * phase (power of i) for gamma. */
static int frame_mul_left(uint8_t *x, uint8_t *z, const uint8_t *ex, const uint8_t *ez, int r, int n)
{
    int e = 2 * r;
    for (int j = 0; j < n; j++) {
        e += ex[j] & ez[j];      /* sigma(1,1) = Y = i X Z */
        e += 2 * (ez[j] & x[j]); /* Z^{ez} X^{x} = (-1)^{ez x} X^{x} Z^{ez} */
        x[j] ^= ex[j];
        z[j] ^= ez[j];
    }
    return e;
}

static int parity_and(const uint8_t *a, const uint8_t *b, int n)
{
    int p = 0;
    for (int j = 0; j < n; j++) p ^= a[j] & b[j];
    return p;
}

static void shot_init(shot_state *S, const program *P)
{
    int n = P->nq;
    S->n = n;
    S->kmax = P->kmax;
    memset(S->tx, 0, (size_t)n);
    memset(S->tz, 0, (size_t)n);
    memset(S->nx, 0, (size_t)n);
    memset(S->nz, 0, (size_t)n);
    size_t dim = (size_t)1 << P->kmax;
    for (size_t i = 0; i < dim; i++) S->phi[i] = 0;
    S->phi[0] = 1;
    S->k = 0;
    for (int q = 0; q < n; q++) S->q_slot[q] = -1;
    S->gamma = 1;
    memset(S->rec, 0, (size_t)(P->nrec + 1));
    memset(S->ev_m, 0, (size_t)(P->nevents + 1));
    memset(S->ev_pn, 0, (size_t)(P->nevents + 1));
    memset(S->det, 0, (size_t)(P->ndet + 1));
    memset(S->obs, 0, (size_t)(P->nobs + 1));
    memset(S->probe, 0, sizeof(double) * (size_t)(P->nprobes + 1));
    S->rejected = 0;
}

static shot_state *shot_alloc(const program *P)
{
    shot_state *S = (shot_state *)calloc(1, sizeof(shot_state));
    int n = P->nq;
    S->tx = (uint8_t *)calloc((size_t)n, 1);
    S->tz = (uint8_t *)calloc((size_t)n, 1);
    S->nx = (uint8_t *)calloc((size_t)n, 1);
    S->nz = (uint8_t *)calloc((size_t)n, 1);
    S->phi = (double complex *)calloc((size_t)1 << P->kmax, sizeof(double complex));
    S->tmp = (double complex *)calloc((size_t)1 << P->kmax, sizeof(double complex));
    S->slot_q = (int *)calloc((size_t)(P->kmax + 1), sizeof(int));
    S->q_slot = (int *)calloc((size_t)n, sizeof(int));
    S->rec = (uint8_t *)calloc((size_t)(P->nrec + 1), 1);
    S->ev_m = (uint8_t *)calloc((size_t)(P->nevents + 1), 1);
    S->ev_pn = (uint8_t *)calloc((size_t)(P->nevents + 1), 1);
    S->det = (uint8_t *)calloc((size_t)(P->ndet + 1), 1);
    S->obs = (uint8_t *)calloc((size_t)(P->nobs + 1), 1);
    S->probe = (double *)calloc((size_t)(P->nprobes + 1), sizeof(double));
    return S;
}

static void shot_free(shot_state *S)
{
    free(S->tx); free(S->tz); free(S->nx); free(S->nz);
    free(S->phi); free(S->tmp); free(S->slot_q); free(S->q_slot);
    free(S->rec); free(S->ev_m); free(S->ev_pn); free(S->det); free(S->obs); free(S->probe);
    free(S);
}

/* Apply a virtual gate to the shot: both frames, gamma, and the active
 * vector when the gate acts on active qubits (Lemma 2 otherwise). */
static void shot_vgate(shot_state *S, int g, int a, int b)
{
    S->gamma *= ipow(frame_conj(S->tx, S->tz, g, a, b));
    (void)frame_conj(S->nx, S->nz, g, a, b);
    size_t dim = (size_t)1 << S->k;
    if (g == G_CX) {
        if (S->q_slot[a] < 0) return; /* dormant control */
        size_t bc = (size_t)1 << S->q_slot[a], bt = (size_t)1 << S->q_slot[b];
        for (size_t i = 0; i < dim; i++)
            if ((i & bc) && !(i & bt)) {
                double complex t = S->phi[i];
                S->phi[i] = S->phi[i | bt];
                S->phi[i | bt] = t;
            }
    } else if (g == G_CZ) {
        if (S->q_slot[a] < 0 || S->q_slot[b] < 0) return;
        size_t ba = (size_t)1 << S->q_slot[a], bb = (size_t)1 << S->q_slot[b];
        for (size_t i = 0; i < dim; i++)
            if ((i & ba) && (i & bb)) S->phi[i] = -S->phi[i];
    } else if (g == G_S) {
        if (S->q_slot[a] < 0) return; /* S|0> = |0> */
        size_t ba = (size_t)1 << S->q_slot[a];
        for (size_t i = 0; i < dim; i++)
            if (i & ba) S->phi[i] *= I;
    } else {
        size_t ba = (size_t)1 << S->q_slot[a];
        double h = 1.0 / sqrt(2.0);
        for (size_t i = 0; i < dim; i++)
            if (!(i & ba)) {
                double complex u = S->phi[i], v = S->phi[i | ba];
                S->phi[i] = h * (u + v);
                S->phi[i | ba] = h * (u - v);
            }
    }
}

/* Remove the slot of qubit v after it has been projected to |0> at the
 * start of the array (order-preserving: slots above shift down). */
static void demote(shot_state *S, int v, const double complex *kept)
{
    int s = S->q_slot[v];
    size_t half = (size_t)1 << (S->k - 1);
    for (size_t i = 0; i < half; i++) S->phi[i] = kept[i];
    for (size_t i = half; i < ((size_t)1 << S->k); i++) S->phi[i] = 0;
    for (int t = s; t < S->k - 1; t++) {
        S->slot_q[t] = S->slot_q[t + 1];
        S->q_slot[S->slot_q[t]] = t;
    }
    S->q_slot[v] = -1;
    S->k--;
}

/* Index of the amplitude with bit s inserted (value bit) into j. */
static size_t insert_bit(size_t j, int s, int bit)
{
    size_t lo = j & (((size_t)1 << s) - 1);
    size_t hi = j >> s;
    return (hi << (s + 1)) | ((size_t)bit << s) | lo;
}

typedef struct {
    const uint8_t *forced_m;  /* per event forced outcome, or NULL */
    const int *fault_at_site; /* per site forced outcome index or -1, or NULL */
    double *probs;            /* per event P(m = 1), or NULL */
    int error;
    int strat_r;              /* >= 0: exactly this many faults (stratified) */
    const double *strat_q;    /* its tail pmf table (strat_tail_pmf) */
} run_opts;

/* Outcome index -> (x,z) letters of the fired Pauli on each qubit. */
static void noise_outcome(int type, int idx, int *la, int *lb)
{
    /* letters: 0 I, 1 X, 2 Y, 3 Z */
    *lb = 0;
    switch (type) {
    case N_DEP1: *la = idx + 1; break;
    case N_DEP2: *la = (idx + 1) >> 2; *lb = (idx + 1) & 3; break;
    case N_XERR: *la = 1; break;
    case N_YERR: *la = 2; break;
    default: *la = 3; break;
    }
}
static int noise_nout(int type) { return type == N_DEP1 ? 3 : type == N_DEP2 ? 15 : 1; }

/* Apply a fired noise Pauli (Appendix B.3): E~ = image of the physical
 * Pauli, multiplied into both frames. */
static void apply_fault(shot_state *S, const program *P, int site, int idx)
{
    const site_t *st = &P->sites[site];
    int n = S->n;
    int la, lb;
    noise_outcome(st->type, idx, &la, &lb);
    pauli e = pauli_new(n);
    int letters[2] = {la, lb};
    for (int qi = 0; qi < 2; qi++) {
        int L = letters[qi];
        if (!L) continue;
        const pauli *ix = &st->img[2 * qi], *iz = &st->img[2 * qi + 1];
        if (L == 1 || L == 2) {
            int ee = pauli_mul_into(&e, ix, n, 0);
            e.r = (ee / 2) & 1;
        }
        if (L == 3 || L == 2) {
            int ee = pauli_mul_into(&e, iz, n, L == 2 ? 1 : 0); /* Y = i X Z */
            e.r = (ee / 2) & 1;
        }
    }
    S->gamma *= ipow(frame_mul_left(S->tx, S->tz, e.x, e.z, e.r, n));
    (void)frame_mul_left(S->nx, S->nz, e.x, e.z, e.r, n);
    pauli_free(&e);
}

/* Sparse noise sampling (Section 3.2): within each chunk, from cursor cur
 * draw u, set tau = u * S[cur]; the next fault is the smallest j >= cur with
 * S[j+1] <= tau, else none in the rest of the chunk.  The fired Pauli is
 * outcome floor(w * n_out / 2^64) with w = (w3 << 32) | w2 of the same draw. */
int oracle_gap_next(const double *S, int len, int cur, double u)
{
    double tau = u * S[cur];
    for (int j = cur; j < len; j++)
        if (S[j + 1] <= tau) return j;
    return -1;
}

static void draw_faults(const program *P, uint64_t shot, uint64_t seed, int *fault_at_site)
{
    for (int s = 0; s < P->nsites; s++) fault_at_site[s] = -1;
    for (int c = 0; c < P->nchunks; c++) {
        int cur = 0;
        uint32_t ordinal = 0;
        for (;;) {
            uint32_t w[4];
            draw(ordinal++, PURPOSE_NOISE | (uint32_t)c, shot, seed, w);
            int j = oracle_gap_next(P->surv[c], P->chunk_len[c], cur, uniform53(w));
            if (j < 0) break;
            int site = c * CHUNK + j;
            uint64_t w64 = ((uint64_t)w[3] << 32) | w[2];
            int nout = noise_nout(P->sites[site].type);
            fault_at_site[site] = (int)(((unsigned __int128)w64 * (unsigned)nout) >> 64);
            cur = j + 1;
        }
    }
}

/* Stratified fault sampling (Section 3.2, rare-event sampling).  Shots are
 * conditioned on exactly r of the N noise sites firing.  Site l fires on its
 * own with probability p_l, so the fault count is Poisson-binomial, and
 *   Q[t][s] = P(exactly s of the sites t .. N-1 fire)
 * satisfies Q[N][0] = 1, Q[N][s > 0] = 0 and
 *   Q[t][s] = (1 - p_t) Q[t+1][s] + p_t Q[t+1][s-1]
 * (condition on site t).  Layout Q[t * (r + 1) + s], t = 0..N, s = 0..r.
 * Plain FP64 products: the table underflows once the probability of no
 * fault at all drops below about 1e-300. */
static double *strat_tail_pmf(const program *P, int r)
{
    const int N = P->nsites;
    const size_t R = (size_t)r + 1;
    double *Q = (double *)calloc((size_t)(N + 1) * R, sizeof(double));
    Q[(size_t)N * R] = 1.0;
    for (int t = N - 1; t >= 0; t--) {
        const double p = P->sites[t].p;
        for (int s = 0; s <= r; s++) {
            double v = (1.0 - p) * Q[(size_t)(t + 1) * R + s];
            if (s > 0) v += p * Q[(size_t)(t + 1) * R + s - 1];
            Q[(size_t)t * R + s] = v;
        }
    }
    return Q;
}

/* The next fault, given that s faults are still to be placed among the
 * sites j .. N-1, lies at or after site t >= j with probability
 *   survival(t) = P(none of j .. t-1 fires) Q[t][s] / Q[j][s]
 * (no fault in between, all s of them from t on).  Inverse transform: for
 * a uniform u the fault is at the smallest t >= j with survival(t+1) <= u,
 * which is at most N - s because Q[t][s] = 0 when fewer than s sites
 * remain. */
static int strat_next(const program *P, const double *Q, int r, int s, int j, double u)
{
    const size_t R = (size_t)r + 1;
    const double qj = Q[(size_t)j * R + s];
    double none = 1.0; /* P(none of j .. t fires) */
    int t = j;
    for (;; t++) {
        none *= 1.0 - P->sites[t].p;
        if (none * Q[(size_t)(t + 1) * R + s] / qj <= u || t + 1 >= P->nsites) break;
    }
    return t;
}

/* Exactly r faults per shot: fault i (i = 0 .. r-1, in site order) is placed
 * by draw i of purpose STRAT from one past the previous fault; its fired
 * Pauli comes from the same draw's 64-bit word as in draw_faults.  Returns
 * 4 when no configuration has r faults (Q[0][r] = 0). */
static int draw_faults_strat(const program *P, int r, const double *Q, uint64_t shot, uint64_t seed, int *fault_at_site)
{
    for (int s = 0; s < P->nsites; s++) fault_at_site[s] = -1;
    if (!(Q[r] > 0.0)) return 4;
    int j = 0;
    for (int i = 0; i < r; i++) {
        uint32_t w[4];
        draw((uint32_t)i, PURPOSE_STRAT, shot, seed, w);
        const int t = strat_next(P, Q, r, r - i, j, uniform53(w));
        const uint64_t w64 = ((uint64_t)w[3] << 32) | w[2];
        fault_at_site[t] = (int)(((unsigned __int128)w64 * (unsigned)noise_nout(P->sites[t].type)) >> 64);
        j = t + 1;
    }
    return 0;
}

static int rbit(uint64_t shot, uint64_t seed, int j)
{
    uint32_t w[4];
    draw((uint32_t)(j >> 7), PURPOSE_RBIT, shot, seed, w);
    int b = j & 127;
    return (int)((w[b >> 5] >> (b & 31)) & 1u);
}

/* Squared norm with Kahan-compensated summation, so that the unit-norm
 * self-check measures the drift of the vector and not of the sum. */
static double sqnorm(const double complex *v, size_t n)
{
    double s = 0, c = 0;
    for (size_t i = 0; i < n; i++) {
        double y = creal(v[i]) * creal(v[i]) + cimag(v[i]) * cimag(v[i]) - c;
        double t = s + y;
        c = (t - s) - y;
        s = t;
    }
    return s;
}

static void check_norm(shot_state *S, run_opts *ro)
{
    double s = sqnorm(S->phi, (size_t)1 << S->k);
    if (fabs(sqrt(s) - 1.0) > 1e-12 && !ro->error) { ro->error = 3; if (getenv("ORACLE_DEBUG")) fprintf(stderr, "norm dev %.3e k=%d\n", sqrt(s) - 1.0, S->k); }
}

/* Execute one shot of the compiled program on the frame-factored state. */
static void run_shot(const program *P, shot_state *S, uint64_t shot, uint64_t seed, run_opts *ro, int *faults)
{
    shot_init(S, P);
    if (ro->fault_at_site) memcpy(faults, ro->fault_at_site, sizeof(int) * (size_t)P->nsites);
    else if (ro->strat_r >= 0) draw_faults_strat(P, ro->strat_r, ro->strat_q, shot, seed, faults);
    else draw_faults(P, shot, seed, faults);
    const double rs2 = 1.0 / sqrt(2.0);
    for (int oi = 0; oi < P->nops; oi++) {
        const oop *o = &P->ops[oi];
        int v = o->a;
        switch (o->kind) {
        case O_VCX: shot_vgate(S, G_CX, o->a, o->b); break;
        case O_VCZ: shot_vgate(S, G_CZ, o->a, o->b); break;
        case O_VS: shot_vgate(S, G_S, o->a, -1); break;
        case O_VH: shot_vgate(S, G_H, o->a, -1); break;
        case O_EXPAND: {
            /* Appendix B.1 case 2: H_v maps |0>_v to |+>_v, v joins A */
            S->gamma *= ipow(frame_conj(S->tx, S->tz, G_H, v, -1));
            (void)frame_conj(S->nx, S->nz, G_H, v, -1);
            size_t dim = (size_t)1 << S->k;
            for (size_t i = 0; i < dim; i++) {
                S->phi[i + dim] = rs2 * S->phi[i];
                S->phi[i] = rs2 * S->phi[i];
            }
            S->slot_q[S->k] = v;
            S->q_slot[v] = S->k;
            S->k++;
            check_norm(S, ro);
            break; }
        case O_ROT: {
            /* Appendix B.1: commuting exp(-i theta Z_v) past the frame flips
             * the angle when the frame anticommutes with Z_v (x_v = 1) */
            double th = S->tx[v] ? -o->theta : o->theta;
            size_t bit = (size_t)1 << S->q_slot[v];
            double complex e0 = cexp(-I * th), e1 = cexp(I * th);
            for (size_t i = 0; i < ((size_t)1 << S->k); i++) S->phi[i] *= (i & bit) ? e1 : e0;
            break; }
        case O_PHASE: {
            int c = parity_and(S->tx, o->mask.z, S->n);
            double th = c ? -o->theta : o->theta;
            S->gamma *= cexp(-I * th);
            break; }
        case O_MSTATIC: {
            int j = o->event;
            int p = parity_and(S->tx, o->mask.z, S->n);
            int pn = parity_and(S->nx, o->mask.z, S->n);
            int m = p ^ o->sign;
            if (ro->forced_m && ro->forced_m[j] != m && !ro->error) ro->error = 2;
            if (ro->probs) ro->probs[j] = m;
            S->ev_m[j] = (uint8_t)m;
            S->ev_pn[j] = (uint8_t)pn;
            if (o->rec >= 0) S->rec[o->rec] = (uint8_t)m;
            break; }
        case O_MRANDOM: {
            int j = o->event;
            int p = S->tz[v], pn = S->nz[v]; /* X_v anticommutes iff z_v */
            int m = ro->forced_m ? ro->forced_m[j] : (rbit(shot, seed, j) ^ pn);
            if (ro->probs) ro->probs[j] = 0.5;
            int b = m ^ o->sign ^ p;
            /* H_v absorbed into U_C (done at compile time) and into the frames */
            S->gamma *= ipow(frame_conj(S->tx, S->tz, G_H, v, -1));
            (void)frame_conj(S->nx, S->nz, G_H, v, -1);
            /* the qubit is now |b>: P~ <- P~ X_v^b */
            if (b && S->tz[v]) S->gamma = -S->gamma;
            S->tx[v] ^= (uint8_t)b;
            S->ev_m[j] = (uint8_t)m;
            S->ev_pn[j] = (uint8_t)pn;
            if (o->rec >= 0) S->rec[o->rec] = (uint8_t)m;
            break; }
        case O_MACTIVE_Z:
        case O_MACTIVE_X: {
            int j = o->event;
            int isx = o->kind == O_MACTIVE_X;
            int p = isx ? S->tz[v] : S->tx[v];
            int pn = isx ? S->nz[v] : S->nx[v];
            int s = S->q_slot[v];
            size_t half = (size_t)1 << (S->k - 1);
            double sb[2];
            for (int bb = 0; bb < 2; bb++) {
                double acc = 0;
                for (size_t jj = 0; jj < half; jj++) {
                    double complex a;
                    if (isx) a = rs2 * (S->phi[insert_bit(jj, s, 0)] + (bb ? -1.0 : 1.0) * S->phi[insert_bit(jj, s, 1)]);
                    else a = S->phi[insert_bit(jj, s, bb)];
                    acc += creal(a) * creal(a) + cimag(a) * cimag(a);
                }
                sb[bb] = acc;
            }
            double tot = sb[0] + sb[1];
            /* physical outcome m corresponds to virtual branch m ^ sign ^ p */
            double p1 = sb[1 ^ o->sign ^ p] / tot;
            int m;
            if (ro->forced_m) {
                m = ro->forced_m[j];
            } else {
                uint32_t w[4];
                draw((uint32_t)j, PURPOSE_AMEAS, shot, seed, w);
                double pref1 = sb[1 ^ pn ^ o->sign ^ p] / tot; /* P(m_ref = 1) */
                int mref = uniform53(w) < pref1;
                m = mref ^ pn;
            }
            if (ro->probs) ro->probs[j] = p1;
            int b = m ^ o->sign ^ p;
            if (!(sb[b] / tot > 1e-300)) {
                if (!ro->error) ro->error = 2;
                sb[b] = 1;
            }
            double scale = 1.0 / sqrt(sb[b]);
            for (size_t jj = 0; jj < half; jj++) {
                double complex a;
                if (isx) a = rs2 * (S->phi[insert_bit(jj, s, 0)] + (b ? -1.0 : 1.0) * S->phi[insert_bit(jj, s, 1)]);
                else a = S->phi[insert_bit(jj, s, b)];
                S->tmp[jj] = a * scale;
            }
            if (isx) {
                S->gamma *= ipow(frame_conj(S->tx, S->tz, G_H, v, -1));
                (void)frame_conj(S->nx, S->nz, G_H, v, -1);
            }
            if (b && S->tz[v]) S->gamma = -S->gamma;
            S->tx[v] ^= (uint8_t)b;
            demote(S, v, S->tmp);
            check_norm(S, ro);
            S->ev_m[j] = (uint8_t)m;
            S->ev_pn[j] = (uint8_t)pn;
            if (o->rec >= 0) S->rec[o->rec] = (uint8_t)m;
            break; }
        case O_CPAULI: {
            int j = o->event;
            if (S->ev_m[j]) S->gamma *= ipow(frame_mul_left(S->tx, S->tz, o->mask.x, o->mask.z, o->mask.r, S->n));
            if (S->ev_pn[j]) (void)frame_mul_left(S->nx, S->nz, o->mask.x, o->mask.z, o->mask.r, S->n);
            break; }
        case O_NOISE:
            if (faults[o->site] >= 0) apply_fault(S, P, o->site, faults[o->site]);
            break;
        case O_EXPVAL: {
            /* <psi|P|psi> with psi = gamma U_C P~ (phi (x) 0_D) and the
             * virtual observable g = U_C^dagger P U_C: P~ g P~ = (-1)^c g,
             * and g takes |0>_D to an orthogonal state when it has X
             * support on a dormant qubit; otherwise only its letters on
             * active qubits act on phi (Z on |0> is 1) */
            const pauli *g = &o->mask;
            int dormant_x = 0;
            for (int q = 0; q < S->n; q++) dormant_x |= g->x[q] && S->q_slot[q] < 0;
            double e = 0;
            if (!dormant_x) {
                size_t dim = (size_t)1 << S->k;
                for (size_t i = 0; i < dim; i++) S->tmp[i] = S->phi[i];
                for (int q = 0; q < S->n; q++) {
                    if (!g->x[q] && !g->z[q]) continue;
                    if (S->q_slot[q] < 0) continue; /* Z on |0>: 1 */
                    size_t b = (size_t)1 << S->q_slot[q];
                    for (size_t i = 0; i < dim; i++) {
                        if (i & b) continue;
                        double complex a0 = S->tmp[i], a1 = S->tmp[i | b];
                        if (g->x[q] && g->z[q]) { S->tmp[i] = -I * a1; S->tmp[i | b] = I * a0; }     /* Y */
                        else if (g->x[q]) { S->tmp[i] = a1; S->tmp[i | b] = a0; }                  /* X */
                        else { S->tmp[i | b] = -a1; }                                               /* Z */
                    }
                }
                double complex acc = 0;
                for (size_t i = 0; i < dim; i++) acc += conj(S->phi[i]) * S->tmp[i];
                int c = parity_and(S->tx, g->z, S->n) ^ parity_and(S->tz, g->x, S->n);
                e = ((c ^ g->r) ? -1.0 : 1.0) * creal(acc);
            }
            S->probe[o->obs] = e;
            break; }
        case O_CFEED:
            /* feed-forward Pauli (Appendix B.3) on the full frame; the noise
             * frame only follows physical faults */
            if (S->rec[o->rec]) S->gamma *= ipow(frame_mul_left(S->tx, S->tz, o->mask.x, o->mask.z, o->mask.r, S->n));
            break;
        case O_DET: {
            int d = 0;
            for (int r = 0; r < o->nref; r++) d ^= S->rec[o->refs[r]];
            S->det[o->rec] = (uint8_t)d;
            if (d && P->det_post && P->det_post[o->rec]) {
                /* rejected: the shot ends here; its observables read 0 and
                 * every later record stays 0 */
                S->rejected = 1;
                memset(S->obs, 0, (size_t)(P->nobs + 1));
                return;
            }
            break; }
        case O_OBS: {
            int d = 0;
            for (int r = 0; r < o->nref; r++) d ^= S->rec[o->refs[r]];
            S->obs[o->obs] ^= (uint8_t)d;
            break; }
        }
    }
}

/* ------------------------------------------------------------------ */
/* C entry points (test infrastructure).                               */
/* ------------------------------------------------------------------ */
int oracle_compile(const char *text, size_t len, void **out, char *err, int errlen)
{
    circuit c;
    memset(&c, 0, sizeof c);
    lexer L = {text, len, 0, 0};
    int rc = parse_block(&c, &L, 0);
    if (rc < 0) {
        if (err && errlen > 0) snprintf(err, (size_t)errlen, "%s", c.err);
        for (int i = 0; i < c.n; i++) { free(c.ops[i].refs); free(c.ops[i].pq); free(c.ops[i].pl); }
        free(c.ops);
        *out = NULL;
        return rc == -2 ? 2 : 1;
    }
    program *P = compile_circuit(&c);
    for (int i = 0; i < c.n; i++) { free(c.ops[i].refs); free(c.ops[i].pq); free(c.ops[i].pl); }
    free(c.ops);
    P->ndet = P->ndet; /* counted during compilation */
    *out = P;
    return 0;
}

void oracle_free(void *h) { prog_free((program *)h); }

void oracle_info(void *h, int64_t *info)
{
    program *P = (program *)h;
    info[0] = P->nq;
    info[1] = P->kmax;
    info[2] = P->nevents;
    info[3] = P->nrec;
    info[4] = P->ndet;
    info[5] = P->nobs;
    info[6] = P->nsites;
    info[7] = P->nops;
    info[8] = P->nchunks;
    info[9] = P->nprobes;
}

void oracle_event_classes(void *h, int *cls)
{
    program *P = (program *)h;
    memcpy(cls, P->event_class, sizeof(int) * (size_t)P->nevents);
}

/* per op: kind, a, b, k after the op */
void oracle_ops(void *h, int *out)
{
    program *P = (program *)h;
    for (int i = 0; i < P->nops; i++) {
        out[4 * i] = P->ops[i].kind;
        out[4 * i + 1] = P->ops[i].a;
        out[4 * i + 2] = P->ops[i].b;
        out[4 * i + 3] = P->ops[i].k_after;
    }
}

int oracle_uclog(void *h, int *out, int cap)
{
    program *P = (program *)h;
    int n = P->nuclog < cap ? P->nuclog : cap;
    memcpy(out, P->uclog, sizeof(int) * (size_t)n);
    return P->nuclog;
}

void oracle_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out) { philox(ctr, key[0], key[1], out); }

int oracle_survival(void *h, int chunk, double *out)
{
    program *P = (program *)h;
    if (chunk < 0 || chunk >= P->nchunks) return -1;
    memcpy(out, P->surv[chunk], sizeof(double) * (size_t)(P->chunk_len[chunk] + 1));
    return P->chunk_len[chunk];
}

int oracle_faults(void *h, uint64_t seed, uint64_t shot, int *fault_at_site)
{
    draw_faults((program *)h, shot, seed, fault_at_site);
    return 0;
}

/* One shot with full trace output.  forced_m (per event) and forced_faults
 * (per site: outcome index or -1) may be NULL (then the Philox contract is
 * used).  Outputs: probs[nevents] = P(m = 1), ev_m[nevents], recs[nrec],
 * dets[ndet], obs[nobs], phi[2 * 2^kmax] (re, im of the final vector),
 * slots[kmax] (virtual qubit per slot), k, gamma[2], faults[nsites],
 * frame[4 * nq] (total x, total z, noise x, noise z). */
int oracle_trace(void *h, uint64_t seed, uint64_t shot, const uint8_t *forced_m, const int *forced_faults,
                 double *probs, uint8_t *ev_m, uint8_t *recs, uint8_t *dets, uint8_t *obs, double *phi,
                 int *slots, int *k, double *gamma, int *faults, uint8_t *frame, double *expvals)
{
    program *P = (program *)h;
    shot_state *S = shot_alloc(P);
    run_opts ro = {forced_m, forced_faults, probs, 0, -1, NULL};
    int *fl = (int *)malloc(sizeof(int) * (size_t)(P->nsites + 1));
    run_shot(P, S, shot, seed, &ro, fl);
    if (ev_m) memcpy(ev_m, S->ev_m, (size_t)P->nevents);
    if (recs) memcpy(recs, S->rec, (size_t)P->nrec);
    if (dets) memcpy(dets, S->det, (size_t)P->ndet);
    if (obs) memcpy(obs, S->obs, (size_t)P->nobs);
    if (phi)
        for (size_t i = 0; i < ((size_t)1 << P->kmax); i++) {
            phi[2 * i] = creal(S->phi[i]);
            phi[2 * i + 1] = cimag(S->phi[i]);
        }
    if (slots)
        for (int s = 0; s < S->k; s++) slots[s] = S->slot_q[s];
    if (k) *k = S->k;
    if (gamma) { gamma[0] = creal(S->gamma); gamma[1] = cimag(S->gamma); }
    if (faults) memcpy(faults, fl, sizeof(int) * (size_t)P->nsites);
    if (expvals) memcpy(expvals, S->probe, sizeof(double) * (size_t)P->nprobes);
    if (frame) {
        memcpy(frame, S->tx, (size_t)P->nq);
        memcpy(frame + P->nq, S->tz, (size_t)P->nq);
        memcpy(frame + 2 * P->nq, S->nx, (size_t)P->nq);
        memcpy(frame + 3 * P->nq, S->nz, (size_t)P->nq);
    }
    free(fl);
    int err = ro.error;
    shot_free(S);
    return err;
}

typedef struct {
    program *P;
    uint64_t s0, s1, offset, seed, words, shots;
    uint64_t *meas, *det, *obs;
    double *expvals;  /* [nprobes][shots] or NULL */
    int strat_r;      /* stratified: faults per shot, or -1 */
    const double *strat_q;
    int error;
} job;

static void *sample_worker(void *arg)
{
    job *J = (job *)arg;
    program *P = J->P;
    shot_state *S = shot_alloc(P);
    int *fl = (int *)malloc(sizeof(int) * (size_t)(P->nsites + 1));
    run_opts ro = {NULL, NULL, NULL, 0, J->strat_r, J->strat_q};
    for (uint64_t s = J->s0; s < J->s1; s++) {
        run_shot(P, S, J->offset + s, J->seed, &ro, fl);
        uint64_t w = s >> 6, bit = (uint64_t)1 << (s & 63);
        if (J->meas)
            for (int r = 0; r < P->nrec; r++)
                if (S->rec[r]) J->meas[(uint64_t)r * J->words + w] |= bit;
        if (J->det)
            for (int d = 0; d < P->ndet; d++)
                if (S->det[d]) J->det[(uint64_t)d * J->words + w] |= bit;
        if (J->obs)
            for (int d = 0; d < P->nobs; d++)
                if (S->obs[d]) J->obs[(uint64_t)d * J->words + w] |= bit;
        if (J->expvals)
            for (int e = 0; e < P->nprobes; e++) J->expvals[(uint64_t)e * J->shots + s] = S->probe[e];
    }
    J->error = ro.error;
    free(fl);
    shot_free(S);
    return NULL;
}

/* Sample `shots` shots with global indices offset .. offset+shots-1.
 * Outputs are record-major bit-packed: out[r * ceil(shots/64) + s/64] bit
 * s%64; the caller zero-fills them.  strat_r >= 0: every shot has exactly
 * that many faults (draw_faults_strat); returns 4 if that count is
 * impossible. */
int oracle_sample(void *h, uint64_t shots, uint64_t seed, uint64_t offset, int nthreads, uint64_t *meas, uint64_t *det,
                  uint64_t *obs, double *expvals, int strat_r)
{
    program *P = (program *)h;
    uint64_t words = (shots + 63) / 64;
    double *Q = NULL;
    if (strat_r >= 0) {
        Q = strat_tail_pmf(P, strat_r);
        if (!(Q[strat_r] > 0.0)) { free(Q); return 4; }
    }
    if (nthreads < 1) nthreads = 1;
    if ((uint64_t)nthreads > words) nthreads = (int)(words ? words : 1);
    job *jobs = (job *)calloc((size_t)nthreads, sizeof(job));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int t = 0; t < nthreads; t++) {
        uint64_t w0 = words * (uint64_t)t / (uint64_t)nthreads, w1 = words * (uint64_t)(t + 1) / (uint64_t)nthreads;
        jobs[t].P = P;
        jobs[t].s0 = w0 * 64;
        jobs[t].s1 = w1 * 64 < shots ? w1 * 64 : shots;
        jobs[t].offset = offset;
        jobs[t].seed = seed;
        jobs[t].words = words;
        jobs[t].meas = meas;
        jobs[t].det = det;
        jobs[t].obs = obs;
        jobs[t].expvals = expvals;
        jobs[t].shots = shots;
        jobs[t].strat_r = strat_r;
        jobs[t].strat_q = Q;
        pthread_create(&th[t], NULL, sample_worker, &jobs[t]);
    }
    int err = 0;
    for (int t = 0; t < nthreads; t++) {
        pthread_join(th[t], NULL);
        if (jobs[t].error && !err) err = jobs[t].error;
    }
    free(jobs);
    free(th);
    free(Q);
    return err;
}

/* Poisson-binomial distribution of the number of faults over all noise
 * sites (Section 3.2, rare-event sampling: the weight of the stratum of r
 * faults): pmf[r] = Q[0][r], r = 0 .. rmax. */
int oracle_fault_pmf(void *h, int rmax, double *pmf)
{
    program *P = (program *)h;
    if (rmax < 0) return -1;
    double *Q = strat_tail_pmf(P, rmax);
    memcpy(pmf, Q, sizeof(double) * (size_t)(rmax + 1));
    free(Q);
    return 0;
}

/* The faults of one stratified shot (per site: outcome index or -1). */
int oracle_faults_strat(void *h, int r, uint64_t seed, uint64_t shot, int *fault_at_site)
{
    program *P = (program *)h;
    if (r < 0) return -1;
    double *Q = strat_tail_pmf(P, r);
    int rc = draw_faults_strat(P, r, Q, shot, seed, fault_at_site);
    free(Q);
    return rc;
}

/* survival(t) of strat_next for s faults left among the sites j .. N-1. */
double oracle_strat_survival(void *h, int s, int j, int t)
{
    program *P = (program *)h;
    double *Q = strat_tail_pmf(P, s);
    const size_t R = (size_t)s + 1;
    double none = 1.0;
    for (int l = j; l < t; l++) none *= 1.0 - P->sites[l].p;
    double v = none * Q[(size_t)t * R + s] / Q[(size_t)j * R + s];
    free(Q);
    return v;
}

/* Mark post-selected detectors: bit d of mask[d / 64] (nwords words).
 * Returns -1 if a set bit names no detector. */
int oracle_set_postselect(void *h, const uint64_t *mask, int nwords)
{
    program *P = (program *)h;
    for (int w = 0; w < nwords; w++)
        for (int b = 0; b < 64; b++)
            if (((mask[w] >> b) & 1u) && (int64_t)w * 64 + b >= P->ndet) return -1;
    free(P->det_post);
    P->det_post = (uint8_t *)calloc((size_t)P->ndet + 1, 1);
    for (int d = 0; d < P->ndet && d / 64 < nwords; d++) P->det_post[d] = (uint8_t)((mask[d / 64] >> (d % 64)) & 1u);
    return 0;
}
