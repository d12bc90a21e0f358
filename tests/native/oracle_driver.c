/*
 * oracle_driver.c -- runs the CPU oracle (oracle/siminf_oracle.c, included
 * below so that the whole oracle is built with the driver's flags) on one
 * model read from a binary file, and writes the result to another.  Test
 * infrastructure: the CPU test suite builds it with AddressSanitizer and
 * UndefinedBehaviorSanitizer and checks that every case runs clean and
 * gives the same bits as the oracle built normally.
 *
 * Input (native byte order): int32 model, Nc, Nt, Nn, Nv, Nld, Ngd, Ntspan,
 * Nev, Ecols, Ncols, nthreads; uint64 seed; uint32 stream; int32 S[Nc*Nt],
 * G[Nt*Nt], u0[Nc*Nn]; double v0[Nv*Nn], ldata[Nld*Nn], gdata[Ngd],
 * tspan[Ntspan]; int32 ev_type, ev_time, ev_node, ev_dest, ev_n, ev_select,
 * ev_shift [Nev each]; double ev_prop[Nev]; int32 E[Nc*Ecols], N[Nc*Ncols].
 * Output: int64 status, err[4], counters[3]; int32 U[Ntspan*Nn*Nc];
 * double V[Ntspan*Nn*Nv].
 */
#include "../../oracle/siminf_oracle.c"

#include <stdio.h>

static void *read_n(FILE *f, size_t elem, size_t n) {
    void *p = malloc(elem * (n ? n : 1));
    if (!p || fread(p, elem, n, f) != n) {
        fprintf(stderr, "short input\n");
        exit(2);
    }
    return p;
}

int main(int argc, char **argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: %s in out\n", argv[0]);
        return 2;
    }
    FILE *f = fopen(argv[1], "rb");
    if (!f)
        return 2;
    int32_t *h = read_n(f, 4, 12);
    oracle_model m;
    memset(&m, 0, sizeof m);
    m.model = h[0]; m.Nc = h[1]; m.Nt = h[2]; m.Nn = h[3]; m.Nv = h[4];
    m.Nld = h[5]; m.Ngd = h[6]; m.Ntspan = h[7]; m.Nev = h[8];
    m.Ecols = h[9]; m.Ncols = h[10];
    int nthreads = h[11];
    uint64_t *seed = read_n(f, 8, 1);
    uint32_t *stream = read_n(f, 4, 1);
    size_t Nc = m.Nc, Nn = m.Nn, Nev = m.Nev;
    m.S = read_n(f, 4, Nc * m.Nt);
    m.G = read_n(f, 4, (size_t)m.Nt * m.Nt);
    m.u0 = read_n(f, 4, Nc * Nn);
    m.v0 = read_n(f, 8, (size_t)m.Nv * Nn);
    m.ldata = read_n(f, 8, (size_t)m.Nld * Nn);
    m.gdata = read_n(f, 8, m.Ngd);
    m.tspan = read_n(f, 8, m.Ntspan);
    m.ev_type = read_n(f, 4, Nev);
    m.ev_time = read_n(f, 4, Nev);
    m.ev_node = read_n(f, 4, Nev);
    m.ev_dest = read_n(f, 4, Nev);
    m.ev_n = read_n(f, 4, Nev);
    m.ev_select = read_n(f, 4, Nev);
    m.ev_shift = read_n(f, 4, Nev);
    m.ev_prop = read_n(f, 8, Nev);
    m.E = read_n(f, 4, Nc * m.Ecols);
    m.N = read_n(f, 4, Nc * m.Ncols);
    fclose(f);
    size_t nU = (size_t)m.Ntspan * Nn * Nc, nV = (size_t)m.Ntspan * Nn * m.Nv;
    int32_t *U = calloc(nU ? nU : 1, 4);
    double *V = calloc(nV ? nV : 1, 8);
    uint64_t counters[3];
    int64_t err[4];
    int rc = oracle_run(&m, *seed, *stream, nthreads, U, V, counters, err);
    FILE *o = fopen(argv[2], "wb");
    if (!o)
        return 2;
    int64_t head[8] = {rc, err[0], err[1], err[2], err[3], (int64_t)counters[0], (int64_t)counters[1],
                       (int64_t)counters[2]};
    fwrite(head, 8, 8, o);
    fwrite(U, 4, nU, o);
    fwrite(V, 8, nV, o);
    fclose(o);
    free(U); free(V); free(h); free(seed); free(stream);
    free((void *)m.S); free((void *)m.G); free((void *)m.u0); free((void *)m.v0);
    free((void *)m.ldata); free((void *)m.gdata); free((void *)m.tspan);
    free((void *)m.ev_type); free((void *)m.ev_time); free((void *)m.ev_node);
    free((void *)m.ev_dest); free((void *)m.ev_n); free((void *)m.ev_select);
    free((void *)m.ev_shift); free((void *)m.ev_prop); free((void *)m.E); free((void *)m.N);
    return 0;
}
