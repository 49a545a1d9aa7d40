"""Bounds check of recorded kernel launches (test infrastructure, CPU only).

The recording HIP stand-in (mock_hip.cpp) runs the library's real host code
and logs every device allocation and every kernel launch with its grid, block
and argument bytes.  For each kernel this module restates, from the kernel's
source, the largest and smallest element index it can touch through each
pointer argument for the recorded grid and arguments, and checks that the
touched byte range lies inside one allocation that is live at the time of the
launch.  Index expressions are evaluated over the whole grid with numpy where
they depend on the thread, or at their extreme values where the kernel clamps
or guards them.
"""
import struct

import numpy as np

# ---------------------------------------------------------------------------
# Log parsing
# ---------------------------------------------------------------------------


class Launch:
    def __init__(self, name, grid, block, shmem, raw):
        self.name = name
        self.grid = grid
        self.block = block
        self.shmem = shmem
        self.raw = raw          # list of bytes objects, one per argument

    def i(self, j):
        """Argument j as a signed integer (any width)."""
        b = self.raw[j]
        return int.from_bytes(b, "little", signed=True)

    def u(self, j):
        return int.from_bytes(self.raw[j], "little", signed=False)

    def f(self, j):
        b = self.raw[j]
        return struct.unpack("<d" if len(b) == 8 else "<f", b)[0]


def parse_log(path):
    events = []
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if not parts:
                continue
            if parts[0] == "alloc":
                events.append(("alloc", int(parts[1]), int(parts[2])))
            elif parts[0] == "free":
                events.append(("free", int(parts[1])))
            elif parts[0] == "launch":
                name = parts[1]
                grid = tuple(int(x) for x in parts[2:5])
                block = tuple(int(x) for x in parts[5:8])
                shmem = int(parts[8])
                nargs = int(parts[9])
                raw = [bytes.fromhex(h) for h in parts[10:10 + nargs]]
                events.append(("launch", Launch(name, grid, block, shmem, raw)))
            elif parts[0] == "copy":
                events.append(("copy", int(parts[1]), int(parts[2]), int(parts[3]), int(parts[4])))
            elif parts[0] == "data":
                events.append(("data", int(parts[1]), bytes.fromhex(parts[2]) if len(parts) > 2 else b""))
    return events


# ---------------------------------------------------------------------------
# Access records: (argument index, element bytes, min index, max index)
# ---------------------------------------------------------------------------
def cdiv(a, b):
    return -(-a // b)


def acc(j, es, lo, hi):
    return (j, es, int(lo), int(hi))


def _qr_init(L):
    # (R, ldr, m, flag, counters, ncnt)
    ldr, m, ncnt = L.i(1), L.i(2), L.i(5)
    out = [acc(0, 8, 0, (m - 1) + (m - 1) * ldr), acc(3, 8, 0, 0)]
    if ncnt > 0:
        out.append(acc(4, 4, 0, ncnt - 1))
    threads = L.grid[0] * L.block[0]
    assert threads >= max(m * m, ncnt, 1)
    return out


def _sketch_reduce(L):
    # (partial, G, k, ncols, scale, out, ldo, part_cols)
    G, k, ncols, ldo, pc = L.i(1), L.i(2), L.i(3), L.i(6), L.i(7)
    nthr_out = L.grid[0] * 64
    assert nthr_out >= k * ncols, "reduction grid does not cover the outputs"
    assert L.block[0] == 16 * 64
    return [acc(0, 8, 0, (k * ncols - 1) + (G - 1) * pc * k),
            acc(5, 8, 0, (k - 1) + (ncols - 1) * ldo)]


def _gram_sty(L):
    # (S, k, K, X0, n0, X1, n1, out0, ldo0, out1, ldo1, out1t, ldo1t)
    k, K, n0, n1 = L.i(1), L.i(2), L.i(4), L.i(6)
    ldo0, ldo1, ldo1t = L.i(8), L.i(10), L.i(12)
    ncol = n0 + n1
    assert L.grid[0] * L.block[0] // 64 >= K * ncol
    out = [acc(0, 8, 0, K * k - 1)]
    if n0 > 0:
        out += [acc(3, 8, 0, n0 * k - 1), acc(7, 8, 0, (K - 1) + (n0 - 1) * ldo0)]
    if n1 > 0:
        out += [acc(5, 8, 0, n1 * k - 1), acc(9, 8, 0, (K - 1) + (n1 - 1) * ldo1)]
        if L.u(11) != 0:
            out.append(acc(11, 8, 0, (n1 - 1) + (K - 1) * ldo1t))
    return out


def _gram_sweep(L):
    # (G, ldg, K, C, Y, ldy, Ynew, ldyn, bw)
    ldg, K, ldy, ldyn, bw = L.i(1), L.i(2), L.i(5), L.i(7), L.i(8)
    assert L.grid[0] * L.block[0] // 16 >= K * bw
    return [acc(0, 8, 0, (K - 1) * ldg + K - 1), acc(3, 8, 0, (K - 1) + (bw - 1) * K),
            acc(4, 8, 0, (bw - 1) * ldy + K - 1), acc(6, 8, 0, (K - 1) + (bw - 1) * ldyn)]


def _resid(L, NC):
    # (P, S, k, K, Y, ldy, E, bw): 16 lanes per row and NC columns; columns of Y
    # clamped to bw - 1
    k, K, ldy, bw = L.i(2), L.i(3), L.i(5), L.i(7)
    assert K >= 1 and bw >= 1
    assert L.grid[0] * L.block[0] // 16 >= k * cdiv(bw, NC)
    return [acc(0, 8, 0, (k - 1) + (bw - 1) * k), acc(1, 8, 0, (k - 1) + (K - 1) * k),
            acc(4, 8, 0, (bw - 1) * ldy + K - 1), acc(6, 8, 0, (k - 1) + (bw - 1) * k)]


def qr_bwp(bw):
    return 4 if bw <= 4 else (8 if bw <= 8 else (16 if bw <= 16 else 32))


def qr_chunk_rows(bw):
    return (256 // qr_bwp(bw)) * 16


def _qr_fused(L):
    # (src, k, bw, stack, counters, ncnt, Rii, ldr, flag, col0)
    k, bw, ncnt, ldr = L.i(1), L.i(2), L.i(5), L.i(7)
    CH = qr_chunk_rows(bw)
    nch = cdiv(k, CH)
    assert L.grid[0] == nch and L.block[0] == 256
    out = [acc(0, 8, 0, (k - 1) + (bw - 1) * k), acc(6, 8, 0, (bw - 1) + (bw - 1) * ldr),
           acc(8, 8, 0, 0)]
    if nch == 1:
        return out
    # grouped tree: level l holds n_l R factors (n_0 = nch), n_(l+1) = ceil(n_l / fan),
    # a counter per group of each level
    fan = CH // bw
    need, n = 0, nch
    while n > 1:
        need += cdiv(n, fan)
        n = cdiv(n, fan)
    if need <= ncnt:
        hi, n, off = -1, nch, 0
        while n > 1:
            hi = max(hi, off + n * bw * bw - 1)
            off += n * bw * bw
            n = cdiv(n, fan)
        return out + [acc(3, 8, 0, hi), acc(4, 4, 0, need - 1)]
    # one group: level 1 rows [b bw, b bw + bw) of a (nch bw) x bw stack, then
    # the further levels of re-chunked stacked rows
    ld1 = nch * bw
    hi = ld1 * bw - 1
    lrows, off = ld1, ld1 * bw
    while lrows > CH:
        n2 = cdiv(lrows, CH)
        out_rows = n2 * bw
        hi = max(hi, off + out_rows * bw - 1)      # writes of this level
        off += out_rows * bw
        lrows = out_rows
    out += [acc(3, 8, 0, hi), acc(4, 4, 0, 0)]
    return out


def _sketch_identity(L, T):
    # (X, ldx, n, ncols, out, ldo)
    es = 4 if T == "f" else 8
    ldx, n, ncols, ldo = L.i(1), L.i(2), L.i(3), L.i(5)
    assert L.grid[0] * L.block[0] >= n * ncols
    return [acc(0, es, 0, (n - 1) + (ncols - 1) * ldx), acc(4, 8, 0, (n - 1) + (ncols - 1) * ldo)]


def _qr_wave(L):
    # (src, k, bw, Rii, ldr, flag, col0)
    k, bw, ldr = L.i(1), L.i(2), L.i(4)
    return [acc(0, 8, 0, (k - 1) + (bw - 1) * k), acc(3, 8, 0, (bw - 1) + (bw - 1) * ldr),
            acc(5, 8, 0, 0)]


def _trmm_upper(L):
    # (A, lda, R, ldr, bw): thread (i, j) = (t % 32, t / 32)
    lda, ldr, bw = L.i(1), L.i(3), L.i(4)
    assert L.grid[0] == 1 and L.block[0] == 1024 and 1 <= bw <= 32
    return [acc(0, 8, 0, (bw - 1) + (bw - 1) * lda), acc(2, 8, 0, (bw - 1) + (bw - 1) * ldr)]


def _hh_absorb(L, RPT, CPW):
    # (Snew, k, c0, bw, HS, tau)
    k, c0, bw = L.i(1), L.i(2), L.i(3)
    assert L.grid[0] == 1 and L.block[0] == 1024
    assert 64 * RPT >= k and 16 * CPW >= bw >= 1 and c0 >= 0
    return [acc(0, 8, 0, (k - 1) + (bw - 1) * k), acc(4, 8, 0, (c0 + bw) * k - 1),
            acc(5, 8, 0, c0 + bw - 1)]


def _hh_solve(L, RPT):
    # (HS, tau, P, k, K, bw, Y, ldy)
    k, K, bw, ldy = L.i(3), L.i(4), L.i(5), L.i(7)
    assert L.grid[0] == 1 and L.block[0] == 1024
    assert 64 * RPT >= k and 1 <= K <= 1024 and 1 <= bw <= 32
    return [acc(0, 8, 0, K * k - 1), acc(1, 8, 0, K - 1), acc(2, 8, 0, (k - 1) + (bw - 1) * k),
            acc(6, 8, 0, (K - 1) + (bw - 1) * ldy)]


def _update_general(L, T, NB):
    # (W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr, nfull, n, K, bw)
    es = 4 if T == "f" else 8
    VEC = 16 // es
    TILE = 4 * 16 * VEC
    ldw, ldq, ldqo, ldr = L.i(1), L.i(3), L.i(5), L.i(8)
    nfull, n, K, bw = L.i(9), L.i(10), L.i(11), L.i(12)
    assert L.grid[0] == cdiv(n, TILE) and L.block[0] == 256
    assert 1 <= bw <= 16 * NB
    assert nfull * TILE <= n
    last = n - 1
    out = [acc(0, es, 0, last + (bw - 1) * ldw), acc(4, es, 0, last + (bw - 1) * ldqo)]
    if K > 0:
        out += [acc(2, es, 0, last + (K - 1) * ldq), acc(6, 8, 0, (K - 1) + (bw - 1) * ldr)]
    if L.u(7) != 0:
        out.append(acc(7, 8, 0, (bw - 1) + (bw - 1) * ldr))
    return out


def _update_persistent(L, T, NB=1, form=None):
    # (W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr, ntiles, nfull, n, K, Kp, bw)
    es = 4 if T == "f" else 8
    VEC = 16 // es
    WAVES = 8
    TILE = WAVES * 16 * VEC
    NCOL = 16 * NB
    ldw, ldq, ldqo, ldr = L.i(1), L.i(3), L.i(5), L.i(8)
    ntiles, nfull, n, K, Kp, bw = L.i(9), L.i(10), L.i(11), L.i(12), L.i(13), L.i(14)
    assert L.block[0] == 64 * WAVES and L.grid[0] <= (512 if NB == 1 else 256)
    assert ntiles == cdiv(n, TILE) and nfull * TILE <= n and bw <= NCOL
    align = 16 if NB == 1 else 32    # whole pairs of the K loop's load groups
    assert Kp == cdiv(K, align) * align <= (512 if NB == 1 else 480)
    assert form == (2 if K > 0 else 0) + (1 if bw == NCOL else 0), "form does not match K, bw"
    assert L.shmem >= (Kp * NCOL + NCOL * NCOL + NCOL) * 8
    assert L.shmem <= 160 * 1024
    last = n - 1
    out = [acc(0, es, 0, last + (bw - 1) * ldw), acc(4, es, 0, last + (bw - 1) * ldqo),
           acc(6, 8, 0, max(0, (K - 1) + (bw - 1) * ldr))]
    if K > 0:
        out.append(acc(2, es, 0, last + (K - 1) * ldq))
    if L.u(7) != 0:
        out.append(acc(7, 8, 0, (bw - 1) + (bw - 1) * ldr))
    return out


def _update_fused(L, T, form, RPT):
    # (W, ldw, Q, ldq, Qout, ldqo, Rk, Rii, ldr, ntiles, nfull, n, K, Kp, bw,
    #  E, k, flag, col0, ready, limit, subst): the persistent update in eight-wave
    # workgroups, the first of which factors the k x bw sketch E into R_(i,i)
    es = 4 if T == "f" else 8
    VEC = 16 // es
    TILE = 8 * 16 * VEC
    ldw, ldq, ldqo, ldr = L.i(1), L.i(3), L.i(5), L.i(8)
    ntiles, nfull, n, K, Kp, bw = L.i(9), L.i(10), L.i(11), L.i(12), L.i(13), L.i(14)
    k = L.i(16)
    assert L.block[0] == 512 and L.grid[0] >= 2
    assert ntiles == cdiv(n, TILE) and nfull * TILE <= n
    assert form == 3 and bw == 16 and 48 <= K <= 512 and Kp == cdiv(K, 16) * 16
    assert bw <= k <= 64 * RPT and RPT in (4, 8, 16)
    assert L.shmem >= max((Kp * 16 + 16 * 16 + 16) * 8, (2 * 64 * RPT + 2 + 16) * 8)
    assert L.shmem <= 160 * 1024
    assert L.u(20) > 0 and L.i(21) == 1, "wait limit, substitution on"
    last = n - 1
    return [acc(0, es, 0, last + (bw - 1) * ldw), acc(4, es, 0, last + (bw - 1) * ldqo),
            acc(2, es, 0, last + (K - 1) * ldq), acc(6, 8, 0, (K - 1) + (bw - 1) * ldr),
            acc(7, 8, 0, (bw - 1) + (bw - 1) * ldr), acc(15, 8, 0, (k - 1) + (bw - 1) * k),
            acc(17, 8, 0, 0), acc(19, 4, 0, 0)]


def _trsm(L, T):
    # (Qb, ldq, Rii, ldr, n, bw)
    es = 4 if T == "f" else 8
    ldq, ldr, n, bw = L.i(1), L.i(3), L.i(4), L.i(5)
    return [acc(0, es, 0, (n - 1) + (bw - 1) * ldq), acc(2, 8, 0, (bw - 1) + (bw - 1) * ldr)]


def _sketch_gauss(L, T, NCG):
    # (X, ldx, n, ncols, row0, k, key0, key1, rows_per_wg, partial, X2, ldx2, n1)
    es = 4 if T == "f" else 8
    ldx, n, ncols, k, rpw = L.i(1), L.i(2), L.i(3), L.i(5), L.i(8)
    ldx2, n1 = L.i(11), L.i(12)
    G = L.grid[0]
    NC = 16 * NCG
    S0 = cdiv(ncols, 16) * 16 if n1 > 0 else ncols
    NS = S0 + n1 if n1 > 0 else ncols
    assert L.block[0] == 256
    assert L.grid[1] * 256 >= k, "targets not covered"
    assert L.grid[2] * NC >= NS, "column slots not covered"
    assert G * rpw >= n, "rows not covered"
    rbeg = np.arange(G, dtype=np.int64) * rpw
    rend = np.minimum(n, rbeg + rpw)
    active = rbeg < rend
    out = []
    if active.any():
        rmax = int(rend[active].max()) - 1
        out.append(acc(0, es, 0, rmax + (ncols - 1) * ldx))
        if n1 > 0:
            out.append(acc(10, es, 0, rmax + (n1 - 1) * ldx2))
    out.append(acc(9, 8, 0, G * NS * k - 1))
    return out


def _sketch_sparse_q(L, T, TPT, MANY):
    # (X, ldx, n, ncols, k, zeta, plan_off, plan_ent, tiles_per_wg, partial, G)
    es = 4 if T == "f" else 8
    ldx, n, ncols, k, zeta, tpw, G = L.i(1), L.i(2), L.i(3), L.i(4), L.i(5), L.i(8), L.i(10)
    if es == 4:
        NT, NC = (1024, 16) if MANY else (1024, 8)
    else:
        NT, NC = (512, 4) if MANY else (1024, 4)
    assert L.block[0] == NT
    assert TPT * NT >= k
    slices = cdiv(ncols, NC)
    assert L.grid[0] == G * slices
    ntiles = cdiv(n, 1024)
    assert G * tpw >= ntiles
    E = 1024 * zeta
    return [acc(0, es, 0, (n - 1) + (ncols - 1) * ldx),
            acc(6, 2, 0, ntiles * (k + 1) - 1),
            acc(7, 2, 0, ntiles * E - 1),
            acc(9, 8, 0, G * ncols * k - 1)]


def _sparse_plan(L):
    # (n, row0, k, zeta, key0, key1, plan_off, plan_ent)
    n, k, zeta = L.i(0), L.i(2), L.i(3)
    ntiles = cdiv(n, 1024)
    assert L.grid[0] == ntiles and L.block[0] == 1024 and k <= 2048 and zeta <= 8
    return [acc(6, 2, 0, ntiles * (k + 1) - 1), acc(7, 2, 0, ntiles * 1024 * zeta - 1)]


def _gram_defect(L):
    # (S, k, m, out)
    k, m = L.i(1), L.i(2)
    assert L.grid[0] * 4 >= m * m
    return [acc(0, 8, 0, (k - 1) + (m - 1) * k), acc(3, 8, 0, m * m - 1)]


def _sketch_resid(L):
    # (S, P, R, ldr, k, m, out, out2)
    ldr, k, m = L.i(3), L.i(4), L.i(5)
    assert L.grid[0] * 256 >= k and L.grid[1] == m
    return [acc(0, 8, 0, (k - 1) + (m - 1) * k), acc(1, 8, 0, (k - 1) + (m - 1) * k),
            acc(2, 8, 0, (m - 1) + (m - 1) * ldr), acc(6, 8, 0, (k - 1) + (m - 1) * k),
            acc(7, 8, 0, (k - 1) + (m - 1) * k)]


def _sum(L):
    # (v, len, out)
    return [acc(0, 8, 0, L.i(1) - 1), acc(2, 8, 0, 0)]


def _finite(L):
    # (S, R, ldr, k, m, out)
    ldr, k, m = L.i(2), L.i(3), L.i(4)
    return [acc(0, 8, 0, k * m - 1), acc(1, 8, 0, (m - 1) + (m - 1) * ldr),
            acc(5, 8, 0, k * m + m * m - 1)]


def _sketch_srht(L, T, TPT):
    # (X, ldx, n, ncols, row0, k, logn, key0, key1, chunks_per_wg, partial)
    es = 4 if T == "f" else 8
    ldx, n, ncols, k = L.i(1), L.i(2), L.i(3), L.i(5)
    G = L.grid[0]
    return [acc(0, es, 0, (n - 1) + (ncols - 1) * ldx), acc(10, 8, 0, G * ncols * k - 1)]


# ---------------------------------------------------------------------------
# Persistent batch.  The descriptors are read from the bytes the host uploaded
# (the "data" events); every access is returned as ("abs", first byte, end
# byte) of device memory.
# ---------------------------------------------------------------------------
MEM = {}          # device address -> uploaded bytes (set by check_events)
PB_FMT = "<13Q4q2I10i"   # struct PbProb: 13 pointers, n, ldw, ldq, ldr, key0, key1, 10 int32
PB_SIZE = struct.calcsize(PB_FMT) + (-struct.calcsize(PB_FMT)) % 8
PB_FIELDS = ("W Q R S P E G Cb Yb part flag plan_off plan_ent n ldw ldq ldr key0 key1 "
             "m p k nb plan_tiles sk_G sk_tpw up_tiles up_nfull pad").split()
PB_LDS = 144 * 1024
PB_TILE = 1024


def uploaded(addr):
    assert addr in MEM, f"no upload at {addr:#x}"
    return MEM[addr]


def pb_problems(addr, count=None):
    raw = uploaded(addr)
    assert len(raw) % PB_SIZE == 0, "descriptor array size"
    np_ = len(raw) // PB_SIZE if count is None else count
    out = []
    for q in range(np_):
        vals = struct.unpack_from(PB_FMT[:-3] + "9i", raw, q * PB_SIZE)
        out.append(dict(zip(PB_FIELDS, vals)))
    return out


def absacc(ptr, es, lo, hi):
    return ("abs", ptr + int(lo) * es, ptr + (int(hi) + 1) * es)


def pb_items(P, kind, block):
    """Items of a stage (restated from the device code)."""
    bw = min(P["p"], P["m"] - block * P["p"])
    red = 4 * 1024
    if kind == "plan":
        return cdiv(P["plan_tiles"], 8)
    if kind == "wsk":
        return P["sk_G"] * cdiv(P["m"], 16)
    if kind == "redw":
        return cdiv(P["k"] * P["m"], red)
    if kind == "small":
        return 1
    if kind == "upd":
        return cdiv(P["up_tiles"], 16)
    if kind == "qsk":
        return P["sk_G"] * cdiv(bw, 16 if bw > 8 else 8)
    return cdiv(P["k"] * bw, red)


def pb_chain(P):
    """Stages of one problem in the order the queue runs them."""
    out = [("plan", 0), ("wsk", 0), ("redw", 0)]
    for b in range(P["nb"]):
        out += [("small", b), ("upd", b)]
        if b + 1 < P["nb"]:
            out += [("qsk", b), ("reds", b)]
    return out


def pb_problem_accesses(P, zeta, ls):
    n, m, p, k = P["n"], P["m"], P["p"], P["k"]
    ldw, ldq, ldr = P["ldw"], P["ldq"], P["ldr"]
    G, tpw = P["sk_G"], P["sk_tpw"]
    assert 1 <= p <= 32 and 1 <= m <= n and m <= k <= 1024 and zeta <= 8 and k % zeta == 0
    assert P["nb"] == cdiv(m, p)
    tiles = cdiv(n, 1024)
    assert P["plan_tiles"] == tiles
    assert G * tpw >= tiles and (G - 1) * tpw < tiles, "sketch row groups"
    assert G <= 16 and (tpw >= 4 or tpw == tiles)
    rows = PB_TILE if p <= 16 else PB_TILE // 2
    assert P["up_tiles"] == cdiv(n, rows)
    assert P["up_nfull"] * rows <= n
    if P["up_nfull"] > 0:
        assert P["W"] % 16 == 0 and P["Q"] % 16 == 0 and ldw % 4 == 0 and ldq % 4 == 0
    ncol = 16 if p <= 16 else 32
    out = [absacc(P["plan_off"], 2, 0, tiles * (k + 1) - 1),
           absacc(P["plan_ent"], 2, 0, tiles * 1024 * zeta - 1),
           absacc(P["flag"], 8, 0, 0)]
    for kind, b in pb_chain(P):
        assert pb_items(P, kind, b) >= 1
        c0 = b * p
        K = c0
        bw = min(p, m - c0)
        if kind == "wsk":
            out += [absacc(P["W"], 4, 0, (n - 1) + (m - 1) * ldw),
                    absacc(P["part"], 8, 0, G * m * k - 1)]
        elif kind == "redw":
            out += [absacc(P["part"], 8, 0, G * m * k - 1), absacc(P["P"], 8, 0, k * m - 1)]
        elif kind == "small":
            if K > 0:
                bp = p
                out += [absacc(P["S"], 8, 0, K * k - 1),                       # S_(1:i-1)
                        absacc(P["P"], 8, K * k, K * k + bw * k - 1),          # P_(i)
                        absacc(P["G"], 8, (K - bp) * m, (K - bp) * m + (K - 1) + (bp - 1) * m),
                        absacc(P["G"], 8, K - bp, (K - bp) + (bp - 1) + (K - 1) * m),
                        absacc(P["G"], 8, 0, (K - 1) * m + K - 1),             # sweeps
                        absacc(P["R"], 8, K * ldr, K * ldr + (K - 1) + (bw - 1) * ldr),
                        absacc(P["E"], 8, 0, k * bw - 1)]
                if ls > 1:
                    out += [absacc(P["Cb"], 8, 0, K * bw - 1), absacc(P["Yb"], 8, 0, K * bw - 1)]
            out.append(absacc(P["R"], 8, c0 + c0 * ldr, c0 + c0 * ldr + (bw - 1) + (bw - 1) * ldr))
            out.append(absacc(P["P"] if K == 0 else P["E"], 8, 0, k * bw - 1))
        elif kind == "upd":
            align = 16 if ncol == 16 else 32
            Kp = cdiv(K, align) * align
            assert (Kp * ncol + ncol * ncol + ncol) * 8 <= PB_LDS, "update factors exceed the LDS pool"
            assert bw <= ncol
            out += [absacc(P["W"], 4, c0 * ldw, (n - 1) + (c0 + bw - 1) * ldw),
                    absacc(P["Q"], 4, c0 * ldq, (n - 1) + (c0 + bw - 1) * ldq),
                    absacc(P["R"], 8, c0 + c0 * ldr, c0 + c0 * ldr + (bw - 1) + (bw - 1) * ldr)]
            if K > 0:
                out += [absacc(P["Q"], 4, 0, (n - 1) + (K - 1) * ldq),
                        absacc(P["R"], 8, c0 * ldr, c0 * ldr + (K - 1) + (bw - 1) * ldr)]
        elif kind == "qsk":
            out += [absacc(P["Q"], 4, c0 * ldq, (n - 1) + (c0 + bw - 1) * ldq),
                    absacc(P["part"], 8, 0, G * bw * k - 1)]
        elif kind == "reds":
            out += [absacc(P["part"], 8, 0, G * bw * k - 1),
                    absacc(P["S"], 8, c0 * k, c0 * k + bw * k - 1)]
    return out


PB_LEVELS = 4
PB_CTL = 16 * PB_LEVELS + 16   # struct PbCtl


def pb_level(nb, kind, block):
    rem = nb if kind in ("plan", "wsk", "redw") else nb - block
    return min(PB_LEVELS - 1, (rem - 1) // 2)


def pb_queue0(L, probs, total):
    """The queue the host uploads: every problem's first stage once, in its
    level's range; ranges that partition [0, total) with room for each level's
    stages."""
    st = struct.unpack("<%di" % (4 * total), uploaded(L.u(2)))
    va = struct.unpack("<%dI" % total, uploaded(L.u(3)))
    c0 = struct.unpack("<20I", uploaded(L.u(4)))
    head, tail, base, end = c0[0:4], c0[4:8], c0[8:12], c0[12:16]
    need = [0] * PB_LEVELS
    for P in probs:
        for kind, b in pb_chain(P):
            need[pb_level(P["nb"], kind, b)] += 1
    assert base[0] == 0 and end[PB_LEVELS - 1] == total
    firsts = {}
    for lv in range(PB_LEVELS):
        assert end[lv] - base[lv] == need[lv], "level range"
        if lv:
            assert base[lv] == end[lv - 1]
        assert head[lv] == base[lv] <= tail[lv] <= end[lv]
        for t in range(base[lv], end[lv]):
            q, kind, blk = st[4 * t:4 * t + 3]
            assert bool(va[t]) == (t < tail[lv])
            if va[t]:
                assert kind == 0 and blk == 0 and q not in firsts
                assert pb_level(probs[q]["nb"], "plan", 0) == lv
                firsts[q] = t
    assert sorted(firsts) == list(range(len(probs)))


def _persistent_init(L):
    # (probs, nprob, stages0, valid0, ctl0, stages, claimed, finished, valid, ctl, total)
    nprob, total = L.i(1), L.u(10)
    probs = pb_problems(L.u(0))
    assert len(probs) == nprob
    pb_queue0(L, probs, total)
    assert L.block[0] == 256 and L.grid[1] == nprob + 1
    assert L.grid[0] * 256 >= total
    out = [absacc(L.u(0), PB_SIZE, 0, nprob - 1), acc(2, 16, 0, total - 1),
           acc(3, 4, 0, total - 1), acc(4, PB_CTL, 0, 0), acc(5, 16, 0, total - 1),
           acc(6, 4, 0, total - 1), acc(7, 4, 0, total - 1), acc(8, 4, 0, total - 1),
           acc(9, PB_CTL, 0, 0)]
    for P in probs:
        m = P["m"]
        assert L.grid[0] * 256 >= m * m
        out += [absacc(P["R"], 8, 0, (m - 1) + (m - 1) * P["ldr"]), absacc(P["flag"], 8, 0, 0)]
    return out


def _persistent_batch(L):
    # (probs, stages, claimed, finished, valid, ctl, total, zeta, ls, limit)
    total, zeta, ls = L.u(6), L.i(7), L.i(8)
    probs = pb_problems(L.u(0))
    assert L.block[0] == 1024 and L.grid[0] >= 1 and L.shmem == 0
    assert total == sum(len(pb_chain(P)) for P in probs) == sum(4 * P["nb"] + 1 for P in probs)
    assert L.u(9) > 0, "wait limit"
    out = [absacc(L.u(0), PB_SIZE, 0, len(probs) - 1), acc(1, 16, 0, total - 1),
           acc(2, 4, 0, total - 1), acc(3, 4, 0, total - 1), acc(4, 4, 0, total - 1),
           acc(5, PB_CTL, 0, 0)]
    for P in probs:
        out += pb_problem_accesses(P, zeta, ls)
    return out


def _template_args(name):
    """Template arguments of a mangled kernel name, e.g. IfdLi2EE -> ['f', 'd', 2]."""
    base = kernel_base(name)
    i = name.find("I", name.find(base) + len(base))
    j = name.find("EE", i)
    if i < 0 or j < 0 or i > j:
        return []
    body = name[i + 1:j + 1]
    out, p = [], 0
    while p < len(body):
        c = body[p]
        if c in "fd":
            out.append(c)
            p += 1
        elif c == "N":                 # a nested class name, e.g. NS_6Bf16x3E
            q = body.find("E", p)
            k = p + 1
            while k < q and not body[k].isdigit():
                k += 1
            m = k
            while m < q and body[m].isdigit():
                m += 1
            out.append(body[m:m + int(body[k:m])] if m > k else body[p + 1:q])
            p = q + 1
        elif c == "b":                 # bool in a literal: Lb0E / Lb1E handled below
            p += 1
        elif c == "L":
            q = body.find("E", p)
            lit = body[p + 1:q]
            if lit.startswith("i"):
                out.append(int(lit[1:]))
            elif lit.startswith("b"):
                out.append(bool(int(lit[1:])))
            p = q + 1
        else:
            p += 1
    return out


MIRRORS = {
    "qr_init_kernel": _qr_init,
    "sketch_reduce_kernel": _sketch_reduce,
    "gram_sty_kernel": _gram_sty,
    "gram_sweep_kernel": _gram_sweep,
    "qr_fused_kernel": _qr_fused,
    "sparse_plan_kernel": _sparse_plan,
    "gram_defect_kernel": _gram_defect,
    "sketch_resid_kernel": _sketch_resid,
    "sum_kernel": _sum,
    "finite_kernel": _finite,
    "trmm_upper_kernel": _trmm_upper,
    "persistent_init_kernel": _persistent_init,
    "persistent_batch_kernel": _persistent_batch,
}
TEMPLATED = {
    "update_kernel": lambda L, t: _update_general(L, t[0], t[2]),
    "update_p_kernel": lambda L, t: _update_persistent(L, t[0], int(t[1]), int(t[2])),
    "update_fused_kernel": lambda L, t: _update_fused(L, t[0], int(t[1]), int(t[2])),
    "trsm_kernel": lambda L, t: _trsm(L, t[0]),
    "resid_cols_kernel": lambda L, t: _resid(L, int(t[0])),
    "sketch_gauss_kernel": lambda L, t: _sketch_gauss(L, t[0], t[2]),
    "sketch_sparse_q_kernel": lambda L, t: _sketch_sparse_q(L, t[0], t[1], t[2]),
    "sketch_srht_kernel": lambda L, t: _sketch_srht(L, t[0], t[1]),
    "qr_wave_kernel": lambda L, t: _qr_wave(L),
    "sketch_identity_kernel": lambda L, t: _sketch_identity(L, t[0]),
    "hh_absorb_kernel": lambda L, t: _hh_absorb(L, t[0], t[1]),
    "hh_solve_kernel": lambda L, t: _hh_solve(L, t[0]),
}


def kernel_base(name):
    """rbgs::<base> from a mangled name _ZN4rbgs<len><base>..."""
    assert name.startswith("_ZN4rbgs")
    p = len("_ZN4rbgs")
    q = p
    while name[q].isdigit():
        q += 1
    ln = int(name[p:q])
    return name[q:q + ln]


def check_events(events):
    """Returns (violations, launches checked, names of kernels seen)."""
    live = {}
    violations = []
    seen = set()
    n = 0
    MEM.clear()
    for ev in events:
        if ev[0] == "data":
            MEM[ev[1]] = ev[2]
        elif ev[0] == "alloc":
            live[ev[1]] = ev[2]
        elif ev[0] == "free":
            live.pop(ev[1], None)
        elif ev[0] == "launch":
            L = ev[1]
            base = kernel_base(L.name)
            seen.add(base)
            if base in MIRRORS:
                accesses = MIRRORS[base](L)
            elif base in TEMPLATED:
                accesses = TEMPLATED[base](L, _template_args(L.name))
            else:
                violations.append(f"no bounds mirror for kernel {base}")
                continue
            n += 1
            for a in accesses:
                if a[0] == "abs":
                    j, (a0, a1) = "(descriptor)", a[1:]
                else:
                    j, es, lo, hi = a
                    ptr = L.u(j)
                    a0, a1 = ptr + lo * es, ptr + (hi + 1) * es
                ok = any(b <= a0 and a1 <= b + sz for b, sz in live.items())
                if not ok:
                    violations.append(f"{base} grid {L.grid}: argument {j} touches "
                                      f"[{a0:#x}, {a1:#x}) outside every live allocation")
    return violations, n, seen
