"""CPU check of the 2D sweep kernel's indexing (no GPU).

The sweep kernel addresses its arrays through wave-uniform bases plus per-lane
and per-step byte offsets; a lane with no work gets an offset at or past 2^31,
which the hardware turns into a dropped access.  This module restates the
planner's chunk, band-group and slot layout and the kernel's index arithmetic
(task -> band group, chunk; wave -> band, group block; lane -> channel, row;
step -> column) and checks, for every launch shape (waves per band 1, 2, 4;
bands per workgroup 1 .. 16; groups per lane 1, 2, 4; FP32 and FP64), on
regular, ragged and degenerate meshes:

* every access of a lane with work lies inside its allocation and inside
  the buffer resource it goes through, with a byte offset below 2^31;
* every lane without work is marked out of range;
* the trace words the publishing wave of a workgroup writes (its top band's
  outflow) are exactly the words the receiving wave of the workgroup above
  reads, and each is written once;
* the LDS hand-off slot a band writes at one step is the slot the band above
  (or the publishing wave) reads at the next barrier interval, the receiving
  wave's slot for column c is written in the interval before the bottom band
  reads it and not overwritten before, and every LDS index stays inside its
  array;
* every wave of a workgroup passes the same number of barriers;
* each moment partial of a (chunk, band, step) is stored once, and the
  finalisation reads only partials of cells inside the mesh.

It is run before kernel changes go to a GPU.
"""
import itertools

import numpy as np
import pytest

from paper_2504_21784_amd import workloads as W

BAND_ROWS, CHANNELS, OOB = 16, 4, 1 << 31
TRACE_LAG = 8


def quadrant_dirs(omega):
    q = []
    for d, (mu, eta, _) in enumerate(omega):
        q.append(0 if (mu > 0 and eta > 0) else 1 if (mu < 0 and eta > 0) else 2 if (mu < 0 and eta < 0) else 3)
    return [[d for d in range(len(q)) if q[d] == k] for k in range(4)]


def plan(nx, ny, G, omega, NW, K):
    """Chunks (quadrant, direction, block of 4 K NW groups) and their slots
    (group block w, channel c, pair k) -> (direction, group) or (-1, -1)."""
    qd = quadrant_dirs(omega)
    GB = 4 * K * NW
    ngb = (G + GB - 1) // GB
    qc_quad, qc_dir, slots = [], [], []
    for q in range(4):
        for d in qd[q]:
            for gb in range(ngb):
                qc_quad.append(q)
                qc_dir.append(d)
                s = []
                for w in range(NW):
                    for c in range(CHANNELS):
                        for k in range(K):
                            g = gb * GB + w * CHANNELS * K + CHANNELS * k + c
                            s.append((d, g) if g < G else (-1, -1))
                slots.append(s)
    nbands = (ny + BAND_ROWS - 1) // BAND_ROWS
    return dict(qc_quad=qc_quad, qc_dir=qc_dir, slots=slots, NQC=len(qc_quad), R=4 * NW * K, nbands=nbands,
                NT=nx + BAND_ROWS - 1)


def prefetch_steps(rs, K, waves):
    """Steps per unrolled round of the kernel's step loop (prefetch depth + 1)."""
    if rs == 4:
        pf = (3 if K == 1 else 1) if waves >= 16 else {1: 4, 2: 3, 4: 1}[K]
    else:
        pf = 1 if waves >= 16 else (2 if K == 1 else 1)
    return pf + 1


def check_shape(nx, ny, G, sn, NW, NBW, K, rs):
    omega, _ = W.level_symmetric_2d(sn)
    nang = len(omega)
    P = plan(nx, ny, G, omega, NW, K)
    NQC, R, nb, NT = P["NQC"], P["R"], P["nbands"], P["NT"]
    TW = rs // 4
    NB = 4 * (nx + ny)
    gslab = nb * NT * BAND_ROWS
    n_groups = (nb + NBW - 1) // NBW
    if n_groups > 1 and NW * NBW > 8:
        return   # the planner rejects it: stacked band groups take at most 8 compute waves
    STEPS = prefetch_steps(rs, K, NW * NBW)
    NTP = (NT + STEPS - 1) // STEPS * STEPS
    # allocations (elements of the unit each array is addressed in)
    n_psi = nang * G * gslab            # r4 records
    n_tab = 4 * G * gslab               # r2 / r4 records of the per-quadrant tables
    n_inf = nang * G * NB               # reals
    slot_words = nx * 2 * TW            # one slot's words in a band's trace block
    n_trace = NQC * nb * R * slot_words
    n_part = NQC * nb * NT * 64         # r2 records
    n_hand = 2 * NBW * NW * K * CHANNELS * 2
    n_ring = 2 * NBW * NW * 64
    n_recv = 2 * NW * K * CHANNELS * 2
    assert CHANNELS * K * nb * NT * BAND_ROWS * 4 * rs < OOB, "planner would reject this mesh"
    written = np.zeros(n_trace, np.int32)
    read_words = np.zeros(n_trace, np.int32)
    part_owner = np.zeros(n_part, np.int32)
    lane = np.arange(64)
    ch, r = lane >> 4, lane & 15
    t = np.arange(NT)
    for qc in range(NQC):
        quad = P["qc_quad"][qc]
        fx, fy = quad in (1, 2), quad in (2, 3)
        slots = P["slots"][qc]
        d = slots[0][0]
        assert d >= 0, "slot 0 of a chunk must be active"
        for bg in range(n_groups):
            hand_w = {}   # LDS hand-off writes: (parity, band slot, w, k, ch, column) -> barrier interval
            barriers = []
            XW = n_groups > 1
            NSLOT = CHANNELS * K * NW
            total = NTP + BAND_ROWS * (NBW - 1)   # barrier intervals after the first barrier
            RP = 4                                # the receiving wave's columns in flight
            active_iv = (nx - 1 + RP - 1) // RP * RP
            # the receiving wave's LDS writes: column c < nx into slot c & 1 in
            # interval c - 1 (column 0 before the first barrier); it writes
            # columns up to active_iv, whose slots nobody reads past nx - 1
            recv_w = {}
            if XW and bg * NBW > 0:
                assert active_iv <= total
                for sl in range(NSLOT):
                    sc, sk, sw = sl % CHANNELS, (sl // CHANNELS) % K, sl // (CHANNELS * K)
                    for c in range(0, active_iv + 1):
                        idx = ((((c & 1) * NW + sw) * K + sk) * CHANNELS + sc) * 2
                        assert 0 <= idx and idx + 1 < n_recv
                        recv_w[(c & 1, sw, sk, sc, c)] = c - 1
            for bw in range(NBW):
                band = bg * NBW + bw
                for w in range(NW):
                    if band >= nb:
                        barriers.append(1 + NTP + BAND_ROWS * (NBW - 1))
                        continue
                    barriers.append(1 + BAND_ROWS * bw + NTP + BAND_ROWS * (NBW - 1 - bw))
                    jc = band * BAND_ROWS + r
                    row_ok = jc < ny
                    jn = np.where(fy, ny - 1 - jc, jc)
                    assert np.all(jn[row_ok] >= 0) and np.all(jn[row_ok] < ny)
                    rd_recv = bw == 0 and band > 0
                    assert not rd_recv or XW, "a band reads the group below without a receiving wave"
                    part_base = (qc * nb + band) * NT * 64
                    pg0 = slots[w * CHANNELS * K]
                    wave_on = pg0[0] >= 0
                    gb0 = pg0[1] if wave_on else 0
                    pbase = ((d * G + gb0) * nb + band) * NT * BAND_ROWS
                    tbase = (quad * G + gb0) * gslab + band * NT * BAND_ROWS
                    span = CHANNELS * K * gslab
                    for k in range(K):
                        slot_idx = (w * CHANNELS + ch) * K + k
                        assert np.all(slot_idx < R)
                        pg = [slots[i] for i in slot_idx]
                        act = np.array([p[0] >= 0 for p in pg]) & row_ok
                        gl = np.array([p[1] - gb0 if p[1] >= 0 else 0 for p in pg])
                        g = gb0 + gl
                        assert np.all(g[act] < G) and np.all(gl[act] < CHANNELS * K) and np.all(gl[act] >= 0)
                        cell = gl * gslab + r
                        vo4 = np.where(act, cell * 4 * rs, OOB)
                        assert np.all(vo4[act] < OOB) and np.all(vo4[~act] >= OOB)
                        # intensity and tables over every step (loads clamp t to NT-1)
                        so = t * BAND_ROWS * 4 * rs
                        off = vo4[act][:, None] + so[None, :]
                        assert off.size == 0 or (off.max() < OOB and off.max() + 4 * rs <= span * 4 * rs)
                        el = pbase + (off // (4 * rs))
                        assert el.size == 0 or (el.min() >= 0 and el.max() < n_psi)
                        el = tbase + (off // (4 * rs))
                        assert el.size == 0 or (el.min() >= 0 and el.max() < n_tab)
                        # boundary inflow (y- side at row 0's column for band 0, x- side per row)
                        yside = 4 * ny + (2 * nx if fy else 0)
                        xside = 2 * ny if fx else 0
                        c0 = np.minimum(t, nx - 1)
                        in0 = np.where(fx, nx - 1 - c0, c0)
                        if band == 0:
                            inf_off = (gl[act][:, None] * NB + yside + 2 * in0[None, :])
                            el = (d * G + gb0) * NB + inf_off
                            assert el.size == 0 or (el.max() + 1 < n_inf and inf_off.max() + 1 < CHANNELS * K * NB)
                        jv = np.where(row_ok, jn, 0)
                        ib = (d * G + gb0 + gl) * NB
                        el = ib[act] + xside + 2 * jv[act] + 1
                        assert el.size == 0 or el.max() < n_inf
                        if rd_recv:
                            # row 0 at step tt < nx reads column tt from the receiving wave's
                            # slot (tt & 1), written in interval tt - 1 (column 0: before the
                            # first barrier, interval -1)
                            for c in range(CHANNELS):
                                for tt in range(min(nx, NTP)):
                                    idx = ((((tt & 1) * NW + w) * K + k) * CHANNELS + c) * 2
                                    assert 0 <= idx and idx + 1 < n_recv
                                    assert recv_w[(tt & 1, w, k, c, tt)] == tt - 1
                        # LDS hand-off: written by the top row at step tt (global
                        # iteration 16 bw + tt) into parity tt & 1 of band slot bw
                        for c in range(CHANNELS):
                            if True:   # every band, the top one for the publishing wave
                                for tt in range(NTP):
                                    idx = ((((tt & 1) * NBW + bw) * NW + w) * K + k) * CHANNELS * 2 + c * 2
                                    assert 0 <= idx and idx + 1 < n_hand
                                    hand_w[(tt & 1, bw, w, k, c, tt - (BAND_ROWS - 1))] = BAND_ROWS * bw + tt
                            if bw > 0:
                                # row 0 at step tt < nx reads column tt from parity (tt + 1) & 1 of band slot bw - 1
                                for tt in range(min(nx, NTP)):
                                    idx = (((((tt + 1) & 1) * NBW + bw - 1) * NW + w) * K + k) * CHANNELS * 2 + c * 2
                                    assert 0 <= idx and idx + 1 < n_hand
                                    key = ((tt + 1) & 1, bw - 1, w, k, c, tt)
                                    assert key in hand_w, "a band reads an LDS slot the band below never wrote"
                                    # written in the previous barrier interval, not overwritten since
                                    assert hand_w[key] == BAND_ROWS * bw + tt - 1
                    # moment partials: block 0 stores each step of the band once
                    if NW > 1:
                        for tt in range(NTP):
                            assert ((((tt & 1) * NBW + bw) * NW + w) * 64 + 63) < n_ring
                    if w == 0:
                        idx = part_base + t[:, None] * 64 + lane[None, :]
                        assert idx.max() < n_part
                        part_owner[idx.ravel()] += 1
            if XW:
                # publishing wave: after interval i - 1 it reads the top band's step
                # ts = i - 1 - 16 (NBW - 1) and stores column ts - 15 of the top band
                top = bg * NBW + NBW - 1
                barriers.append(1 + total)
                if top + 1 < nb:
                    tout_base = (qc * nb + top) * R * slot_words
                    for i in range(total + 1):
                        ts = i - 1 - BAND_ROWS * (NBW - 1)
                        col = ts - (BAND_ROWS - 1)
                        if not (0 <= col < nx):
                            continue
                        for sl in range(NSLOT):
                            sc, sk, sw = sl % CHANNELS, (sl // CHANNELS) % K, sl // (CHANNELS * K)
                            assert hand_w[(ts & 1, NBW - 1, sw, sk, sc, col)] == i - 1
                            o = tout_base + (sl * nx + col) * 2 * TW
                            assert o + 2 * TW <= n_trace
                            written[o: o + 2 * TW] += 1
                # receiving wave: column c < nx into slot c & 1 in interval c - 1, from
                # the trace words of band bg NBW - 1 (active slots only); loads of
                # columns past nx - 1 are clamped to it
                barriers.append(1 + total)
                bottom = bg * NBW
                if bottom > 0:
                    tin_base = (qc * nb + bottom - 1) * R * slot_words
                    for sl in range(NSLOT):
                        sc, sk, sw = sl % CHANNELS, (sl // CHANNELS) % K, sl // (CHANNELS * K)
                        if slots[(sw * CHANNELS + sc) * K + sk][0] < 0:
                            continue
                        cols = [min(TRACE_LAG, nx - 1)] + [min(c, nx - 1) for c in range(0, active_iv + 1 + RP)]
                        for c in cols:
                            o = tin_base + (sl * nx + c) * 2 * TW
                            assert o + 2 * TW <= n_trace
                            read_words[o: o + 2 * TW] += 1
            assert len(set(barriers)) == 1, "the waves of a workgroup pass different numbers of barriers"
    # every word the bottom band of a workgroup reads was published by the top
    # band of the workgroup below, once; words nobody reads are never written
    assert np.all(written <= 1), "a trace word is written twice"
    assert np.all(written[read_words > 0] == 1), "a band reads a trace word nobody writes"
    assert np.all(part_owner == 1), "each moment partial has one owner"
    # the finalisation reads (chunk, band, t, node, row) for cells inside the mesh
    for band in range(nb):
        for tt in range(NT):
            rc = np.arange(16)
            ic, jc = tt - rc, band * BAND_ROWS + rc
            ok = (ic >= 0) & (ic < nx) & (jc < ny)
            assert np.all(((NQC - 1) * nb + band) * NT * 64 + tt * 64 + 3 * 16 + rc[ok] < n_part)


def max_waves(rs, K):
    return 8 if rs * K >= 16 else 16


SHAPES = [(1, 1), (9, 1), (1, 20), (37, 35), (16, 16), (17, 33), (64, 48), (20, 130)]
LAUNCH = [(nw, nb, k) for nw, nb, k in itertools.product((1, 2, 4), (1, 2, 4, 8, 16), (1, 2, 4))]


@pytest.mark.parametrize("nx,ny", SHAPES)
@pytest.mark.parametrize("nw,nb,k", LAUNCH)
@pytest.mark.parametrize("rs", [4, 8])
def test_sweep_indexing_in_bounds(nx, ny, nw, nb, k, rs):
    if rs == 8 and k == 4:
        pytest.skip("four groups per lane is an FP32 shape only")
    if nw * nb > max_waves(rs, k):
        pytest.skip("more waves than the shape's register budget allows (rejected by the planner)")
    for G, sn in ((1, 4), (5, 4), (16, 8), (33, 4)):
        if 4 * k * nw > 2 * max(G, 4) and (nw, k) != (1, 1):
            continue
        check_shape(nx, ny, G, sn, nw, nb, k, rs)


def test_sweep_indexing_benchmark_size():
    """The benchmark's 256^2, S8, 16-group sweep in its default and nearby FP32 shapes."""
    for nw, nb, k in ((1, 16, 1), (2, 8, 1), (1, 8, 2), (4, 4, 1)):
        check_shape(256, 256, 16, 8, nw, nb, k, 4)
