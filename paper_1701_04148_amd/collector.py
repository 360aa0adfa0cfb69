"""Streaming Slim export to a collector in another process.

In the paper's deployment (Sections 1 and 3) a measurement point keeps both
subsketches and sends only the Slim-subsketch to a remote collector.  The
collector answers point queries from it with the query rule of Section 3.1:
the smallest of the key's d Slim counters.  This module is that hand-off on
one host:

* a ring of frames in POSIX shared memory, each able to hold one Slim
  snapshot ([d][w] uint16 after a 64-byte header), and a duplex pipe for
  control messages;
* ``Collector`` (producer side): ``publish`` exports a sketch's Slim with
  sf_export_slim straight into a free frame (one device-to-host copy), then
  names the frame, the sketch and its shape in a message.  ``query`` asks the
  collector for answers;
* ``collector_main`` (the collector process, started with "spawn"): copies
  every published Slim into its own device buffer, keeping the latest one per
  sketch, and hands the frame back.  It answers queries with sf_query_slim on
  its own stream.

The producer never writes to a frame the collector still holds: it blocks
until one comes back.  Each frame header repeats the sequence number and
shape, so a frame can never be read for the wrong message.  Every wait on the
pipe has a time limit; an error in the collector comes back as an exception
and is never left as a hang.
"""
from __future__ import annotations

import os
import struct
import time

import numpy as np

HEADER = 64                                    # bytes before a frame's payload
_MAGIC = 0x534C494D                            # "SLIM"
_HDR = struct.Struct("<IIQIIIII")              # magic, sketch, seq, d, w, z, key_bytes, seed_base


def frame_bytes(d: int, w: int) -> int:
    """Bytes of one frame holding a [d][w] uint16 Slim, rounded to 4 KiB."""
    return (HEADER + 2 * d * w + 4095) & ~4095


def write_header(buf, off: int, sketch: int, seq: int, shape) -> None:
    _HDR.pack_into(buf, off, _MAGIC, sketch, seq, *shape)


def read_header(buf, off: int):
    """(sketch, seq, (d, w, z, key_bytes, seed_base)) of the frame at off."""
    magic, sketch, seq, d, w, z, kb, seed = _HDR.unpack_from(buf, off)
    if magic != _MAGIC:
        raise ValueError("not a Slim frame")
    return sketch, seq, (d, w, z, kb, seed)


class FrameRing:
    """Which frames the producer may write: a frame is free until published,
    then held by the collector until it reports the frame loaded."""

    def __init__(self, frames: int):
        if frames < 1:
            raise ValueError("need at least one frame")
        self.free = list(range(frames))[::-1]
        self.held: dict[int, int] = {}          # frame -> seq in flight

    def take(self, seq: int) -> int:
        if not self.free:
            raise RuntimeError("no free frame")
        f = self.free.pop()
        self.held[f] = seq
        return f

    def give_back(self, frame: int, seq: int) -> None:
        if self.held.get(frame) != seq:
            raise RuntimeError(f"frame {frame} returned for seq {seq}, holds {self.held.get(frame)}")
        del self.held[frame]
        self.free.append(frame)


def collector_main(conn, shm_name: str, frames: int, fbytes: int, device: int) -> None:
    """The collector process: load published Slim snapshots, answer queries."""
    from multiprocessing import shared_memory
    try:
        import torch
        from . import lib, make_config, sf_query_slim
        torch.cuda.set_device(device)
        lib()                                  # fail here, loudly, if libsf.so is missing
        shm = shared_memory.SharedMemory(name=shm_name)
        stream = torch.cuda.Stream(device=device)
        held: dict[int, tuple] = {}            # sketch -> (cfg, device Slim, seq)
        conn.send(("ready", os.getpid()))
    except Exception as e:  # noqa: BLE001 -- reported to the producer, which raises
        conn.send(("error", f"collector start: {e!r}"))
        return
    try:
        while True:
            msg = conn.recv()
            kind = msg[0]
            if kind == "stop":
                break
            if kind == "slim":
                _, frame, seq, sketch = msg
                off = frame * fbytes
                hs, hq, shape = read_header(shm.buf, off)
                if (hs, hq) != (sketch, seq):
                    raise RuntimeError(f"frame {frame} holds sketch {hs} seq {hq}, message says {sketch} {seq}")
                d, w, z, kb, seed = shape
                src = np.ndarray((d * w,), dtype=np.uint16, buffer=shm.buf, offset=off + HEADER)
                cur = held.get(sketch)
                if cur is None or cur[1].numel() != d * w:
                    dev = torch.empty(d * w, dtype=torch.int16, device=f"cuda:{device}")
                else:
                    dev = cur[1]
                with torch.cuda.stream(stream):
                    dev.copy_(torch.from_numpy(src.view(np.int16)))
                stream.synchronize()
                held[sketch] = (make_config(d, w, z, kb, seed), dev, seq)
                del src
                conn.send(("loaded", frame, seq, time.perf_counter()))
            elif kind == "query":
                _, sketch, raw, key_bytes = msg
                if sketch not in held:
                    conn.send(("error", f"no Slim of sketch {sketch} has been published"))
                    continue
                cfg, dev, seq = held[sketch]
                if key_bytes != cfg.key_bytes:
                    conn.send(("error", f"sketch {sketch} takes {cfg.key_bytes}-byte keys"))
                    continue
                keys_h = np.frombuffer(raw, dtype=np.uint8)
                n = keys_h.size // key_bytes
                with torch.cuda.stream(stream):
                    keys = torch.from_numpy(keys_h.copy()).to(f"cuda:{device}")
                    if key_bytes == 4:
                        keys = keys.view(torch.int32)
                    out = torch.empty(n, dtype=torch.int32, device=f"cuda:{device}")
                    sf_query_slim(dev, cfg, keys, out, stream)
                    ans = out.cpu()
                stream.synchronize()
                conn.send(("answers", sketch, seq, ans.numpy().view(np.uint32).tobytes()))
            else:
                raise RuntimeError(f"unknown message {kind!r}")
    except Exception as e:  # noqa: BLE001
        conn.send(("error", repr(e)))
    finally:
        held.clear()
        torch.cuda.synchronize(device)
        shm.close()


class Collector:
    """Producer-side handle of a collector process for Slims of at most
    max_cells = d*w counters, with `frames` shared-memory frames in flight.
    publish() takes a Sketch (anything with d, w, cfg and export_slim(out))."""

    KEEP_TIMES = 1 << 16                          # snapshots whose times latencies() reports, at most

    def __init__(self, max_cells: int, frames: int = 4, device: int = 0, timeout: float = 300.0):
        import multiprocessing as mp
        from multiprocessing import shared_memory
        self.fbytes = frame_bytes(1, max_cells)
        self.max_cells = max_cells
        self.timeout = timeout
        self.ring = FrameRing(frames)
        self.seq = 0
        self.times: dict[int, list] = {}         # seq -> [export start, export end, loaded]
        self.shm = shared_memory.SharedMemory(create=True, size=frames * self.fbytes)
        ctx = mp.get_context("spawn")
        self.conn, child = ctx.Pipe(duplex=True)
        self.proc = ctx.Process(target=collector_main, args=(child, self.shm.name, frames, self.fbytes, device),
                                daemon=True)
        self.proc.start()
        child.close()
        try:
            msg = self._recv(timeout)
            if msg[0] != "ready":
                raise RuntimeError(f"collector sent {msg[0]!r} before it was ready")
        except BaseException:
            self.close()
            raise
        self.pid = msg[1]

    # ---- pipe
    def _recv(self, timeout: float | None = None):
        if not self.conn.poll(self.timeout if timeout is None else timeout):
            raise TimeoutError("collector did not answer in time")
        msg = self.conn.recv()
        if msg[0] == "error":
            raise RuntimeError(f"collector: {msg[1]}")
        return msg

    def _handle(self, msg):
        if msg[0] == "loaded":
            _, frame, seq, t = msg
            self.ring.give_back(frame, seq)
            self.times[seq][2] = t
            return None
        return msg

    def _wait_for(self, kind: str):
        while True:
            msg = self._handle(self._recv())
            if msg is not None:
                if msg[0] != kind:
                    raise RuntimeError(f"collector sent {msg[0]!r}, expected {kind!r}")
                return msg

    # ---- API
    def publish(self, sketch_id: int, sk) -> int:
        """Export sketch `sk`'s Slim into a free frame and hand it to the
        collector as sketch `sketch_id`.  Returns the snapshot's sequence number."""
        d, w = sk.d, sk.w
        if d * w > self.max_cells:
            raise ValueError(f"Slim of {d * w} counters exceeds the frames' {self.max_cells}")
        while not self.ring.free:
            self._handle(self._recv())
        self.seq += 1
        seq = self.seq
        frame = self.ring.take(seq)
        off = frame * self.fbytes
        view = np.ndarray((d, w), dtype=np.uint16, buffer=self.shm.buf, offset=off + HEADER)
        t0 = time.perf_counter()
        sk.export_slim(view)
        t1 = time.perf_counter()
        del view
        c = sk.cfg
        write_header(self.shm.buf, off, sketch_id, seq, (c.d, c.w, c.z, c.key_bytes, c.seed_base))
        self.times[seq] = [t0, t1, None]
        if len(self.times) > self.KEEP_TIMES:
            self.clear_latencies()
        self.conn.send(("slim", frame, seq, sketch_id))
        return seq

    def drain(self) -> None:
        """Wait until the collector has loaded every published snapshot."""
        while self.ring.held:
            self._handle(self._recv())

    def query(self, sketch_id: int, keys: np.ndarray, key_bytes: int = 4):
        """Answers (uint32) of the collector's latest Slim of sketch_id, and
        that snapshot's sequence number.  keys: uint32 [n] or uint8 [n, 13]."""
        raw = np.ascontiguousarray(keys).tobytes()
        self.conn.send(("query", sketch_id, raw, key_bytes))
        _, sid, seq, ans = self._wait_for("answers")
        return np.frombuffer(ans, dtype=np.uint32).copy(), seq

    def clear_latencies(self) -> None:
        """Forget the times of snapshots already loaded (e.g. a warm-up)."""
        self.times = {q: v for q, v in self.times.items() if v[2] is None}

    def latencies(self) -> dict:
        """Per loaded snapshot: export time (into shared memory) and the time
        from the start of the export until the collector's GPU held it."""
        done = [v for v in self.times.values() if v[2] is not None]
        exp = np.array([v[1] - v[0] for v in done]) * 1e3
        e2e = np.array([v[2] - v[0] for v in done]) * 1e3
        return {"snapshots": len(done), "export_ms": exp, "end_to_end_ms": e2e}

    def close(self) -> None:
        """Stop the collector process and remove the shared memory (idempotent)."""
        proc, self.proc = getattr(self, "proc", None), None
        conn, self.conn = getattr(self, "conn", None), None
        shm, self.shm = getattr(self, "shm", None), None
        try:
            if proc is not None and proc.is_alive():
                try:
                    conn.send(("stop",))
                except OSError:
                    pass
                proc.join(60)
        finally:
            if proc is not None and proc.is_alive():
                proc.terminate()
                proc.join(10)
            if conn is not None:
                conn.close()
            if shm is not None:
                shm.close()
                shm.unlink()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 -- interpreter shutdown
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
