"""Checkpointed energy sweeps: the energies of a long sweep are solved in chunks, each chunk's outputs
written to `directory/chunk_<i>.npz` as it completes, with `index.json` describing the sweep.  A later
call with the same directory, energies and chunk size loads the finished chunks and solves only the
rest, so an interrupted sweep resumes where it stopped.  Files are plain numpy arrays (loaded without
pickle) and JSON."""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

OUTPUT_KEYS = ("gr", "gl", "trans", "spectral", "status")


def _digest(energies: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(energies, dtype=np.float64).tobytes()).hexdigest()


def sweep(ctx, tree, energies, directory, chunk=64, solve_fn=None, **solve_kw) -> dict:
    """Solve `energies` (host array) in chunks of `chunk` through `solve_fn` (default: the binding's
    solve) with `solve_kw`; returns host arrays of every output the solve produced, in energy order.
    Raises ValueError when `directory` holds a different sweep (other energies, chunk size or sites)."""
    if solve_fn is None:
        from .hsc import solve as solve_fn
    import torch
    E = np.ascontiguousarray(energies, dtype=np.float64).ravel()
    if chunk < 1:
        raise ValueError("chunk must be >= 1")
    os.makedirs(directory, exist_ok=True)
    index_path = os.path.join(directory, "index.json")
    meta = {"energies_sha256": _digest(E), "n_energies": int(E.size), "chunk": int(chunk), "sites": int(tree.n),
            "want": int(solve_kw.get("want", -1))}
    if os.path.exists(index_path):
        with open(index_path) as f:
            old = json.load(f)
        if {k: old.get(k) for k in meta} != meta:
            raise ValueError(f"{directory} holds another sweep ({old}); expected {meta}")
    else:
        with open(index_path, "w") as f:
            json.dump({**meta, "done": []}, f)
    n_chunks = (E.size + chunk - 1) // chunk
    parts = []
    for i in range(n_chunks):
        path = os.path.join(directory, f"chunk_{i}.npz")
        if os.path.exists(path):
            with np.load(path, allow_pickle=False) as z:
                parts.append({k: z[k] for k in z.files})
            continue
        e = torch.as_tensor(E[i * chunk:(i + 1) * chunk], dtype=torch.float64, device=ctx.torch_device)
        out = solve_fn(ctx, tree, e, **solve_kw)
        host = {k: out[k].cpu().numpy() for k in OUTPUT_KEYS if k in out}
        tmp = path + ".part.npz"
        np.savez(tmp, **host)
        os.replace(tmp, path)   # a chunk file exists only once complete
        with open(index_path) as f:
            idx = json.load(f)
        idx["done"] = sorted(set(idx.get("done", [])) | {i})
        with open(index_path + ".part", "w") as f:
            json.dump(idx, f)
        os.replace(index_path + ".part", index_path)
        parts.append(host)
    keys = [k for k in OUTPUT_KEYS if parts and k in parts[0]]
    return {k: np.concatenate([p[k] for p in parts]) for k in keys}
