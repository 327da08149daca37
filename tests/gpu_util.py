"""Helpers for the GPU tests: storage conversion of test inputs (so the
oracle sees exactly the rounded values the kernels read) and a shared
context.  No method arithmetic here."""
import numpy as np
import torch


def to_storage(z: np.ndarray, prec: str, device="cuda:0"):
    """(device tensor in the engine's complex storage, the stored values as
    complex128)."""
    z = np.ascontiguousarray(z, dtype=np.complex128)
    if prec == "c64":
        t = torch.from_numpy(z.astype(np.complex64)).to(device)
        torch.cuda.synchronize()   # the library runs on its own stream
        return t, t.cpu().numpy().astype(np.complex128)
    dt = torch.float16 if prec.startswith("f16") else torch.bfloat16
    ri = torch.from_numpy(np.stack([z.real, z.imag], axis=-1).astype(np.float32)).to(dt)
    back = ri.to(torch.float64).numpy()
    words = ri.contiguous().view(torch.int32).reshape(z.shape).to(device)
    torch.cuda.synchronize()
    return words, back[..., 0] + 1j * back[..., 1]


def from_storage(t: torch.Tensor, prec: str, scale_log2: int = 0) -> np.ndarray:
    if prec == "c64":
        return t.cpu().numpy().astype(np.complex128)
    dt = torch.float16 if prec.startswith("f16") else torch.bfloat16
    ri = t.cpu().contiguous().view(dt).reshape(*t.shape, 2).to(torch.float64).numpy()
    return (ri[..., 0] + 1j * ri[..., 1]) * (2.0 ** scale_log2)


def empty_storage(shape, prec, device="cuda:0"):
    t = torch.zeros(shape, dtype=torch.complex64 if prec == "c64" else torch.int32, device=device)
    torch.cuda.synchronize()
    return t
