"""Upload helpers: place a CSR system in torch-owned GPU memory and wrap it
for the library.  Marshalling only; the tensors are kept alive by the
returned objects for as long as the wrappers exist."""
from __future__ import annotations

import numpy as np

from . import (apcg_mat_destroy, apcg_mat_wrap_csr, apcg_vec_destroy, apcg_vec_wrap)


class DeviceVec:
    """A float64 GPU tensor and its library wrapper."""

    def __init__(self, data, device: int = 0):
        import torch

        if isinstance(data, torch.Tensor):
            t = data.to(device=f"cuda:{device}", dtype=torch.float64).contiguous()
        else:
            t = torch.from_numpy(np.ascontiguousarray(data, dtype=np.float64)).to(f"cuda:{device}")
        # the copy is on torch's stream; the library's streams start after it
        torch.cuda.current_stream(device).synchronize()
        self.t = t
        self.n = t.numel()
        self.h = apcg_vec_wrap(t)

    @classmethod
    def zeros(cls, n: int, device: int = 0):
        import torch

        return cls(torch.zeros(n, dtype=torch.float64, device=f"cuda:{device}"), device)

    def numpy(self):
        """Host copy through the library accessor (waits on the last writer)."""
        from . import apcg_vec_copy_to_host

        return apcg_vec_copy_to_host(self.h, self.n)

    def close(self):
        if self.h is not None:
            apcg_vec_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceCSR:
    """CSR arrays in GPU tensors and their library wrapper."""

    def __init__(self, A, device: int = 0):
        import torch

        dev = f"cuda:{device}"
        self.n = int(A.n)
        self.nnz = int(A.rowptr[-1])
        self.rowptr = torch.from_numpy(np.ascontiguousarray(A.rowptr, dtype=np.int32)).to(dev)
        self.col = torch.from_numpy(np.ascontiguousarray(A.col, dtype=np.int32)).to(dev)
        self.val = torch.from_numpy(np.ascontiguousarray(A.val, dtype=np.float64)).to(dev)
        torch.cuda.current_stream(device).synchronize()
        self.h = apcg_mat_wrap_csr(self.rowptr, self.col, self.val, host_rowptr=np.asarray(A.rowptr, np.int32))

    @classmethod
    def from_tensors(cls, rowptr, col, val, device: int = 0):
        """Wraps CSR arrays that already live in torch tensors (moved to the
        device if they are not there yet)."""
        import torch

        dev = f"cuda:{device}"
        obj = cls.__new__(cls)
        obj.rowptr = rowptr.to(device=dev, dtype=torch.int32).contiguous()
        obj.col = col.to(device=dev, dtype=torch.int32).contiguous()
        obj.val = val.to(device=dev, dtype=torch.float64).contiguous()
        obj.n = int(obj.rowptr.numel() - 1)
        obj.nnz = int(obj.val.numel())
        host_rowptr = obj.rowptr.cpu().numpy()
        torch.cuda.current_stream(device).synchronize()
        obj.h = apcg_mat_wrap_csr(obj.rowptr, obj.col, obj.val, host_rowptr=host_rowptr)
        return obj

    def close(self):
        if self.h is not None:
            apcg_mat_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
