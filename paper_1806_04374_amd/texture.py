"""Texture classification pipeline of Sec. III-B ("Classifier") over the C ABI.

One dictionary per class is learned with R-K-SVD from training windows of that class's
images; every window of an image is labelled with the class whose dictionary codes it
with the smallest squared error; an image's feature is its label histogram (as
frequencies); a test image takes the class of its chi^2-nearest training image.  Every
step runs in the library's kernels (rsc_project_images, rsc_rksvd_train, rsc_classify,
rsc_label_histogram, rsc_chi2_nearest); this module only arranges the calls.
"""
from __future__ import annotations

import numpy as np

from . import rsc


def upload_batch(images, N: int, device):
    """Host images (a list of 2-D arrays) packed back to back on the device.  Returns
    (ImageBatch, pixels)."""
    import torch
    batch = rsc.ImageBatch([im.shape for im in images], N, device)
    pix = torch.from_numpy(np.concatenate([np.asarray(im, np.float32).ravel() for im in images])).to(device)
    return batch, pix


def window_offsets(batch, device):
    """Device int64 [n + 1]: first window of each image in rsc_project_images' numbering."""
    import torch
    off = np.zeros(batch.n + 1, np.int64)
    off[1:] = np.cumsum(batch.patches_per_image)
    return torch.from_numpy(off).to(device)


class TextureClassifier:
    """Per-class rotational dictionaries, label-histogram features, chi^2 1-NN."""

    def __init__(self, N: int, S: int, T: int, R: int, K: int, prec: str = "fp32", annular: bool = False):
        """annular: the classes use the paper's annular basis at N (S and T are then unused;
        FP32 only)."""
        if annular and prec != "fp32":
            raise ValueError("the annular basis is FP32 only")
        self.N, self.S, self.T, self.R, self.K, self.prec = N, S, T, R, K, prec
        self.annular = annular
        self.handles: list[rsc.Handle] = []
        self.dictionaries: list[np.ndarray] = []
        self.histories: list[np.ndarray] = []
        self.train_hist = None
        self.train_class = None

    def learn(self, class_windows, M: int, n_iter: int, seed: int = 0):
        """class_windows[c]: device [P_c, B] hat coordinates of class c's training windows.
        Each dictionary starts from M of its windows (unit norm) and runs n_iter rounds."""
        rng = np.random.default_rng(seed)
        for c, xh in enumerate(class_windows):
            pick = np.sort(rng.choice(xh.shape[0], M, replace=False))
            d0 = xh[pick].cpu().numpy().astype(np.float64)
            d0 /= np.maximum(np.linalg.norm(d0, axis=1, keepdims=True), 1e-30)
            h = rsc.rsc_create_annular(self.N) if self.annular else rsc.rsc_create(self.N, self.S, self.T, prec=self.prec)
            D, _, hist = rsc.rsc_rksvd_train(h, xh, d0.astype(np.float32), self.R, self.K, n_iter)
            rsc.rsc_set_dictionary(h, D, self.R)
            self.handles.append(h)
            self.dictionaries.append(D)
            self.histories.append(hist)

    def features(self, xhat, offsets, workspace=None, stream=None):
        """Label histograms [n_images, C] (device) of the windows xhat grouped by offsets."""
        label, _ = rsc.rsc_classify(self.handles, xhat, self.K, workspace=workspace, stream=stream)
        return rsc.rsc_label_histogram(label, offsets, len(self.handles), stream=stream)

    def fit(self, train_hist, train_class):
        self.train_hist = train_hist
        self.train_class = np.asarray(train_class)

    def predict(self, test_hist, stream=None):
        nearest, dist = rsc.rsc_chi2_nearest(self.train_hist, test_hist, stream=stream)
        return nearest, dist

    def close(self):
        for h in self.handles:
            h.close()
        self.handles = []
