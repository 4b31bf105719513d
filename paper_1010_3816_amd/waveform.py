"""The field from its azimuthal modes: all modes m = m_min .. m_max of one
(a, s) problem evolved as one batch and summed at observers,
Psi(t, r*, theta, phi) = sum_m e^{i m phi} r^3 Phi_m(t, r*, theta)
(Sec. 3.2: the field is expanded in e^{i m phi} modes, Psi = e^{i m phi} r^3
Phi for each, and the modes evolve independently).

Every mode is one member of a TeukBatch with the same grid, time step and
observers; the batch is sampled after every `sample_every` steps with one
extraction launch, and the mode sum runs in the library
(teuk_assemble_modes).  This module only moves tensors between the calls.
"""
import numpy as np

from . import binding


class ModeSet:
    """Modes m_values of one problem, advanced together.

    observers: list of (rstar, theta, phi)."""

    def __init__(self, a, s, m_values, nr, ntheta, rstar_min, rstar_max, dt, observers, device=None):
        import torch

        self.torch = torch
        self.m_values = [int(m) for m in m_values]
        if len(set(self.m_values)) != len(self.m_values):
            raise ValueError("mode numbers must be distinct")
        obs = np.asarray(observers, dtype=np.float64).reshape(-1, 3)
        self.observers = obs
        members = [dict(a=a, s=s, m=m, nr=nr, ntheta=ntheta, rstar_min=rstar_min, rstar_max=rstar_max, dt=dt,
                        extract_rstar=obs[:, 0].tolist(), extract_theta=obs[:, 1].tolist()) for m in self.m_values]
        self.batch = binding.TeukBatch(members, device=device)
        self.radius = np.array([binding.teuk_radius(a, rs) for rs in obs[:, 0]])
        self.shape = (ntheta, nr)

    def set_initial_data(self, m, phi0, pi0):
        self.batch.set_initial_data(self.m_values.index(int(m)), phi0, pi0)

    def evolve(self, n_samples, sample_every=1):
        """Advance n_samples * sample_every steps; returns the mode samples,
        complex128 [n_samples][n_modes][n_obs], after every sample_every steps."""
        out = self.torch.empty((int(n_samples), len(self.m_values), len(self.observers)),
                               dtype=self.torch.complex128, device=self.batch.device)
        for k in range(int(n_samples)):
            self.batch.step(sample_every)
            self.batch.extract(out[k].view(-1))
        return out

    def assemble(self, samples):
        """Psi at the observers, complex128 [n_samples][n_obs]."""
        samples = samples.contiguous()
        psi = self.torch.empty((samples.shape[0], len(self.observers)), dtype=self.torch.complex128,
                               device=samples.device)
        return binding.teuk_assemble_modes(samples, self.m_values, self.observers[:, 2], self.radius, psi,
                                           self.batch.stream)

    def close(self):
        self.batch.close()
