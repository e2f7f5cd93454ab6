"""Detector geometry, antenna patterns and arrival-time delays (oracle side).

The paper projects each simulated signal onto the detectors on the fly from
the sky position and polarisation angle (section 6, where the extrinsic
parameters are applied to waveforms on the GPU) and uses the time difference
of arrival between sites for sky localisation (section 4).  It does not give
the geometry; the standard long-wavelength response is used:

  * site vertex r_d on the WGS-84 ellipsoid (a = 6378137 m,
    f = 1/298.257223563) at the site's geodetic latitude and longitude,
    elevation and arm tilt ignored;
  * arm unit vectors in the local tangent plane, u = cos(z) N + sin(z) E,
    with azimuth z measured from North toward East;
  * detector tensor D = (x x^T - y y^T) / 2;
  * source direction n = (cos d cos a, cos d sin a, sin d) in Earth-fixed
    axes (right ascension taken as longitude: sidereal time 0);
  * polarisation frame p = cos(psi) e_theta + sin(psi) e_phi,
    q = -sin(psi) e_theta + cos(psi) e_phi, with e_theta, e_phi the
    spherical unit vectors at n;  e+ = p p^T - q q^T,  ex = p q^T + q p^T;
  * F+ = D : e+,  Fx = D : ex;
  * delay relative to the geocentre: dt_d = -(n . r_d) / c.

The site coordinates are public survey facts (geodetic latitude, longitude,
arm azimuths).  Pinned by: psi-invariance of F+^2 + Fx^2; the sign flip under
psi -> psi + pi/2; F+^2 + Fx^2 = 1 at the geodetic zenith and 1/4 along an
arm; the published H1-L1 light travel time.
"""

import math

import numpy as np

C_SI = 299792458.0
WGS84_A = 6378137.0
WGS84_F = 1.0 / 298.257223563

# id: (name, latitude deg N, longitude deg E, x-arm azimuth deg, y-arm azimuth deg)
DETECTOR_SITES = {
    0: ("H1", 46.45514, -119.40766, 324.0000, 234.0000),
    1: ("L1", 30.56289, -90.77424, 252.2835, 162.2835),
    2: ("V1", 43.63141, 10.50450, 19.4326, 289.4326),
}


def detector_geometry(det_id):
    """Return (D 3x3 tensor, vertex position r [m]) for detector id 0/1/2."""
    _, lat_d, lon_d, zx_d, zy_d = DETECTOR_SITES[int(det_id)]
    lat, lon = math.radians(lat_d), math.radians(lon_d)
    e2 = WGS84_F * (2.0 - WGS84_F)
    nu = WGS84_A / math.sqrt(1.0 - e2 * math.sin(lat) ** 2)
    r = np.array([nu * math.cos(lat) * math.cos(lon),
                  nu * math.cos(lat) * math.sin(lon),
                  nu * (1.0 - e2) * math.sin(lat)])
    east = np.array([-math.sin(lon), math.cos(lon), 0.0])
    north = np.array([-math.sin(lat) * math.cos(lon),
                      -math.sin(lat) * math.sin(lon),
                      math.cos(lat)])

    def arm(z_deg):
        z = math.radians(z_deg)
        return math.cos(z) * north + math.sin(z) * east

    x, y = arm(zx_d), arm(zy_d)
    D = 0.5 * (np.outer(x, x) - np.outer(y, y))
    return D, r


def source_direction(ra, dec):
    return np.array([math.cos(dec) * math.cos(ra),
                     math.cos(dec) * math.sin(ra),
                     math.sin(dec)])


def polarisation_tensors(ra, dec, psi):
    e_theta = np.array([math.sin(dec) * math.cos(ra),
                        math.sin(dec) * math.sin(ra),
                        -math.cos(dec)])
    e_phi = np.array([-math.sin(ra), math.cos(ra), 0.0])
    p = math.cos(psi) * e_theta + math.sin(psi) * e_phi
    q = -math.sin(psi) * e_theta + math.cos(psi) * e_phi
    e_plus = np.outer(p, p) - np.outer(q, q)
    e_cross = np.outer(p, q) + np.outer(q, p)
    return e_plus, e_cross


def antenna_patterns(D, ra, dec, psi):
    """(F+, Fx) of a detector with tensor D for a source at (ra, dec, psi)."""
    e_plus, e_cross = polarisation_tensors(ra, dec, psi)
    return float(np.sum(D * e_plus)), float(np.sum(D * e_cross))


def time_delays(r, ra, dec):
    """Arrival time at vertex r minus arrival time at the geocentre [s]."""
    return float(-np.dot(source_direction(ra, dec), r) / C_SI)
