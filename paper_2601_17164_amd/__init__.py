"""MI355X-native hot path of the semiclassical strong-field Herman-Kluk (SFHK) method."""
